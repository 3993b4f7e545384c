"""Launch shapes through the C ABI: every stage launched with 1, 2, 4 or 8
wavefronts per workgroup (options.tune = -w), the active lists built with
every element tile (options.tile = 1..4), and the Euler stages with the EC
fluxes and the GLM-MHD stages run with two directions per phase or one direction
at a time (options.phases = 1, 2), give bit-identical states; so does the autotuner's own choice (tune = 1,
tile = 0, phases = 0), which the tuning report names.

In 2D the active lists keep tiles of each case mesh together and a neighbour that
sits in the same workgroup is read from LDS instead of global memory, so the split
between the two paths changes with the workgroup size.  Cases: three case meshes
whose sizes are not multiples of the tile (partial tiles, periodic wrap inside a
tile, a 2 x 2 mesh whose two x neighbours are the same element), random levels
(partial active lists at the middle stages), FP64 and mixed precision; a 3D mesh
for comparison.  The FP64 states are also checked against the oracle per case.
"""
import numpy as np
import pytest

from tests.helpers import rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

WPB = (1, 2, 4, 8)


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_04991_amd import perrk
    perrk.lib()
    return perrk


def ensemble_2d():
    from paper_2507_04991_amd import tableau as T
    from paper_2507_04991_amd import workloads as W
    tab = T.get_tableau(3, [4, 6, 8, 12])
    rng = np.random.default_rng(11)
    faces, U0s, levs, dts = [], [], [], []
    for n in ((13, 9), (2, 2), (10, 6)):
        fy = W.graded_faces(n[1], 0, 10) if n[1] % 2 == 0 and n[1] >= 4 else W.uniform_faces(n[1], 0, 10)
        f = [W.uniform_faces(n[0], 0, 10), fy]
        U0 = W.vortex_state(W.node_coords(f), strength=rng.uniform(1, 4), centre=tuple(rng.uniform(3, 7, 2)))
        dt, _ = T.assign_levels(tab, W.element_widths(f).min(axis=1), W.max_wave_speed(U0, 2))
        lev = rng.integers(0, len(tab["E"]), size=n[0] * n[1]).astype(np.int32)
        ratio = W.element_widths(f).min(axis=1) / W.max_wave_speed(U0, 2)
        dt = min(dt, 0.5 * float(np.min(np.asarray(tab["h_stab"])[lev] * ratio)))
        faces.append(f), U0s.append(U0), levs.append(lev), dts.append(dt)
    return tab, faces, U0s, levs, dts


def run(P, tab, faces, U0s, levs, dts, precision, w, nsteps=3, tile=1, phases=1, flux=0):
    d = P.Descriptors(faces, levs, tab, precision=precision, surface_flux=flux)
    st = P.Stepper(d, P.default_options(tune=-w, tile=tile, phases=phases) if w > 0 else P.default_options())
    u = torch.tensor(np.concatenate(U0s, axis=1), device="cuda").contiguous()
    gam = []
    for _ in range(nsteps):
        infos = st.step(u, np.array(dts))
        assert all(i["flags"] == 0 for i in infos)
        gam.append([i["gamma"] for i in infos])
    out = u.cpu().numpy()
    if w > 0:
        assert "(not tuned)" in st.tuning() and f"stage_waves_per_workgroup=[{','.join([str(w)] * len(tab['c']))}]" \
            in st.tuning(), st.tuning()
        od = int(phases == 2 and flux == 0)
        assert f"stage_one_direction_at_a_time=[{','.join([str(od)] * len(tab['c']))}]" in st.tuning(), st.tuning()
    else:
        assert "Chosen: tile" in st.tuning(), st.tuning()
    st.close()
    return out, np.array(gam)


@pytest.mark.parametrize("precision", [0, 1])
def test_2d_states_identical_for_every_workgroup_size(P, oracle, precision):
    tab, faces, U0s, levs, dts = ensemble_2d()
    res = {}
    for w in WPB:
        print(f"case 2d ensemble precision={precision} waves per workgroup {w}", flush=True)
        res[w] = run(P, tab, faces, U0s, levs, dts, precision, w)
    for w in WPB[1:]:
        assert np.array_equal(res[w][0], res[1][0]), w
        assert np.array_equal(res[w][1], res[1][1]), w
    if precision == 0:
        Ug, off = res[1][0], 0
        for f, U0, lev, dt in zip(faces, U0s, levs, dts):
            t = oracle.Tableau(tab["order"], tab["c"], tab["b"], tab["a_sub"], tab["E"])
            Uref, _, _ = oracle.run(oracle.Mesh(f), t, lev, U0, dt, 3)
            ne = U0.shape[1]
            assert rel_err(Ug[:, off:off + ne], Uref) < 1e-12
            off += ne


@pytest.mark.parametrize("precision", [0, 1])
def test_3d_states_identical_for_every_workgroup_size(P, precision):
    from tests.helpers import problem_3d
    f, U0, tab, dt, lev = problem_3d(levels="random")
    res = {}
    for w in WPB:
        print(f"case 3d precision={precision} waves per workgroup {w}", flush=True)
        res[w] = run(P, tab, [f], [U0], [lev], [dt], precision, w, nsteps=2)
    for w in WPB[1:]:
        assert np.array_equal(res[w][0], res[1][0]), w
        assert np.array_equal(res[w][1], res[1][1]), w


@pytest.mark.parametrize("dim", ["2d", "3d"])
def test_states_identical_for_every_element_tile(P, dim):
    from tests.helpers import problem_3d
    if dim == "2d":
        tab, faces, U0s, levs, dts = ensemble_2d()
    else:
        f, U0, tab, dt, lev = problem_3d(n=(6, 4, 8), levels="random")
        faces, U0s, levs, dts = [f], [U0], [lev], [dt]
    res = {}
    for tile in range(1, P.TILES + 1):
        print(f"case {dim} mixed precision, element tile {tile}", flush=True)
        res[tile] = run(P, tab, faces, U0s, levs, dts, 1, 4, nsteps=2, tile=tile)
    print(f"case {dim} mixed precision, autotuned", flush=True)
    res[0] = run(P, tab, faces, U0s, levs, dts, 1, 0, nsteps=2)
    for tile in res:
        assert np.array_equal(res[tile][0], res[1][0]), tile
        assert np.array_equal(res[tile][1], res[1][1]), tile


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_2d_states_identical_for_both_phase_structures(P, precision):
    """Quadrilaterals with the EC fluxes: pairs of both directions in one phase
    with the faces in a round of their own, or one direction at a time with the
    faces in the half-empty pair rounds, give the same bits (the same fluxes,
    summed in the same order), at every workgroup size."""
    tab, faces, U0s, levs, dts = ensemble_2d()
    res = {}
    for phases in (1, 2):
        for w in (1, 4, 8):
            print(f"case 2d ensemble precision={precision} phases={phases} waves per workgroup {w}", flush=True)
            res[phases, w] = run(P, tab, faces, U0s, levs, dts, precision, w, nsteps=2, phases=phases)
    for k in res:
        assert np.array_equal(res[k][0], res[1, 1][0]), k
        assert np.array_equal(res[k][1], res[1, 1][1]), k


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_3d_states_identical_for_both_phase_structures(P, precision):
    """Hexahedra with the EC fluxes: z with its faces then x and y in one phase,
    or z, x, y one at a time, each with its faces, give the same bits."""
    from tests.helpers import problem_3d
    f, U0, tab, dt, lev = problem_3d(levels="random")
    res = {}
    for phases in (1, 2):
        for w in (1, 4):
            print(f"case 3d precision={precision} phases={phases} waves per workgroup {w}", flush=True)
            res[phases, w] = run(P, tab, [f], [U0], [lev], [dt], precision, w, nsteps=2, phases=phases)
    for k in res:
        assert np.array_equal(res[k][0], res[1, 1][0]), k
        assert np.array_equal(res[k][1], res[1, 1][1]), k


@pytest.mark.parametrize("setup", ["alfven", "blast"])
def test_glm_mhd_states_identical_for_both_phase_structures(P, setup):
    """GLM-MHD stages with the pair fluxes of both directions per phase and one
    direction at a time (half the pair-flux LDS), at 1 and 2 wavefronts per
    workgroup: the same states and gammas bit for bit (Alfven wave: weak form with
    LLF faces, random levels; 1.5D blast: EC fluxes)."""
    from paper_2507_04991_amd import problems
    prob = problems.alfven(n=16) if setup == "alfven" else problems.mhd_blast()
    res = {}
    for phases in (1, 2):
        for w in (1, 2):
            d = P.Descriptors(prob["faces"], prob["lev"], prob["tab"], gas_gamma=prob["gam"],
                              surface_flux=prob["flux"], volume_integral=prob["volume"], system=1,
                              glm_ch=prob["glm_ch"])
            st = P.Stepper(d, P.default_options(tune=-w, phases=phases))
            u = torch.tensor(prob["U0"], device="cuda").contiguous()
            gam = []
            for _ in range(3):
                infos = st.step(u, prob["dt"])
                assert all(i["flags"] == 0 for i in infos)
                gam.append([i["gamma"] for i in infos])
            od = int(phases == 2)
            assert f"stage_one_direction_at_a_time=[{','.join([str(od)] * len(prob['tab']['c']))}]" in st.tuning()
            res[(phases, w)] = (u.cpu().numpy(), np.array(gam))
            st.close()
    for key, (uu, gg) in res.items():
        assert np.array_equal(uu, res[(1, 1)][0]) and np.array_equal(gg, res[(1, 1)][1]), key


def test_phases_option_ignored_where_it_does_not_apply(P):
    """The HLL surface flux keeps its one phase structure."""
    tab, faces, U0s, levs, dts = ensemble_2d()
    a = run(P, tab, faces, U0s, levs, dts, 1, 4, nsteps=2, phases=1, flux=P.FLUX_HLL)
    b = run(P, tab, faces, U0s, levs, dts, 1, 4, nsteps=2, phases=2, flux=P.FLUX_HLL)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_autotuner_reports_the_phase_structure(P):
    tab, faces, U0s, levs, dts = ensemble_2d()
    d = P.Descriptors(faces, levs, tab, precision=1)
    st = P.Stepper(d, P.default_options())
    u = torch.tensor(np.concatenate(U0s, axis=1), device="cuda").contiguous()
    st.step(u, np.array(dts))
    rep = st.tuning()
    st.close()
    assert "then the same one direction at a time" in rep, rep
    od = rep.split("stage_one_direction_at_a_time=[")[1].split("]")[0].split(",")
    assert len(od) == len(tab["c"]) and set(od) <= {"0", "1"}, rep
