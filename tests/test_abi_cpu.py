"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and its host-side validation accepts good descriptors and
rejects bad ones with PERRK_EINVAL."""
import os
import re

import numpy as np
import pytest

from paper_2507_04991_amd import perrk as P
from paper_2507_04991_amd import tableau as T
from paper_2507_04991_amd import workloads as W

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "perrk.h")


def declared_functions():
    src = open(HDR).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|size_t|const char \*)\s*(perrk_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    L = P.lib()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(P.EXPORTS)
    assert b"gfx950" in L.perrk_version()


def desc(**over):
    f = [W.graded_faces(6, 0, 10), W.graded_faces(4, 0, 10)]
    tab = dict(T.get_tableau(2, [3, 6]))
    tab.update(over.pop("tab", {}))
    lev = over.pop("lev", np.zeros(24, dtype=np.int32))
    return P.Descriptors([f], [lev], tab, **over)


def test_validate_accepts_good_descriptors():
    st, msg = desc().validate(P.default_options())
    assert st == P.OK, msg
    for order, E in [(3, [4, 6, 8, 12]), (4, [5, 9, 14])]:
        d = desc(tab=T.get_tableau(order, E))
        assert d.validate()[0] == P.OK
    # classic RK4: four nonzero weights, one level evaluating every stage
    st, msg = desc(tab=T.classic_rk4()).validate()
    assert st == P.OK, msg


@pytest.mark.parametrize("mutate,expect", [
    (lambda t: t["b"].__setitem__(-1, 0.9), "order 1"),
    (lambda t: t["c"].__setitem__(-1, 0.51), "order 2"),
    (lambda t: t["a_sub"].__setitem__((0, 2), 0.1), "skipped or first evaluated"),
    (lambda t: t["b"].__setitem__(2, 0.1), "needs every level to evaluate stage 3"),
    (lambda t: t["E"].__setitem__(0, 7), "outside"),
])
def test_validate_rejects_bad_tableaux(mutate, expect):
    t = {k: (np.array(v, copy=True) if isinstance(v, (list, np.ndarray)) else v)
         for k, v in T.get_tableau(2, [3, 6]).items()}
    mutate(t)
    st, msg = desc(tab=t).validate()
    assert st == P.EINVAL and expect in msg, msg


def test_validate_rejects_bad_mesh_and_levels():
    d = desc(lev=np.full(24, 5, dtype=np.int32))
    assert d.validate()[0] == P.EINVAL
    d = desc()
    d.faces[3] = d.faces[2]  # non-increasing faces
    assert d.validate()[0] == P.EINVAL
    d = desc(gas_gamma=0.9)
    assert d.validate()[0] == P.EINVAL
    d = desc(surface_flux=7)
    assert d.validate()[0] == P.EINVAL
    d = desc(surface_flux=-1)
    assert d.validate()[0] == P.EINVAL
    for flux in range(5):
        for volume in (0, 1):
            assert desc(surface_flux=flux, volume_integral=volume).validate()[0] == P.OK
    st, msg = desc(volume_integral=2).validate()
    assert st == P.EINVAL and "volume" in msg, msg
    assert desc(surface_flux=P.FLUX_CENTRAL).validate()[0] == P.EINVAL  # central: GLM-MHD only


def test_validate_glm_mhd_descriptors():
    ok = dict(system=P.SYSTEM_GLM_MHD, glm_ch=1.0)
    for flux in (P.FLUX_EC, P.FLUX_LLF, P.FLUX_CENTRAL):
        for volume in (0, 1):
            assert desc(surface_flux=flux, volume_integral=volume, **ok).validate()[0] == P.OK
    for bad, word in [(dict(surface_flux=P.FLUX_HLL), "surface flux"), (dict(precision=P.MIXED), "FP64"),
                      (dict(glm_ch=-1.0), "glm_ch"), (dict(glm_ch=float("nan")), "glm_ch")]:
        st, msg = desc(**dict(ok, **bad)).validate()
        assert st == P.EINVAL and word in msg, msg
    st, msg = desc(system=7).validate()
    assert st == P.EINVAL and "system" in msg, msg


def test_validate_viscous_descriptors():
    ok = dict(viscous=1, mu=0.15, prandtl=0.75)
    assert desc(**ok).validate()[0] == P.OK
    assert desc(bc_x=1, **ok).validate()[0] == P.OK
    for bad, word in [(dict(precision=P.MIXED), "FP64"), (dict(mu=-1.0), "mu"), (dict(prandtl=0.0), "prandtl"),
                      (dict(system=P.SYSTEM_GLM_MHD, glm_ch=1.0), "Euler"), (dict(viscous=2), "viscous")]:
        st, msg = desc(**dict(ok, **bad)).validate()
        assert st == P.EINVAL and word in msg, msg
    st, msg = desc(bc_x=1).validate()  # the shock boundaries need the viscous terms
    assert st == P.EINVAL and "viscous" in msg, msg
    d = desc()
    assert d.validate(P.default_options(fast_passes=0))[0] == P.EINVAL
    assert d.validate(P.default_options(bisect_lo=1.1))[0] == P.EINVAL
    for tune in (1, 0, -1, -2, -4, -8):
        assert d.validate(P.default_options(tune=tune))[0] == P.OK
    for tune in (2, -3, -16):
        st, msg = d.validate(P.default_options(tune=tune))
        assert st == P.EINVAL and "tune" in msg, msg
    for tile in range(0, P.TILES + 1):
        assert d.validate(P.default_options(tile=tile))[0] == P.OK
    for tile in (-1, P.TILES + 1):
        st, msg = d.validate(P.default_options(tile=tile))
        assert st == P.EINVAL and "tile" in msg, msg
    for phases in (0, 1, 2):
        assert d.validate(P.default_options(phases=phases))[0] == P.OK
    for phases in (-1, 3):
        st, msg = d.validate(P.default_options(phases=phases))
        assert st == P.EINVAL and "phases" in msg, msg
    for guess in (P.GUESS_PREV, P.GUESS_MLP, P.GUESS_EXTRAP):
        assert d.validate(P.default_options(guess=guess))[0] == P.OK
    for guess in (-1, 3):
        st, msg = d.validate(P.default_options(guess=guess))
        assert st == P.EINVAL and "guess" in msg, msg


def test_validate_node_limit_and_case_count():
    """All cases together must hold fewer than 2^29 nodes, so that an FP64 field of
    a node array spans less than 4 GiB and its byte range fits a 32-bit buffer
    descriptor (at exactly 2^29 it would wrap to 0).  2D meshes of 2^25 - 1, 2^25
    and 2^25 + 1 quadrilaterals (2^29 - 16, 2^29 and 2^29 + 16 nodes): the first is
    accepted, the other two rejected; a 3D mesh of 2^23 hexahedra (2^29 nodes) is
    rejected too; no cases at all is rejected."""
    from paper_2507_04991_amd import tableau as T
    tab = T.get_tableau(2, [3, 6])
    # 2^25 - 1 = 18631 * 1801, 2^25 = 4096 * 8192, 2^25 + 1 = 8283 * 4051
    for (nx, ny), ok in (((18631, 1801), True), ((4096, 8192), False), ((8283, 4051), False)):
        assert nx * ny * 16 - (1 << 29) in ((-16,) if ok else (0, 16))
        f = [W.uniform_faces(nx, 0, 1), W.uniform_faces(ny, 0, 1)]
        lev = np.zeros(nx * ny, dtype=np.int32)
        st, msg = P.Descriptors([f], [lev], tab).validate()
        assert (st == P.OK) == ok, (nx, ny, msg)
        if not ok:
            assert "2^29" in msg, msg
        del lev
    f = [W.uniform_faces(2048, 0, 1), W.uniform_faces(2048, 0, 1), W.uniform_faces(2, 0, 1)]
    st, msg = P.Descriptors([f], [np.zeros(2048 * 2048 * 2, dtype=np.int32)], tab).validate()
    assert st == P.EINVAL and "2^29" in msg, msg
    d = desc()
    d.mesh.n_cases = 0
    assert d.validate()[0] == P.EINVAL
