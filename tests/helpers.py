"""Shared set-up of test problems: inputs only (meshes, states, tableaux, levels)."""
import numpy as np

from paper_2507_04991_amd import tableau as T
from paper_2507_04991_amd import workloads as W


def problem_2d(nx=10, ny=6, order=2, E=(3, 6), flux=0, levels="cfl", seed=0, ic="vortex", box=10.0):
    f = [W.graded_faces(nx, 0, box), W.graded_faces(ny, 0, box)]
    co = W.node_coords(f)
    if ic == "vortex":
        U0 = W.vortex_state(co, centre=(box / 2, box / 2), box=(0.0, box))
    elif ic == "blast":
        U0 = W.weak_blast_x_state([co[0] - box / 2, co[1]])
    else:
        U0 = W.random_smooth_state(co, seed=seed)
    tab = T.get_tableau(order, list(E))
    dt, lev = T.assign_levels(tab, W.element_widths(f).min(axis=1), W.max_wave_speed(U0, 2))
    lev = pick_levels(levels, lev, len(E), len(lev), seed)
    dt = min(dt, stable_dt(tab, f, U0, lev))
    return f, U0, tab, dt, lev


def stable_dt(tab, f, U0, lev, cfl=0.5):
    """Largest step every element's level is stable for (local CFL of its own level)."""
    dim = len(f)
    ratio = W.element_widths(f).min(axis=1) / W.max_wave_speed(U0, dim)
    return cfl * float(np.min(np.asarray(tab["h_stab"])[lev] * ratio))


def problem_3d(n=(4, 4, 6), order=4, E=(5, 9, 14), flux=0, levels="cfl", seed=0, mach=0.3):
    f = [W.graded_faces(k, 0, 2 * np.pi) for k in n]
    co = W.node_coords(f)
    rng = np.random.default_rng(seed)
    U0 = W.taylor_green_state(co, mach=mach, phase=tuple(rng.uniform(0, 2 * np.pi, 3)))
    tab = T.get_tableau(order, list(E))
    dt, lev = T.assign_levels(tab, W.element_widths(f).min(axis=1), W.max_wave_speed(U0, 3))
    lev = pick_levels(levels, lev, len(E), len(lev), seed)
    dt = min(dt, stable_dt(tab, f, U0, lev))
    return f, U0, tab, dt, lev


def pick_levels(kind, lev, R, n, seed):
    if kind == "cfl":
        return lev
    if kind == "random":
        return np.random.default_rng(seed + 17).integers(0, R, size=n).astype(np.int32)
    if kind == "roundrobin":
        return (np.arange(n) % R).astype(np.int32)
    if kind == "single":  # every element on the largest-E level: the single-level method
        return np.full(n, R - 1, dtype=np.int32)
    if kind == "lowest":  # every element on the smallest-E level: the stages in between have no active element
        return np.zeros(n, dtype=np.int32)
    raise ValueError(kind)


def rel_err(a, b):
    """Relative error of the whole state vector in the max norm: max |a - b| / max |b|."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def field_errors(a, b):
    """Per-field max |a - b| / max |b| (reported, not asserted)."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return [float(np.abs(a[v] - b[v]).max() / max(np.abs(b[v]).max(), 1e-300)) for v in range(b.shape[0])]


def flux_scale(U, dim, gam=W.GAMMA):
    """Largest magnitude of the physical Euler flux over all nodes, fields and directions."""
    rho = U[0]
    vel = [U[1 + d] / rho for d in range(dim)]
    p = (gam - 1.0) * (U[dim + 1] - 0.5 * rho * sum(v * v for v in vel))
    m = 0.0
    for d in range(dim):
        m = max(m, np.abs(U[1 + d]).max())
        for k in range(dim):
            m = max(m, np.abs(U[1 + k] * vel[d] + (p if k == d else 0.0)).max())
        m = max(m, np.abs((U[dim + 1] + p) * vel[d]).max())
    return float(m)


def mixed_step_amplification(tab, cfl=0.5, all_stages=False):
    """Bound factor A of one mixed-precision step: |U_{n+1} - U_{n+1}^exact| <= A dt B
    when every single-precision stage right-hand side is within B of the exact one.

    Linearised stage chain (the test equation U' = lambda U, per level): an error e
    in K_j enters U_{n,k} = U_n + dt((c_k - a_k) K_1 + a_k K_{k-1}) of the later
    stages and so U_{n+1} = U_n + dt sum_k b_k K_k as dt R_j(z) e, z = dt lambda,
    R_j = sum_k b_k dK_k with dK_j = 1, dK_k = z ((c_k - a_k) dK_1 + a_k dK_{k-1}).
    A = max over levels of sum over the level's single-precision stages (b_j = 0,
    or every stage with all_stages) of max |R_j(z)| over z on the model spectrum
    scaled to the level's step (cfl h_stab).  Every stage of a level evaluates
    the same error bound, so the sum is the worst case."""
    c, b = np.asarray(tab["c"]), np.asarray(tab["b"])
    S = len(c)
    spec = T.model_spectrum()
    best = 0.0
    for r, E in enumerate(tab["E"]):
        a = np.asarray(tab["a_sub"][r])
        z = cfl * float(tab["h_stab"][r]) * spec
        z = np.concatenate([z, np.conj(z)])
        total = 0.0
        for j in [0] + list(range(S - E + 1, S)):
            if b[j] != 0.0 and not all_stages:
                continue
            dK = [np.zeros_like(z) for _ in range(S)]
            dK[j] = np.ones_like(z)
            for k in range(j + 1, S):
                ak = a[k] if k >= 2 else 0.0
                dK[k] = z * ((c[k] - ak) * dK[0] + ak * dK[k - 1])
            total += float(np.abs(sum(b[k] * dK[k] for k in range(S))).max())
        best = max(best, total)
    return best
