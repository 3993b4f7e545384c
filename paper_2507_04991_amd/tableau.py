"""P-ERK tableau construction (host-side preparation, run once per set-up).

Builds the shared abscissae c, shared weights b and the per-level sub-diagonal
coefficients a^{(r)}_{i,i-1} of the archetype tableaux of Appendix A
(second order: Sec. 2.2 example; third order: Shu-Osher based archetype;
fourth order: the one-parameter family with the printed base coefficients).
The free coefficients come from a stability polynomial per level, optimised
for the largest stable step on a model spectrum (Sec. 2.2: the number of free
coefficients of P^{(r)} is E^{(r)} - p).

The model spectrum is the 2D linear advection DGSEM (degree 3, a = (1,1),
Rusanov/upwind surface flux, unit elements), the spectrum the paper uses to
illustrate optimised stability domains.  The optimiser maximises the step h by
bisection; for fixed h it minimises, by a linear program, the largest value of
Re(exp(-i theta_m) P(h lambda)) over spectrum samples and 64 polygon directions
(a polygonal outer bound of |P|).  The stable step reported per level is the
largest h with max |P(h lambda)| <= 1 + STAB_TOL on the samples.

Everything here runs on the host in float64 numpy/scipy.
"""
from __future__ import annotations

import functools
import json
import math
import os

import numpy as np

# |P| tolerance of the stable step: the polygon bound above lets |P| exceed 1 by up to
# 1/cos(pi/64) - 1 = 1.2e-3 near the imaginary axis
STAB_TOL = 2e-3

# fourth-order base coefficients (Appendix A.3)
P4_C_SM2 = 0.479274057836310
P4_A_SM2_NUM = 0.114851811257441
P4_A_SM1 = 0.648906880894214
P4_A_S = 0.0283121635129678


# --------------------------------------------------------------------------
# model spectrum
# --------------------------------------------------------------------------

def _lgl3():
    xi = np.array([-1.0, -1.0 / math.sqrt(5.0), 1.0 / math.sqrt(5.0), 1.0])
    lam = np.array([1.0 / np.prod([xi[j] - xi[k] for k in range(4) if k != j]) for j in range(4)])
    D = np.zeros((4, 4))
    for i in range(4):
        for j in range(4):
            if i != j:
                D[i, j] = (lam[j] / lam[i]) / (xi[i] - xi[j])
        D[i, i] = -D[i].sum()
    q = np.array([1, 5, 5, 1]) / 6.0
    return xi, q, D


@functools.lru_cache(maxsize=None)
def advection_spectrum_1d(n: int = 16) -> np.ndarray:
    """Eigenvalues of the periodic 1D DGSEM (degree 3) for u_t + u_x = 0 with the
    upwind flux on n unit elements (strong form)."""
    _, q, D = _lgl3()
    N = 4 * n
    L = np.zeros((N, N))
    for e in range(n):
        o = 4 * e
        L[o:o + 4, o:o + 4] -= 2.0 * D
        # left face: f* = u of left neighbour's last node; correction (f* - u_0)/q_0
        left = 4 * ((e - 1) % n) + 3
        L[o + 0, left] += 2.0 / q[0]
        L[o + 0, o + 0] -= 2.0 / q[0]
        # right face: upwind flux is the own trace, correction vanishes
    return np.linalg.eigvals(L)


@functools.lru_cache(maxsize=None)
def model_spectrum(n: int = 16, samples: int = 600) -> np.ndarray:
    """Samples of the 2D (a = (1,1)) spectrum lambda_x + lambda_y, upper half plane,
    thinned to at most ``samples`` points while keeping the outer envelope."""
    l1 = advection_spectrum_1d(n)
    l2 = (l1[:, None] + l1[None, :]).ravel()
    l2 = l2[l2.imag >= -1e-12]
    # keep the envelope: for each imaginary band, the points of extreme real part
    bands = np.linspace(0.0, l2.imag.max() * (1 + 1e-9), samples // 2 + 1)
    keep = []
    idx = np.digitize(l2.imag, bands)
    for b in np.unique(idx):
        sel = np.nonzero(idx == b)[0]
        keep.append(sel[np.argmin(l2.real[sel])])
        keep.append(sel[np.argmax(l2.real[sel])])
    pts = np.unique(l2[np.array(keep)])
    return pts


# --------------------------------------------------------------------------
# stability-polynomial optimisation
# --------------------------------------------------------------------------

def _fixed_coeffs(p: int) -> list[float]:
    return [1.0 / math.factorial(j) for j in range(p + 1)]


def _lp_min_max(spec_h, E, p, eq_rows=None, n_dirs=64):
    """min over the free coefficients of max_{k,m} Re(exp(-i theta_m) P(z_k)),
    z_k = h lambda_k, theta_m = 2 pi m / n_dirs: a polygonal outer bound of max_k |P|
    (it exceeds the true maximum by at most a factor 1/cos(pi/n_dirs)).
    Returns (bound, alpha[0..E]).  The monomial basis is scaled by s = max|z|."""
    from scipy.optimize import linprog

    s = max(np.abs(spec_h).max(), 1e-12)
    w = spec_h / s
    nf = E - p
    fixed = np.array(_fixed_coeffs(p)) * s ** np.arange(p + 1)
    pfix = (w[:, None] ** np.arange(p + 1)[None, :]) @ fixed
    if nf == 0:
        return float(np.abs(pfix).max()), np.array(_fixed_coeffs(p))
    pvar = w[:, None] ** np.arange(p + 1, E + 1)[None, :]
    rot = np.exp(-2j * math.pi * np.arange(n_dirs) / n_dirs)
    A = (rot[:, None, None] * pvar[None, :, :]).real.reshape(-1, nf)
    A_ub = np.hstack([A, -np.ones((A.shape[0], 1))])
    b_ub = -(rot[:, None] * pfix[None, :]).real.reshape(-1)
    A_eq = b_eq = None
    if eq_rows is not None:
        rows, rhs = [], []
        for z0, val in eq_rows:
            wz = z0 / s
            rows.append(np.concatenate([wz ** np.arange(p + 1, E + 1), [0.0]]))
            rhs.append(val - np.sum(fixed * wz ** np.arange(p + 1)))
        A_eq, b_eq = np.array(rows), np.array(rhs)
    c = np.zeros(nf + 1)
    c[-1] = 1.0
    res = linprog(c, A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=b_eq,
                  bounds=[(None, None)] * (nf + 1), method="highs")
    if res.status != 0:
        return np.inf, None
    beta = res.x[:nf]
    return float(res.x[-1]), np.concatenate([_fixed_coeffs(p), beta / s ** np.arange(p + 1, E + 1)])


def optimise_polynomial(E: int, p: int, spectrum=None, eq_fn=None, h_hi=None, iters=40):
    """Largest h (and coefficients) with max |P(h lambda)| <= 1 (polygonal bound).
    eq_fn(h) -> list of linear equality rows (z0, value) imposed on P."""
    spec = model_spectrum() if spectrum is None else spectrum
    rho = np.abs(spec).max()
    lo, hi = 0.0, (h_hi if h_hi is not None else 1.5 * E * E / rho + 4.0 / rho)
    best = None
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        val, alpha = _lp_min_max(mid * spec, E, p, None if eq_fn is None else eq_fn(mid))
        if alpha is not None and val <= 1.0:
            lo, best = mid, alpha
        else:
            hi = mid
    if best is None:
        _, best = _lp_min_max(1e-3 * spec, E, p, None if eq_fn is None else eq_fn(1e-3))
        lo = 0.0
    return lo, best


def poly_max_abs(alpha, z) -> float:
    return float(np.abs(np.polyval(np.asarray(alpha)[::-1], z)).max())


# --------------------------------------------------------------------------
# archetype recursions: stability polynomial <-> a_{i,i-1}
# --------------------------------------------------------------------------

def _pmul(a, b):
    return np.convolve(a, b)


def _peel(T, c_i, a_i):
    """Given T = k_i = z + (c_i - a_i) z^2 + a_i z k_{i-1} (coefficient arrays, index =
    power), return k_{i-1}."""
    rest = T.copy()
    rest[1] -= 1.0
    rest[2] -= (c_i - a_i)
    # rest = a_i z k_{i-1}: shift down by one and divide
    return rest[1:] / a_i


def stage_polynomials(c, a_sub_row, E, S):
    """k_i(z) coefficient arrays of one level (for the linear test equation)."""
    k = [None] * S
    k[0] = np.array([0.0, 1.0])
    for i in range(1, S):
        a = a_sub_row[i] if i >= 2 else 0.0
        base = np.zeros(3)
        base[1] = 1.0
        base[2] = c[i] - a
        if a != 0.0:
            kk = np.zeros(len(k[i - 1]) + 1)
            kk[1:] = a * k[i - 1]
            n = max(len(base), len(kk))
            k[i] = np.pad(base, (0, n - len(base))) + np.pad(kk, (0, n - len(kk)))
        else:
            k[i] = base
    return k


def level_polynomial(c, b, a_sub_row, E, S):
    """P(z) = 1 + sum_i b_i k_i(z) of one level."""
    k = stage_polynomials(c, a_sub_row, E, S)
    n = max(len(x) for x in k)
    P = np.zeros(n)
    P[0] = 1.0
    for i in range(S):
        if b[i] != 0.0:
            P[: len(k[i])] += b[i] * k[i]
    return np.trim_zeros(P, "b")


def _chain_down(T, c, a_row, top, first_active):
    """Peel k_top = T down to the first evaluated stage, filling a_row[top..first+1]."""
    for i in range(top, first_active, -1):
        a = T[3] / c[i - 1] if len(T) > 3 else 0.0
        a_row[i] = a
        if a == 0.0:
            raise ValueError("degenerate stability polynomial (zero chain coefficient)")
        T = _peel(T, c[i], a)
    return T


def abscissae(order: int, S: int) -> np.ndarray:
    c = np.zeros(S)
    if order == 2:
        # c_i = (i-1) / (2 (S-1)): reproduces the S = 6 example (c_i = (i-1)/10), c_S = 1/2
        c[:] = np.arange(S) / (2.0 * (S - 1))
    elif order == 3:
        if S == 3:
            c[:] = [0.0, 1.0, 0.5]
        else:
            c[: S - 2] = np.arange(S - 2) / (S - 3.0)
            c[S - 2] = 1.0
            c[S - 1] = 0.5
    elif order == 4:
        assert S >= 5
        c[1: S - 3] = 1.0
        c[S - 3] = P4_C_SM2
        c[S - 2] = 0.5 + math.sqrt(3.0) / 6.0
        c[S - 1] = 0.5 - math.sqrt(3.0) / 6.0
    else:
        raise ValueError(order)
    return c


def weights(order: int, S: int) -> np.ndarray:
    b = np.zeros(S)
    if order == 2:
        b[S - 1] = 1.0
    elif order == 3:
        b[0], b[S - 2], b[S - 1] = 1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0
    elif order == 4:
        b[S - 2] = b[S - 1] = 0.5
    return b


def level_row_from_polynomial(order: int, S: int, E: int, alpha) -> np.ndarray:
    """a_{i,i-1} of one level whose stability polynomial is alpha[0..E]."""
    c = abscissae(order, S)
    a = np.zeros(S)
    first = S - E + 1  # zero-based index of the first evaluated stage after K_1
    P = np.array(alpha, dtype=np.float64)
    if order == 2:
        T = P.copy()
        T[0] = 0.0
        if E > 2:
            _chain_down(T, c, a, S - 1, first)
    elif order == 3:
        if E == 3:
            a[S - 1] = 0.25
            return a
        # P - 1 - 5z/6 - (1/3 - 2 a_S/3) z^2 = k_{S-1} (1/6 + 2 a_S z / 3); the divisor's
        # root z* = -1/(4 a_S) must be a root of the left side.
        def g(aS):
            z = -1.0 / (4.0 * aS)
            return np.polyval(P[::-1], z) - 1.0 - 5.0 * z / 6.0 - (1.0 / 3.0 - 2.0 * aS / 3.0) * z * z
        # scan for sign changes in a_S in (0, 1/4]
        grid = np.linspace(1e-4, 0.25, 4001)
        vals = np.array([g(x) for x in grid])
        roots = []
        for j in range(len(grid) - 1):
            if np.sign(vals[j]) != np.sign(vals[j + 1]):
                lo_, hi_ = grid[j], grid[j + 1]
                for _ in range(100):
                    mid = 0.5 * (lo_ + hi_)
                    if np.sign(g(mid)) == np.sign(g(lo_)):
                        lo_ = mid
                    else:
                        hi_ = mid
                roots.append(0.5 * (lo_ + hi_))
        best = None
        for aS in roots:
            try:
                row = np.zeros(S)
                row[S - 1] = aS
                lhs = P.copy()
                lhs[0] -= 1.0
                lhs[1] -= 5.0 / 6.0
                lhs[2] -= (1.0 / 3.0 - 2.0 * aS / 3.0)
                # polynomial division by (1/6 + 2 aS z / 3), from the top
                deg = len(lhs) - 1
                q = np.zeros(deg)
                rem = lhs.copy()
                for j in range(deg, 0, -1):
                    q[j - 1] = rem[j] / (2.0 * aS / 3.0)
                    rem[j] -= q[j - 1] * 2.0 * aS / 3.0
                    rem[j - 1] -= q[j - 1] / 6.0
                T = q
                _chain_down(T, c, row, S - 2, first)
                score = np.max(np.abs(row))
                if np.all(row >= -1e-14) and (best is None or score < best[0]):
                    best = (score, row)
            except (ValueError, FloatingPointError):
                continue
        if best is None:
            raise ValueError(f"no admissible third-order tableau for E={E}")
        a = best[1]
    elif order == 4:
        a[S - 1] = P4_A_S
        a[S - 2] = P4_A_SM1
        a[S - 3] = P4_A_SM2_NUM / c[S - 4]
        if E == 5:
            return a
        # 2(P-1) - z - (c_S - a_S) z^2 = k_{S-1} (1 + a_S z)
        lhs = 2.0 * P.copy()
        lhs[0] -= 2.0
        lhs[1] -= 1.0
        lhs[2] -= (c[S - 1] - a[S - 1])
        deg = len(lhs) - 1
        q = np.zeros(deg + 1)
        rem = lhs.copy()
        for j in range(deg, 0, -1):
            q[j - 1] = rem[j] / a[S - 1]
            rem[j] -= q[j - 1] * a[S - 1]
            rem[j - 1] -= q[j - 1]
        T = np.trim_zeros(q, "b")
        T = _peel(T, c[S - 2], a[S - 2])
        T = _peel(T, c[S - 3], a[S - 3])
        _chain_down(T, c, a, S - 4, first)
    return a


def p4_equality(h, S):
    """Divisibility condition of the fourth-order construction: with z* = -1/a_S,
    2 (P(z*) - 1) - z* - (c_S - a_S) z*^2 = 0, as a row on P in unscaled z."""
    c = abscissae(4, S)
    z0 = -1.0 / P4_A_S
    val = 1.0 + 0.5 * (z0 + (c[S - 1] - P4_A_S) * z0 * z0)
    return [(z0, val)]


# --------------------------------------------------------------------------
# full tableaux
# --------------------------------------------------------------------------

def build_tableau(order: int, E_levels, spectrum=None):
    """Returns dict(order, S, E, c, b, a_sub, h_stab): h_stab[r] is the optimised
    stable step of level r on the unit model spectrum."""
    E_levels = [int(e) for e in E_levels]
    S = max(E_levels)
    c, b = abscissae(order, S), weights(order, S)
    a_sub = np.zeros((len(E_levels), S))
    hs = []
    for r, E in enumerate(E_levels):
        eq = (lambda h, S=S: p4_equality(h, S)) if (order == 4 and E > 5) else None
        if order == 4 and E == 5:
            row = level_row_from_polynomial(4, S, 5, np.zeros(6))
            P = level_polynomial(c, b, row, 5, S)
            h = _stable_step_of(P, spectrum)
            a_sub[r] = row
            hs.append(h)
            continue
        h, alpha = optimise_polynomial(E, order if order < 4 else 4, spectrum, eq_fn=eq)
        row = level_row_from_polynomial(order, S, E, alpha)
        a_sub[r] = row
        P = level_polynomial(c, b, row, E, S)
        hs.append(_stable_step_of(P, spectrum))
    return dict(order=order, S=S, E=E_levels, c=c, b=b, a_sub=a_sub, h_stab=np.array(hs))


def _stable_step_of(P, spectrum=None, tol=STAB_TOL) -> float:
    """Largest h with max |P(h lambda)| <= 1 + tol on the model spectrum (bisection)."""
    spec = model_spectrum() if spectrum is None else spectrum
    rho = np.abs(spec).max()
    lo, hi = 0.0, 4.0 * len(P) ** 2 / rho
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if poly_max_abs(P, mid * spec) <= 1.0 + tol:
            lo = mid
        else:
            hi = mid
    return lo


def classic_rk4():
    """The classic fourth-order Runge-Kutta method (the paper's relaxed comparison
    method R-RK_{4;4}) in the library's tableau form: one level with E = S = 4,
    c = (0, 1/2, 1/2, 1), b = (1/6, 1/3, 1/3, 1/6), a_{2,1} = 1/2, a_{3,2} = 1/2,
    a_{4,3} = 1 (every row couples to a single earlier stage, so a_{i,1} =
    c_i - a_{i,i-1} with a_sub = (0, 0, 1/2, 1)); h_stab from its stability
    polynomial 1 + z + z^2/2 + z^3/6 + z^4/24 on the model spectrum."""
    P = np.array(_fixed_coeffs(4))
    return dict(order=4, S=4, E=[4], c=np.array([0.0, 0.5, 0.5, 1.0]),
                b=np.array([1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0]),
                a_sub=np.array([[0.0, 0.0, 0.5, 1.0]]), h_stab=np.array([_stable_step_of(P)]))


_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tableaux.json")


def _key(order, E_levels):
    return f"p{order}_E" + "-".join(str(int(e)) for e in E_levels)


def get_tableau(order: int, E_levels):
    """Cached tableau (float64 values stored as hex strings for exact round trips)."""
    key = _key(order, E_levels)
    data = {}
    if os.path.exists(_CACHE):
        with open(_CACHE) as f:
            data = json.load(f)
    if key not in data:
        t = build_tableau(order, E_levels)
        data[key] = dict(order=t["order"], S=t["S"], E=t["E"],
                         c=[float(x).hex() for x in t["c"]], b=[float(x).hex() for x in t["b"]],
                         a_sub=[[float(x).hex() for x in row] for row in t["a_sub"]],
                         h_stab=[float(x).hex() for x in t["h_stab"]])
        with open(_CACHE, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
    d = data[key]
    return dict(order=d["order"], S=d["S"], E=list(d["E"]),
                c=np.array([float.fromhex(x) for x in d["c"]]),
                b=np.array([float.fromhex(x) for x in d["b"]]),
                a_sub=np.array([[float.fromhex(x) for x in row] for row in d["a_sub"]]),
                h_stab=np.array([float.fromhex(x) for x in d["h_stab"]]))


# --------------------------------------------------------------------------
# level assignment
# --------------------------------------------------------------------------

def assign_levels(tab, h_elem, speed_elem, cfl: float = 0.5, geometric: bool = True):
    """Local-CFL level assignment (TimestepConstraintLocal): the step is set by the
    most restrictive element with the largest-E level; each element takes the
    smallest E whose stable step cfl * h_stab(E) * h / speed is >= dt.  With
    geometric=True (the paper's choice: levels from the shortest edge length) one
    speed, the largest over all elements, is used everywhere, so the assignment
    stays valid while the flow moves.  Returns (dt, level index per element)."""
    hs = np.asarray(tab["h_stab"])
    E = np.asarray(tab["E"])
    speed = np.asarray(speed_elem, dtype=np.float64)
    if geometric:
        speed = np.full_like(speed, speed.max())
    ratio = np.asarray(h_elem) / speed
    rmax = int(np.argmax(E))
    dt = cfl * hs[rmax] * ratio.min()
    order = np.argsort(E, kind="stable")
    ok = cfl * hs[order][None, :] * ratio[:, None] >= dt * (1.0 - 1e-12)  # [elem][level by E]
    first = np.argmax(ok, axis=1)
    lev = np.where(ok.any(axis=1), order[first], rmax).astype(np.int32)
    return dt, lev
