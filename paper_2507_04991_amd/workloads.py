"""Seeded synthetic inputs: graded periodic Cartesian meshes and initial states.

This module holds no arithmetic of the time integrator or of the spatial
operator: it only places nodes and evaluates analytic initial conditions.  It
feeds both the HIP path and the CPU oracle so that both start from
bit-identical data.

State layout: float64 array U[v][elem][node]; v = rho, rho v_1..rho v_dim,
rho e; elem = ix + nx (iy + ny iz); node = i + 4 j + 16 k.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 1.4
LGL_XI = np.array([-1.0, -1.0 / math.sqrt(5.0), 1.0 / math.sqrt(5.0), 1.0])


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------

def uniform_faces(n: int, lo: float, hi: float) -> np.ndarray:
    return lo + (hi - lo) * np.arange(n + 1) / n


def graded_faces(n: int, lo: float, hi: float, ratio: float = 4.0) -> np.ndarray:
    """Face coordinates of n cells whose widths grow geometrically from the centre
    (finest) to both ends (coarsest); largest / smallest width = ratio.
    Half the cells have widths h0 q^j, j = 0..n/2-1, q = ratio^(1/(n/2-1)),
    mirrored about the centre."""
    assert n % 2 == 0 and n >= 4
    half = n // 2
    q = ratio ** (1.0 / (half - 1))
    w = q ** np.arange(half)
    w = w * (0.5 * (hi - lo) / w.sum())
    widths = np.concatenate([w[::-1], w])
    f = lo + np.concatenate([[0.0], np.cumsum(widths)])
    f[-1] = hi
    return f


def node_coords(faces) -> list[np.ndarray]:
    """Physical coordinates of every node, one array [elem][node] per direction."""
    dim = len(faces)
    n = [len(f) - 1 for f in faces]
    nelem = int(np.prod(n))
    npe = 4 ** dim
    e = np.arange(nelem)
    l = np.arange(npe)
    eidx = [e % n[0], (e // n[0]) % n[1]] + ([e // (n[0] * n[1])] if dim == 3 else [])
    lidx = [l % 4, (l // 4) % 4] + ([l // 16] if dim == 3 else [])
    out = []
    for d in range(dim):
        f = np.asarray(faces[d], dtype=np.float64)
        left = f[eidx[d]][:, None]
        h = (f[eidx[d] + 1] - f[eidx[d]])[:, None]
        out.append(left + 0.5 * (LGL_XI[lidx[d]][None, :] + 1.0) * h)
    return out


def element_widths(faces) -> np.ndarray:
    """[elem][dim] element widths."""
    dim = len(faces)
    n = [len(f) - 1 for f in faces]
    e = np.arange(int(np.prod(n)))
    eidx = [e % n[0], (e // n[0]) % n[1]] + ([e // (n[0] * n[1])] if dim == 3 else [])
    return np.stack([np.diff(np.asarray(faces[d]))[eidx[d]] for d in range(dim)], axis=1)


def conserved(rho, vel, p, gam=GAMMA) -> np.ndarray:
    kin = 0.5 * rho * sum(v * v for v in vel)
    return np.stack([rho] + [rho * v for v in vel] + [p / (gam - 1.0) + kin]).astype(np.float64)


# --------------------------------------------------------------------------
# initial conditions
# --------------------------------------------------------------------------

def vortex_state(coords, t=0.0, strength=5.0, centre=(5.0, 5.0), box=(0.0, 10.0), radius=1.0,
                 mach=1.0 / math.sqrt(GAMMA), vinf=(1.0, 1.0), gam=GAMMA):
    """Isentropic vortex (Sec. 4.1.2 parametrisation): Gaussian g = exp((1-|c|^2)/(2R^2)),
    rho = (1 - I^2 M^2 (gamma-1) g^2 / (8 pi^2))^(1/(gamma-1)),
    v = v_inf + I g / (2 pi R) (-c_y, c_x), p = rho^gamma / (gamma M^2),
    c = x - x_c - v_inf t taken as the nearest periodic image.
    With I = 5, R = 1, M = 1/sqrt(gamma) this is Shu's vortex; p = rho^gamma."""
    x, y = coords
    L = box[1] - box[0]
    cx = x - centre[0] - vinf[0] * t
    cy = y - centre[1] - vinf[1] * t
    cx = cx - L * np.round(cx / L)
    cy = cy - L * np.round(cy / L)
    g = np.exp((1.0 - (cx * cx + cy * cy)) / (2.0 * radius * radius))
    rho = (1.0 - strength ** 2 * mach ** 2 * (gam - 1.0) * g * g / (8.0 * math.pi ** 2)) ** (1.0 / (gam - 1.0))
    amp = strength * g / (2.0 * math.pi * radius)
    vx = vinf[0] - amp * cy
    vy = vinf[1] + amp * cx
    p = rho ** gam / (gam * mach ** 2)
    return conserved(rho, [vx, vy], p, gam)


def kelvin_helmholtz_state(coords, phase=0.0, rho_inner=1.0, rho_outer=0.5, gam=GAMMA):
    """Kelvin-Helmholtz shear layer on [-1,1]^2 (Sec. 3.2.2 set-up, densities 0.5/1):
    b = tanh(15y + 7.5) - tanh(15y - 7.5), rho = rho_out + (rho_in - rho_out) b / 2,
    v_x = (b - 1)/2, v_y = sin(2 pi x + phase)/10, p = 1."""
    x, y = coords
    b = np.tanh(15.0 * y + 7.5) - np.tanh(15.0 * y - 7.5)
    rho = rho_outer + 0.5 * (rho_inner - rho_outer) * b
    vx = 0.5 * (b - 1.0)
    vy = 0.1 * np.sin(2.0 * math.pi * x + phase)
    p = np.ones_like(x)
    return conserved(rho, [vx, vy], p, gam)


def taylor_green_state(coords, mach=0.1, phase=(0.0, 0.0, 0.0), gam=GAMMA):
    """Taylor-Green vortex on [0, 2 pi]^3 with shifted arguments X = x + phase_x etc.:
    rho = 1, v = (sin X cos Y cos Z, -cos X sin Y cos Z, 0),
    p = 1/(gamma Ma^2) + (cos 2X + cos 2Y)(cos 2Z + 2)/16."""
    X, Y, Z = (coords[d] + phase[d] for d in range(3))
    rho = np.ones_like(X)
    vx = np.sin(X) * np.cos(Y) * np.cos(Z)
    vy = -np.cos(X) * np.sin(Y) * np.cos(Z)
    vz = np.zeros_like(X)
    p = 1.0 / (gam * mach ** 2) + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
    return conserved(rho, [vx, vy, vz], p, gam)


def weak_blast_x_state(coords, gam=GAMMA):
    """Discontinuous weak blast in x only (Sec. 4.1.1 data), on any 2D/3D periodic box
    centred at x = 0: inner |x| <= 0.5: rho 1.1691, v_x 0.1882 sgn(x), p 1.245."""
    x = coords[0]
    inner = np.abs(x) <= 0.5
    rho = np.where(inner, 1.1691, 1.0)
    vx = np.where(inner, 0.1882 * np.sign(x), 0.0)
    p = np.where(inner, 1.245, 1.0)
    vel = [vx] + [np.zeros_like(x) for _ in coords[1:]]
    return conserved(rho, vel, p, gam)


# ---------------------------------------------------------------- viscous shock
def viscous_shock_faces(n: int) -> np.ndarray:
    """[-2, 2] with n cells (n a multiple of 6): cells of width 8/(3n)... more
    precisely n/6 cells in each of [-2, -1] and [1, 2] and 2n/3 cells (half the
    width) in [-1, 1] (the Sec. 4.3.2 refinement by two in the centre)."""
    assert n % 6 == 0
    k = n // 6
    return np.concatenate([np.linspace(-2.0, -1.0, k + 1)[:-1], np.linspace(-1.0, 1.0, 4 * k + 1)[:-1],
                           np.linspace(1.0, 2.0, k + 1)])


def viscous_shock_state(coords, t=0.0, gam=5.0 / 3.0, mu=0.15):
    """Becker's viscous shock (Sec. 4.3.2, Margolin's explicit profile at
    Ma = 2/sqrt(3 - gamma)): rho_0 = 1, shock speed 1, moving in +x; no
    variation in y.  rho = 1/w, v_x = 1 - w, p = p_0/w (1 + (gamma-1)/2 Ma^2 (1 - w^2))
    with w = 1 + (1 - sqrt(1 + 2 chi^2))/(2 chi^2), chi = 2 exp((x - t)/(2 l)),
    p_0 = 1/(gamma Ma^2) and the length scale l = 2 gamma (4/3 mu)/(gamma + 1) of the
    Navier-Stokes-Fourier equations with Stokes stress and Pr = 3/4."""
    x = coords[0]
    Ma = 2.0 / math.sqrt(3.0 - gam)
    p0 = 1.0 / (gam * Ma * Ma)
    ln = 2.0 * gam * (4.0 / 3.0 * mu) / (gam + 1.0)
    chi = 2.0 * np.exp((x - t) / (2.0 * ln))
    w = 1.0 + (1.0 - np.sqrt(1.0 + 2.0 * chi * chi)) / (2.0 * chi * chi)
    rho = 1.0 / w
    vx = 1.0 - w
    p = p0 / w * (1.0 + 0.5 * (gam - 1.0) * Ma * Ma * (1.0 - w * w))
    return conserved(rho, [vx, np.zeros_like(x)], p, gam)


# ---------------------------------------------------------------- ideal GLM-MHD
# u = (rho, rho v_1..3, E, B_1..3, psi), E = p/(gamma-1) + rho |v|^2/2 + |B|^2/2 + psi^2/2

def mhd_conserved(rho, vel3, p, B3, psi, gam=GAMMA) -> np.ndarray:
    kin = 0.5 * rho * sum(v * v for v in vel3)
    mag = 0.5 * sum(b * b for b in B3)
    E = p / (gam - 1.0) + kin + mag + 0.5 * psi * psi
    return np.stack([rho] + [rho * v for v in vel3] + [E] + list(B3) + [psi]).astype(np.float64)


def mhd_weak_blast_state(coords, gam=GAMMA):
    """1.5D MHD weak blast (Sec. 4.1.1): the Euler weak-blast data in x with
    v_y = v_z = 0, B = (1, 1, 1), psi = 0; no variation in y."""
    x = coords[0]
    inner = np.abs(x) <= 0.5
    rho = np.where(inner, 1.1691, 1.0)
    vx = np.where(inner, 0.1882 * np.sign(x), 0.0)
    p = np.where(inner, 1.245, 1.0)
    z, one = np.zeros_like(x), np.ones_like(x)
    return mhd_conserved(rho, [vx, z, z], p, [one, one, one], z, gam)


def mhd_alfven_state(coords, t=0.0, gam=5.0 / 3.0, amp=0.1):
    """Circularly polarised Alfven wave on [0, sqrt 2]^2 (Sec. 4.3.3 set-up):
    along x_par = (x + y)/sqrt 2 with B_par = 1, rho = 1, p = 0.1, v_par = 0,
    v_perp = amp sin(theta), v_z = amp cos(theta), B_perp = v_perp, B_z = v_z,
    theta = 2 pi (x_par + t) (period 1 in t), psi = 0; e_perp = (-1, 1)/sqrt 2."""
    x, y = coords
    s2 = math.sqrt(2.0)
    th = 2.0 * math.pi * ((x + y) / s2 + t)
    vperp, vz = amp * np.sin(th), amp * np.cos(th)
    vx, vy = -vperp / s2, vperp / s2
    Bx, By = 1.0 / s2 - vperp / s2, 1.0 / s2 + vperp / s2
    one = np.ones_like(x)
    return mhd_conserved(one, [vx, vy, vz], 0.1 * one, [Bx, By, vz], 0.0 * one, gam)


def mhd_max_wave_speed(U, dim, gam=GAMMA) -> np.ndarray:
    """Per-element max over nodes and directions of |v_d| + c_f,d (fast
    magnetosonic speed), for level assignment."""
    rho = U[0]
    v = [U[1 + k] / rho for k in range(3)]
    B = [U[5 + k] for k in range(3)]
    p = (gam - 1.0) * (U[4] - 0.5 * rho * sum(w * w for w in v) - 0.5 * sum(b * b for b in B) - 0.5 * U[8] ** 2)
    a2 = gam * p / rho
    b2 = sum(b * b for b in B) / rho
    s = []
    for d in range(dim):
        cf = np.sqrt(0.5 * (a2 + b2 + np.sqrt((a2 + b2) ** 2 - 4.0 * a2 * B[d] ** 2 / rho)))
        s.append(np.abs(v[d]) + cf)
    return np.max(np.stack(s), axis=0).max(axis=1)


def free_stream_state(coords, rho=1.3, vel=None, p=0.9, gam=GAMMA):
    dim = len(coords)
    vel = vel if vel is not None else [0.3, -0.2, 0.1][:dim]
    one = np.ones_like(coords[0])
    return conserved(rho * one, [v * one for v in vel], p * one, gam)


def random_smooth_state(coords, seed=0, amp=0.1, gam=GAMMA):
    """Smooth random periodic perturbation of a uniform state (test input)."""
    rng = np.random.default_rng(seed)
    dim = len(coords)
    f = np.zeros_like(coords[0])
    fields = []
    for _ in range(dim + 2):
        k = rng.integers(1, 3, size=dim)
        ph = rng.uniform(0, 2 * math.pi, size=dim)
        f = np.ones_like(coords[0])
        for d in range(dim):
            f = f * np.sin(2 * math.pi * k[d] * coords[d] / 10.0 + ph[d])
        fields.append(f)
    rho = 1.0 + amp * fields[0]
    vel = [0.5 * amp * fields[1 + d] for d in range(dim)]
    p = 1.0 + amp * fields[dim + 1]
    return conserved(rho, vel, p, gam)


def max_wave_speed(U, dim, gam=GAMMA) -> np.ndarray:
    """Per-element max over nodes and directions of |v_d| + c (for level assignment)."""
    rho = U[0]
    vel = [U[1 + d] / rho for d in range(dim)]
    p = (gam - 1.0) * (U[dim + 1] - 0.5 * rho * sum(v * v for v in vel))
    c = np.sqrt(gam * p / rho)
    s = np.max(np.stack([np.abs(v) + c for v in vel]), axis=0)
    return s.max(axis=1)


def vortex_ensemble(n_cases=256, seed=0, sizes=(16, 32, 48, 64), box=10.0, ratio=4.0):
    """Independent isentropic-vortex cases for batched stepping: strength U[1, 6],
    centre U[3, 7]^2, mesh size drawn from ``sizes`` (graded, ratio 4).  Case i takes
    its parameters from a generator seeded with (seed, i).
    Returns a list of dicts (faces, U0, strength, centre, n)."""
    out = []
    for i in range(n_cases):
        rng = np.random.default_rng([seed, i])
        n = int(rng.choice(sizes))
        strength = float(rng.uniform(1.0, 6.0))
        centre = tuple(float(x) for x in rng.uniform(3.0, 7.0, 2))
        f = [graded_faces(n, 0.0, box, ratio)] * 2
        U0 = vortex_state(node_coords(f), strength=strength, centre=centre, box=(0.0, box))
        out.append(dict(faces=f, U0=U0, strength=strength, centre=centre, n=n))
    return out
