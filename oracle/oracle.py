"""Python access to the FP64 CPU oracle (``perrk_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  The product path never imports this module.

Arrays use the interface layout U[v][elem][node] (node fastest, x index
fastest within a node and within the element numbering), float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "perrk_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ENOMEM, ENONPHYS, ENONFINITE = 0, -1, -2, -4, -5
FLAG_BISECT, FLAG_FALLBACK, FLAG_TRIVIAL = 1, 2, 4


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3),
                ("faces", ctypes.POINTER(ctypes.c_double)), ("gam", ctypes.c_double),
                ("surface_flux", ctypes.c_int), ("volume_integral", ctypes.c_int),
                ("physics", ctypes.c_int), ("c_h", ctypes.c_double), ("viscous", ctypes.c_int),
                ("mu", ctypes.c_double), ("prandtl", ctypes.c_double), ("bc_x", ctypes.c_int),
                ("time", ctypes.c_double)]


class _Tableau(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int), ("S", ctypes.c_int), ("R", ctypes.c_int),
                ("E", ctypes.POINTER(ctypes.c_int)), ("c", ctypes.POINTER(ctypes.c_double)),
                ("b", ctypes.POINTER(ctypes.c_double)), ("a_sub", ctypes.POINTER(ctypes.c_double))]


class _Relax(ctypes.Structure):
    _fields_ = [("relax", ctypes.c_int), ("max_newton", ctypes.c_int), ("tol_r", ctypes.c_double),
                ("tol_step", ctypes.c_double), ("anchor", ctypes.c_int), ("H0", ctypes.c_double),
                ("bis_lo", ctypes.c_double), ("bis_hi", ctypes.c_double),
                ("max_bisect", ctypes.c_int), ("gamma0", ctypes.c_double), ("t0", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("r", ctypes.c_double), ("dH", ctypes.c_double),
                ("H_old", ctypes.c_double), ("H_new", ctypes.c_double), ("passes", ctypes.c_int),
                ("newton_iters", ctypes.c_int), ("flags", ctypes.c_int), ("pad", ctypes.c_int),
                ("e", ctypes.c_double * 64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        d, i, p = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        _lib.or_logmean.restype = d
        _lib.or_logmean.argtypes = [d, d]
        _lib.or_entropy.restype = d
        _lib.or_entropy.argtypes = [i, p, d]
        _lib.or_entropy_diff.restype = d
        _lib.or_entropy_diff.argtypes = [i, p, p, d]
        for fn in ("or_flux_ec", "or_flux_hll", "or_flux_llf", "or_flux_hlle", "or_flux_hllc"):
            getattr(_lib, fn).argtypes = [i, i, p, p, d, p]
        _lib.or_flux_phys.argtypes = [i, i, p, d, p]
        _lib.or_mhd_flux_phys.argtypes = [i, p, d, d, p]
        for fn in ("or_mhd_flux_ec", "or_mhd_flux_llf", "or_mhd_flux_central"):
            getattr(_lib, fn).argtypes = [i, p, p, d, d, p]
        _lib.or_mhd_nonconservative.argtypes = [i, p, d, p, p]
        _lib.or_mhd_cfast.restype = d
        _lib.or_mhd_cfast.argtypes = [i, p, d]
        _lib.or_mhd_entropy.restype = d
        _lib.or_mhd_entropy.argtypes = [p, d]
        _lib.or_mhd_entropy_vars.argtypes = [p, d, p]
        _lib.or_mhd_entropy_diff.restype = d
        _lib.or_mhd_entropy_diff.argtypes = [p, p, d]
        _lib.or_viscous_shock_prim.argtypes = [d, d, d, d, p, p, p]
        _lib.or_ns_viscous_flux.argtypes = [i, d, d, p, d, d, p]
        _lib.or_entropy_vars.argtypes = [i, p, d, p]
        _lib.or_lgl.argtypes = [p, p, p, p]
        _lib.or_rhs.restype = i
        _lib.or_rhs.argtypes = [ctypes.POINTER(_Mesh), p, p, p]
        _lib.or_check_state.restype = i
        _lib.or_check_state.argtypes = [ctypes.POINTER(_Mesh), p]
        _lib.or_total_entropy.restype = d
        _lib.or_total_entropy.argtypes = [ctypes.POINTER(_Mesh), p]
        _lib.or_total_conserved.argtypes = [ctypes.POINTER(_Mesh), p, p]
        _lib.or_entropy_production.restype = d
        _lib.or_entropy_production.argtypes = [ctypes.POINTER(_Mesh), p, p]
        _lib.or_relax_eval.argtypes = [ctypes.POINTER(_Mesh), p, p, d, d, d, d, p, p]
        _lib.or_dense_A.argtypes = [ctypes.POINTER(_Tableau), i, p]
        for fn in ("or_step", "or_step_dense"):
            getattr(_lib, fn).restype = i
            getattr(_lib, fn).argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Tableau), p,
                                          ctypes.POINTER(_Relax), p, d, ctypes.POINTER(_Info)]
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# point-wise functions
# --------------------------------------------------------------------------

def lgl():
    """(xi, q, D, Dsplit) of the degree-3 LGL rule."""
    xi, q = np.zeros(4), np.zeros(4)
    D, Ds = np.zeros((4, 4)), np.zeros((4, 4))
    lib().or_lgl(_ptr(xi), _ptr(q), _ptr(D), _ptr(Ds))
    return xi, q, D, Ds


def logmean(a: float, b: float) -> float:
    return lib().or_logmean(float(a), float(b))


def flux_ec(dim, direction, uL, uR, gam=1.4):
    uL, uR, f = _f64(uL), _f64(uR), np.zeros(dim + 2)
    lib().or_flux_ec(dim, direction, _ptr(uL), _ptr(uR), gam, _ptr(f))
    return f


def flux_hll(dim, direction, uL, uR, gam=1.4):
    uL, uR, f = _f64(uL), _f64(uR), np.zeros(dim + 2)
    lib().or_flux_hll(dim, direction, _ptr(uL), _ptr(uR), gam, _ptr(f))
    return f


def flux_llf(dim, direction, uL, uR, gam=1.4):
    uL, uR, f = _f64(uL), _f64(uR), np.zeros(dim + 2)
    lib().or_flux_llf(dim, direction, _ptr(uL), _ptr(uR), gam, _ptr(f))
    return f


def flux_hlle(dim, direction, uL, uR, gam=1.4):
    uL, uR, f = _f64(uL), _f64(uR), np.zeros(dim + 2)
    lib().or_flux_hlle(dim, direction, _ptr(uL), _ptr(uR), gam, _ptr(f))
    return f


def flux_hllc(dim, direction, uL, uR, gam=1.4):
    uL, uR, f = _f64(uL), _f64(uR), np.zeros(dim + 2)
    lib().or_flux_hllc(dim, direction, _ptr(uL), _ptr(uR), gam, _ptr(f))
    return f


def flux_phys(dim, direction, u, gam=1.4):
    u, f = _f64(u), np.zeros(dim + 2)
    lib().or_flux_phys(dim, direction, _ptr(u), gam, _ptr(f))
    return f


def mhd_flux_phys(direction, u, gam=1.4, c_h=0.0):
    u, f = _f64(u), np.zeros(9)
    lib().or_mhd_flux_phys(direction, _ptr(u), gam, c_h, _ptr(f))
    return f


def _mhd2(fn, direction, uL, uR, gam, c_h):
    uL, uR, f = _f64(uL), _f64(uR), np.zeros(9)
    getattr(lib(), fn)(direction, _ptr(uL), _ptr(uR), gam, c_h, _ptr(f))
    return f


def mhd_flux_ec(direction, uL, uR, gam=1.4, c_h=0.0):
    return _mhd2("or_mhd_flux_ec", direction, uL, uR, gam, c_h)


def mhd_flux_llf(direction, uL, uR, gam=1.4, c_h=0.0):
    return _mhd2("or_mhd_flux_llf", direction, uL, uR, gam, c_h)


def mhd_flux_central(direction, uL, uR, gam=1.4, c_h=0.0):
    return _mhd2("or_mhd_flux_central", direction, uL, uR, gam, c_h)


def mhd_cfast(direction, u, gam=1.4) -> float:
    """Fast magnetosonic speed in direction n (the LLF wave speed of GLM-MHD)."""
    return lib().or_mhd_cfast(direction, _ptr(_f64(u)), gam)


def mhd_nonconservative(direction, u, gam=1.4):
    u, phi, phin = _f64(u), np.zeros(9), np.zeros(9)
    lib().or_mhd_nonconservative(direction, _ptr(u), gam, _ptr(phi), _ptr(phin))
    return phi, phin


def viscous_shock_prim(x, t, gam=5.0 / 3.0, mu=0.15):
    r, u, p = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().or_viscous_shock_prim(float(x), float(t), gam, mu, ctypes.byref(r), ctypes.byref(u), ctypes.byref(p))
    return r.value, u.value, p.value


def ns_viscous_flux(direction, vx, vy, grad, mu, kappa):
    g, f = _f64(grad).reshape(8), np.zeros(4)
    lib().or_ns_viscous_flux(direction, float(vx), float(vy), _ptr(g), mu, kappa, _ptr(f))
    return f


def mhd_entropy(u, gam=1.4) -> float:
    return lib().or_mhd_entropy(_ptr(_f64(u)), gam)


def mhd_entropy_vars(u, gam=1.4):
    u, w = _f64(u), np.zeros(9)
    lib().or_mhd_entropy_vars(_ptr(u), gam, _ptr(w))
    return w


def mhd_entropy_diff(u, du, gam=1.4) -> float:
    return lib().or_mhd_entropy_diff(_ptr(_f64(u)), _ptr(_f64(du)), gam)


def entropy(dim, u, gam=1.4) -> float:
    u = _f64(u)
    return lib().or_entropy(dim, _ptr(u), gam)


def entropy_vars(dim, u, gam=1.4):
    u, w = _f64(u), np.zeros(dim + 2)
    lib().or_entropy_vars(dim, _ptr(u), gam, _ptr(w))
    return w


def entropy_diff(dim, u, du, gam=1.4) -> float:
    u, du = _f64(u), _f64(du)
    return lib().or_entropy_diff(dim, _ptr(u), _ptr(du), gam)


# --------------------------------------------------------------------------
# mesh-level functions
# --------------------------------------------------------------------------

class Mesh:
    """Periodic Cartesian mesh: ``faces`` is a list of per-direction face coordinates."""

    def __init__(self, faces, gam: float = 1.4, surface_flux: int = 0, volume_integral: int = 0,
                 physics: int = 0, c_h: float = 0.0, viscous: int = 0, mu: float = 0.0, prandtl: float = 0.75,
                 bc_x: int = 0, time: float = 0.0):
        self.dim = len(faces)
        self.faces_list = [_f64(f) for f in faces]
        self.n = [len(f) - 1 for f in self.faces_list] + ([1] if self.dim == 2 else [])
        self.faces = _f64(np.concatenate(self.faces_list))
        self.gam = gam
        self.surface_flux = surface_flux
        self.volume_integral = volume_integral
        self.physics = physics
        self.c_h = c_h
        self.viscous, self.mu, self.prandtl, self.bc_x = viscous, mu, prandtl, bc_x
        self.nelem = int(np.prod(self.n[: self.dim]))
        self.npe = 4 ** self.dim
        self.V = 9 if physics == 1 else self.dim + 2
        self._s = _Mesh(self.dim, (ctypes.c_int * 3)(*self.n),
                        self.faces.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), gam, surface_flux,
                        volume_integral, physics, c_h, viscous, mu, prandtl, bc_x, time)

    @property
    def shape(self):
        return (self.V, self.nelem, self.npe)

    def ref(self):
        return ctypes.byref(self._s)


class Tableau:
    def __init__(self, order, c, b, a_sub, E):
        self.order = int(order)
        self.c, self.b = _f64(c), _f64(b)
        self.a_sub = _f64(a_sub)
        self.E = np.ascontiguousarray(E, dtype=np.int32)
        self.S, self.R = len(self.c), len(self.E)
        assert self.a_sub.shape == (self.R, self.S)
        self._s = _Tableau(self.order, self.S, self.R,
                           self.E.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                           self.c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           self.b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           self.a_sub.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))

    def ref(self):
        return ctypes.byref(self._s)

    def dense_A(self, r: int) -> np.ndarray:
        A = np.zeros((self.S, self.S))
        lib().or_dense_A(self.ref(), r, _ptr(A))
        return A


def rhs(mesh: Mesh, U, active=None, K=None):
    U = _f64(U)
    K = np.zeros_like(U) if K is None else K
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    st = lib().or_rhs(mesh.ref(), _ptr(U), None if act is None else _ptr(act), _ptr(K))
    if st:
        raise ValueError(f"oracle rhs status {st}")
    return K


def check_state(mesh: Mesh, U) -> int:
    U = _f64(U)
    return lib().or_check_state(mesh.ref(), _ptr(U))


def total_entropy(mesh: Mesh, U) -> float:
    U = _f64(U)
    return lib().or_total_entropy(mesh.ref(), _ptr(U))


def total_conserved(mesh: Mesh, U):
    U, out = _f64(U), np.zeros(mesh.V)
    lib().or_total_conserved(mesh.ref(), _ptr(U), _ptr(out))
    return out


def entropy_production(mesh: Mesh, U, K) -> float:
    U, K = _f64(U), _f64(K)
    return lib().or_entropy_production(mesh.ref(), _ptr(U), _ptr(K))


def relax_eval(mesh: Mesh, Un, d, dt, gamma, dH, offset=0.0):
    Un, d = _f64(Un), _f64(d)
    r, rp = ctypes.c_double(), ctypes.c_double()
    lib().or_relax_eval(mesh.ref(), _ptr(Un), _ptr(d), dt, gamma, dH, offset,
                        ctypes.byref(r), ctypes.byref(rp))
    return r.value, rp.value


def relax_options(relax=True, max_newton=10, tol_r=1e-12, tol_step=1e-15, anchor=0, H0=0.0,
                  bis_lo=0.8, bis_hi=1.2, max_bisect=60, gamma0=1.0, t0=0.0) -> _Relax:
    return _Relax(int(relax), max_newton, tol_r, tol_step, anchor, H0, bis_lo, bis_hi, max_bisect,
                  gamma0, t0)


def step(mesh: Mesh, tab: Tableau, level, U, dt, opts: _Relax | None = None, dense=False):
    """One P-ERRK step.  Returns (U_{n+1}, info dict); U is not modified."""
    Uw = np.array(U, dtype=np.float64, copy=True, order="C")
    lev = np.ascontiguousarray(level, dtype=np.int32)
    opts = opts if opts is not None else relax_options()
    info = _Info()
    fn = lib().or_step_dense if dense else lib().or_step
    st = fn(mesh.ref(), tab.ref(), _ptr(lev), ctypes.byref(opts), _ptr(Uw), float(dt),
            ctypes.byref(info))
    out = dict(status=st, gamma=info.gamma, r=info.r, dH=info.dH, H_old=info.H_old,
               H_new=info.H_new, passes=info.passes, newton_iters=info.newton_iters,
               flags=info.flags, e=np.array(info.e[: tab.S]))
    return Uw, out


def run(mesh: Mesh, tab: Tableau, level, U0, dt, nsteps, relax=True, anchor=0, dense=False,
        **kw):
    """Advance nsteps; Newton starts from 1 at the first step, then from the previous gamma."""
    U = np.array(U0, dtype=np.float64, copy=True)
    H0 = total_entropy(mesh, U)
    g, t, hist = 1.0, 0.0, []
    for _ in range(nsteps):
        opts = relax_options(relax=relax, anchor=anchor, H0=H0, gamma0=g, t0=t, **kw)
        U, info = step(mesh, tab, level, U, dt, opts, dense=dense)
        if info["status"] != OK:
            raise ValueError(f"oracle step status {info['status']}")
        g = info["gamma"]
        t += g * dt
        hist.append(info)
    return U, t, hist


def relax_solve(mesh: Mesh, Un, d, dt, dH, offset=0.0, opts: _Relax | None = None):
    """Scalar root find of r(gamma) = 0 (Newton, then bisection, then gamma = 1)."""
    Un, d = _f64(Un), _f64(d)
    opts = opts if opts is not None else relax_options()
    info = _Info()
    f = lib().or_relax_solve
    f.argtypes = [ctypes.POINTER(_Mesh), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                  ctypes.c_double, ctypes.c_double, ctypes.POINTER(_Relax), ctypes.POINTER(_Info)]
    f(mesh.ref(), _ptr(Un), _ptr(d), float(dt), float(dH), float(offset), ctypes.byref(opts),
      ctypes.byref(info))
    return dict(gamma=info.gamma, r=info.r, passes=info.passes, newton_iters=info.newton_iters,
                flags=info.flags)
