"""Thin ctypes binding of libperrk (include/perrk.h).

Argument marshalling only: every step of the P-ERRK path runs in the HIP
library.  PyTorch provides device memory and the stream.  Loading fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from collections import namedtuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libperrk.so")

OK, EINVAL, ENOMEM, EHIP, ENONPHYS, ENONFINITE, WARN_FALLBACK = 0, -1, -2, -3, -4, -5, 1
FLUX_EC, FLUX_HLL, FLUX_LLF, FLUX_HLLE, FLUX_HLLC, FLUX_CENTRAL = 0, 1, 2, 3, 4, 5
VOLUME_FLUX_DIFFERENCING, VOLUME_WEAK = 0, 1
SYSTEM_EULER, SYSTEM_GLM_MHD = 0, 1
FP64, MIXED, MIXED_ALL = 0, 1, 2
ANCHOR_STEP, ANCHOR_INITIAL = 0, 1
GUESS_PREV, GUESS_MLP, GUESS_EXTRAP = 0, 1, 2
TILES = 4  # PERRK_TILES
FLAG_BISECT, FLAG_FALLBACK, FLAG_TRIVIAL = 1, 2, 4


RelaxationState = namedtuple("RelaxationState", "gamma_prev h_offset t gamma_hist n_steps")


class PerrkError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"perrk status {status}: {msg}")
        self.status = status


class MeshDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_cases", ctypes.c_int32),
                ("n_elem_dir", ctypes.POINTER(ctypes.c_int32)),
                ("face_coords", ctypes.POINTER(ctypes.c_double)), ("gas_gamma", ctypes.c_double),
                ("surface_flux", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("volume_integral", ctypes.c_int32), ("system", ctypes.c_int32), ("glm_ch", ctypes.c_double),
                ("viscous", ctypes.c_int32), ("mu", ctypes.c_double), ("prandtl", ctypes.c_double),
                ("bc_x", ctypes.c_int32)]


class PartitionDesc(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("elem_level", ctypes.POINTER(ctypes.c_int32))]


class TableauDesc(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("S", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("E", ctypes.POINTER(ctypes.c_int32)), ("c", ctypes.POINTER(ctypes.c_double)),
                ("b", ctypes.POINTER(ctypes.c_double)), ("a_sub", ctypes.POINTER(ctypes.c_double))]


class Options(ctypes.Structure):
    _fields_ = [("relax", ctypes.c_int32), ("max_newton", ctypes.c_int32), ("tol_r", ctypes.c_double),
                ("tol_step", ctypes.c_double), ("anchor", ctypes.c_int32), ("max_bisect", ctypes.c_int32),
                ("bisect_lo", ctypes.c_double), ("bisect_hi", ctypes.c_double), ("guess", ctypes.c_int32),
                ("fast_passes", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("tune", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("phases", ctypes.c_int32)]


class StepInfo(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("r", ctypes.c_double), ("dH", ctypes.c_double),
                ("H_delta", ctypes.c_double), ("e", ctypes.c_double * 8), ("t", ctypes.c_double),
                ("passes", ctypes.c_int32), ("flags", ctypes.c_int32)]


class KernelStat(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("bytes", ctypes.c_double), ("launches", ctypes.c_int64)]


K_CLASSES = ["stage_first", "stage_mid", "stage_last", "residual", "solver", "update"]

EXPORTS = ["perrk_default_options", "perrk_validate", "perrk_init", "perrk_step", "perrk_entropy",
           "perrk_rhs", "perrk_get_relaxation_state", "perrk_set_relaxation_state",
           "perrk_set_guess_model", "perrk_set_profiling", "perrk_get_kernel_stats", "perrk_get_stage_stats",
           "perrk_get_tuning", "perrk_last_error", "perrk_version", "perrk_destroy",
           "perrk_mlp_workspace_bytes", "perrk_mlp_forward", "perrk_mlp_loss_grad", "perrk_mlp_loss_grad_static",
           "perrk_mlp_adam"]

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it with paper_2507_04991_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        p, i32, d, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
        L.perrk_default_options.argtypes = [ctypes.POINTER(Options)]
        L.perrk_default_options.restype = None
        L.perrk_validate.argtypes = [ctypes.POINTER(MeshDesc), ctypes.POINTER(PartitionDesc),
                                     ctypes.POINTER(TableauDesc), ctypes.POINTER(Options),
                                     ctypes.c_char_p, sz]
        L.perrk_validate.restype = ctypes.c_int
        L.perrk_init.argtypes = [ctypes.POINTER(MeshDesc), ctypes.POINTER(PartitionDesc),
                                 ctypes.POINTER(TableauDesc), ctypes.POINTER(Options), p,
                                 ctypes.POINTER(p)]
        L.perrk_init.restype = ctypes.c_int
        L.perrk_step.argtypes = [p, p, ctypes.POINTER(d), ctypes.POINTER(StepInfo)]
        L.perrk_step.restype = ctypes.c_int
        L.perrk_entropy.argtypes = [p, p, ctypes.POINTER(d)]
        L.perrk_entropy.restype = ctypes.c_int
        L.perrk_rhs.argtypes = [p, p, p]
        L.perrk_rhs.restype = ctypes.c_int
        for fn in ("perrk_get_relaxation_state", "perrk_set_relaxation_state"):
            getattr(L, fn).argtypes = [p, ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(d),
                                       ctypes.POINTER(d), ctypes.POINTER(ctypes.c_int32)]
            getattr(L, fn).restype = ctypes.c_int
        L.perrk_set_guess_model.argtypes = [p, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                            ctypes.POINTER(ctypes.c_float)]
        L.perrk_set_guess_model.restype = ctypes.c_int
        L.perrk_set_profiling.argtypes = [p, ctypes.c_int]
        L.perrk_set_profiling.restype = ctypes.c_int
        L.perrk_get_kernel_stats.argtypes = [p, ctypes.POINTER(KernelStat), ctypes.c_int]
        L.perrk_get_kernel_stats.restype = ctypes.c_int
        L.perrk_get_stage_stats.argtypes = [p, ctypes.POINTER(KernelStat), ctypes.c_int, ctypes.c_int]
        L.perrk_get_stage_stats.restype = ctypes.c_int
        L.perrk_get_tuning.argtypes = [p, ctypes.c_char_p, sz]
        L.perrk_get_tuning.restype = ctypes.c_int
        L.perrk_last_error.argtypes = [p]
        L.perrk_last_error.restype = ctypes.c_char_p
        L.perrk_version.argtypes = []
        L.perrk_version.restype = ctypes.c_char_p
        L.perrk_destroy.argtypes = [p]
        L.perrk_destroy.restype = None
        L.perrk_mlp_workspace_bytes.argtypes = [ctypes.c_int64]
        L.perrk_mlp_workspace_bytes.restype = ctypes.c_size_t
        L.perrk_mlp_forward.argtypes = [p, p, ctypes.c_int64, p, p]
        L.perrk_mlp_forward.restype = ctypes.c_int
        L.perrk_mlp_loss_grad.argtypes = [p, p, p, ctypes.c_int64, p, p, p, sz, p]
        L.perrk_mlp_loss_grad.restype = ctypes.c_int
        L.perrk_mlp_loss_grad_static.argtypes = [p, p, p, ctypes.c_int64, p, p, p]
        L.perrk_mlp_loss_grad_static.restype = ctypes.c_int
        L.perrk_mlp_adam.argtypes = [p, p, p, p, ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, p]
        L.perrk_mlp_adam.restype = ctypes.c_int
        _lib = L
    return _lib


def default_options(**kw) -> Options:
    o = Options()
    lib().perrk_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class Descriptors:
    """Host-side descriptors (keeps the numpy buffers alive)."""

    def __init__(self, faces_per_case, levels, tableau, gas_gamma=1.4, surface_flux=FLUX_EC,
                 precision=FP64, volume_integral=VOLUME_FLUX_DIFFERENCING, system=SYSTEM_EULER, glm_ch=0.0,
                 viscous=0, mu=0.0, prandtl=0.75, bc_x=0):
        self.dim = len(faces_per_case[0])
        self.n_cases = len(faces_per_case)
        n = []
        coords = []
        for faces in faces_per_case:
            nn = [len(f) - 1 for f in faces] + ([1] if self.dim == 2 else [])
            n.extend(nn)
            coords.extend(np.asarray(f, dtype=np.float64) for f in faces)
        self.n = np.ascontiguousarray(n, dtype=np.int32)
        self.faces = np.ascontiguousarray(np.concatenate(coords), dtype=np.float64)
        self.levels = np.ascontiguousarray(np.concatenate([np.asarray(x) for x in levels]), dtype=np.int32)
        self.E = np.ascontiguousarray(tableau["E"], dtype=np.int32)
        self.c = np.ascontiguousarray(tableau["c"], dtype=np.float64)
        self.b = np.ascontiguousarray(tableau["b"], dtype=np.float64)
        self.a_sub = np.ascontiguousarray(tableau["a_sub"], dtype=np.float64)
        self.mesh = MeshDesc(self.dim, self.n_cases, _ip(self.n), _dp(self.faces), gas_gamma, surface_flux,
                             precision, volume_integral, system, glm_ch, viscous, mu, prandtl, bc_x)
        self.part = PartitionDesc(len(self.E), _ip(self.levels))
        self.tab = TableauDesc(int(tableau["order"]), len(self.c), len(self.E), _ip(self.E), _dp(self.c),
                               _dp(self.b), _dp(self.a_sub))
        self.nelem = int(sum(np.prod(self.n[3 * i:3 * i + self.dim]) for i in range(self.n_cases)))
        self.npe = 4 ** self.dim
        self.V = 9 if system == SYSTEM_GLM_MHD else self.dim + 2

    def validate(self, opts: Options | None = None):
        msg = ctypes.create_string_buffer(512)
        st = lib().perrk_validate(ctypes.byref(self.mesh), ctypes.byref(self.part), ctypes.byref(self.tab),
                                  None if opts is None else ctypes.byref(opts), msg, 512)
        return st, msg.value.decode()


class Stepper:
    """One context of libperrk.  ``u`` arguments are torch float64 tensors of shape
    [V, total elements, nodes] on the current HIP device."""

    def __init__(self, desc: Descriptors, opts: Options | None = None, stream=None):
        import torch

        self.desc = desc
        self.opts = opts if opts is not None else default_options()
        self._torch = torch
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        ctx = ctypes.c_void_p()
        st = lib().perrk_init(ctypes.byref(desc.mesh), ctypes.byref(desc.part), ctypes.byref(desc.tab),
                              ctypes.byref(self.opts), ctypes.c_void_p(s.cuda_stream), ctypes.byref(ctx))
        if st != OK:
            raise PerrkError(st, "perrk_init failed (see stderr)")
        self.ctx = ctx
        self.n_cases = desc.n_cases
        self.n_stages = len(desc.c)
        self._infos = (StepInfo * desc.n_cases)()

    def _check(self, st):
        if st < 0:
            raise PerrkError(st, lib().perrk_last_error(self.ctx).decode())
        return st

    def _u(self, u):
        t = self._torch
        assert u.is_cuda and u.dtype == t.float64 and u.is_contiguous()
        assert tuple(u.shape) == (self.desc.V, self.desc.nelem, self.desc.npe)
        return ctypes.c_void_p(u.data_ptr())

    def step(self, u, dt, info=True):
        """Advance every case by one step in place; returns a list of dicts (or None)."""
        dts = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (self.n_cases,)))
        st = lib().perrk_step(self.ctx, self._u(u), _dp(dts), self._infos if info else None)
        self._check(st)
        if not info:
            return None
        return [dict(gamma=i.gamma, r=i.r, dH=i.dH, H_delta=i.H_delta, e=list(i.e), t=i.t,
                     passes=i.passes, flags=i.flags, status=st) for i in self._infos]

    def entropy(self, u):
        H = np.zeros(self.n_cases)
        self._check(lib().perrk_entropy(self.ctx, self._u(u), _dp(H)))
        return H

    def rhs(self, u):
        t = self._torch
        dtype = t.float64 if self.desc.mesh.precision == FP64 else t.float32
        k = t.empty_like(u, dtype=dtype)
        self._check(lib().perrk_rhs(self.ctx, self._u(u), ctypes.c_void_p(k.data_ptr())))
        return k

    def relaxation_state(self):
        """RelaxationState(gamma_prev, h_offset, t, gamma_hist [n, 3], n_steps) per case."""
        n = self.n_cases
        g, h, tt, gh = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros((n, 3))
        ns = np.zeros(n, dtype=np.int32)
        self._check(lib().perrk_get_relaxation_state(self.ctx, _dp(g), _dp(h), _dp(tt), _dp(gh),
                                                     ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return RelaxationState(g, h, tt, gh, ns)

    def set_relaxation_state(self, gamma_prev=None, h_offset=None, t=None, gamma_hist=None, n_steps=None):
        n = self.n_cases
        arr = [None if x is None else np.ascontiguousarray(np.broadcast_to(x, (n,)), dtype=np.float64)
               for x in (gamma_prev, h_offset, t)]
        arr.append(None if gamma_hist is None
                   else np.ascontiguousarray(np.broadcast_to(gamma_hist, (n, 3)), dtype=np.float64))
        ptrs = [None if x is None else _dp(x) for x in arr]
        ns = None if n_steps is None else np.ascontiguousarray(np.broadcast_to(n_steps, (n,)), dtype=np.int32)
        ptrs.append(None if ns is None else ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        self._check(lib().perrk_set_relaxation_state(self.ctx, *ptrs))

    def set_guess_model(self, weights, mean, scale):
        w = np.ascontiguousarray(weights, dtype=np.float32)
        m = np.ascontiguousarray(mean, dtype=np.float32)
        s = np.ascontiguousarray(scale, dtype=np.float32)
        fp = ctypes.POINTER(ctypes.c_float)
        self._check(lib().perrk_set_guess_model(self.ctx, w.ctypes.data_as(fp), m.ctypes.data_as(fp),
                                                s.ctypes.data_as(fp)))

    def set_profiling(self, on: bool):
        self._check(lib().perrk_set_profiling(self.ctx, int(bool(on))))

    def kernel_stats(self, reset=True):
        arr = (KernelStat * len(K_CLASSES))()
        self._check(lib().perrk_get_kernel_stats(self.ctx, arr, int(reset)))
        return {name: dict(ms=s.ms, bytes=s.bytes, launches=s.launches) for name, s in zip(K_CLASSES, arr)}

    def stage_stats(self, reset=True):
        """Per-stage profiling statistics: list of dict(ms, bytes, launches), stage 1 first."""
        arr = (KernelStat * self.n_stages)()
        self._check(lib().perrk_get_stage_stats(self.ctx, arr, self.n_stages, int(reset)))
        return [dict(ms=s.ms, bytes=s.bytes, launches=s.launches) for s in arr]

    def tuning(self):
        buf = ctypes.create_string_buffer(16384)
        lib().perrk_get_tuning(self.ctx, buf, 16384)
        return buf.value.decode()

    def close(self):
        if getattr(self, "ctx", None):
            lib().perrk_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------
# learned-guess network on device tensors
# --------------------------------------------------------------------------

MLP_NW = 1377


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def mlp_forward(w, x):
    """y = network(w, x) for float32 device tensors w[1377], x[n][8]."""
    import torch

    y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    st = lib().perrk_mlp_forward(_ptr(w), _ptr(x), x.shape[0], _ptr(y), _stream(torch))
    if st != OK:
        raise PerrkError(st, "perrk_mlp_forward")
    return y


def mlp_loss_grad(w, x, t, work=None):
    """(loss tensor [1] float64, grad [1377] float32) of the mean squared error."""
    import torch

    n = x.shape[0]
    nbytes = lib().perrk_mlp_workspace_bytes(n)
    if work is None or work.numel() < nbytes:
        work = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    g = torch.empty(MLP_NW, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float64, device=x.device)
    st = lib().perrk_mlp_loss_grad(_ptr(w), _ptr(x), _ptr(t), n, _ptr(g), _ptr(loss), _ptr(work), nbytes,
                                   _stream(torch))
    if st != OK:
        raise PerrkError(st, "perrk_mlp_loss_grad")
    return loss, g


MLP_STATIC_MAX_N = 131072  # PERRK_MLP_STATIC_MAX_N


def mlp_loss_grad_static(w, x, t, loss=None, grad=None):
    """mlp_loss_grad with the library's static scratch instead of a workspace
    (perrk_mlp_loss_grad_static: allocates nothing when loss and grad are given)."""
    import torch

    n = x.shape[0]
    g = grad if grad is not None else torch.empty(MLP_NW, dtype=torch.float32, device=x.device)
    lo = loss if loss is not None else torch.empty(1, dtype=torch.float64, device=x.device)
    st = lib().perrk_mlp_loss_grad_static(_ptr(w), _ptr(x), _ptr(t), n, _ptr(g), _ptr(lo), _stream(torch))
    if st != OK:
        raise PerrkError(st, f"perrk_mlp_loss_grad_static (n = {n}, at most {MLP_STATIC_MAX_N})")
    return lo, g


def mlp_adam(w, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    import torch

    st = lib().perrk_mlp_adam(_ptr(w), _ptr(g), _ptr(m), _ptr(v), int(step), lr, beta1, beta2, eps, _stream(torch))
    if st != OK:
        raise PerrkError(st, "perrk_mlp_adam")
