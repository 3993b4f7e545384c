"""Complete synthetic problem set-ups: mesh, initial state, tableau, levels and step.

  vortex16   2D isentropic vortex (strength 5, centre (5, 5)) on [0, 10]^2, 16^2 graded
             quads, p = 2 with E = {3, 6}.
  kh64       2D Kelvin-Helmholtz shear layer on [-1, 1]^2, 64^2 graded quads, HLL surface
             flux, p = 3 with E = {4, 6, 8, 12}; perturbation phase from the seed.
  tgv32      3D Taylor-Green vortex, Mach 0.1, [0, 2 pi]^3, 32^3 graded hexahedra,
             p = 4 with E = {5, 9, 14}; phase offsets from the seed.
  ensemble   256 isentropic vortices (strength U[1, 6], centre U[3, 7]^2) on graded
             16^2..64^2 meshes, p = 3 with E = {4, 6, 8, 12}, per-case step and levels.

  mhd_blast  1.5D ideal GLM-MHD weak blast (Sec. 4.1.1): [-2, 2] x [0, 1/4] with 64 x 2
             cells of widths 1/8, 1/16, 1/32 (finest in [-1/2, 1/2]), B = (1, 1, 1),
             EC volume and surface flux, p = 3 with E = {4, 7, 13}, c_h = 1.
  alfven     2D ideal GLM-MHD Alfven wave (Sec. 4.3.3) on [0, sqrt 2]^2, n^2 uniform
             cells, gamma = 5/3, weak-form volume term, LLF surface flux, p = 3 with
             E = {10, ..., 14} assigned to the cells at random, c_h = 1.

  viscous_shock  1.5D Navier-Stokes-Fourier viscous shock (Sec. 4.3.2): [-2, 2] x [0, 8/n]
             with n cells in x (widths halved in [-1, 1]) and 2 in y, gamma = 5/3,
             mu = 0.15, Pr = 3/4, HLLE surface flux, weak-form volume term, BR1,
             exact inflow / outflow / moving isothermal walls at the x ends, p = 4 with
             E = {6, 10} (10 on the fine cells), dt = 0.035 dx_min^2 / v.

Levels by the shortest edge with one speed per case, step at 0.5 of the optimised
stable step of the largest level (random assignments: of every assigned level).
Every Euler mesh is graded geometrically (ratio 4, finest at the centre).
"""
from __future__ import annotations

import numpy as np

from . import tableau as T
from . import workloads as W


def _levels(tab, faces, U, dim):
    return T.assign_levels(tab, W.element_widths(faces).min(axis=1), W.max_wave_speed(U, dim))


def vortex16(seed=0):
    f = [W.graded_faces(16, 0.0, 10.0)] * 2
    U0 = W.vortex_state(W.node_coords(f))
    tab = T.get_tableau(2, [3, 6])
    dt, lev = _levels(tab, f, U0, 2)
    return dict(kind="vortex", name="vortex16_p2_E3-6", faces=[f], U0=U0, tab=tab, dt=np.array([dt]), lev=[lev],
                flux=0, cases=[dict(faces=f, U0=U0, strength=5.0, centre=(5.0, 5.0), n=16)])


def kh64(seed=0):
    f = [W.graded_faces(64, -1.0, 1.0)] * 2
    rng = np.random.default_rng(seed)
    U0 = W.kelvin_helmholtz_state(W.node_coords(f), phase=float(rng.uniform(0, 2 * np.pi)))
    tab = T.get_tableau(3, [4, 6, 8, 12])
    dt, lev = _levels(tab, f, U0, 2)
    return dict(kind="kh", name="kh64_p3_E4-6-8-12_hll", faces=[f], U0=U0, tab=tab, dt=np.array([dt]), lev=[lev],
                flux=1)


def tgv32(seed=0, n=32):
    f = [W.graded_faces(n, 0.0, 2 * np.pi)] * 3
    rng = np.random.default_rng(seed)
    U0 = W.taylor_green_state(W.node_coords(f), mach=0.1, phase=tuple(rng.uniform(0, 2 * np.pi, 3)))
    tab = T.get_tableau(4, [5, 9, 14])
    dt, lev = _levels(tab, f, U0, 3)
    return dict(kind="tgv", name=f"tgv{n}_p4_E5-9-14", faces=[f], U0=U0, tab=tab, dt=np.array([dt]), lev=[lev],
                flux=0)


def ensemble(seed=0, n_cases=256):
    cases = W.vortex_ensemble(n_cases, seed)
    tab = T.get_tableau(3, [4, 6, 8, 12])
    dts, levs = [], []
    for c in cases:
        dt, lev = _levels(tab, c["faces"], c["U0"], 2)
        dts.append(dt)
        levs.append(lev)
    U0 = np.ascontiguousarray(np.concatenate([c["U0"] for c in cases], axis=1))
    return dict(kind="ensemble", name=f"vortex_ensemble{n_cases}_p3_E4-6-8-12", faces=[c["faces"] for c in cases],
                U0=U0, tab=tab, dt=np.array(dts), lev=levs, cases=cases, flux=0)


def mhd_blast(seed=0):
    fx = np.concatenate([np.linspace(-2.0, -1.0, 9)[:-1], np.linspace(-1.0, -0.5, 9)[:-1],
                         np.linspace(-0.5, 0.5, 33)[:-1], np.linspace(0.5, 1.0, 9)[:-1], np.linspace(1.0, 2.0, 9)])
    f = [fx, W.uniform_faces(2, 0.0, 0.25)]
    U0 = W.mhd_weak_blast_state(W.node_coords(f))
    tab = T.get_tableau(3, [4, 7, 13])
    dt, lev = T.assign_levels(tab, W.element_widths(f).min(axis=1), W.mhd_max_wave_speed(U0, 2))
    return dict(kind="mhd_blast", name="mhd_blast1p5d_p3_E4-7-13", faces=[f], U0=U0, tab=tab, dt=np.array([dt]),
                lev=[lev], flux=0, volume=0, system=1, glm_ch=1.0, gam=W.GAMMA)


def alfven(seed=0, n=16):
    gam = 5.0 / 3.0
    f = [W.uniform_faces(n, 0.0, float(np.sqrt(2.0)))] * 2
    U0 = W.mhd_alfven_state(W.node_coords(f), 0.0, gam)
    tab = T.get_tableau(3, list(range(10, 15)))
    lev = np.random.default_rng(seed + 17).integers(0, len(tab["E"]), size=n * n).astype(np.int32)
    speed = float(W.mhd_max_wave_speed(U0, 2, gam).max())
    h = W.element_widths(f).min(axis=1)
    dt = 0.5 * float(np.min(np.asarray(tab["h_stab"])[lev] * h / speed))
    return dict(kind="alfven", name=f"alfven{n}_p3_E10-14_random", faces=[f], U0=U0, tab=tab, dt=np.array([dt]),
                lev=[lev], flux=2, volume=1, system=1, glm_ch=1.0, gam=gam)


def viscous_shock(seed=0, n=24):
    gam, mu = 5.0 / 3.0, 0.15
    fx = W.viscous_shock_faces(n)
    f = [fx, W.uniform_faces(2, 0.0, 8.0 / n)]
    U0 = W.viscous_shock_state(W.node_coords(f), 0.0, gam, mu)
    tab = T.get_tableau(4, [6, 10])
    wx = W.element_widths(f)[:, 0]
    lev = np.where(wx < 0.75 * wx.max(), 1, 0).astype(np.int32)
    dt = 0.035 * wx.min() ** 2
    return dict(kind="viscous_shock", name=f"viscous_shock{n}_p4_E6-10", faces=[f], U0=U0, tab=tab,
                dt=np.array([dt]), lev=[lev], flux=3, volume=1, system=0, viscous=1, mu=mu, prandtl=0.75, bc_x=1,
                gam=gam)
