#!/usr/bin/env python3
"""Throughput of the P-ERRK step on one MI355X.

Default workload: 3D compressible Euler Taylor-Green vortex (Mach 0.1, random
phase offsets from seed 0) on the periodic [0, 2 pi]^3 box, 32^3 hexahedra
graded geometrically (ratio 4, finest at the centre), DGSEM degree 3
(64 nodes per element, 10.5 M DOF), Ranocha EC volume and surface flux,
fourth-order P-ERRK with stage-evaluation levels E = {5, 9, 14} assigned by
local CFL.  The headline variant computes fluxes in FP32 (FP32 accumulation,
FP32 stage storage) and the stage combinations, entropy sums and the gamma
solve in FP64; the FP64-plain variant is timed beside it on the same inputs,
and the L2 distance between the two is compared with the temporal error of
the FP64 run (dt vs dt/2) to check that they are at equal L2 error.

Prints one JSON line (see the keys below).  Inputs are synthetic and seeded.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "P-ERRK DOF-updates/s on 1 GPU; mixed/learned vs FP64 plain at equal L2 error"
HBM_PEAK_GBS = 8000.0


def workload_tgv(n=32, seed=0):
    from paper_2507_04991_amd import tableau as T
    from paper_2507_04991_amd import workloads as W

    f = [W.graded_faces(n, 0.0, 2 * np.pi, 4.0)] * 3
    co = W.node_coords(f)
    rng = np.random.default_rng(seed)
    U0 = W.taylor_green_state(co, mach=0.1, phase=tuple(rng.uniform(0, 2 * np.pi, 3)))
    tab = T.get_tableau(4, [5, 9, 14])
    dt, lev = T.assign_levels(tab, W.element_widths(f).min(axis=1), W.max_wave_speed(U0, 3))
    return dict(name=f"tgv{n}_p4_E5-9-14", faces=f, U0=U0, tab=tab, dt=dt, lev=lev,
                desc=f"3D Euler Taylor-Green Mach 0.1, {n}^3 graded (ratio 4) periodic hexes, DGSEM k=3, "
                     f"Ranocha EC volume+surface flux, P-ERRK p=4 E={{5,9,14}}")


def run_variant(P, torch, wl, precision, steps, warmup, profile=False):
    d = P.Descriptors([wl["faces"]], [wl["lev"]], wl["tab"], precision=precision)
    st = P.Stepper(d, P.default_options())
    u = torch.tensor(wl["U0"], dtype=torch.float64, device="cuda").contiguous()
    for _ in range(warmup):
        st.step(u, wl["dt"], info=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st.step(u, wl["dt"], info=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g, _, tt = st.relaxation_state()
    out = dict(seconds=t1 - t0, u=u, gamma=float(g[0]), t=float(tt[0]), stepper=st)
    if profile:
        # the same kernels, launched one by one with HIP events around each launch
        st.set_profiling(True)
        st.kernel_stats(reset=True)
        up = u.clone()
        for _ in range(steps):
            st.step(up, wl["dt"], info=False)
        out["stats"] = st.kernel_stats(reset=True)
        st.set_profiling(False)
    return out


def l2_rel(a, b, tab_w=None):
    diff = (a - b).double()
    return float(torch_norm(diff) / torch_norm(b.double()))


def torch_norm(x):
    return (x * x).sum().sqrt()


def cpu_baseline(wl):
    """The FP64 CPU oracle on one full step of the same workload (single thread)."""
    from oracle import oracle as O

    m = O.Mesh(wl["faces"])
    t = O.Tableau(wl["tab"]["order"], wl["tab"]["c"], wl["tab"]["b"], wl["tab"]["a_sub"], wl["tab"]["E"])
    t0 = time.perf_counter()
    U1, info = O.step(m, t, wl["lev"], wl["U0"], wl["dt"])
    sec = time.perf_counter() - t0
    M = wl["U0"].size
    return dict(value=M / sec, unit="DOF-updates/s", cores=1, kind="oracle",
                sample=f"one full P-ERRK step of the same workload ({M} DOF, {sec:.1f} s, single thread)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mesh", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64-plain and dt/2 runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the path is single-GPU "
                                   "(multi-GPU sharding is described, not built)", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2507_04991_amd import perrk as P

    P.lib()
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    wl = workload_tgv(args.mesh)
    M = wl["U0"].size
    print(f"# workload {wl['name']}: {M} DOF, dt={wl['dt']:.4e}, levels={np.bincount(wl['lev']).tolist()}",
          file=sys.stderr, flush=True)

    mixed = run_variant(P, torch, wl, P.MIXED, args.steps, args.warmup, profile=True)
    print(f"# mixed: {mixed['seconds'] / args.steps * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
    extra = {}
    if not args.no_compare:
        fp64 = run_variant(P, torch, wl, P.FP64, args.steps, args.warmup)
        print(f"# fp64: {fp64['seconds'] / args.steps * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
        # temporal error of the FP64 run: same end time with half the step
        wl2 = dict(wl)
        wl2["dt"] = wl["dt"] / 2
        half = run_variant(P, torch, wl2, P.FP64, 2 * (args.steps + args.warmup), 0)
        extra = dict(
            fp64_plain_value=M * args.steps / fp64["seconds"],
            fp64_plain_ms_per_step=fp64["seconds"] / args.steps * 1e3,
            speedup_mixed_vs_fp64=fp64["seconds"] / mixed["seconds"],
            l2_rel_mixed_vs_fp64=l2_rel(mixed["u"], fp64["u"]),
            l2_rel_temporal_fp64=l2_rel(fp64["u"], half["u"]),
            t_end_mixed=mixed["t"], t_end_fp64=fp64["t"], t_end_half=half["t"])
        extra["equal_l2_error"] = extra["l2_rel_mixed_vs_fp64"] < 0.1 * extra["l2_rel_temporal_fp64"]

    stats = mixed["stats"]
    dom = max(stats, key=lambda k: stats[k]["ms"])
    s = stats[dom]
    achieved = s["bytes"] / (s["ms"] * 1e-3) / 1e9 if s["ms"] > 0 else 0.0
    roofline = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=achieved / HBM_PEAK_GBS, traffic=None, kernel=f"stage kernel ({dom})",
                    avg_launch_us=s["ms"] / max(s["launches"], 1) * 1e3,
                    bytes_per_launch=s["bytes"] / max(s["launches"], 1))
    breakdown = {k: dict(ms_per_step=v["ms"] / args.steps, launches_per_step=v["launches"] / args.steps,
                         GBps=(v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] > 0 and v["bytes"] > 0 else None))
                 for k, v in stats.items()}

    ms_per_step = mixed["seconds"] / args.steps * 1e3
    line = {
        "metric": METRIC,
        "value": M * args.steps / mixed["seconds"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 fluxes + f64 relaxation",
        "data": "synthetic",
        "config": {"workload": wl["name"], "description": wl["desc"], "dof": int(M),
                   "elements": int(wl["U0"].shape[1]), "dt": wl["dt"],
                   "level_counts": np.bincount(wl["lev"], minlength=3).tolist(), "variant": "mixed",
                   "newton_guess": "previous gamma"},
        "roofline": roofline,
        "kernel_breakdown": breakdown,
    }
    line.update(extra)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
