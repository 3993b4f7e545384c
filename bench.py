#!/usr/bin/env python3
"""Throughput of the P-ERRK step on one MI355X.

Default workload (--workload ensemble): 256 independent 2D isentropic-vortex
cases (strength U[1, 6], centre U[3, 7]^2, periodic [0, 10]^2) on graded
meshes (ratio 4, finest at the centre) of 16^2, 32^2, 48^2 or 64^2 elements,
DGSEM degree 3, Ranocha EC volume and surface flux, third-order P-ERRK with
stage-evaluation levels E = {4, 6, 8, 12} assigned by each element's shortest
edge with one wave speed per case, and a per-case step size; all cases advance together (one launch per stage over
every case's active elements, the step captured in a hipGraph).
--workload tgv: 3D Taylor-Green vortex, Mach 0.1, 32^3 graded hexahedra,
fourth-order P-ERRK with E = {5, 9, 14}.
--workload alfven: 2D ideal GLM-MHD Alfven wave, 256^2 uniform cells, weak form
with LLF surface flux and the Powell / GLM terms, p = 3 with E = {10..14} at
random (the GLM-MHD path is double precision only; no comparisons).
--viscous MU: the 2D Euler workload with Navier-Stokes-Fourier terms (BR1,
Pr = 0.72, double precision only; no comparisons).
--surface-flux / --volume: the same workload with a dissipative surface flux
(HLL, LLF, HLLE, HLLC) and/or the standard weak-form volume term (Sec. 4.2, 4.3
and 5 use these), which runs the stage kernel's dissipative instantiation.

Variants on identical inputs (same mesh, dt, steps and initial state):
  mixed(+learned)      single-precision fluxes, flux accumulation, stage states and
                       K storage in the stages with b_i = 0; the stages entering d
                       and dH, d, entropy sums and the gamma solve in double precision;
  mixed_all(+learned)  the same single precision in every stage; d and the stage
                       entropy production accumulated in double precision;
  fp64                 double precision throughout;
"+learned": the first Newton point is the previous gamma plus the learned
increment (otherwise the previous gamma); "fp64+extrapolated" (ensemble only):
fp64 starting from the linear extrapolation of the root history, beside the
plain fp64 baseline (previous gamma).  The headline is mixed+learned
(mixed where no network applies); mixed_all is faster but its states deviate
from FP64 about ten times more, enough to miss "equal L2 error" on some cases.
For the ensemble the L2 error of each case against the exact advected vortex at
the case's own relaxed end time decides "equal L2 error" (within 1 % of FP64's).

Prints one JSON line.  Inputs are synthetic and seeded.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "P-ERRK DOF-updates/s on 1 GPU; mixed/learned vs FP64 plain at equal L2 error"
HBM_PEAK_GBS = 8000.0
FLUX_NAMES = ["ec", "hll", "llf", "hlle", "hllc"]  # PERRK_FLUX_* order
VOLUME_NAMES = ["flux_differencing", "weak"]  # PERRK_VOLUME_* order
Q1 = np.array([1.0, 5.0, 5.0, 1.0]) / 6.0


def workload_ensemble(n_cases=256, seed=0):
    from paper_2507_04991_amd import problems

    wl = problems.ensemble(seed, n_cases)
    wl["desc"] = (f"{n_cases} 2D Euler isentropic vortices (strength U[1,6], centre U[3,7]^2) on graded "
                  f"(ratio 4) periodic meshes of 16^2..64^2 quads, DGSEM k=3, Ranocha EC volume+surface "
                  f"flux, P-ERRK p=3 E={{4,6,8,12}}, per-case dt and levels (shortest edge, CFL 0.5)")
    return wl


def workload_tgv(n=32, seed=0):
    from paper_2507_04991_amd import problems

    wl = problems.tgv32(seed, n)
    wl["desc"] = (f"3D Euler Taylor-Green Mach 0.1, {n}^3 graded (ratio 4) periodic hexes, DGSEM k=3, "
                  f"Ranocha EC volume+surface flux, P-ERRK p=4 E={{5,9,14}}")
    return wl


def workload_alfven(n=256, seed=0):
    from paper_2507_04991_amd import problems

    wl = problems.alfven(seed, n)
    wl["desc"] = (f"2D ideal GLM-MHD Alfven wave (gamma 5/3, c_h 1) on [0, sqrt 2]^2, {n}^2 uniform quads, "
                  f"DGSEM k=3, weak-form volume term, LLF surface flux, Powell and GLM terms, P-ERRK p=3 "
                  f"E={{10..14}} assigned to the cells at random")
    return wl


def run_variant(P, torch, wl, precision, steps, warmup, profile=False, guess=0, model=None):
    d = P.Descriptors(wl["faces"], wl["lev"], wl["tab"], surface_flux=wl.get("flux", 0), precision=precision,
                      volume_integral=wl.get("volume", 0), gas_gamma=wl.get("gam", 1.4),
                      system=wl.get("system", 0), glm_ch=wl.get("glm_ch", 0.0), viscous=wl.get("viscous", 0),
                      mu=wl.get("mu", 0.0), prandtl=wl.get("prandtl", 0.75), bc_x=wl.get("bc_x", 0))
    st = P.Stepper(d, P.default_options(guess=guess))
    if model is not None:
        st.set_guess_model(*model)
    u = torch.tensor(wl["U0"], dtype=torch.float64, device="cuda").contiguous()
    for _ in range(warmup):
        st.step(u, wl["dt"], info=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st.step(u, wl["dt"], info=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rs = st.relaxation_state()
    g, tt = rs.gamma_prev, rs.t
    out = dict(seconds=t1 - t0, u=u.clone(), gamma=g, t=tt)
    # untimed: two synchronous steps on a copy to sample the solver statistics
    us = u.clone()
    infos = st.step(us, wl["dt"]) + st.step(us, wl["dt"])
    out["passes_mean"] = float(np.mean([i["passes"] for i in infos]))
    out["r_max"] = float(max(abs(i["r"]) for i in infos))
    out["fallbacks"] = int(sum(1 for i in infos if i["flags"] & P.FLAG_FALLBACK))
    if profile:
        # the same kernels launched one by one with HIP events around each launch
        st.set_profiling(True)
        st.kernel_stats(reset=True)
        up = u.clone()
        for _ in range(steps):
            st.step(up, wl["dt"], info=False)
        out["stats"] = st.kernel_stats(reset=True)
        out["stage_stats"] = st.stage_stats(reset=True)
        st.set_profiling(False)
    out["tuning"] = st.tuning()
    st.close()
    return out


ARITHMETIC = {
    "mixed_all": "fluxes, flux accumulation, stage states and K storage in f32 in every stage; d, stage entropy "
                 "production, entropy sums and the gamma solve in f64",
    "mixed": "fluxes, stage states and K storage of the stages with b_i = 0 in f32; stages with b_i != 0, d, "
             "entropy sums and the gamma solve in f64",
    "fp64": "f64 throughout",
}


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary kept under profiles/ (scaled by the copy-kernel calibration), or None
    when there is none for this workload or the kernel source has changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    src = os.path.join(ROOT, "paper_2507_04991_amd", "csrc", "perrk_kernels.hip")
    with open(src, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    if t.get("kernel_source_sha256") != digest:
        return None
    e = t.get("entries", {}).get(f"{workload}|{kernel}")
    return None if e is None else e["bytes_per_launch"]


def fp32_mid_active_dof(wl, precision):
    """Active DOF summed over the single-precision middle stages of one step."""
    b = np.asarray(wl["tab"]["b"])
    E = np.asarray(wl["tab"]["E"])
    S = len(b)
    V = wl["U0"].shape[0]
    npe = wl["U0"].shape[2]
    per_level = sum(np.bincount(np.asarray(lv), minlength=len(E)) for lv in wl["lev"])
    total = 0
    for i in range(1, S - 1):
        if precision == 0 or (precision == 1 and b[i] != 0.0):
            continue
        total += int(per_level[E >= S - i + 1].sum())  # stage i + 1 runs the levels with E >= S - i + 1
    return float(total) * V * npe


def stage_groups(wl, stage_stats, precision):
    """Sums the per-stage profiling statistics by stage-kernel instantiation:
    <dim, flux type, storage type, kind> (precision 0 = FP64, 1 = MIXED, whose
    stages with b_i != 0 compute their fluxes in double precision, 2 = MIXED_ALL)."""
    dim = len(wl["faces"][0])
    b = np.asarray(wl["tab"]["b"])
    S = len(b)
    out = {}
    for i, s in enumerate(stage_stats):
        if s["launches"] == 0:
            continue
        kind = "first" if i == 0 else ("last" if i == S - 1 else "mid")
        ft = "double" if precision == 0 or (precision == 1 and b[i] != 0.0) else "float"
        st = "double" if precision == 0 else "float"
        name = f"stage_kernel<{dim}, {ft}, {st}, {kind}>"
        if wl.get("system", 0) == 1:
            name = f"mhd_stage_kernel<{kind}>"
        elif wl.get("viscous", 0):
            name = f"ns_grad_kernel+ns_stage_kernel<{kind}>"
        g = out.setdefault(name, dict(ms=0.0, bytes=0.0, launches=0))
        g["ms"] += s["ms"]
        g["bytes"] += s["bytes"]
        g["launches"] += s["launches"]
    return out


def ensemble_l2_errors(wl, U, t):
    """Per case: || U - U_exact(t_case) ||_L2 / || U_exact ||_L2 (quadrature weighted)."""
    from paper_2507_04991_amd import workloads as W

    errs = []
    off = 0
    for k, c in enumerate(wl["cases"]):
        ne = c["U0"].shape[1]
        co = W.node_coords(c["faces"])
        Ue = W.vortex_state(co, t=float(t[k]), strength=c["strength"], centre=c["centre"])
        w = W.element_widths(c["faces"])
        J = (w[:, 0] * w[:, 1] / 4.0)[:, None] * np.outer(Q1, Q1).reshape(1, 16)  # ordering i + 4 j
        Uk = U[:, off:off + ne]
        errs.append(math.sqrt(float(((Uk - Ue) ** 2 * J).sum()) / float((Ue ** 2 * J).sum())))
        off += ne
    return np.array(errs)


def _oracle_case_step(O, t, wl, k, U):
    faces = wl["faces"][k]
    m = O.Mesh(faces, gam=wl.get("gam", 1.4), surface_flux=wl.get("flux", 0),
               volume_integral=wl.get("volume", 0), physics=wl.get("system", 0), c_h=wl.get("glm_ch", 0.0),
               viscous=wl.get("viscous", 0), mu=wl.get("mu", 0.0), prandtl=wl.get("prandtl", 0.75))
    O.step(m, t, wl["lev"][k], U, float(wl["dt"][k]))
    return U.size


def host_cores():
    """Host threads this process may use (at most 16, the CPU share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(wl, target_dof=12.0e6, pool_dof=40.0e6):
    """The FP64 CPU oracle on the host: one step of a leading subset of the
    workload's cases, single-threaded, and the same oracle on every host core
    (at most 16) with the cases of a larger leading subset stepped in parallel
    (independent cases; the oracle's C code releases the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O

    t = O.Tableau(wl["tab"]["order"], wl["tab"]["c"], wl["tab"]["b"], wl["tab"]["a_sub"], wl["tab"]["E"])
    offs = np.cumsum([0] + [np.asarray(lv).shape[0] for lv in wl["lev"]])
    cases = [wl["U0"][:, offs[k]:offs[k + 1]] for k in range(len(wl["faces"]))]
    dof, sec, ncase = 0, 0.0, 0
    for k, U in enumerate(cases):
        t0 = time.perf_counter()
        _oracle_case_step(O, t, wl, k, U)
        sec += time.perf_counter() - t0
        dof += U.size
        ncase += 1
        if dof >= target_dof:
            break
    single = dict(value=dof / sec, unit="DOF-updates/s", cores=1, kind="oracle",
                  sample=f"one P-ERRK step of the first {ncase} of {len(cases)} cases of the same workload "
                         f"({dof} DOF, {sec:.1f} s, single thread)")
    sel, pdof = [], 0
    for k, U in enumerate(cases):
        sel.append(k)
        pdof += U.size
        if pdof >= pool_dof:
            break
    threads = min(host_cores(), len(sel))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        done = sum(ex.map(lambda k: _oracle_case_step(O, t, wl, k, cases[k]), sel))
    psec = time.perf_counter() - t0
    return dict(value=done / psec, unit="DOF-updates/s", cores=threads, kind="oracle",
                sample=f"one P-ERRK step of the first {len(sel)} of {len(cases)} cases of the same workload "
                       f"({done} DOF, {psec:.1f} s on {threads} host threads, one case per task)",
                single_thread=single)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["ensemble", "tgv", "alfven"], default="ensemble")
    ap.add_argument("--surface-flux", choices=FLUX_NAMES, default=None,
                    help="surface flux instead of the workload's own (EC)")
    ap.add_argument("--volume", choices=VOLUME_NAMES, default="flux_differencing",
                    help="volume term: EC flux differencing or the standard weak form")
    ap.add_argument("--viscous", type=float, default=None, metavar="MU",
                    help="add the Navier-Stokes-Fourier terms (BR1, Pr 0.72) with viscosity MU (2D Euler workloads; "
                         "double precision)")
    ap.add_argument("--tgv-n", type=int, default=32, metavar="N",
                    help="elements per direction of the Taylor-Green mesh (64: 84 M DOF, beyond the Infinity Cache)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="time the mixed variant only")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 5 times (calibrates HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the path is single-GPU "
                                   "(multi-GPU sharding is described, not built)", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2507_04991_amd import learned_guess as LG
    from paper_2507_04991_amd import perrk as P

    P.lib()
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / 5
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "seconds_per_copy": sec,
                          "GBps_read_plus_write": 2 * n * 8 / sec / 1e9}), flush=True)
        return
    wl = {"ensemble": workload_ensemble, "tgv": lambda: workload_tgv(n=args.tgv_n),
          "alfven": workload_alfven}[args.workload]()
    mhd = wl.get("system", 0) == 1
    if args.viscous is not None:
        if mhd or len(wl["faces"][0]) != 2:
            sys.exit("--viscous applies to the 2D Euler workloads")
        wl.update(viscous=1, mu=args.viscous, prandtl=0.72)
        wl["name"] += f"_ns_mu{args.viscous:g}"
        wl["desc"] += f"; Navier-Stokes-Fourier terms by BR1, mu = {args.viscous:g}, Pr = 0.72"
    fp64_only = mhd or args.viscous is not None
    if args.surface_flux is not None or args.volume != "flux_differencing":
        fl = FLUX_NAMES.index(args.surface_flux) if args.surface_flux is not None else wl.get("flux", 0)
        wl["flux"], wl["volume"] = fl, VOLUME_NAMES.index(args.volume)
        wl["name"] += f"_{FLUX_NAMES[fl]}_{args.volume}"
        wl["desc"] += f"; surface flux {FLUX_NAMES[fl]}, volume term {args.volume} (instead of EC)"
    M = wl["U0"].size
    print(f"# workload {wl['name']}: {M} DOF, {len(wl['faces'])} case(s)", file=sys.stderr, flush=True)

    # variants on identical inputs: name -> (precision, initial guess of the Newton
    # iteration); the first is the headline (the learned guess needs the network
    # trained on the ensemble).  fp64 is the plain baseline (previous gamma);
    # fp64+extrapolated starts from the linear extrapolation of the root history.
    learned = wl["kind"] == "ensemble" and os.path.exists(LG.DEFAULT_MODEL)
    MLP, PREV, EXTRAP = P.GUESS_MLP, P.GUESS_PREV, P.GUESS_EXTRAP
    plan = [("mixed+learned", P.MIXED, MLP), ("mixed", P.MIXED, PREV), ("mixed_all+learned", P.MIXED_ALL, MLP),
            ("mixed_all", P.MIXED_ALL, PREV), ("fp64", P.FP64, PREV)]
    if wl["kind"] == "ensemble":
        plan.append(("fp64+extrapolated", P.FP64, EXTRAP))
    if not learned:
        plan = [(n, p, g) for n, p, g in plan if g != MLP]
    if fp64_only:  # the GLM-MHD and viscous paths are double precision only
        plan = [("fp64", P.FP64, PREV)]
    if args.no_compare:
        plan = plan[:1]
    head_name = plan[0][0]
    runs = {}
    model = LG.load(LG.DEFAULT_MODEL) if learned else None
    for k, (name, prec, guess) in enumerate(plan):
        runs[name] = run_variant(P, torch, wl, prec, args.steps, args.warmup, profile=(k == 0),
                                 guess=guess, model=model if guess == MLP else None)
    extra = {"variants": {}}
    for name, r in runs.items():
        print(f"# {name}: {r['seconds'] / args.steps * 1e3:.3f} ms/step, passes {r['passes_mean']}",
              file=sys.stderr, flush=True)
        extra["variants"][name] = dict(value=M * args.steps / r["seconds"], ms_per_step=r["seconds"] / args.steps * 1e3,
                                       newton_passes_per_step=r["passes_mean"], max_abs_r=r["r_max"],
                                       fallback_steps=r["fallbacks"])
    mixed = runs[head_name]
    if "fp64" in runs:
        fp64 = runs["fp64"]
        uf = fp64["u"].cpu().numpy()
        ef = ensemble_l2_errors(wl, uf, fp64["t"]) if wl["kind"] == "ensemble" else None
        names = ["rho"] + [f"m{k}" for k in range(uf.shape[0] - 2)] + ["E"]
        for name, r in runs.items():
            v = extra["variants"][name]
            v["speedup_vs_fp64"] = fp64["seconds"] / r["seconds"]
            if name == "fp64":
                continue
            um = r["u"].cpu().numpy()
            v["field_rel_l2_diff_vs_fp64"] = {n: float(np.linalg.norm(um[i] - uf[i]) / np.linalg.norm(uf[i]))
                                             for i, n in enumerate(names)}
            if ef is not None:
                em = ensemble_l2_errors(wl, um, r["t"])
                rel = np.abs(em - ef) / ef
                v.update(l2_error_mean=float(em.mean()), l2_error_rel_diff_vs_fp64_max=float(rel.max()),
                         equal_l2_error=bool(rel.max() <= 0.01))
            else:
                v.update(gamma=float(r["gamma"][0]), gamma_fp64=float(fp64["gamma"][0]))
        if ef is not None:
            extra["variants"]["fp64"]["l2_error_mean"] = float(ef.mean())

    stats = mixed["stats"]
    breakdown = {k: dict(ms_per_step=v["ms"] / args.steps, launches_per_step=v["launches"] / args.steps,
                         GBps=(v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] > 0 and v["bytes"] > 0 else None))
                 for k, v in stats.items()}
    # stage launches grouped by kernel instantiation (the mixed variant runs the
    # stages with b_i != 0 with double-precision fluxes)
    groups = stage_groups(wl, mixed["stage_stats"], plan[0][1])
    dom = max(groups, key=lambda k: groups[k]["ms"])
    g = groups[dom]
    achieved = g["bytes"] / (g["ms"] * 1e-3) / 1e9
    roofline = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=measured_traffic(wl["name"], dom), kernel=dom,
                    avg_launch_us=g["ms"] / g["launches"] * 1e3, bytes_per_launch=g["bytes"] / g["launches"],
                    launches_per_step=g["launches"] / args.steps)
    if ", float, float, mid>" in dom:
        # the single-precision stages read U_n from its single-precision copy (4 B per
        # DOF); counted with U_n in double precision, as the planned 20 B per active DOF
        u64_bytes = 4.0 * fp32_mid_active_dof(wl, plan[0][1]) * args.steps
        b20 = g["bytes"] + u64_bytes
        roofline.update(bytes_per_launch_fp64_state=b20 / g["launches"],
                        achieved_fp64_state=b20 / (g["ms"] * 1e-3) / 1e9,
                        frac_fp64_state=b20 / (g["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS)
    stage_breakdown = {k: dict(ms_per_step=v["ms"] / args.steps, launches_per_step=v["launches"] / args.steps,
                               avg_launch_us=v["ms"] / v["launches"] * 1e3,
                               GBps=v["bytes"] / (v["ms"] * 1e-3) / 1e9) for k, v in groups.items()}

    line = {
        "metric": METRIC,
        "value": M * args.steps / mixed["seconds"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["seconds"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head_name == "fp64" else "f32/f64",
        "data": "synthetic",
        "config": {"workload": wl["name"], "description": wl["desc"], "dof": int(M),
                   "elements": int(wl["U0"].shape[1]), "cases": len(wl["faces"]), "variant": head_name,
                   "arithmetic": ARITHMETIC[head_name.replace("+learned", "")]},
        "roofline": roofline,
        "kernel_breakdown": breakdown,
        "stage_kernel_breakdown": stage_breakdown,
        "tuning": mixed["tuning"],
    }
    # right-hand-side evaluations per step, counted in DOF: sum_r E^(r) M^(r)
    E = np.asarray(wl["tab"]["E"])
    n_rhs = float(sum(E[np.asarray(lv)].sum() for lv in wl["lev"])) * (M / wl["U0"].shape[1])
    if not args.no_compare and not fp64_only:
        # the paper's comparison: the same mesh, dt and steps with every element on the
        # largest-E level (the single-level method P-ERRK_{p;S_max}); tau / tau* and
        # N_RHS / N_RHS* with * = multirate
        R = len(E)
        wl1 = dict(wl, lev=[np.full_like(np.asarray(lv), R - 1) for lv in wl["lev"]])
        head = plan[0]
        one = run_variant(P, torch, wl1, head[1], args.steps, args.warmup,
                          guess=head[2], model=model if head[2] == MLP else None)
        n_rhs1 = float(E[-1]) * M
        cmp = dict(variant=head_name, single_level_ms_per_step=one["seconds"] / args.steps * 1e3,
                   multirate_ms_per_step=mixed["seconds"] / args.steps * 1e3,
                   tau_ratio=one["seconds"] / mixed["seconds"], n_rhs_ratio=n_rhs1 / n_rhs,
                   single_level_newton_passes_per_step=one["passes_mean"], single_level_max_abs_r=one["r_max"])
        if wl["kind"] == "ensemble":
            e1 = ensemble_l2_errors(wl, one["u"].cpu().numpy(), one["t"])
            em = ensemble_l2_errors(wl, mixed["u"].cpu().numpy(), mixed["t"])
            cmp.update(l2_error_mean_single_level=float(e1.mean()), l2_error_mean_multirate=float(em.mean()))
        print(f"# single level: {cmp['single_level_ms_per_step']:.3f} ms/step, tau/tau* {cmp['tau_ratio']:.3f}, "
              f"N_RHS/N_RHS* {cmp['n_rhs_ratio']:.3f}", file=sys.stderr, flush=True)
        extra["multirate_vs_single_level"] = cmp
        # relaxed classic RK4 (R-RK_{4;4}) at its own stable step, compared per unit of
        # simulated time: tau / tau* = (ms per step / dt) ratio, with * = multirate
        from paper_2507_04991_amd import tableau as T
        from paper_2507_04991_amd import workloads as W
        rk4 = T.classic_rk4()
        dim = len(wl["faces"][0])
        dts4, levs4, off = [], [], 0
        for k, faces in enumerate(wl["faces"]):
            ne = np.asarray(wl["lev"][k]).shape[0]
            dt4, lv4 = T.assign_levels(rk4, W.element_widths(faces).min(axis=1),
                                       W.max_wave_speed(wl["U0"][:, off:off + ne], dim))
            dts4.append(dt4)
            levs4.append(lv4)
            off += ne
        wl4 = dict(wl, tab=rk4, lev=levs4, dt=np.array(dts4))
        r4 = run_variant(P, torch, wl4, head[1], args.steps, args.warmup)
        ratio_dt = float(np.mean(np.asarray(wl["dt"]) / np.array(dts4)))
        ms4 = r4["seconds"] / args.steps * 1e3
        ms_m = mixed["seconds"] / args.steps * 1e3
        rk = dict(precision_mode=head_name.replace("+learned", ""), rk4_ms_per_step=ms4,
                  dt_ratio_multirate_over_rk4=ratio_dt, tau_ratio=ms4 * ratio_dt / ms_m,
                  n_rhs_ratio=4.0 * M * ratio_dt / n_rhs, rk4_newton_passes_per_step=r4["passes_mean"],
                  rk4_max_abs_r=r4["r_max"])
        print(f"# relaxed RK4: {ms4:.3f} ms/step at dt x {1 / ratio_dt:.3f}, tau/tau* {rk['tau_ratio']:.3f}, "
              f"N_RHS/N_RHS* {rk['n_rhs_ratio']:.3f}", file=sys.stderr, flush=True)
        extra["multirate_vs_relaxed_rk4"] = rk
    extra.update(rhs_dof_evals_per_step=n_rhs, rhs_dof_evals_per_s=n_rhs * args.steps / mixed["seconds"],
                 newton_passes_per_step=mixed["passes_mean"], max_abs_r=mixed["r_max"])
    line.update(extra)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
