"""Benchmark: space-time unknowns per second to a 1e-8 relative residual on one MI355X.

A step is one complete ParaDiag-II solve of the all-at-once system of the
workload (right-hand side resident in HBM): flexible GMRES with the
alpha-circulant preconditioner -- time FFTs, x-transforms, line solves or the
Schur back-sweep, matvec, Gram-Schmidt -- until ||b - A u|| <= 1e-8 ||b||.
The mixed-precision preconditioner (float32 FFT and line solves, bf16 MFMA
x-transform) is timed next to the plain float64 one on the same problem;
`value` is the mixed-precision rate.

The default workload is 2D advection-diffusion on 512 x 512 interior points,
Nt = 1024 trapezoidal steps, with a batch of 8 source terms solved in one
launch (2.15e9 space-time unknowns).

The JSON line also carries
* the roofline of the dominant kernel (algorithmic bytes or flops per launch
  over the average launch time, both measured by the library with HIP events
  on the solve's stream during the timed steps);
* the error of right-hand side 0 against the float64 oracle's sequential time
  stepper over the whole horizon, for both precisions (computed after the
  timed region);
* CPU baselines: the oracle's sequential stepper on that right-hand side
  (one core; it also yields the error reference), and a sample of the
  oracle's own ParaDiag-II preconditioner with Step-(b) spread over the host
  cores, scaled to a whole solve.
* a ParaDiag-I leg (key `paradiag_i`): the direct float64 solve of the hybrid
  time discretisation on the wave problem of Table Ex2Tab1 (511^2 x 512), its
  rate, its error against the exact solution and its dominant kernel's
  roofline.
One extra solve before the timed region, with every stage timed, gives the
per-stage breakdown and picks the dominant stage; inside the timed region only
that stage records events, since every event pair costs a few microseconds of
stream time.
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

PEAK = {  # MI355X published peaks
    "hbm_GBs": 8000.0,
    "mfma_TFs": {"fp64": 78.6, "fp32": 157.3, "fp32_bf16gemm": 2500.0, "fp32_bf16x1": 2500.0},
    "vector_TFs": {"fp64": 78.6, "fp32": 157.3, "fp32_bf16gemm": 157.3, "fp32_bf16x1": 157.3},
}

# bound of each stage of the library's accounting
STAGE_BOUND = {"fft_fwd": "hbm", "fft_inv": "hbm", "line_solve": "hbm", "matvec": "hbm",
               "dot": "hbm", "update": "hbm", "other": "hbm", "xform_fwd": "mfma",
               "xform_inv": "mfma"}

STAGE_KERNEL = {"fft_fwd": "k_fft_fwd", "fft_inv": "k_fft_inv", "line_solve": "k_schur_sweep",
                "matvec": "k_matvec", "dot": "k_mdot", "update": "k_update", "other": "k_reduce",
                "xform_fwd": "k_gemm", "xform_inv": "k_gemm"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg3", choices=["cfg1", "cfg2", "cfg3", "cfg4", "cfg5"])
    ap.add_argument("--mixed", default=None, choices=["fp32", "fp32_bf16gemm", "fp32_bf16x1"],
                    help="reduced-precision preconditioner (default: the workload's own; float32 "
                         "for the wave equation, split-bf16 x-transform otherwise)")
    ap.add_argument("--restart", type=int, default=8)
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--skip-paradiag-i", action="store_true",
                    help="skip the ParaDiag-I (hybrid time discretisation) leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle", action="store_true",
                    help="skip the oracle's sequential solve (no error_vs_oracle, no cpu_baseline)")
    ap.add_argument("--traffic", default=None,
                    help="profile summary holding a 'traffic: {...}' line with the measured HBM "
                         "bytes per launch of the dominant kernel (default: profiles/<kernel>_<workload>_traffic.md)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized float64 tensor 3 times (HBM counter calibration)")
    return ap.parse_args()


def copy_probe(mib: int) -> None:
    """A plain device-to-device copy of known size, for calibrating HBM byte counters."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8}), flush=True)


def make_inputs(cfg, torch, pd):
    from workloads import initial_state, initial_velocity, source_term_torch
    U0 = torch.from_numpy(initial_state(cfg)).cuda()
    U0 = U0.reshape(1, cfg.ny, cfg.nx).expand(cfg.batch, cfg.ny, cfg.nx).contiguous()
    u1 = None
    if cfg.scheme == "lf":
        u1 = torch.from_numpy(initial_velocity(cfg)).cuda().reshape(1, cfg.ny, cfg.nx)
        u1 = u1.expand(cfg.batch, cfg.ny, cfg.nx).contiguous()
    f = None
    if cfg.with_source:
        f = torch.empty(pd.source_shape, dtype=torch.float64, device="cuda")
        for s in range(cfg.batch):
            f[s] = source_term_torch(cfg, cfg.seed + 1 + s, "cuda")
    return U0, u1, f


def run_precision(cfg, prec, args, torch):
    from paper_2005_09158_amd import ParaDiag
    # the FGMRES workspace holds restart+1 float64 and restart preconditioned
    # vectors: a shorter restart where the requested one does not fit in HBM
    # (with the right-hand side, the solution and the source term beside it)
    restart, pd = args.restart, None
    while pd is None:
        try:
            pd = ParaDiag(dim=cfg.dim, nx=cfg.nx, ny=cfg.ny, nt=cfg.nt, scheme=cfg.scheme, T=cfg.T,
                          nu=cfg.nu, ax=cfg.ax, ay=cfg.ay, alpha=cfg.alpha, batch=cfg.batch,
                          prec=prec, restart=restart)
            U0, u1, f = make_inputs(cfg, torch, pd)
            b = pd.build_rhs(U0, u1, f)
            del f
            u = torch.empty_like(b)
        except torch.OutOfMemoryError:
            pd = U0 = u1 = f = b = None
            torch.cuda.empty_cache()
            if restart <= 2:
                raise
            restart -= 1
            print(f"[bench] {prec}: does not fit in HBM, restart {restart}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        pd.solve(b, u, rtol=cfg.rtol, max_iter=200, restart=restart)
    # one solve with every stage timed, outside the timed region: the per-stage
    # breakdown, and the dominant stage
    pd.set_timing(True)
    pd.stage_times(reset=True)
    pd.solve(b, u, rtol=cfg.rtol, max_iter=200, restart=restart)
    stages = pd.stage_times(reset=True)
    dominant = max(stages, key=lambda k: stages[k][0])
    # timed region: only the dominant stage records events (they cost time)
    pd.set_timing(True, stages=[dominant])
    pd.stage_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(args.steps):
        _, res = pd.solve(b, u, rtol=cfg.rtol, max_iter=200, restart=restart)
        results.append(res)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timed = pd.stage_times(reset=True)
    pd.set_timing(False)
    ms = (t1 - t0) * 1e3 / args.steps
    out = dict(prec=prec, ms_per_step=ms, restart=restart, iters=[r.iters for r in results],
               rel_resid=max(r.rel_resid for r in results),
               converged=all(r.converged for r in results), stages=stages, dominant=dominant,
               dominant_timed=timed[dominant])
    # right-hand side 0 of the last timed solve, for the error against the
    # oracle (outside the timed region)
    u0 = u[0].cpu().numpy().reshape(cfg.nt, -1)
    del b, u, pd
    torch.cuda.empty_cache()
    return out, u0


KERNEL_SOURCES = {"k_schur_sweep": ("kernels_sweep.hip", "tri_device.h")}


def measured_traffic(path, kernel, workload, prec):
    """HBM bytes per launch from a committed counter summary, or None.

    The summary's 'traffic:' line names the kernel, workload and precision it was
    measured on and the sha256 of the kernel's sources; any mismatch (the kernel
    changed since the counters were read) gives None.
    """
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = path or os.path.join(here, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCES:
        return None
    rec = None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic: "):
                rec = json.loads(line[len("traffic: "):])
    if not rec or (rec.get("kernel"), rec.get("workload"), rec.get("prec")) != (kernel, workload, prec):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(here, "paper_2005_09158_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec.get("source_sha256"):
        return None
    return rec.get("bytes_per_launch")


def roofline(run, cfg, traffic_file):
    name = run["dominant"]
    ms, cnt, by, fl = run["dominant_timed"]   # events of the timed region
    bound = STAGE_BOUND[name]
    if name == "line_solve" and cfg.dim == 2 and cfg.ax != 0.0:
        bound = "mfma"  # Schur back-sweep: the coupling product runs on MFMA
    avg_s = ms / 1e3 / max(cnt, 1)
    if bound == "hbm":
        achieved = by / max(cnt, 1) / avg_s / 1e9
        peak, unit = PEAK["hbm_GBs"], "GB/s"
    elif bound == "mfma":
        achieved = fl / max(cnt, 1) / avg_s / 1e12
        # the back-sweep's products run in the line precision (float32 in mixed modes)
        key = run["prec"] if name != "line_solve" else ("fp64" if run["prec"] == "fp64" else "fp32")
        peak, unit = PEAK["mfma_TFs"][key], "TFLOP/s"
    else:
        achieved = fl / max(cnt, 1) / avg_s / 1e12
        peak, unit = PEAK["vector_TFs"][run["prec"]], "TFLOP/s"
    traffic = measured_traffic(traffic_file, STAGE_KERNEL[name], cfg.name, run["prec"])
    return {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4), "traffic": traffic, "kernel": STAGE_KERNEL[name],
            "stage": name, "launches": cnt, "avg_launch_ms": round(ms / max(cnt, 1), 5),
            "algorithmic_bytes_per_launch": by / max(cnt, 1),
            "algorithmic_flops_per_launch": fl / max(cnt, 1)}


def stage_rooflines(run):
    """Per-stage average launch time and achieved rate against the stage's bound."""
    out = {}
    for name, (ms, cnt, by, fl) in run["stages"].items():
        if cnt == 0:
            continue
        avg_s = ms / 1e3 / cnt
        rec = {"launches": cnt, "avg_launch_ms": round(ms / cnt, 5),
               "GBs": round(by / cnt / avg_s / 1e9, 1),
               "hbm_frac": round(by / cnt / avg_s / 1e9 / PEAK["hbm_GBs"], 4)}
        if fl:
            rec["TFs"] = round(fl / cnt / avg_s / 1e12, 2)
        out[name] = rec
    return out


def oracle_reference(cfg):
    """The oracle's right-hand side 0 and its solution by sequential float64
    time stepping over the whole horizon (one sparse LU, then Nt triangular
    solves, one thread), with the wall time of the stepping."""
    from threadpoolctl import threadpool_limits
    from oracle import Problem, rhs, solve
    from workloads import initial_state, initial_velocity, source_term
    p = Problem.from_kwargs(**cfg.problem_kwargs())
    with threadpool_limits(1):
        U0 = initial_state(cfg)
        f = source_term(cfg, cfg.seed + 1) if cfg.with_source else None
        u1 = initial_velocity(cfg) if cfg.scheme == "lf" else None
        b = rhs.build_rhs(p, U0, u1, f)
        del f
        t0 = time.perf_counter()
        ref = solve.sequential(p, b)
        dt = time.perf_counter() - t0
    return p, ref, dt


def error_vs_oracle(u, ref):
    """Relative error of one right-hand side's solution: max norm and 2-norm."""
    d = u - ref
    return {"max_rel": float(np.abs(d).max() / np.abs(ref).max()),
            "l2_rel": float(np.linalg.norm(d) / np.linalg.norm(ref))}


def _stepb_worker(args):
    """One Step-(b) solve of the oracle at frequency n (a worker process)."""
    kw, n = args
    from threadpoolctl import threadpool_limits
    from oracle import Problem, precond
    p = Problem.from_kwargs(**kw)
    s1 = np.random.default_rng(n).standard_normal(p.nspace) + 1j * np.random.default_rng(n + 1).standard_normal(p.nspace)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        precond.frequency_solve(p, n, s1)
        return time.perf_counter() - t0


def cpu_paradiag_sample(cfg, cores):
    """Wall time of Step-(b) of the oracle's ParaDiag-II preconditioner on
    `cores` frequencies at once, one sparse LU and solve per frequency and per
    worker process: the paper's own parallelisation across time points on one
    node.  Run before the GPU is touched (the workers are forked)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    kw = cfg.problem_kwargs()
    freqs = [1 + (k * (cfg.nt - 1)) // cores for k in range(cores)]
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("fork")) as ex:
        per = list(ex.map(_stepb_worker, [(kw, n) for n in freqs]))
    wall = time.perf_counter() - t0
    return {"wall_s": wall, "freqs": len(freqs), "per_freq_s": float(np.mean(per))}


def cpu_baselines(cfg, ref_dt, sample, iters):
    """cpu_baseline (sequential oracle stepper) and the scaled CPU ParaDiag-II figure."""
    U1 = cfg.nx * cfg.ny * cfg.nt   # unknowns of one right-hand side
    base = {"value": U1 / ref_dt, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
            "sample": f"sequential float64 time stepping of right-hand side 0 of {cfg.batch} "
                      f"(one sparse LU + {cfg.nt} triangular solves, the whole horizon, "
                      f"{cfg.nx * cfg.ny} unknowns per step); {ref_dt:.1f} s"}
    if sample is None:
        return base, None
    cores = sample["freqs"]
    # one preconditioner application needs nt frequency solves; `cores` ran
    # side by side in sample["wall_s"]
    per_app = sample["wall_s"] * cfg.nt / cores
    solve_s = per_app * iters
    para = {"value": U1 / solve_s, "unit": "unknowns/s", "cores": cores, "kind": "oracle",
            "sample": f"Step-(b) of the oracle's ParaDiag-II preconditioner (complex sparse LU and "
                      f"solve per frequency) on {cores} of {cfg.nt} frequencies, one per worker "
                      f"process, {sample['wall_s']:.1f} s wall ({sample['per_freq_s']:.1f} s per "
                      f"frequency); scaled to {cfg.nt} frequencies x {iters} preconditioner "
                      f"applications (the float64 FGMRES count) for right-hand side 0. Steps (a), "
                      f"(c), the matvec and Gram-Schmidt are left out, so this overstates the rate"}
    return base, para


def run_paradiag_i(args, torch):
    """ParaDiag-I leg: the direct solve of the hybrid time discretisation on the
    wave problem of Table Ex2Tab1 (511^2 points, Nt = 512, T = 2), float64,
    with the right-hand side resident in HBM.  Reports unknowns/s of whole
    direct solves (time transforms with V^{-1} and V, Step-(b), and the
    residual check), the error against the exact solution (the table prints
    7.88e-05), and the roofline of the dominant kernel."""
    from paper_2005_09158_amd import ParaDiag
    from workloads import CONFIGS, hybrid_wave_data, hybrid_wave_exact
    cfg = CONFIGS["hyb"]
    pd = ParaDiag(dim=cfg.dim, nx=cfg.nx, ny=cfg.ny, nt=cfg.nt, scheme=cfg.scheme, T=cfg.T, nu=cfg.nu,
                  alpha=cfg.alpha, batch=cfg.batch, prec="fp64", mode="direct")
    U0, V0, f = hybrid_wave_data(cfg)
    b = pd.build_rhs(torch.from_numpy(U0).reshape(pd.field_shape).cuda(),
                     torch.from_numpy(V0).reshape(pd.field_shape).cuda(),
                     torch.from_numpy(f).reshape(pd.source_shape).cuda())
    u = torch.empty_like(b)
    for _ in range(args.warmup):
        pd.solve(b, u, mode="direct", rtol=1e-8, max_iter=1)
    pd.set_timing(True)
    pd.stage_times(reset=True)
    pd.solve(b, u, mode="direct", rtol=1e-8, max_iter=1)
    stages = pd.stage_times(reset=True)
    dominant = max(stages, key=lambda k: stages[k][0])
    pd.set_timing(True, stages=[dominant])
    pd.stage_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, res = pd.solve(b, u, mode="direct", rtol=1e-8, max_iter=1)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    timed = pd.stage_times(reset=True)
    pd.set_timing(False)
    un = u.cpu().numpy().reshape(cfg.nt, -1)
    err = float(np.abs(un - hybrid_wave_exact(cfg).reshape(cfg.nt, -1)).max())
    tms, cnt, by, fl = timed[dominant]
    avg_s = tms / 1e3 / max(cnt, 1)
    bound = "mfma" if dominant in ("fft_fwd", "fft_inv", "xform_fwd", "xform_inv") else "hbm"
    if bound == "mfma":
        achieved, peak, unit = fl / max(cnt, 1) / avg_s / 1e12, PEAK["mfma_TFs"]["fp64"], "TFLOP/s"
    else:
        achieved, peak, unit = by / max(cnt, 1) / avg_s / 1e9, PEAK["hbm_GBs"], "GB/s"
    kernel = {"fft_fwd": "k_time_gemm (V^-1)", "fft_inv": "k_time_gemm (V)"}.get(dominant, STAGE_KERNEL[dominant])
    U = cfg.unknowns
    return {
        "workload": f"hyb: 2D wave equation {cfg.nx}x{cfg.ny}, Nt {cfg.nt}, T {cfg.T}, hybrid "
                    f"midpoint/backward-Euler time discretisation, direct ParaDiag-I solve (Table Ex2Tab1)",
        "unknowns": U, "ms_per_step": ms, "value": U / (ms / 1e3), "unit": "unknowns/s",
        "dtype": "f64", "rel_resid": res.rel_resid,
        "error_vs_exact": err, "error_printed_in_paper": 7.88e-05,
        "stage_ms_per_step": {k: round(v[0], 4) for k, v in stages.items()},
        "roofline": {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                     "frac": round(achieved / peak, 4), "kernel": kernel, "stage": dominant,
                     "launches": cnt, "avg_launch_ms": round(tms / max(cnt, 1), 5),
                     "algorithmic_flops_per_launch": fl / max(cnt, 1),
                     "algorithmic_bytes_per_launch": by / max(cnt, 1)},
    }


def workload_name(cfg):
    if cfg.dim == 1:
        return (f"{cfg.name}: 1D advection-diffusion {cfg.nx} points, Nt {cfg.nt}, "
                f"{cfg.scheme.upper()}, alpha {cfg.alpha}, batch {cfg.batch}")
    pde = "2D wave equation" if cfg.scheme == "lf" else "2D advection-diffusion"
    scheme = {"lf": "implicit leap-frog", "tr": "TR", "be": "BE"}[cfg.scheme]
    return (f"{cfg.name}: {pde} {cfg.nx}x{cfg.ny}, Nt {cfg.nt}, {scheme}, alpha {cfg.alpha}, "
            f"batch {cfg.batch}")


DTYPE = {"fp32_bf16gemm": "f64 krylov + f32 fft/line solves + split-bf16 mfma x-transform",
         "fp32_bf16x1": "f64 krylov + f32 fft/line solves + bf16 mfma x-transform",
         "fp32": "f64 krylov + f32 preconditioner"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path is "
              f"single-GPU in this build", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    from workloads import CONFIGS
    cfg = CONFIGS[args.workload]
    mixed_prec = args.mixed or (cfg.prec if cfg.prec != "fp64" else "fp32_bf16gemm")
    # the CPU ParaDiag-II sample forks worker processes: before the GPU is touched
    sample = None
    if not args.no_cpu_baseline:
        cores = max(1, min(16, os.cpu_count() or 1))
        print(f"[bench] CPU ParaDiag-II sample on {cores} worker processes", file=sys.stderr, flush=True)
        sample = cpu_paradiag_sample(cfg, cores)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    print(f"[bench] workload {cfg.name} {cfg.nx}x{cfg.ny}x{cfg.nt} batch {cfg.batch} "
          f"scheme {cfg.scheme} alpha {cfg.alpha}", file=sys.stderr, flush=True)
    mixed, um = run_precision(cfg, mixed_prec, args, torch)
    print(f"[bench] {mixed_prec}: {mixed['ms_per_step']:.3f} ms/solve iters {mixed['iters']} "
          f"resid {mixed['rel_resid']:.2e}", file=sys.stderr, flush=True)
    fp64, u64 = None, None
    if not args.skip_fp64:
        fp64, u64 = run_precision(cfg, "fp64", args, torch)
        print(f"[bench] fp64: {fp64['ms_per_step']:.3f} ms/solve iters {fp64['iters']} "
              f"resid {fp64['rel_resid']:.2e}", file=sys.stderr, flush=True)
    U = cfg.unknowns
    value = U / (mixed["ms_per_step"] / 1e3)
    line = {
        "metric": "space-time unknowns/s to 1e-8 residual, mixed-prec vs FP64 ParaDiag-II, 1 GPU",
        "value": value,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[mixed_prec],
        "data": "synthetic",
        "config": {"workload": workload_name(cfg), "nx": cfg.nx, "ny": cfg.ny, "nt": cfg.nt,
                   "batch": cfg.batch, "unknowns": U, "rtol": cfg.rtol, "restart": args.restart},
        "mixed": {k: v for k, v in mixed.items() if k not in ("stages", "dominant_timed")},
        "fp64": None if fp64 is None else {k: v for k, v in fp64.items()
                                           if k not in ("stages", "dominant_timed")},
        "fp64_value": None if fp64 is None else U / (fp64["ms_per_step"] / 1e3),
        "mixed_speedup_vs_fp64": None if fp64 is None else fp64["ms_per_step"] / mixed["ms_per_step"],
        # per-stage figures come from one extra solve (before the timed region) with
        # every stage timed
        "stage_ms_per_step": {k: round(v[0], 4) for k, v in mixed["stages"].items()},
        "stage_ms_per_step_fp64": None if fp64 is None else
        {k: round(v[0], 4) for k, v in fp64["stages"].items()},
        "roofline": roofline(mixed, cfg, args.traffic),
        "stage_roofline": stage_rooflines(mixed),
    }
    if not args.no_oracle:
        print("[bench] float64 oracle: sequential time stepping of right-hand side 0", file=sys.stderr,
              flush=True)
        _, ref, ref_dt = oracle_reference(cfg)
        line["error_vs_oracle"] = {
            "rhs": 0, "oracle": "sequential float64 time stepping, whole horizon",
            "mixed": error_vs_oracle(um, ref),
            "fp64": None if u64 is None else error_vs_oracle(u64, ref)}
        iters64 = max(fp64["iters"]) if fp64 else max(mixed["iters"])
        base, para = cpu_baselines(cfg, ref_dt, sample, iters64)
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = base
            if para:
                line["cpu_baseline_paradiag_ii"] = para
    if not args.skip_paradiag_i:
        print("[bench] ParaDiag-I leg (hybrid wave, 511^2 x 512)", file=sys.stderr, flush=True)
        line["paradiag_i"] = run_paradiag_i(args, torch)
        print(f"[bench] ParaDiag-I: {line['paradiag_i']['ms_per_step']:.3f} ms/solve error vs exact "
              f"{line['paradiag_i']['error_vs_exact']:.3e}", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
