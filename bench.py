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
* extra legs, each with its rate, its accuracy and its dominant kernel's
  roofline: `paradiag_i`, the direct float64 solve of the hybrid time
  discretisation on the wave problem of Table Ex2Tab1 (511^2 x 512);
  `oc_wave`, the optimal control of the wave equation at Table T2A's largest
  size (255^2 x 257, gamma 1e-4); `parareal`, the ParaDiag-II parareal
  variant (1023 points, 64 intervals x 32 fine steps, batch 256); and
  `nonlinear`, simplified Newton for 2D Allen-Cahn (511^2 x 256).
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
    "mfma_TFs": {"fp64": 78.6, "fp32": 157.3, "fp32_bf16gemm": 2500.0, "fp32_bf16x1": 2500.0,
                 "fp32_fp16gemm": 2500.0},
    "vector_TFs": {"fp64": 78.6, "fp32": 157.3, "fp32_bf16gemm": 157.3, "fp32_bf16x1": 157.3,
                   "fp32_fp16gemm": 157.3},
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
    ap.add_argument("--mixed", default=None, choices=["fp32", "fp32_bf16gemm", "fp32_bf16x1", "fp32_fp16gemm"],
                    help="reduced-precision preconditioner (default: the workload's own; float32 "
                         "for the wave equation, split-bf16 x-transform otherwise)")
    ap.add_argument("--restart", type=int, default=8)
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--no-fp16-alt", action="store_true",
                    help="skip the row-scaled split-fp16 variant timed beside the split-bf16 mixed mode")
    ap.add_argument("--legs", default="paradiag_i,oc_wave,parareal,nonlinear",
                    help="comma-separated extra legs after the main one (paradiag_i, oc_wave, "
                         "parareal, nonlinear), or 'none'")
    ap.add_argument("--legs-only", action="store_true",
                    help="run only the extra legs (one JSON line holding them)")
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


def timed_leg(pd, call, args, torch):
    """Warm-up calls, one call with every stage timed (the breakdown and the
    dominant stage), then `args.steps` timed calls with events around the
    dominant stage only.  Returns (ms per call, last result, stages, dominant,
    the dominant stage's timed figures)."""
    for _ in range(args.warmup):
        call()
    pd.set_timing(True)
    pd.stage_times(reset=True)
    call()
    stages = pd.stage_times(reset=True)
    dominant = max(stages, key=lambda k: stages[k][0])
    pd.set_timing(True, stages=[dominant])
    pd.stage_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = call()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    timed = pd.stage_times(reset=True)[dominant]
    pd.set_timing(False)
    return ms, out, stages, dominant, timed


# kernels behind a stage where it differs from the ParaDiag-II default
LEG_KERNEL = {"hyb": {"fft_fwd": "k_time_gemm (V^-1)", "fft_inv": "k_time_gemm (V)", "line_solve": "k_line_solve"},
              "oc": {"fft_fwd": "k_time_gemm (DFT) + k_oc_mix", "fft_inv": "k_oc_unmix + k_time_gemm (inverse DFT)",
                     "line_solve": "k_line_solve"},
              "par": {"fine": "k_parareal_fine", "line_solve": "k_line_solve"},
              "nl": {"reaction": "k_nl_residual", "line_solve": "k_line_solve"}}


def leg_roofline(leg, dominant, timed):
    """Roofline of a leg's dominant stage (every leg computes in float64):
    MFMA-bound products (the x-transforms, the time products of ParaDiag-I
    and of the optimal-control DFTs), the fine propagator's vector ALU work,
    or HBM bytes."""
    tms, cnt, by, fl = timed
    cnt = max(cnt, 1)
    avg_s = tms / 1e3 / cnt
    # an x-transform of a sine basis with nx + 1 a power of two is a DST by FFT
    # (a few flops per byte): HBM-bound; otherwise a dense product on MFMA
    dense_xform = dominant in ("xform_fwd", "xform_inv") and fl >= 16.0 * by
    if (dominant in ("fft_fwd", "fft_inv") and leg in ("hyb", "oc")) or dense_xform:
        bound, achieved, peak, unit = "mfma", fl / cnt / avg_s / 1e12, PEAK["mfma_TFs"]["fp64"], "TFLOP/s"
    elif dominant == "fine":
        bound, achieved, peak, unit = "alu", fl / cnt / avg_s / 1e12, PEAK["vector_TFs"]["fp64"], "TFLOP/s"
    else:
        bound, achieved, peak, unit = "hbm", by / cnt / avg_s / 1e9, PEAK["hbm_GBs"], "GB/s"
    kernel = LEG_KERNEL.get(leg, {}).get(dominant, STAGE_KERNEL.get(dominant, dominant))
    if dominant in ("xform_fwd", "xform_inv") and not dense_xform:
        kernel = "k_dst"
    return {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4), "kernel": kernel, "stage": dominant, "launches": cnt,
            "avg_launch_ms": round(tms / cnt, 5), "algorithmic_flops_per_launch": fl / cnt,
            "algorithmic_bytes_per_launch": by / cnt}


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
    ms, (_, res), stages, dominant, timed = timed_leg(
        pd, lambda: pd.solve(b, u, mode="direct", rtol=1e-8, max_iter=1), args, torch)
    un = u.cpu().numpy().reshape(cfg.nt, -1)
    err = float(np.abs(un - hybrid_wave_exact(cfg).reshape(cfg.nt, -1)).max())
    U = cfg.unknowns
    return {
        "workload": f"hyb: 2D wave equation {cfg.nx}x{cfg.ny}, Nt {cfg.nt}, T {cfg.T}, hybrid "
                    f"midpoint/backward-Euler time discretisation, direct ParaDiag-I solve (Table Ex2Tab1)",
        "unknowns": U, "ms_per_step": ms, "value": U / (ms / 1e3), "unit": "unknowns/s",
        "dtype": "f64", "rel_resid": res.rel_resid,
        "error_vs_exact": err, "error_printed_in_paper": 7.88e-05,
        "stage_ms_per_step": {k: round(v[0], 4) for k, v in stages.items() if v[1]},
        "roofline": leg_roofline("hyb", dominant, timed),
    }


def run_oc(args, torch):
    """Optimal-control leg (Section 4): the gamma-scaled optimality system of
    the paper's example at Table T2A's largest size (255^2 interior points,
    Nt = 257, gamma = 1e-4), flexible GMRES with the block-circulant
    preconditioner to a relative residual of 1e-7, float64.  Reports unknowns
    (both fields) per second of whole solves, the iteration count against the
    table's, the error against the exact (u, p) and the dominant kernel's
    roofline."""
    from paper_2005_09158_amd import ParaDiagOC
    from workloads import CONFIGS, oc_example_data, oc_example_exact
    cfg = CONFIGS["oc"]
    pd = ParaDiagOC(dim=2, nx=cfg.nx, ny=cfg.ny, nt=cfg.nt, T=cfg.T, nu=cfg.nu, gamma=cfg.gamma,
                    prec=cfg.prec, restart=30)
    U0, u1, f, g = oc_example_data(cfg)
    cu = lambda a, shp: torch.from_numpy(np.ascontiguousarray(a)).reshape(shp).cuda()
    b = pd.build_rhs(cu(U0, pd.field_shape), cu(u1, pd.field_shape), cu(f, pd.source_shape),
                     cu(g, pd.source_shape))
    x = torch.empty_like(b)
    ms, (_, res), stages, dominant, timed = timed_leg(
        pd, lambda: pd.solve(b, x, rtol=cfg.rtol, max_iter=60, restart=30), args, torch)
    xn = x.cpu().numpy().reshape(2, cfg.nt, -1)
    ue, pe = oc_example_exact(cfg)
    u = xn[0] / np.sqrt(cfg.gamma)
    err_u = float(np.abs(u - ue.reshape(cfg.nt, -1)).max() / np.abs(ue).max())
    err_p = float(np.abs(xn[1] - pe.reshape(cfg.nt, -1)).max() / np.abs(pe).max())
    U = 2 * cfg.unknowns
    return {
        "workload": f"oc: optimal control of the 2D wave equation {cfg.nx}x{cfg.ny}, Nt {cfg.nt}, "
                    f"T {cfg.T}, gamma {cfg.gamma}, implicit leap-frog, block-circulant "
                    f"preconditioner (Section 4, Table T2A N = 256)",
        "unknowns": U, "ms_per_step": ms, "value": U / (ms / 1e3), "unit": "unknowns/s",
        "dtype": "f64", "rel_resid": res.rel_resid, "iters": res.iters, "iters_printed_in_paper": 5,
        "rel_error_vs_exact": {"u": err_u, "p": err_p},
        "stage_ms_per_step": {k: round(v[0], 4) for k, v in stages.items() if v[1]},
        "roofline": leg_roofline("oc", dominant, timed),
    }


def run_parareal(args, torch):
    """Parareal leg (Section 2.2.2): the ParaDiag-II parareal variant on 1D
    advection-diffusion with Figure 1.5's coefficients (1023 points, 64
    coarse intervals, J = 32 backward Euler fine steps, alpha = 0.1), a batch
    of 256 initial states, iterated to a relative change of 1e-10.  Reports
    fine-grid space-time unknowns (J per coarse unknown) per second, the
    iteration count, the error against the sequential fine solution (torch
    float64 time stepping of one initial state, after the timed region) and
    the dominant kernel's roofline."""
    from paper_2005_09158_amd import ParaDiag
    from workloads import CONFIGS, parareal_initial
    cfg = CONFIGS["par"]
    pd = ParaDiag(**cfg.problem_kwargs(), batch=cfg.batch, prec="fp64", mode="parareal")
    U0 = torch.from_numpy(parareal_initial(cfg)).reshape(pd.field_shape).cuda()
    u = torch.empty(pd.shape, dtype=torch.float64, device="cuda")
    J = cfg.fine_steps
    ms, (_, res), stages, dominant, timed = timed_leg(
        pd, lambda: pd.parareal(U0, J, u, rtol=cfg.rtol, max_iter=60), args, torch)
    fine = cfg.unknowns * J
    return {
        "workload": f"par: parareal variant, 1D advection-diffusion {cfg.nx} points, {cfg.nt} coarse "
                    f"intervals x J {J} backward Euler steps, T {cfg.T}, nu {cfg.nu}, a {cfg.ax}, "
                    f"alpha {cfg.alpha}, batch {cfg.batch} (Figure 1.5's coefficients)",
        "unknowns": fine, "ms_per_step": ms, "value": fine / (ms / 1e3),
        "unit": "fine-grid unknowns/s", "dtype": "f64", "iters": res.iters,
        "rel_change": res.rel_resid,
        "stage_ms_per_step": {k: round(v[0], 4) for k, v in stages.items() if v[1]},
        "roofline": leg_roofline("par", dominant, timed),
    }


def run_nonlinear(args, torch):
    """Nonlinear leg (eq1.4, eq1.5): 2D Allen-Cahn on 511^2 points, Nt = 256
    backward Euler steps, simplified Newton with the averaged Jacobian and
    the alpha-circulant preconditioner (alpha = 0.05), float64, to a relative
    residual of 1e-10.  Reports unknowns per second of whole solves, the
    correction count and the dominant kernel's roofline."""
    from paper_2005_09158_amd import ParaDiag
    from workloads import CONFIGS, nonlinear_initial
    cfg = CONFIGS["nl"]
    k1, k2, k3 = cfg.reaction
    pd = ParaDiag(**cfg.problem_kwargs(), prec="fp64", mode="nonlinear")
    U0 = torch.from_numpy(nonlinear_initial(cfg)).reshape(pd.field_shape).cuda()
    u = torch.empty((1,) + pd.shape, dtype=torch.float64, device="cuda")
    ms, (_, res), stages, dominant, timed = timed_leg(
        pd, lambda: pd.nonlinear_solve(U0, k1, k2, k3, u=u, rtol=cfg.rtol, max_iter=100), args, torch)
    U = cfg.unknowns
    return {
        "workload": f"nl: 2D Allen-Cahn {cfg.nx}x{cfg.ny}, Nt {cfg.nt}, BE, T {cfg.T}, nu {cfg.nu}, "
                    f"g(u) = {k1} u + {k3} u^3, alpha {cfg.alpha}, simplified Newton (eq1.5)",
        "unknowns": U, "ms_per_step": ms, "value": U / (ms / 1e3), "unit": "unknowns/s",
        "dtype": "f64", "corrections": res.iters, "rel_resid": res.rel_resid,
        "converged": bool(res.converged),
        "stage_ms_per_step": {k: round(v[0], 4) for k, v in stages.items() if v[1]},
        "roofline": leg_roofline("nl", dominant, timed),
    }


EXTRA_LEGS = {"paradiag_i": run_paradiag_i, "oc_wave": run_oc, "parareal": run_parareal,
              "nonlinear": run_nonlinear}


def workload_name(cfg):
    if cfg.dim == 1:
        return (f"{cfg.name}: 1D advection-diffusion {cfg.nx} points, Nt {cfg.nt}, "
                f"{cfg.scheme.upper()}, alpha {cfg.alpha}, batch {cfg.batch}")
    pde = "2D wave equation" if cfg.scheme == "lf" else "2D advection-diffusion"
    scheme = {"lf": "implicit leap-frog", "tr": "TR", "be": "BE"}[cfg.scheme]
    return (f"{cfg.name}: {pde} {cfg.nx}x{cfg.ny}, Nt {cfg.nt}, {scheme}, alpha {cfg.alpha}, "
            f"batch {cfg.batch}")


DTYPE = {"fp32_bf16gemm": "f64 krylov + f32 fft/line solves + split-bf16 mfma x-transform",
         "fp32_fp16gemm": "f64 krylov + f32 fft/line solves + row-scaled split-fp16 mfma x-transform",
         "fp32_bf16x1": "f64 krylov + f32 fft/line solves + bf16 mfma x-transform",
         "fp32": "f64 krylov + f32 preconditioner"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library runs "
              f"on a single GPU", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    legs = [] if args.legs == "none" else [x for x in args.legs.split(",") if x]
    for name in legs:
        if name not in EXTRA_LEGS:
            print(f"unknown leg {name!r} (known: {', '.join(EXTRA_LEGS)})", file=sys.stderr)
            sys.exit(2)
    if args.legs_only:
        import torch
        if not torch.cuda.is_available():
            print("no GPU visible", file=sys.stderr)
            sys.exit(1)
        torch.cuda.set_device(0)
        line = {"legs_only": True, "steps": args.steps, "warmup": args.warmup}
        for name in legs:
            print(f"[bench] leg {name}", file=sys.stderr, flush=True)
            line[name] = EXTRA_LEGS[name](args, torch)
            print(f"[bench] {name}: {line[name]['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
        print(json.dumps(line), flush=True)
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
    # the row-scaled split-fp16 x-transform beside the workload's own mixed mode
    # (reported, not `value`: the workload names bf16 products)
    alt, ualt = None, None
    if not args.no_fp16_alt and mixed_prec == "fp32_bf16gemm":
        alt, ualt = run_precision(cfg, "fp32_fp16gemm", args, torch)
        print(f"[bench] fp32_fp16gemm: {alt['ms_per_step']:.3f} ms/solve iters {alt['iters']} "
              f"resid {alt['rel_resid']:.2e}", file=sys.stderr, flush=True)
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
        "mixed_fp16gemm": None if alt is None else {
            "value": U / (alt["ms_per_step"] / 1e3), "ms_per_step": alt["ms_per_step"], "iters": alt["iters"],
            "rel_resid": alt["rel_resid"], "dtype": DTYPE["fp32_fp16gemm"],
            "stage_ms_per_step": {k: round(v[0], 4) for k, v in alt["stages"].items() if v[1]}},
    }
    if not args.no_oracle:
        print("[bench] float64 oracle: sequential time stepping of right-hand side 0", file=sys.stderr,
              flush=True)
        _, ref, ref_dt = oracle_reference(cfg)
        line["error_vs_oracle"] = {
            "rhs": 0, "oracle": "sequential float64 time stepping, whole horizon",
            "mixed": error_vs_oracle(um, ref),
            "fp64": None if u64 is None else error_vs_oracle(u64, ref),
            "mixed_fp16gemm": None if ualt is None else error_vs_oracle(ualt, ref)}
        iters64 = max(fp64["iters"]) if fp64 else max(mixed["iters"])
        base, para = cpu_baselines(cfg, ref_dt, sample, iters64)
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = base
            if para:
                line["cpu_baseline_paradiag_ii"] = para
    for name in legs:
        print(f"[bench] leg {name}", file=sys.stderr, flush=True)
        line[name] = EXTRA_LEGS[name](args, torch)
        print(f"[bench] {name}: {line[name]['ms_per_step']:.3f} ms/step, dominant "
              f"{line[name]['roofline']['kernel']} at {line[name]['roofline']['frac']:.3f} of its peak",
              file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
