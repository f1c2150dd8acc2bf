"""Parity at the full sizes of the five workloads, in the launch configuration bench.py uses.

The oracle solves every workload over its whole horizon by sequential float64
time stepping (cfg3: right-hand side 0 of the 8; about half a minute of host
time each for cfg3 and a minute for cfg5).  Every right-hand side of cfg3 also
has its true relative residual ||b - A u|| / ||b|| formed by the oracle's
block-wise product with A (the exact definition).
Tolerances: float64 solves to rtol 1e-12 agree with the oracle to 1e-10
(relative, max norm); mixed-precision solves meet rtol 1e-8 on the float64
residual, and their relative 2-norm distance to the oracle solution is at most
kappa_2(A) times that residual, with kappa_2(A) bounded from the structure of A
(tests/bounds.py: 1.26e4 for cfg3, 1.87e6 for cfg5); cfg2 is checked at 1e-6
in the max norm.
"""

import numpy as np
import pytest

from oracle import Problem, adjoint as o_adj, operators as ops, rhs as o_rhs, solve as o_solve
from tests.bounds import kappa2_bound
from tests.gpu_util import announce, rel_err, torch_gpu
from workloads import (CONFIGS, initial_state, initial_velocity, source_term, source_term_torch,
                       tracking_target, fd_directions)

pytestmark = pytest.mark.gpu


def _pd(cfg, prec, restart=8, batch=None):
    from paper_2005_09158_amd import ParaDiag
    return ParaDiag(dim=cfg.dim, nx=cfg.nx, ny=cfg.ny, nt=cfg.nt, scheme=cfg.scheme, T=cfg.T,
                    nu=cfg.nu, ax=cfg.ax, ay=cfg.ay, alpha=cfg.alpha, batch=batch or cfg.batch,
                    prec=prec, restart=restart)


def _rhs_np(cfg, seed_offset=0):
    p = Problem.from_kwargs(**cfg.problem_kwargs())
    U0 = initial_state(cfg)
    u1 = initial_velocity(cfg) if cfg.scheme == "lf" else None
    f = source_term(cfg, cfg.seed + 1 + seed_offset) if cfg.with_source else None
    return p, o_rhs.build_rhs(p, U0, u1, f)


def test_cfg1_full():
    announce("cfg1 full solve fp64")
    torch = torch_gpu()
    cfg = CONFIGS["cfg1"]
    p, b = _rhs_np(cfg)
    pd = _pd(cfg, "fp64")
    bg = torch.from_numpy(b).reshape(pd.shape).cuda()
    # the workload's own tolerance
    u, res = pd.solve(bg, rtol=cfg.rtol, max_iter=100)
    assert res.converged and res.rel_resid <= cfg.rtol
    # parity solve
    u, res = pd.solve(bg, rtol=1e-12, max_iter=100)
    ref = o_solve.sequential(p, b)
    err = rel_err(u.cpu().numpy().reshape(p.nt, -1), ref)
    print(f"  cfg1 iters {res.iters} resid {res.rel_resid:.2e} err {err:.2e}")
    assert err < 1e-10
    # the GPU right-hand side equals the oracle's
    U0 = torch.from_numpy(initial_state(cfg)).reshape(pd.field_shape).cuda()
    assert rel_err(pd.build_rhs(U0).cpu().numpy().reshape(p.nt, -1), b) < 1e-13


@pytest.mark.parametrize("prec", ["fp64", "fp32_bf16gemm", "fp32", "fp32_fp16gemm"])
def test_cfg2_full(prec):
    announce(f"cfg2 full solve {prec}")
    torch = torch_gpu()
    cfg = CONFIGS["cfg2"]
    p, b = _rhs_np(cfg)
    pd = _pd(cfg, prec)
    bg = torch.from_numpy(b).reshape(pd.shape).cuda()
    rtol = 1e-12 if prec == "fp64" else cfg.rtol
    u, res = pd.solve(bg, rtol=rtol, max_iter=100)
    assert res.converged
    un = u.cpu().numpy().reshape(p.nt, -1)
    true_res = np.linalg.norm(b - ops.apply_A(p, un)) / np.linalg.norm(b)
    ref = o_solve.sequential(p, b)
    err = rel_err(un, ref)
    print(f"  cfg2 {prec} iters {res.iters} resid {res.rel_resid:.2e} true {true_res:.2e} err {err:.2e}")
    assert true_res <= rtol * 1.01
    assert err < (1e-10 if prec == "fp64" else 1e-6)


def _full_error(p, b_row, u_row):
    """Whole-horizon error of one right-hand side against the oracle's time stepper."""
    ref = o_solve.sequential(p, b_row)
    d = u_row - ref
    return (float(np.linalg.norm(d) / np.linalg.norm(ref)),
            float(np.abs(d).max() / np.abs(ref).max()))


@pytest.mark.timeout(900)
def test_cfg3_batch_mixed():
    announce("cfg3 512x512x1024 batch 8 split-bf16, restart 8: residuals + whole-horizon error")
    torch = torch_gpu()
    cfg = CONFIGS["cfg3"]
    pd = _pd(cfg, "fp32_bf16gemm", restart=8)
    U0 = torch.from_numpy(initial_state(cfg)).cuda().reshape(1, cfg.ny, cfg.nx)
    U0 = U0.expand(cfg.batch, cfg.ny, cfg.nx).contiguous()
    f = torch.empty(pd.source_shape, dtype=torch.float64, device="cuda")
    for s in range(cfg.batch):
        f[s] = source_term_torch(cfg, cfg.seed + 1 + s, "cuda")
    b = pd.build_rhs(U0, None, f)
    del f
    u, res = pd.solve(b, rtol=cfg.rtol, max_iter=40)
    print(f"  cfg3 iters {res.iters_per_rhs} resid {res.resid_per_rhs}", flush=True)
    assert res.converged and max(res.resid_per_rhs) <= cfg.rtol
    bh = b.cpu().numpy().reshape(cfg.batch, cfg.nt, -1)
    uh = u.cpu().numpy().reshape(cfg.batch, cfg.nt, -1)
    del u, b, pd
    torch.cuda.empty_cache()
    p, b0 = _rhs_np(cfg, 0)
    # the GPU right-hand side 0 equals the oracle's
    assert rel_err(bh[0], b0) < 1e-12
    # every right-hand side meets the tolerance on the oracle's residual
    true_res = []
    for k in range(cfg.batch):
        true_res.append(np.linalg.norm(bh[k] - ops.apply_A(p, uh[k])) / np.linalg.norm(bh[k]))
    print(f"  cfg3 oracle true residuals {['%.2e' % r for r in true_res]}", flush=True)
    assert max(true_res) <= cfg.rtol * 1.01
    # right-hand side 0 against the oracle's solution over the whole horizon
    kappa = kappa2_bound(cfg)
    e2, emax = _full_error(p, b0, uh[0])
    print(f"  cfg3 rhs0 whole-horizon error: 2-norm {e2:.2e} max-norm {emax:.2e} "
          f"(bound kappa2 x residual = {kappa * true_res[0]:.2e})", flush=True)
    assert e2 <= kappa * true_res[0] * 1.01


def test_cfg4_gradient():
    announce("cfg4 gradient via the adjoint solve")
    torch = torch_gpu()
    from paper_2005_09158_amd import ParaDiagSolve
    cfg = CONFIGS["cfg4"]
    p = Problem.from_kwargs(**cfg.problem_kwargs())
    pd = _pd(cfg, "fp64")
    U0 = initial_state(cfg, seed=101)
    f = source_term(cfg, 102)
    target = tracking_target(cfg, 100)
    beta = cfg.beta
    tg = torch.from_numpy(target).reshape(pd.field_shape).cuda()

    def J_gpu(U0n, fn, grad=False):
        U0g = torch.from_numpy(U0n).reshape(pd.field_shape).cuda().requires_grad_(grad)
        fg = torch.from_numpy(fn).reshape(pd.source_shape).cuda().requires_grad_(grad)
        u = ParaDiagSolve.apply(pd, U0g, fg, 1e-13)
        J = 0.5 * ((u[:, -1] - tg) ** 2).sum() + 0.5 * beta * (fg ** 2).sum()
        if grad:
            J.backward()
            return J.item(), U0g.grad.cpu().numpy().ravel(), fg.grad.cpu().numpy().reshape(p.nt + 1, -1)
        return J.item()

    J, gU0, gf = J_gpu(U0, f, grad=True)
    Jr, gU0r, gfr = o_adj.gradient(p, U0.ravel(), f.reshape(p.nt + 1, -1), target.ravel(), beta)
    print(f"  J gpu {J:.12e} oracle {Jr:.12e}")
    assert abs(J - Jr) <= 1e-10 * abs(Jr)
    assert rel_err(gU0, gU0r) < 1e-8
    assert rel_err(gf, gfr) < 1e-8
    # central differences of the exact J (the oracle's direct time stepper: J is
    # quadratic, so the only error is rounding / h); an iterative J would add
    # its solve tolerance / h to every difference.
    # Tolerance per direction: 1e-6 relative plus the cancellation floor of the
    # difference of two O(|J|) numbers, 4 eps |J| / h (J ~ 657 here).
    h = 1e-6
    floor = 4 * np.finfo(float).eps * abs(Jr) / h
    worst = 0.0
    U0r, fr, tr = U0.ravel(), f.reshape(p.nt + 1, -1), target.ravel()
    for d0, df in fd_directions(cfg, 20, 200):
        fd = o_adj.finite_difference(p, U0r, fr, tr, beta, d0.ravel(), df.reshape(p.nt + 1, -1), h)
        an = float(gU0 @ d0.ravel() + np.sum(gf * df.reshape(p.nt + 1, -1)))
        worst = max(worst, abs(fd - an) / (1e-6 * abs(an) + floor))
    print(f"  worst FD mismatch / tolerance over 20 directions {worst:.2e} (floor {floor:.1e})")
    assert worst <= 1.0


@pytest.mark.timeout(900)
def test_cfg5_wave_fp32():
    announce("cfg5 wave 512x512x2048 fp32 preconditioner: residual + whole-horizon error")
    torch = torch_gpu()
    cfg = CONFIGS["cfg5"]
    p, b = _rhs_np(cfg)
    pd = _pd(cfg, "fp32")
    bg = torch.from_numpy(b).reshape(pd.shape).cuda()
    u, res = pd.solve(bg, rtol=cfg.rtol, max_iter=60)
    print(f"  cfg5 iters {res.iters} resid {res.rel_resid:.2e}", flush=True)
    assert res.converged and res.rel_resid <= cfg.rtol
    un = u.cpu().numpy().reshape(p.nt, -1)
    del u, bg, pd
    torch.cuda.empty_cache()
    true_res = np.linalg.norm(b - ops.apply_A(p, un)) / np.linalg.norm(b)
    assert true_res <= cfg.rtol * 1.01
    kappa = kappa2_bound(cfg)
    e2, emax = _full_error(p, b, un)
    print(f"  cfg5 true resid {true_res:.2e} whole-horizon error: 2-norm {e2:.2e} max-norm "
          f"{emax:.2e} (bound kappa2 x residual = {kappa * true_res:.2e})", flush=True)
    assert e2 <= kappa * true_res * 1.01
