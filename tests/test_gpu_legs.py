"""Parity at the full sizes of the parareal and nonlinear workloads, in the
launch configuration bench.py times (the optimal-control workload is covered
at its full size by tests/test_gpu_oc.py, the hybrid one by
tests/test_gpu_hybrid.py).

* Parareal (Section 2.2.2), 1023 points x 64 intervals x J = 32, batch 256:
  iterated to a relative change of 1e-10, every batch entry sampled here
  (the first, a middle and the last) must equal the oracle's sequential fine
  solution.  With the change below 1e-10 and the iteration contracting, the
  distance to the fixed point is at most a few times 1e-10 relative; the bound
  is 1e-8 (max norm).
* Nonlinear (eq1.4, eq1.5), 2D Allen-Cahn 511^2 x 256: the converged iterate's
  residual R(u) = b - (B1 (x) I) u - (B2 (x) I) F(u), formed by the oracle at
  the full size, is at most 1.01 x 1e-10 ||b||; and since the system is
  block lower triangular in time, U_1 and U_2 depend only on U0: they must
  equal the oracle's Newton time stepping over two steps within 1e-9
  (relative, max norm; the residual bound times the backward Euler step's
  condition, at most 1 + dt ||K|| ~ 5e3, is below 1e-6, and the error of
  the first rows is far smaller since nothing from later rows flows back).
"""

import numpy as np
import pytest

from oracle import Problem, nonlinear, parareal
from tests.gpu_util import announce, rel_err, torch_gpu
from workloads import CONFIGS, nonlinear_initial, parareal_initial

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_parareal_full_size_equals_fine_solution():
    cfg = CONFIGS["par"]
    announce(f"parareal full size {cfg.nx} x {cfg.nt} x J {cfg.fine_steps}, batch {cfg.batch}")
    torch = torch_gpu()
    from paper_2005_09158_amd import ParaDiag
    pd = ParaDiag(**cfg.problem_kwargs(), batch=cfg.batch, prec="fp64", mode="parareal")
    U0 = parareal_initial(cfg)
    u, res = pd.parareal(torch.from_numpy(U0).reshape(pd.field_shape).cuda(), cfg.fine_steps,
                         rtol=cfg.rtol, max_iter=60)
    print(f"  iterations {res.iters}, last relative change {res.rel_resid:.2e}")
    assert res.converged and res.rel_resid <= cfg.rtol
    p = Problem.from_kwargs(**cfg.problem_kwargs())
    un = u.cpu().numpy().reshape(cfg.batch, cfg.nt, -1)
    for b in (0, cfg.batch // 2, cfg.batch - 1):
        ref = parareal.fine_solution(p, cfg.fine_steps, U0[b])
        err = rel_err(un[b], ref)
        print(f"  entry {b}: error vs fine solution {err:.2e}")
        assert err <= 1e-8


@pytest.mark.timeout(600)
def test_nonlinear_full_size_residual_and_first_steps():
    cfg = CONFIGS["nl"]
    announce(f"nonlinear full size {cfg.nx}x{cfg.ny} x {cfg.nt}")
    torch = torch_gpu()
    from paper_2005_09158_amd import ParaDiag
    k1, k2, k3 = cfg.reaction
    pd = ParaDiag(**cfg.problem_kwargs(), prec="fp64", mode="nonlinear")
    U0 = nonlinear_initial(cfg)
    u, res = pd.nonlinear_solve(torch.from_numpy(U0).reshape(pd.field_shape).cuda(), k1, k2, k3,
                                rtol=cfg.rtol, max_iter=100)
    print(f"  corrections {res.iters}, relative residual {res.rel_resid:.2e}")
    assert res.converged and res.rel_resid <= cfg.rtol
    un = u.cpu().numpy().reshape(cfg.nt, -1)
    del u
    g = nonlinear.Cubic(k1=k1, k2=k2, k3=k3)
    p = Problem.from_kwargs(**cfg.problem_kwargs())
    b = nonlinear.rhs(p, g, U0)
    r = np.linalg.norm(nonlinear.residual(p, g, un, b)) / np.linalg.norm(b)
    print(f"  oracle residual {r:.2e}")
    assert r <= 1.01 * cfg.rtol
    p2 = Problem.from_kwargs(**{**cfg.problem_kwargs(), "nt": 2, "T": 2 * cfg.dt})
    ref = nonlinear.sequential(p2, g, U0, newton_tol=1e-14)
    err = rel_err(un[:2], ref)
    print(f"  first two steps vs Newton time stepping: {err:.2e}")
    assert err <= 1e-9
