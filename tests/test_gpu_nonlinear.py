"""GPU parity of nonlinear ParaDiag (eq1.4, eq1.5) and windowing against the oracle.

The library's simplified Newton iterates (residual and averaged slope in one
pass, the shifted time symbols uploaded, P_alpha(u)^{-1} by the usual three
steps) are compared with ``oracle.nonlinear.simplified_newton`` after the same
number of corrections from the same start.  Both run the same float64
arithmetic up to rounding order; the iteration contracts, so the difference
stays at rounding level amplified by the preconditioner (bound 1e-11,
relative, max norm).  Converged solutions are compared with the oracle's
Newton time stepping, windows with the oracle's windowed iteration.
"""

import numpy as np
import pytest

from oracle import Problem, nonlinear
from tests.gpu_util import announce, make, rel_err, to_gpu

pytestmark = pytest.mark.gpu

AC = nonlinear.Cubic(k1=-4.0, k3=4.0)

CASES = {
    "1d-be": dict(dim=1, nx=40, ny=1, nt=32, scheme="be", T=0.5, nu=5e-2, ax=0.4, alpha=0.05),
    "1d-tr-ragged": dict(dim=1, nx=37, ny=1, nt=16, scheme="tr", T=0.5, nu=5e-2, ax=-0.4, alpha=0.05),
    "2d-tr-schur": dict(dim=2, nx=24, ny=20, nt=16, scheme="tr", T=0.5, nu=5e-2, ax=0.4, ay=-0.3, alpha=0.05),
    "2d-be-sine": dict(dim=2, nx=30, ny=18, nt=32, scheme="be", T=0.5, nu=5e-2, alpha=0.05),
}


def _u0(p):
    x = np.arange(1, p.nx + 1) / (p.nx + 1)
    if p.dim == 1:
        return 0.9 * np.sin(np.pi * x) + 0.3 * np.sin(3 * np.pi * x)
    y = np.arange(1, p.ny + 1) / (p.ny + 1)
    return (0.9 * np.outer(np.sin(np.pi * y), np.sin(np.pi * x)) + 0.2 * np.outer(np.sin(2 * np.pi * y), np.sin(np.pi * x))).ravel()


@pytest.mark.parametrize("case", list(CASES))
def test_simplified_newton_iterates_match_oracle(case):
    params = CASES[case]
    announce(f"nonlinear iterates {case}")
    torch, pd, prob = make(params, "fp64", mode="nonlinear")
    U0 = _u0(prob)
    U0g = to_gpu(torch, U0, pd.field_shape)
    ref_its = nonlinear.simplified_newton(prob, AC, U0, iters=6)
    for k in (1, 3, 6):
        u, res = pd.nonlinear_solve(U0g, AC.k1, AC.k2, AC.k3, max_iter=k, rtol=1e-300)
        assert res.iters == k
        err = rel_err(u[0].cpu().numpy().reshape(prob.nt, -1), ref_its[k - 1])
        print(f"  k={k}: rel err {err:.2e}")
        assert err <= 1e-11
    # residual history: the GPU's relative residual before correction k equals the oracle's
    b = nonlinear.rhs(prob, AC, U0)
    r6 = np.linalg.norm(nonlinear.residual(prob, AC, ref_its[-1], b)) / np.linalg.norm(b)
    assert res.history[-1] == pytest.approx(r6, rel=1e-6, abs=1e-15)


@pytest.mark.parametrize("case", ["1d-tr-ragged", "2d-tr-schur"])
def test_nonlinear_converges_to_time_stepping(case):
    params = CASES[case]
    announce(f"nonlinear to convergence {case}")
    torch, pd, prob = make(params, "fp64", mode="nonlinear")
    U0 = _u0(prob)
    u, res = pd.nonlinear_solve(to_gpu(torch, U0, pd.field_shape), AC.k1, AC.k2, AC.k3, max_iter=80,
                                rtol=1e-12)
    ref = nonlinear.sequential(prob, AC, U0)
    err = rel_err(u[0].cpu().numpy().reshape(prob.nt, -1), ref)
    print(f"  corrections {res.iters} residual {res.rel_resid:.2e} error vs time stepping {err:.2e}")
    assert res.converged and res.rel_resid <= 1e-12 and err <= 1e-10


def test_windows_match_oracle_and_restore_the_plan():
    params = CASES["1d-be"]
    announce("nonlinear windowing, 3 windows")
    torch, pd, prob = make(params, "fp64", mode="nonlinear")
    U0 = _u0(prob)
    r = np.random.default_rng(2).standard_normal((prob.nt, prob.nspace))
    z_before = pd.apply_precond(to_gpu(torch, r, pd.shape)).cpu().numpy()
    u, res = pd.nonlinear_solve(to_gpu(torch, U0, pd.field_shape), AC.k1, AC.k2, AC.k3, windows=3,
                                max_iter=40, rtol=1e-300)
    ref = nonlinear.windowed(prob, AC, U0, windows=3, iters=40)
    err = rel_err(u.cpu().numpy().reshape(3 * prob.nt, -1), ref)
    print(f"  windows: rel err {err:.2e}")
    assert err <= 1e-11
    # the plan's own preconditioner is intact afterwards
    z_after = pd.apply_precond(to_gpu(torch, r, pd.shape)).cpu().numpy()
    assert np.array_equal(z_before, z_after)


def test_nonlinear_rejects_batches_and_other_schemes():
    announce("nonlinear: unsupported plans")
    from paper_2005_09158_amd import _lib
    for params, batch in ((CASES["1d-be"], 2), ({**CASES["1d-be"], "scheme": "lf"}, 1)):
        torch, pd, prob = make(params, "fp64", batch=batch, mode="nonlinear")
        U0 = torch.zeros(pd.field_shape, dtype=torch.float64, device="cuda")
        with pytest.raises(_lib.ParaDiagError) as e:
            pd.nonlinear_solve(U0, 1.0)
        assert e.value.status == _lib.PD_ERR_UNSUPPORTED
