"""GPU parity of the ParaDiag-II parareal variant (Section 2.2.2) against the oracle.

The library runs parareal with J fine backward Euler steps per coarse
interval (on-chip, one wave per interval) and the alpha-periodic coarse-grid
correction solved by the alpha-circulant preconditioner of the backward Euler
plan.  Each iterate u^k is compared with the oracle's ``parareal.paradiag_ii``
iterate from the same start: the two differ only by rounding, amplified by
the alpha-circulant transform (Cond_2 at most 1/alpha) and by the shifted
solves (condition at most 1 + dT ||K||, ||K|| <= 4 nu / h^2 + |a| / h), so the
bound is 8 u (1 + dT ||K||) / alpha with u = 2^-53 (relative, max norm).  The
converged iterate is compared with the oracle's sequential fine solution.
"""

import numpy as np
import pytest

from oracle import Problem, parareal
from tests.gpu_util import announce, make, rel_err, to_gpu

pytestmark = pytest.mark.gpu

CASES = {
    # Figure 1.5's coefficients on [0, 1] with Dirichlet data (63 points, dT = 1/16, J = 32)
    "fig15": (dict(dim=1, nx=63, ny=1, nt=64, scheme="be", T=4.0, nu=0.1, ax=1.0, alpha=0.1), 32, 1),
    # ragged length, batch of 3, small alpha, several rows per lane
    "ragged": (dict(dim=1, nx=300, ny=1, nt=16, scheme="be", T=1.0, nu=2e-2, ax=-0.7, alpha=0.05), 6, 3),
    "nx1000": (dict(dim=1, nx=1000, ny=1, nt=8, scheme="be", T=0.5, nu=1e-2, ax=0.4, alpha=0.2), 3, 1),
}


def _u0(prob, batch, seed):
    x = np.arange(1, prob.nx + 1) / (prob.nx + 1)
    rng = np.random.default_rng(seed)
    return np.stack([np.exp(-30.0 * (x - 0.5) ** 2) + 0.1 * rng.standard_normal(prob.nx) for _ in range(batch)])


@pytest.mark.parametrize("case", list(CASES))
def test_parareal_iterates_match_oracle(case):
    params, J, batch = CASES[case]
    announce(f"parareal iterates {case} J={J} batch {batch}")
    torch, pd, prob = make(params, "fp64", batch=batch, mode="parareal")
    U0 = _u0(prob, batch, 3)
    init = np.random.default_rng(4).standard_normal((batch, prob.nt, prob.nspace))
    U0g = to_gpu(torch, U0, pd.field_shape)
    h = 1.0 / (prob.nx + 1)
    knorm = 4.0 * prob.nu / h ** 2 + abs(prob.ax) / h
    tol = 8.0 * 2.0 ** -53 * (1.0 + prob.dt * knorm) / prob.alpha
    for k in (1, 2, 4):
        u, res = pd.parareal(U0g, J, max_iter=k, rtol=1e-300, x0=to_gpu(torch, init, pd.shape))
        assert res.iters == k
        un = u.cpu().numpy().reshape(batch, prob.nt, -1)
        for b in range(batch):
            ref = parareal.paradiag_ii(prob, J, U0[b], prob.alpha, iters=k, u_init=init[b])[-1]
            err = rel_err(un[b], ref)
            print(f"  k={k} rhs {b}: rel err {err:.2e} (tol {tol:.1e})")
            assert err <= tol


def test_parareal_converges_to_fine_solution():
    params, J, batch = CASES["fig15"]
    announce("parareal to convergence (Figure 1.5 coefficients)")
    torch, pd, prob = make(params, "fp64", batch=batch, mode="parareal")
    U0 = _u0(prob, batch, 5)
    u, res = pd.parareal(to_gpu(torch, U0, pd.field_shape), J, max_iter=60, rtol=1e-13)
    ref = parareal.fine_solution(prob, J, U0[0])
    err = rel_err(u.cpu().numpy().reshape(prob.nt, -1), ref)
    print(f"  iters {res.iters} last change {res.rel_resid:.2e} error vs fine solution {err:.2e}")
    assert res.converged and err <= 1e-11
    assert res.history[-1] <= 1e-13 and res.history[0] > 1e-3


def test_parareal_rejects_unsupported_plans():
    announce("parareal: unsupported plans and options")
    from paper_2005_09158_amd import _lib
    torch, pd, prob = make(dict(dim=2, nx=8, ny=6, nt=8, scheme="be", T=1.0, nu=0.1, alpha=0.1), "fp64",
                           mode="parareal")
    U0 = torch.zeros(pd.field_shape, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.ParaDiagError) as e:
        pd.parareal(U0, 4)
    assert e.value.status == _lib.PD_ERR_UNSUPPORTED
    torch, pd, prob = make(dict(dim=1, nx=8, ny=1, nt=8, scheme="tr", T=1.0, nu=0.1, alpha=0.1), "fp64",
                           mode="parareal")
    U0 = torch.zeros(pd.field_shape, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.ParaDiagError) as e:
        pd.parareal(U0, 4)
    assert e.value.status == _lib.PD_ERR_UNSUPPORTED
