"""Pins of the nonlinear ParaDiag oracle (eq1.4, eq1.5, windowing)."""

import numpy as np
import pytest

from oracle import Problem, krylov, nonlinear, precond

AC = nonlinear.Cubic(k1=-4.0, k3=4.0)        # Allen-Cahn reaction with eps^2 = 1/4


def _prob(scheme="be", nt=32, dim=1, alpha=0.05):
    if dim == 1:
        return Problem(dim=1, nx=40, ny=1, nt=nt, scheme=scheme, T=0.5, nu=5e-2, ax=0.4, alpha=alpha)
    return Problem(dim=2, nx=12, ny=10, nt=nt, scheme=scheme, T=0.5, nu=5e-2, ax=0.4, ay=-0.3, alpha=alpha)


def _u0(p):
    x = np.arange(1, p.nx + 1) / (p.nx + 1)
    if p.dim == 1:
        return 0.9 * np.sin(np.pi * x) + 0.3 * np.sin(3 * np.pi * x)
    y = np.arange(1, p.ny + 1) / (p.ny + 1)
    return (0.9 * np.outer(np.sin(np.pi * y), np.sin(np.pi * x))).ravel()


@pytest.mark.parametrize("dim", [1, 2])
def test_three_steps_equal_assembled_preconditioner(dim):
    p = _prob(dim=dim, nt=16)
    r = np.random.default_rng(1).standard_normal((p.nt, p.nspace))
    for cbar in (0.0, -3.7, 2.5):
        z = nonlinear.apply_P_inverse(p, r, cbar)
        z2 = np.linalg.solve(nonlinear.assembled_P(p, cbar).toarray(), r.ravel()).reshape(p.nt, -1)
        assert np.abs(z - z2).max() <= 1e-12 * np.abs(z2).max()


def test_linear_g_is_the_linear_stationary_iteration():
    """g(u) = k1 u: the iteration is eq5.1 for K + k1 I, whose iterates the
    linear oracle reproduces (cbar = k1 exactly)."""
    p = _prob(scheme="tr", nt=16)
    lin = nonlinear.Cubic(k1=0.7)
    U0 = _u0(p)
    its = nonlinear.simplified_newton(p, lin, U0, iters=12, u_init=np.zeros((p.nt, p.nspace)))
    b = nonlinear.rhs(p, lin, U0)
    # the linear problem with K + 0.7 I: residual of the converged iterate, and
    # the fixed point is the sequential solution
    ref = nonlinear.sequential(p, lin, U0)
    assert np.abs(its[-1] - ref).max() <= 1e-9 * np.abs(ref).max()
    assert np.abs(nonlinear.residual(p, lin, ref, b)).max() <= 1e-10 * np.abs(b).max()


@pytest.mark.parametrize("scheme", ["be", "tr"])
@pytest.mark.parametrize("dim", [1, 2])
def test_simplified_newton_converges_to_time_stepping(scheme, dim):
    p = _prob(scheme=scheme, dim=dim)
    U0 = _u0(p)
    ref = nonlinear.sequential(p, AC, U0)
    its = nonlinear.simplified_newton(p, AC, U0, iters=60)
    errs = [np.abs(u - ref).max() / np.abs(ref).max() for u in its]
    print(scheme, dim, ["%.1e" % e for e in errs[::6]])
    assert errs[-1] <= 1e-11
    # linear convergence (the averaged Jacobian makes it a contraction, not Newton)
    assert errs[10] <= 0.1 * errs[0]


def test_windowing_reproduces_the_single_window_solution():
    p = _prob(nt=32)
    U0 = _u0(p)
    full = nonlinear.sequential(p, AC, U0)
    half = Problem(**{**p.__dict__, "nt": 16, "T": p.T / 2})
    w = nonlinear.windowed(half, AC, U0, windows=2, iters=30)
    assert w.shape == full.shape
    assert np.abs(w - full).max() <= 1e-10 * np.abs(full).max()
