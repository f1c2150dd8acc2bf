"""Pins of the parareal oracle (Section 2.2.2): classical parareal and its
ParaDiag-II variant with the alpha-periodic coarse-grid correction."""

import numpy as np
import pytest

from oracle import Problem, operators as ops, parareal


def _fig15_problem(nt=64, periodic=False):
    """The setting of Figure 1.5: u_t - nu u_xx + u_x = 0 with nu = 0.1 on the
    periodic interval (-1, 1), dx = 1/64, u(x, 0) = exp(-30 x^2) (eq2.1),
    T = 4, dT = 1/16 (Nt = 64 coarse intervals), J = 32.  The oracle's periodic
    grid lives on [0, 1) with h = 1/n, so x' = (x + 1)/2 maps the problem onto
    it with n = 128 points, nu' = nu/4 and speed 1/2 (the same discrete system).
    periodic=False: the same coefficients with homogeneous Dirichlet data."""
    if periodic:
        return Problem(dim=1, nx=128, ny=1, nt=nt, scheme="be", T=4.0 * nt / 64, nu=0.025, ax=0.5,
                       periodic=True)
    return Problem(dim=1, nx=63, ny=1, nt=nt, scheme="be", T=4.0 * nt / 64, nu=0.1, ax=1.0)


def _u0(p):
    if p.periodic:
        x = 2.0 * np.arange(p.nx) / p.nx - 1.0
        return np.exp(-30.0 * x ** 2)
    x = np.arange(1, p.nx + 1) / (p.nx + 1)
    return np.exp(-30.0 * (x - 0.5) ** 2)


def _err(it, ref):
    return [float(np.abs(u - ref).max() / np.abs(ref).max()) for u in it]


def test_coarse_system_is_the_be_alpha_circulant():
    """The alpha-periodic coarse-grid correction solves (C1^(alpha) (x) I + I (x) K) u = b,
    which is P_alpha of backward Euler on the coarse grid (C2^(alpha) = I)."""
    p = Problem(dim=1, nx=9, ny=1, nt=6, scheme="be", T=1.0, nu=0.3, ax=0.5)
    pc = parareal.coarse_problem(p, 0.2)
    C1, C2 = ops.circulant_time_matrices(pc)
    assert np.array_equal(C2, np.eye(p.nt))
    want = np.eye(p.nt) - np.eye(p.nt, k=-1)
    want[0, -1] = -0.2
    assert np.allclose(C1, want / p.dt)


def test_classical_parareal_finite_termination():
    """After k iterations the classical iterate equals the fine solution on the
    first k coarse intervals (exactly, up to rounding)."""
    p = _fig15_problem(nt=12)
    J = 8
    U0 = _u0(p)
    ref = parareal.fine_solution(p, J, U0)
    its = parareal.classical(p, J, U0, iters=6)
    for k, u in enumerate(its, start=1):
        assert np.abs(u[:k] - ref[:k]).max() <= 1e-13 * np.abs(ref).max()
        if k < p.nt:
            assert np.abs(u[k:] - ref[k:]).max() > 1e-10   # not trivially exact beyond


def test_paradiag_parareal_fixed_point_is_the_fine_solution():
    p = _fig15_problem(nt=16)
    J = 8
    U0 = _u0(p)
    ref = parareal.fine_solution(p, J, U0)
    # the fine solution reproduces itself through one ParaDiag-II step
    b = parareal.paradiag_rhs(p, J, U0, ref, 0.1)
    from oracle import precond
    u = precond.assembled(parareal.coarse_problem(p, 0.1), b)
    assert np.abs(u - ref).max() <= 1e-12 * np.abs(ref).max()
    its = parareal.paradiag_ii(p, J, U0, 0.1, iters=16)
    assert _err(its, ref)[-1] <= 1e-11


def test_thm_the1_3_small_alpha_converges_like_classical():
    """Thm the1.3 (BE coarse propagator, L-stable fine one, real non-negative
    spectrum): the ParaDiag-II parareal contracts like the classical one for
    alpha below alpha* (about 0.3); the paper's Figure 1.5 run (periodic, from
    a random initial guess) agrees for alpha <= 1/5.  For alpha near 1 the
    first iterations are slower."""
    p = _fig15_problem(periodic=True)
    J = 32
    U0 = _u0(p)
    ref = parareal.fine_solution(p, J, U0)
    u_init = np.random.default_rng(15).standard_normal((p.nt, p.nspace))
    it = 10
    e_cl = _err(parareal.classical(p, J, U0, iters=it, u_init=u_init), ref)
    print("classical", ["%.1e" % e for e in e_cl])
    for alpha in (0.05, 0.1, 0.2):
        e = _err(parareal.paradiag_ii(p, J, U0, alpha, iters=it, u_init=u_init), ref)
        print(f"alpha {alpha}", ["%.1e" % v for v in e])
        # the same geometric rate: within a factor 3 at every iteration
        assert all(a <= 3.0 * b + 1e-14 for a, b in zip(e, e_cl))
    e_big = _err(parareal.paradiag_ii(p, J, U0, 0.9, iters=it, u_init=u_init), ref)
    print("alpha 0.9", ["%.1e" % v for v in e_big])
    assert e_big[-1] > 10.0 * e_cl[-1]
