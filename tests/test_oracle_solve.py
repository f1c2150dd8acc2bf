"""Pins of the oracle's all-at-once solution and of its discretisation."""

import numpy as np
import pytest

from oracle import Problem, operators as ops, rhs, solve
from tests.conftest import load_golden


@pytest.mark.parametrize("scheme", ["be", "tr", "lf"])
@pytest.mark.parametrize("dim", [1, 2])
def test_three_routes_agree(scheme, dim):
    p = Problem(dim=dim, nx=7, ny=5 if dim == 2 else 1, nt=9, scheme=scheme, T=0.7,
                nu=0.05, ax=1.0 if scheme != "lf" else 0.0, ay=-0.5 if scheme != "lf" else 0.0)
    b = np.random.default_rng(3).standard_normal((p.nt, p.nspace))
    u1 = solve.sequential(p, b)
    u2 = solve.all_at_once(p, b)
    u3 = solve.dense(p, b)
    s = np.abs(u3).max()
    assert np.abs(u1 - u3).max() / s < 1e-12
    assert np.abs(u2 - u3).max() / s < 1e-12
    assert solve.relative_residual(p, u1, b) < 1e-13


def test_all_at_once_matvec_matches_dense():
    p = Problem(dim=2, nx=4, ny=3, nt=6, scheme="lf", T=1.0, nu=0.3)
    u = np.random.default_rng(1).standard_normal((p.nt, p.nspace))
    A = ops.all_at_once_sparse(p)
    np.testing.assert_allclose(ops.apply_A(p, u).ravel(), A @ u.ravel(), rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(ops.apply_AT(p, u).ravel(), A.T @ u.ravel(), rtol=1e-13, atol=1e-12)
    P = ops.preconditioner_sparse(p)
    np.testing.assert_allclose(ops.apply_P(p, u).ravel(), P @ u.ravel(), rtol=1e-13, atol=1e-12)


def _adv_diff_error(scheme, n, nt, nu=0.1, a=1.0, T=0.5):
    """max-in-time error of the all-at-once solution for u = sin(pi x) e^{-t}."""
    p = Problem(dim=1, nx=n, ny=1, nt=nt, scheme=scheme, T=T, nu=nu, ax=a)
    x = np.arange(1, n + 1) / (n + 1)
    t = np.arange(nt + 1) * p.dt
    ue = np.sin(np.pi * x)[None, :] * np.exp(-t)[:, None]
    f = ((-1 + nu * np.pi ** 2) * np.sin(np.pi * x)[None, :]
         + a * np.pi * np.cos(np.pi * x)[None, :]) * np.exp(-t)[:, None]
    b = rhs.build_rhs(p, ue[0], None, f)
    u = solve.sequential(p, b)
    return np.abs(u - ue[1:]).max()


def test_backward_euler_first_order_in_time():
    e = [_adv_diff_error("be", 400, nt) for nt in (8, 16, 32)]
    orders = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all(np.abs(orders - 1.0) < 0.15), orders


def test_trapezoidal_second_order():
    e = [_adv_diff_error("tr", n, nt) for n, nt in ((15, 8), (31, 16), (63, 32))]
    orders = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all(np.abs(orders - 2.0) < 0.15), orders


def _wave_error(N, T=2.0):
    """T4A problem: u = sin(pi x) sin(pi y) e^t, mesh width 1/N, N steps; L^inf(0,T;L^2) error."""
    n = N - 1
    p = Problem(dim=2, nx=n, ny=n, nt=N, scheme="lf", T=T, nu=1.0)
    x = np.arange(1, n + 1) / N
    X, Y = np.meshgrid(x, x)
    s = (np.sin(np.pi * X) * np.sin(np.pi * Y)).ravel()
    t = np.arange(N + 1) * p.dt
    f = (1 + 2 * np.pi ** 2) * s[None, :] * np.exp(t)[:, None]
    b = rhs.build_rhs(p, s, s, f)
    u = solve.sequential(p, b)
    ue = s[None, :] * np.exp(t[1:])[:, None]
    h = 1.0 / N
    return np.max(np.sqrt(h * h * np.sum((u - ue) ** 2, axis=1)))


def test_leapfrog_order_matches_table_t4a():
    g = load_golden("table_t4a.json")
    errs = {N: _wave_error(N) for N in (16, 32, 64)}
    for row in g["rows"]:
        N = row["N"]
        if N in errs and N // 2 in errs:
            order = np.log2(errs[N // 2] / errs[N])
            assert abs(order - row["order"]) <= 0.1 + 1e-9, (N, order, row["order"])
