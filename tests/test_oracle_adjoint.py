"""Pins of the oracle's transposed solve and gradient."""

import numpy as np
import pytest

from oracle import Problem, adjoint, operators as ops, rhs, solve


@pytest.mark.parametrize("scheme", ["be", "tr", "lf"])
def test_rhs_transpose_dot_product(scheme):
    p = Problem(dim=2, nx=5, ny=4, nt=7, scheme=scheme, T=1.0, nu=0.1,
                ax=0.7 if scheme != "lf" else 0.0, ay=-0.4 if scheme != "lf" else 0.0)
    rng = np.random.default_rng(1)
    U0, u1 = rng.standard_normal(p.nspace), rng.standard_normal(p.nspace)
    f = rng.standard_normal((p.nt + 1, p.nspace))
    lam = rng.standard_normal((p.nt, p.nspace))
    b = rhs.build_rhs(p, U0, u1 if scheme == "lf" else None, f)
    gU0, gu1, gf = rhs.rhs_transpose(p, lam)
    lhs = np.vdot(b, lam)
    rhs_val = np.vdot(U0, gU0) + (np.vdot(u1, gu1) if scheme == "lf" else 0.0) + np.vdot(f, gf)
    assert abs(lhs - rhs_val) <= 1e-12 * (abs(lhs) + 1)


@pytest.mark.parametrize("scheme", ["be", "tr", "lf"])
def test_transpose_solve_dot_product(scheme):
    # <A^{-1} b, g> = <b, A^{-T} g>, with the forward stepper on one side
    p = Problem(dim=2, nx=6, ny=5, nt=9, scheme=scheme, T=1.0, nu=0.05,
                ax=1.0 if scheme != "lf" else 0.0, ay=0.5 if scheme != "lf" else 0.0)
    rng = np.random.default_rng(2)
    b, g = rng.standard_normal((2, p.nt, p.nspace))
    u = solve.sequential(p, b)
    lam = adjoint.sequential_transpose(p, g)
    assert abs(np.vdot(u, g) - np.vdot(b, lam)) <= 1e-11 * np.abs(u).max() * np.abs(g).sum()
    # and A^T lam = g
    assert np.abs(ops.apply_AT(p, lam) - g).max() < 1e-10 * np.abs(g).max() * max(1, np.abs(lam).max())


def test_gradient_equals_dense_gradient():
    p = Problem(dim=2, nx=4, ny=3, nt=5, scheme="be", T=1.0, nu=0.1, ax=1.0, ay=0.5)
    S, nt = p.nspace, p.nt
    rng = np.random.default_rng(4)
    U0 = rng.standard_normal(S)
    f = rng.standard_normal((nt + 1, S))
    target = rng.standard_normal(S)
    beta = 1e-2
    # brute force: the matrices of U0 -> b and f -> b column by column, dense A
    RU = np.stack([rhs.build_rhs(p, e, None, None).ravel() for e in np.eye(S)], axis=1)
    Rf = np.stack([rhs.build_rhs(p, np.zeros(S), None, e.reshape(nt + 1, S)).ravel()
                   for e in np.eye((nt + 1) * S)], axis=1)
    B1, B2 = ops.time_matrices(p)
    A = np.kron(B1, np.eye(S)) + np.kron(B2, ops.spatial_operator(p).toarray())
    Ainv = np.linalg.inv(A)
    sel = np.zeros((S, nt * S))
    sel[:, (nt - 1) * S:] = np.eye(S)
    u = Ainv @ (RU @ U0 + Rf @ f.ravel())
    d = sel @ u - target
    gU0_dense = (sel @ Ainv @ RU).T @ d
    gf_dense = (sel @ Ainv @ Rf).T @ d + beta * f.ravel()
    J, gU0, gf = adjoint.gradient(p, U0, f, target, beta)
    np.testing.assert_allclose(gU0, gU0_dense, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(gf.ravel(), gf_dense, rtol=1e-10, atol=1e-12)
    assert abs(J - (0.5 * d @ d + 0.5 * beta * np.sum(f * f))) < 1e-12 * abs(J)


def test_gradient_matches_central_differences():
    # cfg4-shaped (backward Euler, advection-diffusion), reduced size; J is quadratic,
    # so central differences are exact up to rounding.
    p = Problem(dim=2, nx=8, ny=8, nt=12, scheme="be", T=1.0, nu=5e-3, ax=1.0, ay=0.5)
    rng = np.random.default_rng(9)
    U0 = rng.standard_normal(p.nspace)
    f = rng.standard_normal((p.nt + 1, p.nspace))
    target = rng.standard_normal(p.nspace)
    beta = 1e-4
    J, gU0, gf = adjoint.gradient(p, U0, f, target, beta)
    for i in range(20):
        r = np.random.default_rng(200 + i)
        d0 = r.standard_normal(p.nspace)
        df = r.standard_normal((p.nt + 1, p.nspace))
        nrm = np.sqrt(d0 @ d0 + np.sum(df * df))
        d0, df = d0 / nrm, df / nrm
        fd = adjoint.finite_difference(p, U0, f, target, beta, d0, df, h=1e-6)
        an = gU0 @ d0 + np.sum(gf * df)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * abs(J)), (i, fd, an)
