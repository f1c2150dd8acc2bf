"""Pins of the oracle's operators against the paper and against mathematics."""

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

from oracle import Problem, operators as ops
from tests.conftest import load_golden


def _match(a, b):
    """Max distance between two multisets of complex numbers under the best matching."""
    D = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(D)
    return float(D[r, c].max())


def test_theta_circulants_match_eq2_11b():
    g = load_golden("eq2_11b_circulants.json")
    nt, dt, alpha = g["nt"], g["dt"], g["alpha"]
    c1, c2 = ops.time_columns("tr", dt)
    C1 = ops.alpha_circulant(c1, nt, alpha)
    C2 = ops.alpha_circulant(c2, nt, alpha)
    np.testing.assert_allclose(C1 * dt, np.array(g["C1_times_dt"]), atol=1e-15)
    np.testing.assert_allclose(C2, np.array(g["C2_tr"]), atol=1e-15)
    _, c2be = ops.time_columns("be", dt)
    np.testing.assert_allclose(ops.alpha_circulant(c2be, nt, alpha), np.array(g["C2_be"]), atol=1e-15)


def test_leapfrog_circulants_match_eq3_4():
    g = load_golden("eq3_4_circulants.json")
    nt, dt, alpha = g["nt"], g["dt"], g["alpha"]
    c1, c2 = ops.time_columns("lf", dt)
    np.testing.assert_allclose(ops.alpha_circulant(c1, nt, alpha) * dt ** 2,
                               np.array(g["C1_times_dt2"]), atol=1e-14)
    np.testing.assert_allclose(ops.alpha_circulant(c2, nt, alpha), np.array(g["C2"]), atol=1e-15)


def test_toeplitz_is_alpha_zero_limit():
    # P_alpha -> A as alpha -> 0 (Section 1): the circulant at alpha = 0 is B.
    for s in ("be", "tr", "lf"):
        c1, c2 = ops.time_columns(s, 0.1)
        for c in (c1, c2):
            np.testing.assert_array_equal(ops.alpha_circulant(c, 9, 0.0), ops.toeplitz_lower(c, 9))


@pytest.mark.parametrize("scheme", ["be", "tr", "lf"])
@pytest.mark.parametrize("alpha", [1e-3, 0.1, 1.0])
def test_time_symbols_are_eigenvalues(scheme, alpha):
    # Lemma 1: eig(C_j^(alpha)) = fft(Gamma_alpha c_j)
    p = Problem(dim=1, nx=3, ny=1, nt=16, scheme=scheme, T=1.0, nu=1.0, alpha=alpha)
    C1, C2 = ops.circulant_time_matrices(p)
    l1, l2 = ops.time_symbols(p)
    for C, lam in ((C1, l1), (C2, l2)):
        ev = np.linalg.eigvals(C)
        scale = max(1.0, np.abs(lam).max())
        assert _match(ev, lam) / scale < 1e-12


@pytest.mark.parametrize("scheme", ["be", "tr", "lf"])
def test_time_symbols_simultaneous_diagonalisation(scheme):
    # Lemma 1: C_j = V D_j V^{-1} with the same V = Gamma^{-1} F^* for j = 1, 2.
    p = Problem(dim=1, nx=3, ny=1, nt=8, scheme=scheme, T=1.0, nu=1.0, alpha=0.05)
    C1, C2 = ops.circulant_time_matrices(p)
    l1, l2 = ops.time_symbols(p)
    nt = p.nt
    g = ops.gamma(nt, p.alpha)
    Finv = np.fft.ifft(np.eye(nt), axis=0)            # inverse DFT matrix
    V = np.diag(1.0 / g) @ Finv
    Vinv = np.fft.fft(np.eye(nt), axis=0) @ np.diag(g)
    np.testing.assert_allclose(V @ np.diag(l1) @ Vinv, C1, atol=1e-11 * np.abs(C1).max())
    np.testing.assert_allclose(V @ np.diag(l2) @ Vinv, C2, atol=1e-12)
    # Cond2(V) <= 1/alpha (eq2.13)
    assert np.linalg.cond(V) <= 1.0 / p.alpha * (1 + 1e-12)


def test_persymmetry():
    # J C^T J = C for Toeplitz and alpha-circulant matrices (used by the adjoint).
    for s in ("be", "tr", "lf"):
        c1, _ = ops.time_columns(s, 0.1)
        J = np.eye(10)[::-1]
        for M in (ops.toeplitz_lower(c1, 10), ops.alpha_circulant(c1, 10, 0.3)):
            np.testing.assert_array_equal(J @ M.T @ J, M)


def test_spatial_operator_consistency_2d():
    # K u ~ -nu Lap u + a . grad u for a smooth u vanishing on the boundary, error O(h^2)
    errs = []
    for n in (32, 64, 128):
        p = Problem(dim=2, nx=n, ny=n + 3, nt=4, scheme="be", T=1.0, nu=0.3, ax=1.3, ay=-0.7)
        x = np.arange(1, p.nx + 1) / (p.nx + 1)
        y = np.arange(1, p.ny + 1) / (p.ny + 1)
        X, Y = np.meshgrid(x, y)         # [ny][nx]
        u = np.sin(np.pi * X) * np.sin(2 * np.pi * Y) * np.exp(X)
        ux = (np.pi * np.cos(np.pi * X) + np.sin(np.pi * X)) * np.sin(2 * np.pi * Y) * np.exp(X)
        uxx = (-np.pi ** 2 * np.sin(np.pi * X) + 2 * np.pi * np.cos(np.pi * X)
               + np.sin(np.pi * X)) * np.sin(2 * np.pi * Y) * np.exp(X)
        uy = 2 * np.pi * np.sin(np.pi * X) * np.cos(2 * np.pi * Y) * np.exp(X)
        uyy = -4 * np.pi ** 2 * u
        exact = -p.nu * (uxx + uyy) + p.ax * ux + p.ay * uy
        Ku = (ops.spatial_operator(p) @ u.ravel()).reshape(u.shape)
        errs.append(np.abs(Ku - exact).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.8) and orders[-1] > 1.9, orders


def test_dst_diagonalises_symmetric_factor():
    # Symmetric factor (zero velocity): Q_jk = sqrt(2/(n+1)) sin(jk pi/(n+1)),
    # eigenvalues (4 nu / h^2) sin^2(k pi / (2(n+1))).
    n, nu = 23, 0.7
    K = ops.k1d(n, nu, 0.0).toarray()
    j = np.arange(1, n + 1)
    Q = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(j, j) * np.pi / (n + 1))
    h = 1.0 / (n + 1)
    t = 4 * nu / h ** 2 * np.sin(j * np.pi / (2 * (n + 1))) ** 2
    np.testing.assert_allclose(Q.T @ K @ Q, np.diag(t), atol=1e-10 * t.max())


def test_advection_factor_spectrum():
    # Dirichlet Toeplitz tridiagonal: eigenvalues 2d - 2 sqrt(bc) cos(k pi/(n+1)) (real when Pe < 1)
    n, nu, a = 30, 0.05, 1.0
    h = 1 / (n + 1)
    K = ops.k1d(n, nu, a).toarray()
    b = -nu / h ** 2 - a / (2 * h)
    c = -nu / h ** 2 + a / (2 * h)
    k = np.arange(1, n + 1)
    ev = 2 * nu / h ** 2 - 2 * np.sqrt(b * c) * np.cos(k * np.pi / (n + 1))
    got = np.sort(np.linalg.eigvals(K).real)
    np.testing.assert_allclose(got, np.sort(ev), rtol=1e-8)


@pytest.mark.parametrize("n", [5, 8, 16])
def test_periodic_factor_is_the_circulant_of_eq2_2b(n):
    # Periodic boundaries (eq2.2b with its corner entries): K is circulant, so
    # the Fourier modes w_j = e^{2 pi i k j / n} are eigenvectors with the
    # closed-form eigenvalues (4 nu / h^2) sin^2(pi k / n) + i (a / h) sin(2 pi k / n).
    nu, a = 0.03, 1.7
    K = ops.k1d(n, nu, a, periodic=True).toarray()
    h = ops.mesh_width(n, periodic=True)
    assert h == 1.0 / n
    k = np.arange(n)
    lam = 4 * nu / h ** 2 * np.sin(np.pi * k / n) ** 2 + 1j * (a / h) * np.sin(2 * np.pi * k / n)
    W = np.exp(2j * np.pi * np.outer(np.arange(n), k) / n)
    np.testing.assert_allclose(K @ W, W * lam[None, :], atol=1e-12 * np.abs(lam).max())
    # every row holds the same stencil, wrapped at the ends
    for i in range(n):
        np.testing.assert_allclose(np.roll(K[i], -i), np.roll(K[0], 0), atol=0)
