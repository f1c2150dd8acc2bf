"""Pins of the oracle's P_alpha^{-1}: two routes, exact spectra, alpha limit."""

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

from oracle import Problem, operators as ops, precond, solve
from tests.conftest import load_golden


def _match(a, b):
    D = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(D)
    return float(D[r, c].max())


@pytest.mark.parametrize("scheme", ["be", "tr", "lf"])
@pytest.mark.parametrize("alpha", [1e-3, 0.1, 1.0])
def test_two_routes_agree(scheme, alpha):
    p = Problem(dim=2, nx=6, ny=5, nt=8, scheme=scheme, T=1.0, nu=0.05,
                ax=0.8 if scheme != "lf" else 0.0, ay=0.3 if scheme != "lf" else 0.0, alpha=alpha)
    r = np.random.default_rng(7).standard_normal((p.nt, p.nspace))
    z1 = precond.assembled(p, r)
    z2 = precond.three_steps(p, r)
    assert np.abs(z1 - z2).max() / np.abs(z1).max() < 1e-11
    # defining property at any size: P_alpha z = r
    assert np.abs(ops.apply_P(p, z2) - r).max() / np.abs(r).max() < 1e-11


def _dense_ev(p):
    A = ops.all_at_once_sparse(p).toarray()
    P = ops.preconditioner_sparse(p).toarray()
    return np.linalg.eigvals(np.linalg.solve(P, A))


@pytest.mark.parametrize("scheme", ["be", "tr"])
def test_one_step_spectrum_closed_form(scheme):
    # P^{-1}A has eigenvalue 1 with multiplicity (Nt-1)Nx and 1/(1 - alpha r_j^Nt),
    # r_j the amplification factor of the scheme at the eigenvalue mu_j of K.
    p = Problem(dim=1, nx=7, ny=1, nt=12, scheme=scheme, T=1.0, nu=0.1, ax=1.0, alpha=0.05)
    mu = np.linalg.eigvals(ops.spatial_operator(p).toarray())
    dt = p.dt
    th = 1.0 if scheme == "be" else 0.5
    r = (1 - (1 - th) * dt * mu) / (1 + th * dt * mu)
    expected = np.concatenate([np.ones((p.nt - 1) * p.nx), 1.0 / (1 - p.alpha * r ** p.nt)])
    assert _match(_dense_ev(p), expected) < 1e-9


@pytest.mark.parametrize("alpha", [0.1, 0.5])
def test_leapfrog_spectrum_theorem_the3_1(alpha):
    p = Problem(dim=1, nx=6, ny=1, nt=12, scheme="lf", T=1.0, nu=1.0, alpha=alpha)
    K = ops.spatial_operator(p).toarray()
    lam = np.sort(np.linalg.eigvalsh(np.eye(p.nx) + 0.5 * p.dt ** 2 * K))
    th = np.arctan(np.sqrt(lam ** 2 - 1))
    nontriv = np.concatenate([1 / (1 - alpha * np.exp(1j * p.nt * th)),
                              1 / (1 - alpha * np.exp(-1j * p.nt * th))])
    expected = np.concatenate([np.ones((p.nt - 2) * p.nx), nontriv])
    ev = _dense_ev(p)
    assert _match(ev, expected) < 1e-9
    d = np.abs(ev - 1)
    d = d[d > 1e-8]
    assert np.all(d >= alpha / (1 + alpha) - 1e-10)
    assert np.all(d <= alpha / (1 - alpha) + 1e-10)


def test_leapfrog_strang_circulant_alpha_one():
    # alpha = 1 (the Strang circulant of eq3.3): spectrum {1} U {1/2 +- i/2 cot(Nt theta_j/2)}
    p = Problem(dim=1, nx=5, ny=1, nt=10, scheme="lf", T=1.0, nu=1.0, alpha=1.0)
    K = ops.spatial_operator(p).toarray()
    lam = np.sort(np.linalg.eigvalsh(np.eye(p.nx) + 0.5 * p.dt ** 2 * K))
    th = np.arctan(np.sqrt(lam ** 2 - 1))
    cot = 1 / np.tan(p.nt * th / 2)
    expected = np.concatenate([np.ones((p.nt - 2) * p.nx), 0.5 + 0.5j * cot, 0.5 - 0.5j * cot])
    assert _match(_dense_ev(p), expected) < 1e-8


def test_alpha_to_zero_limit():
    # P_alpha -> A as alpha -> 0: ||P^{-1} b - A^{-1} b|| = O(alpha)
    base = dict(dim=1, nx=9, ny=1, nt=16, scheme="tr", T=1.0, nu=0.05, ax=1.0)
    b = np.random.default_rng(2).standard_normal((16, 9))
    u = solve.sequential(Problem(**base), b)
    errs = []
    for a in (1e-2, 1e-3, 1e-4):
        z = precond.three_steps(Problem(**base, alpha=a), b)
        errs.append(np.abs(z - u).max() / np.abs(u).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(np.log10(ratios) - 1.0) < 0.1), errs


def test_hermitian_half_spectrum():
    # real data and real symbols: S_{Nt-n} = conj(S_n) and lambda_{Nt-n} = conj(lambda_n)
    p = Problem(dim=1, nx=4, ny=1, nt=16, scheme="lf", T=1.0, nu=1.0, alpha=0.01)
    l1, l2 = ops.time_symbols(p)
    for lam in (l1, l2):
        np.testing.assert_allclose(lam[1:][::-1], np.conj(lam[1:]), atol=1e-12 * np.abs(lam).max())
