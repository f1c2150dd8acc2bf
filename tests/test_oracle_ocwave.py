"""Pins of the oracle for the optimal control of the wave equation (Section 4)."""

import numpy as np
import pytest

from oracle import ocwave
from tests.conftest import load_golden


def test_theorem_route_equals_assembled_preconditioner():
    p = ocwave.wave_problem(8, 9)
    r = np.random.default_rng(0).standard_normal(2 * p.nt * p.nspace)
    for gamma in (1e-2, 1e-6):
        z = ocwave.apply_P_inverse(p, gamma, r)
        z2 = np.linalg.solve(ocwave.assembled(p, gamma, circulant=True).toarray(), r)
        assert np.abs(z - z2).max() <= 1e-11 * np.abs(z2).max()


def test_block_eigenvectors_are_perfectly_conditioned():
    """Thm the4: the 2 x 2 eigenvector matrices have Cond_2 = 1 and diagonalise G_n."""
    nt, dt, gamma = 17, 2.0 / 17, 1e-4
    d1, d2 = ocwave.symbols(nt)
    s1, s2, E = ocwave.block_eigen(nt, dt, gamma)
    beta = dt * dt / np.sqrt(gamma)
    for n in range(nt):
        a, q = d1[n] / d2[n], 1.0 / d2[n]
        assert abs(a.imag) <= 1e-12 * max(1.0, abs(a))       # d1/d2 real for alpha = 1
        G = np.array([[a, -beta * np.conj(q)], [beta * q, np.conj(a)]])
        W = np.array([[1, 1], [-1j * E[n], 1j * E[n]]])
        assert np.linalg.cond(W) == pytest.approx(1.0, abs=1e-12)
        assert np.abs(G @ W - W @ np.diag([s1[n], s2[n]])).max() <= 1e-12 * np.abs(G).max()


def test_c2_singular_when_four_divides_nt():
    with pytest.raises(ValueError):
        ocwave.block_eigen(16, 0.1, 1e-4)


def test_discrete_solution_is_second_order():
    """The exact (u, p) of Section 4's example; readings OC1-OC3 give a
    second-order consistent discretisation (a slip in the time indexing of the
    coupling or of the half rows would drop it to first order)."""
    errs = []
    for n in (8, 16, 32):
        p = ocwave.wave_problem(n, n + 1)
        gamma = 1e-2
        # the preconditioned GMRES solve (checked against the direct solve below)
        x, its, _ = ocwave.gmres(p, gamma, ocwave.rhs(p, gamma), tol=1e-13)
        u, q = ocwave.unscale(p, gamma, x)
        ue, qe = ocwave.exact_fields(p)
        errs.append(max(np.abs(u - ue).max() / np.abs(ue).max(), np.abs(q - qe).max() / np.abs(qe).max()))
        if n == 8:
            assert np.abs(x - ocwave.solve(p, gamma, ocwave.rhs(p, gamma))).max() <= 1e-10 * np.abs(x).max()
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print("errors", errs, "rates", rates)
    assert np.all(rates > 1.8)


@pytest.mark.parametrize("n", [16, 32, 64])
def test_table_t2a_iteration_counts(n):
    """GMRES with P to tol 1e-7 on the paper's example: Table T2A's counts,
    within one iteration (the paper's Matlab GMRES variant and stopping norm
    are not stated; reading OC5)."""
    rows = {r["N"]: r for r in load_golden("table_t2a.json")["rows"]}
    p = ocwave.wave_problem(n, n + 1)
    for gamma, key in ((1e-2, "g1e-2"), (1e-4, "g1e-4"), (1e-6, "g1e-6"), (1e-8, "g1e-8"), (1e-10, "g1e-10")):
        b = ocwave.rhs(p, gamma)
        x, its, hist = ocwave.gmres(p, gamma, b, tol=1e-7)
        print(f"N {n} gamma {gamma}: {its} iterations (printed {rows[n][key]})")
        assert abs(its - rows[n][key]) <= 1
        assert np.linalg.norm(b - ocwave.assembled(p, gamma) @ x) <= 1.01e-7 * np.linalg.norm(b)
