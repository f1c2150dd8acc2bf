"""Pins of the oracle's right-hand side rows that no order-of-accuracy test separates.

With K = 0 (nu = 0, no velocity) every scheme reduces to a quadrature of the
source, whose discrete solution is known in closed form.  That fixes:

* the theta-method source weighting theta f_n + (1 - theta) f_{n-1} (our
  reading of eq2.5 with a source): backward Euler must add dt f(t_n), not
  dt f(t_{n-1}), at step n;
* the first two leap-frog rows (our reading of eq3.2 with the central ghost
  value U_{-1} = U_1 - 2 dt u_1): for u'' = c the central second difference is
  exact on quadratics, so U_n = U_0 + u_1 t_n + c t_n^2 / 2 at every level.
"""

import numpy as np
import pytest

from oracle import Problem, rhs, solve


def _flat(scheme, nt, T=1.0):
    # nu = 0 and zero velocity: the spatial operator is the zero matrix
    return Problem(dim=1, nx=3, ny=1, nt=nt, scheme=scheme, T=T, nu=0.0, ax=0.0)


def test_backward_euler_adds_the_source_at_the_new_level():
    # U_n = U_{n-1} + dt f(t_n) with f(t) = t: U_n = U_0 + dt^2 n (n + 1) / 2.
    # Weighting with f(t_{n-1}) instead would give U_0 + dt^2 n (n - 1) / 2.
    p = _flat("be", 10)
    t = np.arange(p.nt + 1) * p.dt
    U0 = np.array([1.0, -2.0, 0.5])
    f = np.repeat(t[:, None], 3, axis=1)
    u = solve.sequential(p, rhs.build_rhs(p, U0, None, f))
    n = np.arange(1, p.nt + 1)
    expect = U0[None, :] + (p.dt ** 2 * n * (n + 1) / 2)[:, None]
    np.testing.assert_allclose(u, expect, rtol=0, atol=1e-13)


def test_trapezoidal_rule_integrates_linear_sources_exactly():
    # U_n = U_{n-1} + dt (f_n + f_{n-1}) / 2 is exact for f(t) = 3 t - 1:
    # U_n = U_0 + 3 t_n^2 / 2 - t_n.
    p = _flat("tr", 12, T=2.0)
    t = np.arange(p.nt + 1) * p.dt
    U0 = np.array([0.25, 0.0, -1.0])
    f = np.repeat((3 * t - 1)[:, None], 3, axis=1)
    u = solve.sequential(p, rhs.build_rhs(p, U0, None, f))
    expect = U0[None, :] + (1.5 * t[1:] ** 2 - t[1:])[:, None]
    np.testing.assert_allclose(u, expect, rtol=0, atol=1e-13)


@pytest.mark.parametrize("nt", [2, 3, 11])
def test_leapfrog_start_rows_exact_on_quadratics(nt):
    # u'' = c, u(0) = U0, u'(0) = v: exact solution U0 + v t + c t^2 / 2, which
    # the leap-frog rows reproduce exactly when row 1 carries the ghost value
    # and half the source f_0, and row 2 moves U_0 to the right-hand side.
    p = _flat("lf", nt, T=1.5)
    t = np.arange(p.nt + 1) * p.dt
    U0 = np.array([1.0, 2.0, -3.0])
    v = np.array([0.5, -1.0, 2.0])
    c = np.array([2.0, 0.0, -4.0])
    f = np.repeat(c[None, :], p.nt + 1, axis=0)
    u = solve.sequential(p, rhs.build_rhs(p, U0, v, f))
    tt = t[1:, None]
    expect = U0[None, :] + v[None, :] * tt + 0.5 * c[None, :] * tt ** 2
    np.testing.assert_allclose(u, expect, rtol=0, atol=1e-11)
