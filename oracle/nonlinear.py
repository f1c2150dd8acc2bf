"""Nonlinear ParaDiag: simplified Newton with an averaged Jacobian (eq1.4, eq1.5)
and windowing, float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Problem: U' + K U + g(U) = 0 with a pointwise cubic g(u) = k1 u + k2 u^2 +
k3 u^3 (Allen-Cahn for k1 = -1/eps^2, k3 = 1/eps^2), discretised by the
theta-method (backward Euler or the trapezoidal rule), so that with
F(U) = K U + g(U) the all-at-once system is eq1.4,

    (B1 (x) I) u + (B2 (x) I) F(u) = b,

B1, B2 the Toeplitz matrices of eq2.5b and b_1 = U0/dt - (1-theta) F(U0)
(U0 known), b_n = 0 otherwise (no source).

* ``residual``: R(u) = b - (B1 (x) I) u - (B2 (x) I) F(u).
* ``sequential``: the plain definition of the solution: time stepping, each
  step solved by full Newton iteration to rounding level.
* ``simplified_newton`` (eq1.5): P_alpha(u^{k-1}) du = R(u^{k-1}),
  u^k = u^{k-1} + du, with P_alpha(u) = C1^(alpha) (x) I + C2^(alpha) (x)
  (K + cbar I): the averaged Jacobian of the paper with the average taken over
  the Nt time points and also over space (reading N1: cbar is the mean of
  g'(U_n) over all n and all points, so Step-(b) keeps the structure of K).
  P_alpha^{-1} is applied by the three steps of eq1.3 with the time symbols
  of the theta-method: Step-(b) solves ((lambda1_n + cbar lambda2_n) I +
  lambda2_n K).
* ``windowed``: the horizon split into windows of Nt steps, each solved by
  ``simplified_newton`` from the last state of the previous one.

Pins (tests/test_oracle_nonlinear.py): the three-step P_alpha(u)^{-1} equals a
sparse solve with the assembled matrix; the simplified Newton iteration
converges to the sequential solution; with g linear it is the linear
ParaDiag-II stationary iteration with K + k1 I; windowing reproduces the
single-window solution of the same time grid.  Beyond that, the paper prints
no values for this method: parity unpinned.
"""

from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operators import THETA, gamma, spatial_operator, time_matrices, time_symbols
from .problem import Problem


@dataclasses.dataclass(frozen=True)
class Cubic:
    k1: float = 0.0
    k2: float = 0.0
    k3: float = 0.0

    def g(self, u):
        return self.k1 * u + self.k2 * u * u + self.k3 * u * u * u

    def dg(self, u):
        return self.k1 + 2.0 * self.k2 * u + 3.0 * self.k3 * u * u


def _theta(p: Problem) -> float:
    if p.scheme not in THETA:
        raise ValueError("the nonlinear oracle covers the theta-method (be, tr)")
    return THETA[p.scheme]


def rhs(p: Problem, g: Cubic, U0) -> np.ndarray:
    """b of eq1.4 with the known initial state: b_1 = U0/dt - (1-theta) F(U0)."""
    th = _theta(p)
    K = spatial_operator(p)
    U0 = np.asarray(U0, dtype=np.float64).reshape(p.nspace)
    b = np.zeros((p.nt, p.nspace))
    b[0] = U0 / p.dt - (1.0 - th) * (K @ U0 + g.g(U0))
    return b


def residual(p: Problem, g: Cubic, u, b) -> np.ndarray:
    """R(u) = b - (B1 (x) I) u - (B2 (x) I) F(u), F(U) = K U + g(U)."""
    B1, B2 = time_matrices(p)
    K = spatial_operator(p)
    U = np.asarray(u, dtype=np.float64).reshape(p.nt, p.nspace)
    F = (K @ U.T).T + g.g(U)
    return np.asarray(b).reshape(p.nt, -1) - B1 @ U - B2 @ F


def sequential(p: Problem, g: Cubic, U0, newton_tol: float = 1e-14) -> np.ndarray:
    """Time stepping: (U_n - U_{n-1})/dt + theta F(U_n) + (1-theta) F(U_{n-1}) = 0,
    each step by Newton's method with the exact Jacobian."""
    th = _theta(p)
    K = spatial_operator(p).tocsc()
    I = sp.identity(p.nspace, format="csc")
    U = np.zeros((p.nt, p.nspace))
    x = np.asarray(U0, dtype=np.float64).reshape(p.nspace)
    for n in range(p.nt):
        known = x / p.dt - (1.0 - th) * (K @ x + g.g(x))
        y = x.copy()
        for _ in range(50):
            res = known - (y / p.dt + th * (K @ y + g.g(y)))
            J = (I / p.dt + th * (K + sp.diags(g.dg(y)))).tocsc()
            dy = spla.spsolve(J, res)
            y = y + dy
            if np.abs(dy).max() <= newton_tol * max(1.0, np.abs(y).max()):
                break
        U[n] = y
        x = y
    return U


def average_slope(g: Cubic, u) -> float:
    """cbar: the mean of g'(U_n) over every time point and grid point (reading N1)."""
    return float(np.mean(g.dg(np.asarray(u))))


def apply_P_inverse(p: Problem, r, cbar: float) -> np.ndarray:
    """P_alpha(u)^{-1} r by the three steps of eq1.3 (full complex FFTs)."""
    lam1, lam2 = time_symbols(p)
    gm = gamma(p.nt, p.alpha)
    K = spatial_operator(p).astype(np.complex128)
    I = sp.identity(p.nspace, dtype=np.complex128, format="csc")
    R = np.asarray(r, dtype=np.float64).reshape(p.nt, p.nspace)
    S1 = np.fft.fft(gm[:, None] * R, axis=0)
    S2 = np.empty_like(S1)
    for n in range(p.nt):
        M = ((lam1[n] + cbar * lam2[n]) * I + lam2[n] * K).tocsc()
        S2[n] = spla.splu(M).solve(S1[n])
    return ((1.0 / gm)[:, None] * np.fft.ifft(S2, axis=0)).real


def assembled_P(p: Problem, cbar: float) -> sp.csc_matrix:
    from .operators import circulant_time_matrices
    C1, C2 = circulant_time_matrices(p)
    K = spatial_operator(p)
    I = sp.identity(p.nspace, format="csr")
    return (sp.kron(sp.csr_matrix(C1), I) + sp.kron(sp.csr_matrix(C2), K + cbar * I)).tocsc()


def simplified_newton(p: Problem, g: Cubic, U0, iters: int, u_init=None):
    """The iteration eq1.5 from u_init (default: U0 repeated); returns the iterates."""
    b = rhs(p, g, U0)
    U0 = np.asarray(U0, dtype=np.float64).reshape(p.nspace)
    u = np.tile(U0, (p.nt, 1)) if u_init is None else np.array(u_init, dtype=np.float64).reshape(p.nt, -1)
    out = []
    for _ in range(iters):
        cbar = average_slope(g, u)
        u = u + apply_P_inverse(p, residual(p, g, u, b), cbar)
        out.append(u.copy())
    return out


def windowed(p: Problem, g: Cubic, U0, windows: int, iters: int) -> np.ndarray:
    """Windows of p.nt steps one after another; returns [windows * nt][nspace]."""
    out = []
    x = np.asarray(U0, dtype=np.float64).reshape(p.nspace)
    for _ in range(windows):
        u = simplified_newton(p, g, x, iters)[-1]
        out.append(u)
        x = u[-1]
    return np.vstack(out)
