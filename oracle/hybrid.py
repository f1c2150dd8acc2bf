"""ParaDiag-I with the hybrid time discretisation (Section 2.1.2), float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Scheme (neq2.9a): explicit midpoint for the first Nt - 1 steps, backward Euler
for the last one, on U' + K U = f:

    (U_{n+1} - U_{n-1}) / (2 dt) + K U_n = f(t_n),   n = 1 .. Nt-1
    (U_Nt - U_{Nt-1}) / dt + K U_Nt = f(t_Nt)

With u = (U_1 .. U_Nt) the all-at-once system is (B (x) I + I (x) K) u = b
(neq2.9b), B the tridiagonal matrix of neq2.9c and b_1 = U_0/(2 dt) + f_1,
b_n = f_n (f_n = f(t_n); the paper prints b for f = 0, the source term is
reading H1).

Second-order problems U'' + K U = f, U(0) = U_0, U'(0) = V_0 (neq2.14a): the
scheme applied to the first-order system neq2.14b with the velocity
eliminated at the discrete level gives (B^2 (x) I + I (x) K) u = b2, with
B^2 the matrix printed in neq2.15 and (reading H2, derived here: V = B u -
b_U from the displacement rows, substituted into the velocity rows)

    b2_1 = V_0 / (2 dt) + f_1,   b2_2 = f_2 - U_0 / (4 dt^2),   b2_n = f_n (n >= 3).

Eigendecomposition (Thm thmCondU): B = V D V^{-1}; the eigenvalues are
lambda_n = i x_n / dt (the theorem's "i dt x_n" is read as i x_n / dt, reading
H3; that is what B v = lambda v gives with the stated eigenvectors), where x_n
are the Nt roots of U_{Nt-1}(x) - i T_Nt(x) (e-value; T, U the Chebyshev
polynomials of the first and second kind) and v_{n,l} = i^l U_l(x_n)
(e-vector, Vformula).

Functions and how each is pinned (tests/test_oracle_hybrid.py):

* ``time_matrix``, ``time_matrix_2nd``: neq2.9c, and B @ B; pinned against the
  matrix printed in neq2.15 (golden fixture).
* ``chebyshev_roots``: Newton's iteration on (e-value), started from the
  eigenvalues of the assembled B (numpy) times dt / i.  Pinned: the roots
  make B V = V D hold with V of Vformula; they agree with numpy's eigenvalues;
  Cond_2(V) grows no faster than Nt^2 (condUorder).
* ``rhs``: readings H1, H2; pinned by the uniform second order of the scheme
  (manufactured solutions) and, for H2, by the errors of Table Ex2Tab1.
* ``reference_solve``: u = A^{-1} b by a sparse LU of the assembled
  all-at-once matrix (the plain definition; small sizes).
* ``reference_solve_sine``: the same for a symmetric K (Dirichlet Laplacian
  scaled by nu): in the sine eigenbasis of K the system splits into one
  banded Nt x Nt system (B + mu I or B^2 + mu I) per spatial mode, solved by
  LAPACK's banded solver.  Pinned against ``reference_solve``; with it the
  errors of Table Ex2Tab1 are reproduced at Nt = 4 .. 512 on the paper's
  511 x 511 grid (Nt = 2 is not: 1.07e-2 against 9.19e-3 printed, reading H4).
* ``direct_solve``: the method itself, the three steps of eq1.3 with V:
  S1 = V^{-1} b (np.linalg.solve), S2_n = (d_n I + K)^{-1} S1_n with d_n =
  lambda_n (first order) or lambda_n^2 (second order), u = V S2.  Pinned
  against ``reference_solve`` to within Cond_2(V) times the unit roundoff.
* ``apply_A``: y = A u blockwise.
"""

from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operators import spatial_operator
from .problem import Problem


def time_matrix(nt: int, dt: float) -> np.ndarray:
    """B of neq2.9c: rows n = 1..Nt-1 are (-1/2, 0, 1/2)/dt, the last row (-1, 1)/dt."""
    if nt < 2:
        raise ValueError("the hybrid scheme needs nt >= 2")
    B = np.zeros((nt, nt))
    for r in range(nt - 1):
        if r > 0:
            B[r, r - 1] = -0.5
        B[r, r + 1] = 0.5
    B[nt - 1, nt - 2] = -1.0
    B[nt - 1, nt - 1] = 1.0
    return B / dt


def time_matrix_2nd(nt: int, dt: float) -> np.ndarray:
    """B_2nd = B^2 (neq2.15): the time matrix of the second-order problem."""
    B = time_matrix(nt, dt)
    return B @ B


def _order(p: Problem) -> int:
    if p.scheme == "hyb":
        return 1
    if p.scheme == "hyb2":
        return 2
    raise ValueError(f"not a hybrid scheme: {p.scheme!r}")


def _time(p: Problem) -> np.ndarray:
    return time_matrix(p.nt, p.dt) if _order(p) == 1 else time_matrix_2nd(p.nt, p.dt)


def rhs(p: Problem, U0, V0=None, f=None) -> np.ndarray:
    """All-at-once right-hand side [nt][nspace] (readings H1, H2).

    f, when given, holds f(t_0) .. f(t_Nt) ([nt+1][nspace]); f(t_0) is unused.
    V0 (the initial velocity) is used by the second-order form only."""
    dt = p.dt
    b = np.zeros((p.nt, p.nspace))
    U0 = np.asarray(U0, dtype=np.float64).reshape(p.nspace)
    if f is not None:
        b += np.asarray(f, dtype=np.float64).reshape(p.nt + 1, p.nspace)[1:]
    if _order(p) == 1:
        b[0] += U0 / (2.0 * dt)
    else:
        if V0 is not None:
            b[0] += np.asarray(V0, dtype=np.float64).reshape(p.nspace) / (2.0 * dt)
        b[1] -= U0 / (4.0 * dt * dt)
    return b


def apply_A(p: Problem, u) -> np.ndarray:
    """y = (B (x) I + I (x) K) u, or with B^2 for the second-order form."""
    Bt = _time(p)
    K = spatial_operator(p)
    U = np.asarray(u, dtype=np.float64).reshape(p.nt, p.nspace)
    return Bt @ U + (K @ U.T).T


def assembled(p: Problem) -> sp.csc_matrix:
    Bt = sp.csr_matrix(_time(p))
    K = spatial_operator(p)
    return (sp.kron(Bt, sp.identity(p.nspace)) + sp.kron(sp.identity(p.nt), K)).tocsc()


def reference_solve(p: Problem, b) -> np.ndarray:
    """u = A^{-1} b by a sparse direct solve of the assembled system."""
    x = spla.spsolve(assembled(p), np.asarray(b, dtype=np.float64).reshape(-1))
    return x.reshape(p.nt, p.nspace)


def _sine_eigenvalues(n: int, nu: float) -> np.ndarray:
    h = 1.0 / (n + 1)
    return 4.0 * nu / h ** 2 * np.sin(np.arange(1, n + 1) * np.pi / (2 * (n + 1))) ** 2


def reference_solve_sine(p: Problem, b) -> np.ndarray:
    """u = A^{-1} b for a symmetric K = nu (-Laplacian), Dirichlet, by the
    sine eigenbasis of K and one banded time solve per spatial mode."""
    if p.ax != 0.0 or p.ay != 0.0 or p.periodic:
        raise ValueError("reference_solve_sine needs the Dirichlet Laplacian")
    Bt = _time(p)
    bw = 1 if _order(p) == 1 else 2
    # banded storage of the time matrix (LAPACK's (l, u) form)
    ab0 = np.zeros((2 * bw + 1, p.nt))
    for d in range(-bw, bw + 1):
        diag = np.diagonal(Bt, offset=d)
        if d >= 0:
            ab0[bw - d, d:] = diag
        else:
            ab0[bw - d, :d] = diag
    shape = (p.nt, p.ny, p.nx) if p.dim == 2 else (p.nt, p.nx)
    axes = (1, 2) if p.dim == 2 else (1,)
    bh = sfft.dstn(np.asarray(b, dtype=np.float64).reshape(shape), type=1, axes=axes, norm="ortho")
    mu = _sine_eigenvalues(p.nx, p.nu)
    if p.dim == 2:
        mu = (_sine_eigenvalues(p.ny, p.nu)[:, None] + mu[None, :]).ravel()
    bh = bh.reshape(p.nt, -1)
    uh = np.empty_like(bh)
    for j in range(mu.size):
        ab = ab0.copy()
        ab[bw] += mu[j]
        uh[:, j] = sla.solve_banded((bw, bw), ab, bh[:, j], check_finite=False)
    u = sfft.idstn(uh.reshape(shape), type=1, axes=axes, norm="ortho")
    return u.reshape(p.nt, p.nspace)


def _cheb_pair(x: np.ndarray, nt: int):
    """U_{nt-1}(x), T_nt(x) and their derivatives by the three-term recurrences (nt >= 2)."""
    T0, T1 = np.ones_like(x), x.copy()
    dT0, dT1 = np.zeros_like(x), np.ones_like(x)
    for _ in range(2, nt + 1):
        T0, T1, dT0, dT1 = T1, 2 * x * T1 - T0, dT1, 2 * T1 + 2 * x * dT1 - dT0
    U0, U1 = np.ones_like(x), 2 * x
    dU0, dU1 = np.zeros_like(x), 2 * np.ones_like(x)
    for _ in range(2, nt):
        U0, U1, dU0, dU1 = U1, 2 * x * U1 - U0, dU1, 2 * U1 + 2 * x * dU1 - dU0
    return U1, dU1, T1, dT1


def chebyshev_roots(nt: int, iters: int = 8) -> np.ndarray:
    """The nt roots of U_{nt-1}(x) - i T_nt(x) (e-value) by Newton's iteration,
    started from dt/i times numpy's eigenvalues of the assembled B."""
    x = np.linalg.eigvals(time_matrix(nt, 1.0)) / 1j
    for _ in range(iters):
        U, dU, T, dT = _cheb_pair(x, nt)
        step = (U - 1j * T) / (dU - 1j * dT)
        x = x - step
    return x


def eigenvectors(x: np.ndarray) -> np.ndarray:
    """V of Vformula: column n is v_{n,l} = i^l U_l(x_n), l = 0..nt-1."""
    nt = x.size
    U = np.zeros((nt, nt), dtype=np.complex128)
    U[0] = 1.0
    if nt > 1:
        U[1] = 2.0 * x
    for l in range(2, nt):
        U[l] = 2.0 * x * U[l - 1] - U[l - 2]
    return (1j ** np.arange(nt))[:, None] * U


def eigendecomposition(nt: int, dt: float):
    """(lambda, V) with B = V diag(lambda) V^{-1} (Thm thmCondU)."""
    x = chebyshev_roots(nt)
    return 1j * x / dt, eigenvectors(x)


def direct_solve(p: Problem, b) -> np.ndarray:
    """ParaDiag-I: u = (V (x) I)(D (x) I + I (x) K)^{-1}(V^{-1} (x) I) b, the
    three steps of eq1.3 with the eigendecomposition of B (or of B^2 = V D^2
    V^{-1} for the second-order form, neq2.15)."""
    lam, V = eigendecomposition(p.nt, p.dt)
    d = lam if _order(p) == 1 else lam ** 2
    R = np.asarray(b, dtype=np.float64).reshape(p.nt, p.nspace)
    S1 = np.linalg.solve(V, R.astype(np.complex128))             # Step-(a)
    K = spatial_operator(p).astype(np.complex128)
    I = sp.identity(p.nspace, dtype=np.complex128, format="csc")
    S2 = np.empty_like(S1)
    for n in range(p.nt):                                        # Step-(b)
        S2[n] = spla.splu((d[n] * I + K).tocsc()).solve(S1[n])
    return (V @ S2).real                                         # Step-(c)
