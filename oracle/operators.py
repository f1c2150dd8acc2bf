"""Spatial and temporal matrices of the all-at-once system (float64).

Spatial operator (method of lines, M = I for finite differences):

* 1D: centred differences for ``-nu u_xx + a u_x``: the diffusion part
  ``(nu/h^2) tridiag(-1, 2, -1)`` plus the advection part
  ``(a/(2h)) tridiag(-1, 0, 1)`` (eq2.2b).  With Dirichlet boundaries the
  periodic corner entries of eq2.2b are absent and h = 1/(n+1); the periodic
  variant keeps them with h = 1/n.
* 2D: the Kronecker sum ``I_y (x) K_x + K_y (x) I_x`` on a grid stored with x
  fastest.
* Wave equation (eq3.1): the negative Laplacian scaled by c^2, i.e. the same
  matrices with zero velocity and nu = c^2.

Time discretisation (uniform step dt): the all-at-once matrix is
``A = B1 (x) I + B2 (x) K`` (eq1.1) where B1, B2 are lower-triangular
Toeplitz matrices given by their first columns:

* theta-method (eq2.5b with constant steps): c1 = (1, -1)/dt,
  c2 = (theta, 1 - theta); backward Euler theta = 1, trapezoidal theta = 1/2.
* implicit leap-frog (eq3.2b): c1 = (1, -2, 1)/dt^2, c2 = (1/2, 0, 1/2).

The alpha-circulant matrices C_j^(alpha) (eq2.11b, eq3.4) wrap the entries
that fall above the diagonal into the top-right corner multiplied by alpha.
Lemma 1: C^(alpha) = V D V^{-1} with D = diag(fft(Gamma c)), Gamma =
diag(alpha^{n/Nt}), n = 0..Nt-1 (numpy's forward-transform sign convention).

Pins (tests/test_oracle_*.py): the assembled alpha-circulant matrices equal
the matrices printed in eq2.11b and eq3.4 (golden fixtures); the eigenvalues
of the assembled C^(alpha) equal the time symbols; the spatial matrices
reproduce manufactured solutions at the expected order.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .problem import Problem

THETA = {"be": 1.0, "tr": 0.5}


def mesh_width(n: int, periodic: bool = False) -> float:
    return 1.0 / n if periodic else 1.0 / (n + 1)


def k1d(n: int, nu: float, a: float, periodic: bool = False) -> sp.csr_matrix:
    """Centred-difference matrix of ``-nu d2/dx2 + a d/dx`` on n points (eq2.2b)."""
    h = mesh_width(n, periodic)
    diff = nu / h ** 2
    adv = a / (2.0 * h)
    lower = np.full(n - 1, -diff - adv)   # coefficient of u_{i-1}
    main = np.full(n, 2.0 * diff)
    upper = np.full(n - 1, -diff + adv)   # coefficient of u_{i+1}
    K = sp.diags([lower, main, upper], [-1, 0, 1], shape=(n, n), format="lil")
    if periodic and n > 2:
        K[0, n - 1] += -diff - adv        # u_{-1} == u_{n-1}
        K[n - 1, 0] += -diff + adv        # u_{n} == u_0
    return K.tocsr()


def spatial_factors(p: Problem):
    """(K_x, K_y) one-dimensional factors; K_y is None in 1D."""
    Kx = k1d(p.nx, p.nu, p.ax, p.periodic)
    Ky = k1d(p.ny, p.nu, p.ay, p.periodic) if p.dim == 2 else None
    return Kx, Ky


def spatial_operator(p: Problem) -> sp.csr_matrix:
    """K acting on a field stored [ny][nx] with x fastest."""
    Kx, Ky = spatial_factors(p)
    if p.dim == 1:
        return Kx
    Ix = sp.identity(p.nx, format="csr")
    Iy = sp.identity(p.ny, format="csr")
    return (sp.kron(Iy, Kx) + sp.kron(Ky, Ix)).tocsr()


def time_columns(scheme: str, dt: float):
    """First columns (c1, c2) of the Toeplitz matrices B1, B2."""
    if scheme in THETA:
        th = THETA[scheme]
        return np.array([1.0, -1.0]) / dt, np.array([th, 1.0 - th])
    if scheme == "lf":
        return np.array([1.0, -2.0, 1.0]) / dt ** 2, np.array([0.5, 0.0, 0.5])
    raise ValueError(f"unknown scheme {scheme!r}")


def toeplitz_lower(c: np.ndarray, nt: int) -> np.ndarray:
    """Dense lower-triangular Toeplitz matrix with first column c (zero padded)."""
    B = np.zeros((nt, nt))
    for k, ck in enumerate(c):
        if k < nt:
            B += ck * np.eye(nt, k=-k)
    return B


def alpha_circulant(c: np.ndarray, nt: int, alpha: float) -> np.ndarray:
    """Dense alpha-circulant matrix built from first column c (eq2.11b, eq3.4).

    Entry (j, k) is c[(j - k) mod nt], multiplied by alpha when k > j.
    """
    col = np.zeros(nt)
    col[: len(c)] = c[:nt]
    C = np.zeros((nt, nt))
    for j in range(nt):
        for k in range(nt):
            v = col[(j - k) % nt]
            C[j, k] = v if k <= j else alpha * v
    return C


def time_matrices(p: Problem):
    c1, c2 = time_columns(p.scheme, p.dt)
    return toeplitz_lower(c1, p.nt), toeplitz_lower(c2, p.nt)


def circulant_time_matrices(p: Problem, alpha: float | None = None):
    a = p.alpha if alpha is None else alpha
    c1, c2 = time_columns(p.scheme, p.dt)
    return alpha_circulant(c1, p.nt, a), alpha_circulant(c2, p.nt, a)


def gamma(nt: int, alpha: float) -> np.ndarray:
    """Diagonal of Gamma_alpha: alpha^(n/Nt), n = 0..Nt-1 (Lemma 1)."""
    return alpha ** (np.arange(nt) / nt)


def time_symbols(p: Problem, alpha: float | None = None):
    """Eigenvalues (lambda_1, lambda_2) of C_1^(alpha), C_2^(alpha): fft(Gamma c) (Lemma 1)."""
    a = p.alpha if alpha is None else alpha
    c1, c2 = time_columns(p.scheme, p.dt)
    g = gamma(p.nt, a)
    col1 = np.zeros(p.nt)
    col2 = np.zeros(p.nt)
    col1[: len(c1)] = c1
    col2[: len(c2)] = c2
    return np.fft.fft(g * col1), np.fft.fft(g * col2)


def all_at_once_sparse(p: Problem) -> sp.csr_matrix:
    """A = B1 (x) I + B2 (x) K assembled (eq1.1); small problems only."""
    B1, B2 = time_matrices(p)
    K = spatial_operator(p)
    I = sp.identity(p.nspace, format="csr")
    return (sp.kron(sp.csr_matrix(B1), I) + sp.kron(sp.csr_matrix(B2), K)).tocsc()


def preconditioner_sparse(p: Problem, alpha: float | None = None) -> sp.csr_matrix:
    """P_alpha = C1 (x) I + C2 (x) K assembled (eq1.2); small problems only."""
    C1, C2 = circulant_time_matrices(p, alpha)
    K = spatial_operator(p)
    I = sp.identity(p.nspace, format="csr")
    return (sp.kron(sp.csr_matrix(C1), I) + sp.kron(sp.csr_matrix(C2), K)).tocsc()


def apply_A(p: Problem, u: np.ndarray) -> np.ndarray:
    """y = A u blockwise: y_n = sum_k (c1_k I + c2_k K) u_{n-k}, u_{m<1} = 0 (eq1.1).

    u has shape [nt][nspace] (or anything reshapeable to it).
    """
    c1, c2 = time_columns(p.scheme, p.dt)
    K = spatial_operator(p)
    U = np.asarray(u, dtype=np.float64).reshape(p.nt, p.nspace)
    Y = np.zeros_like(U)
    for n in range(p.nt):
        for k in range(len(c1)):
            m = n - k
            if m < 0:
                continue
            if c1[k] != 0.0:
                Y[n] += c1[k] * U[m]
            if c2[k] != 0.0:
                Y[n] += c2[k] * (K @ U[m])
    return Y


def apply_AT(p: Problem, v: np.ndarray) -> np.ndarray:
    """y = A^T v blockwise: y_m = sum_k (c1_k I + c2_k K^T) v_{m+k}."""
    c1, c2 = time_columns(p.scheme, p.dt)
    KT = spatial_operator(p).T.tocsr()
    V = np.asarray(v, dtype=np.float64).reshape(p.nt, p.nspace)
    Y = np.zeros_like(V)
    for m in range(p.nt):
        for k in range(len(c1)):
            n = m + k
            if n >= p.nt:
                continue
            if c1[k] != 0.0:
                Y[m] += c1[k] * V[n]
            if c2[k] != 0.0:
                Y[m] += c2[k] * (KT @ V[n])
    return Y


def apply_P(p: Problem, u: np.ndarray, alpha: float | None = None) -> np.ndarray:
    """y = P_alpha u blockwise with the alpha wrap of eq2.11b / eq3.4."""
    a = p.alpha if alpha is None else alpha
    c1, c2 = time_columns(p.scheme, p.dt)
    K = spatial_operator(p)
    U = np.asarray(u, dtype=np.float64).reshape(p.nt, p.nspace)
    Y = np.zeros_like(U)
    for n in range(p.nt):
        for k in range(len(c1)):
            m = n - k
            w = 1.0
            if m < 0:
                m += p.nt
                w = a
            Y[n] += w * (c1[k] * U[m] + c2[k] * (K @ U[m]))
    return Y
