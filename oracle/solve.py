"""The solution u = A^{-1} b three independent ways (float64).

A = B1 (x) I + B2 (x) K (eq1.1) is block lower triangular with the constant
diagonal block E = c1_0 I + c2_0 K, so u is classical time stepping: one
sparse LU of E, then U_n = E^{-1} (b_n - sum_{k>=1} (c1_k I + c2_k K) U_{n-k})
for n = 1..Nt.  This is the primary reference (``sequential``).

``all_at_once`` solves the assembled sparse Kronecker system and ``dense``
the dense one; on small inputs the three agree to rounding, which pins the
block structure (tests/test_oracle_solve.py).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operators import (all_at_once_sparse, spatial_operator, time_columns,
                        time_matrices)
from .problem import Problem


def diagonal_block(p: Problem) -> sp.csc_matrix:
    c1, c2 = time_columns(p.scheme, p.dt)
    K = spatial_operator(p)
    return (c1[0] * sp.identity(p.nspace) + c2[0] * K).tocsc()


def sequential(p: Problem, b) -> np.ndarray:
    """Time stepping: u with shape [nt][nspace]."""
    c1, c2 = time_columns(p.scheme, p.dt)
    K = spatial_operator(p)
    lu = spla.splu(diagonal_block(p))
    B = np.asarray(b, dtype=np.float64).reshape(p.nt, p.nspace)
    U = np.zeros_like(B)
    for n in range(p.nt):
        r = B[n].copy()
        for k in range(1, len(c1)):
            m = n - k
            if m < 0:
                continue
            r -= c1[k] * U[m] + c2[k] * (K @ U[m])
        U[n] = lu.solve(r)
    return U


def all_at_once(p: Problem, b) -> np.ndarray:
    """Sparse direct solve of the assembled all-at-once system."""
    A = all_at_once_sparse(p)
    x = spla.spsolve(A, np.asarray(b, dtype=np.float64).reshape(-1))
    return x.reshape(p.nt, p.nspace)


def dense(p: Problem, b) -> np.ndarray:
    """Dense Kronecker solve (tiny problems)."""
    B1, B2 = time_matrices(p)
    K = spatial_operator(p).toarray()
    A = np.kron(B1, np.eye(p.nspace)) + np.kron(B2, K)
    x = sla.solve(A, np.asarray(b, dtype=np.float64).reshape(-1))
    return x.reshape(p.nt, p.nspace)


def relative_residual(p: Problem, u, b) -> float:
    from .operators import apply_A
    B = np.asarray(b, dtype=np.float64).reshape(p.nt, p.nspace)
    r = B - apply_A(p, u)
    return float(np.linalg.norm(r) / np.linalg.norm(B))
