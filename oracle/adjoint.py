"""Transposed solve A^T lam = g and the gradient of a tracking cost (float64).

A^T = B1^T (x) I + B2^T (x) K^T is block *upper* triangular with diagonal block
E^T, so lam follows by backward substitution in time:
    lam_n = E^{-T} (g_n - sum_{k>=1} (c1_k I + c2_k K^T) lam_{n+k}),  n = Nt..1.

Tracking cost (the reduced optimal-control setting of Section 4, with plain
Euclidean sums in place of the L2 norms -- our reading):
    J(U0, f) = 1/2 ||U_Nt - target||^2 + beta/2 * sum_{n=0..Nt} ||f_n||^2
with u = A^{-1} b(U0, f).  Then dJ/du = g = (0, ..., 0, U_Nt - target),
lam = A^{-T} g, and by the chain rule through b:
    dJ/dU0 = (db/dU0)^T lam,   dJ/df = (db/df)^T lam + beta f.

Pins: <A^{-1} b, g> = <b, A^{-T} g> (dot-product test against the forward
stepper); the gradient equals the dense-matrix gradient on tiny inputs and
central finite differences (J is quadratic, so exact up to rounding).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import rhs as rhs_mod
from . import solve as solve_mod
from .operators import spatial_operator, time_columns
from .problem import Problem


def sequential_transpose(p: Problem, g) -> np.ndarray:
    c1, c2 = time_columns(p.scheme, p.dt)
    KT = spatial_operator(p).T.tocsr()
    lu = spla.splu(solve_mod.diagonal_block(p).T.tocsc())
    G = np.asarray(g, dtype=np.float64).reshape(p.nt, p.nspace)
    L = np.zeros_like(G)
    for n in range(p.nt - 1, -1, -1):
        r = G[n].copy()
        for k in range(1, len(c1)):
            m = n + k
            if m >= p.nt:
                continue
            r -= c1[k] * L[m] + c2[k] * (KT @ L[m])
        L[n] = lu.solve(r)
    return L


def tracking_cost(p: Problem, U0, f, target, beta: float, u1=None) -> float:
    b = rhs_mod.build_rhs(p, U0, u1, f)
    u = solve_mod.sequential(p, b)
    d = u[-1] - np.asarray(target, dtype=np.float64).reshape(-1)
    F = np.zeros((p.nt + 1, p.nspace)) if f is None else np.asarray(f).reshape(p.nt + 1, -1)
    return 0.5 * float(d @ d) + 0.5 * beta * float(np.sum(F * F))


def gradient(p: Problem, U0, f, target, beta: float, u1=None):
    """(J, dJ/dU0 [nspace], dJ/df [nt+1][nspace]) via the transposed solve."""
    b = rhs_mod.build_rhs(p, U0, u1, f)
    u = solve_mod.sequential(p, b)
    d = u[-1] - np.asarray(target, dtype=np.float64).reshape(-1)
    g = np.zeros_like(u)
    g[-1] = d
    lam = sequential_transpose(p, g)
    gU0, _gu1, gf = rhs_mod.rhs_transpose(p, lam)
    F = np.zeros((p.nt + 1, p.nspace)) if f is None else np.asarray(f).reshape(p.nt + 1, -1)
    J = 0.5 * float(d @ d) + 0.5 * beta * float(np.sum(F * F))
    return J, gU0, gf + beta * F


def finite_difference(p: Problem, U0, f, target, beta: float, d0, df, h: float = 1e-6) -> float:
    """Central difference (J(p + h d) - J(p - h d)) / (2h) along direction (d0, df)."""
    U0 = np.asarray(U0, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    jp = tracking_cost(p, U0 + h * d0, f + h * df, target, beta)
    jm = tracking_cost(p, U0 - h * d0, f - h * df, target, beta)
    return (jp - jm) / (2.0 * h)
