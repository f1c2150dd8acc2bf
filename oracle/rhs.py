"""All-at-once right-hand side b(U0, u1, f) and its transpose (float64).

theta-method (eq2.4 with uniform step, all-at-once form eq2.5): row n of
A u = b reads (U_n - U_{n-1})/dt + K(theta U_n + (1-theta) U_{n-1}) =
theta f_n + (1-theta) f_{n-1}, so the known U_0 moves to the first row:

    b_1 = (I/dt - (1-theta) K) U_0 + theta f_1 + (1-theta) f_0
    b_n = theta f_n + (1-theta) f_{n-1},   n = 2..Nt.

(The paper prints b only for f = 0: b = (b_1, 0, ..., 0) with
b_1 = (I/dt - (1-theta) A) U_0.  The source weighting is our reading.)

implicit leap-frog (eq3.2): row n >= 3 is the scheme centred at t_{n-1},
(U_n - 2U_{n-1} + U_{n-2})/dt^2 + K (U_n + U_{n-2})/2 = f_{n-1}.  Row 2
moves U_0 to the right; row 1 is half the scheme at t_0 with the ghost value
U_{-1} = U_1 - 2 dt u_1 (central difference of the initial velocity u_1):

    b_1 = f_0/2 + U_0/dt^2 + u_1/dt + (dt/2) K u_1
    b_2 = f_1 - U_0/dt^2 - (1/2) K U_0
    b_n = f_{n-1},  n = 3..Nt.

Source f is sampled at the Nt+1 time levels t_0..t_Nt, shape [nt+1][nspace].

Pins: manufactured solutions converge at the order of the scheme
(tests/test_oracle_solve.py); with K = 0 every scheme reduces to a quadrature
of the source with a closed-form discrete solution, which separates f_n from
f_{n-1} in the backward Euler row and fixes the two leap-frog start rows
(tests/test_oracle_rhs.py); the transpose passes the dot-product identity
(tests/test_oracle_adjoint.py).
"""

from __future__ import annotations

import numpy as np

from .operators import THETA, spatial_operator
from .problem import Problem


def build_rhs(p: Problem, U0, u1=None, f=None) -> np.ndarray:
    """b with shape [nt][nspace]."""
    S, nt, dt = p.nspace, p.nt, p.dt
    K = spatial_operator(p)
    U0 = np.asarray(U0, dtype=np.float64).reshape(S)
    F = None if f is None else np.asarray(f, dtype=np.float64).reshape(nt + 1, S)
    b = np.zeros((nt, S))
    if p.scheme in THETA:
        th = THETA[p.scheme]
        b[0] = U0 / dt - (1.0 - th) * (K @ U0)
        if F is not None:
            b += th * F[1:] + (1.0 - th) * F[:-1]
        return b
    if p.scheme == "lf":
        v = np.zeros(S) if u1 is None else np.asarray(u1, dtype=np.float64).reshape(S)
        b[0] = U0 / dt ** 2 + v / dt + 0.5 * dt * (K @ v)
        if nt > 1:
            b[1] = -U0 / dt ** 2 - 0.5 * (K @ U0)
        if F is not None:
            b[0] += 0.5 * F[0]
            b[1:] += F[1:nt]
        return b
    raise ValueError(p.scheme)


def rhs_transpose(p: Problem, lam) -> tuple:
    """Transpose of the linear map (U0, u1, f) -> b, applied to lam [nt][nspace].

    Returns (g_U0 [nspace], g_u1 [nspace], g_f [nt+1][nspace]).
    """
    S, nt, dt = p.nspace, p.nt, p.dt
    KT = spatial_operator(p).T.tocsr()
    L = np.asarray(lam, dtype=np.float64).reshape(nt, S)
    gf = np.zeros((nt + 1, S))
    if p.scheme in THETA:
        th = THETA[p.scheme]
        gU0 = L[0] / dt - (1.0 - th) * (KT @ L[0])
        gu1 = np.zeros(S)
        gf[1:] += th * L
        gf[:-1] += (1.0 - th) * L
        return gU0, gu1, gf
    if p.scheme == "lf":
        gU0 = L[0] / dt ** 2
        gu1 = L[0] / dt + 0.5 * dt * (KT @ L[0])
        if nt > 1:
            gU0 = gU0 - L[1] / dt ** 2 - 0.5 * (KT @ L[1])
        gf[0] = 0.5 * L[0]
        gf[1:nt] += L[1:]
        return gU0, gu1, gf
    raise ValueError(p.scheme)
