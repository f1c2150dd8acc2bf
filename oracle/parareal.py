"""The ParaDiag-II parareal variant (Section 2.2.2, eq2.15, Thm the1.3), float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Problem: U' + K U = 0 on (0, T], U(0) = U0, K the spatial operator of the
Problem (``operators.spatial_operator``); Nt coarse intervals of length
dT = T / Nt, each split into J fine steps of dt = dT / J.

* Fine propagator F: J backward Euler steps of size dt (the first of the
  paper's choices of F; L-stable, as Thm the1.3 asks).
* Coarse propagator G: one backward Euler step of size dT.
* Classical parareal (eq2.15): U^k_{n+1} = F(U^{k-1}_n) + G(U^k_n) - G(U^{k-1}_n),
  with U^k_0 = U0 and a sequential coarse-grid correction.
* ParaDiag-II parareal: the coarse-grid correction is applied to the slightly
  wrong problem U(0) = alpha U(T), which makes it the alpha-circulant backward
  Euler system (C1^(alpha) (x) I + I (x) K) u^k = b^k, with
      b^k_1 = (I/dT + K) Ut_1 - alpha U^{k-1}_Nt / dT,
      b^k_n = (I/dT + K) Ut_n - U^{k-1}_{n-1} / dT,   n >= 2,
  and Ut_{n+1} = F(U^{k-1}_n), U^{k-1}_0 = U0.  That matrix is P_alpha of the
  backward Euler scheme on the coarse grid, so u^k = P_alpha^{-1} b^k is
  computed by the oracle's preconditioner (``precond.three_steps``, pinned
  elsewhere); the fixed point of the iteration is the fine solution.

Pins (tests/test_oracle_parareal.py): the classical iteration reproduces the
fine solution exactly on the first k intervals after k iterations (the finite
termination of parareal); both iterations converge to the fine solution; the
ParaDiag-II variant contracts like the classical one for small alpha and
slower for alpha near 1 (Thm the1.3, alpha* about 0.3; the paper's Figure 1.5
setting converges as fast as classical parareal for alpha <= 1/5).
"""

from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import precond
from .operators import spatial_operator
from .problem import Problem


def coarse_problem(p: Problem, alpha: float) -> Problem:
    """The backward Euler problem on the coarse grid, with the given alpha."""
    return dataclasses.replace(p, scheme="be", alpha=alpha)


def _be_solver(p: Problem, step: float):
    K = spatial_operator(p)
    lu = spla.splu((sp.identity(p.nspace) + step * K).tocsc())
    return lu.solve


def fine_propagate(p: Problem, J: int, U: np.ndarray) -> np.ndarray:
    """F applied to every row of U ([m][nspace]): J backward Euler steps of dT/J."""
    solve = _be_solver(p, p.dt / J)
    out = np.array(U, dtype=np.float64, copy=True).reshape(-1, p.nspace)
    for r in range(out.shape[0]):
        x = out[r]
        for _ in range(J):
            x = solve(x)
        out[r] = x
    return out


def coarse_propagate(p: Problem, U: np.ndarray) -> np.ndarray:
    """G applied to every row of U: one backward Euler step of dT."""
    solve = _be_solver(p, p.dt)
    out = np.array(U, dtype=np.float64, copy=True).reshape(-1, p.nspace)
    for r in range(out.shape[0]):
        out[r] = solve(out[r])
    return out


def fine_solution(p: Problem, J: int, U0) -> np.ndarray:
    """Sequential fine propagation: U_n at the coarse points t_1 .. t_Nt."""
    U = np.zeros((p.nt, p.nspace))
    x = np.asarray(U0, dtype=np.float64).reshape(p.nspace)
    for n in range(p.nt):
        x = fine_propagate(p, J, x[None])[0]
        U[n] = x
    return U


def classical(p: Problem, J: int, U0, iters: int, u_init=None):
    """Classical parareal; returns the iterates u^1 .. u^iters ([nt][nspace] each)."""
    U0 = np.asarray(U0, dtype=np.float64).reshape(p.nspace)
    u = np.zeros((p.nt, p.nspace)) if u_init is None else np.array(u_init, dtype=np.float64).reshape(p.nt, -1)
    out = []
    for _ in range(iters):
        prev = np.vstack([U0[None], u[:-1]])               # U^{k-1}_0 .. U^{k-1}_{Nt-1}
        corr = fine_propagate(p, J, prev) - coarse_propagate(p, prev)
        new = np.zeros_like(u)
        x = U0
        for n in range(p.nt):                              # sequential coarse-grid correction
            x = coarse_propagate(p, x[None])[0] + corr[n]
            new[n] = x
        u = new
        out.append(u.copy())
    return out


def paradiag_rhs(p: Problem, J: int, U0, u_prev, alpha: float) -> np.ndarray:
    """b^k of the alpha-periodic coarse-grid correction from the iterate u^{k-1}."""
    K = spatial_operator(p)
    dT = p.dt
    U0 = np.asarray(U0, dtype=np.float64).reshape(p.nspace)
    u_prev = np.asarray(u_prev, dtype=np.float64).reshape(p.nt, p.nspace)
    prev = np.vstack([U0[None], u_prev[:-1]])
    Ut = fine_propagate(p, J, prev)
    b = Ut / dT + (K @ Ut.T).T
    b[0] -= alpha * u_prev[-1] / dT
    b[1:] -= u_prev[:-1] / dT
    return b


def paradiag_ii(p: Problem, J: int, U0, alpha: float, iters: int, u_init=None):
    """ParaDiag-II parareal; returns the iterates u^1 .. u^iters."""
    pc = coarse_problem(p, alpha)
    u = np.zeros((p.nt, p.nspace)) if u_init is None else np.array(u_init, dtype=np.float64).reshape(p.nt, -1)
    out = []
    for _ in range(iters):
        b = paradiag_rhs(p, J, U0, u, alpha)
        u = precond.three_steps(pc, b)
        out.append(u.copy())
    return out
