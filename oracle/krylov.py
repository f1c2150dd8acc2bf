"""Outer iterations around P_alpha^{-1} (float64 replay of the GPU algorithms).

Krylov variant (the preconditioned system P^{-1} A u = P^{-1} b of Section 1,
solved as in the wave example of Section 3: zero initial guess, stopping on
the relative residual).  Our reading fixes the details the paper leaves open:

* right-preconditioned *flexible* GMRES(m): x = x0 + Z y with z_j = P^{-1} v_j;
* Arnoldi with classical Gram-Schmidt applied twice (CGS2);
* Givens rotations give the residual estimate |g_{j+1}|; a cycle ends when
  the estimate reaches rtol * ||b||, at m steps, or at the iteration limit;
* after each cycle the true residual ||b - A x|| decides convergence, and a
  new cycle starts from it otherwise.

Stationary variant (eq5.1, the same iteration as the waveform relaxation of
eq2.10): u^{k+1} = u^k + P^{-1}(b - A u^k), stopping on the true relative
residual.  Its error contracts by at most alpha/(1-alpha) per step for stable
one-step schemes and leap-frog (Thm the1.2, eq5.4).

Pins: GMRES iteration counts of the wave table T4A; the contraction bound of
the stationary iteration; convergence to the sequential solution.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class SolveInfo:
    converged: bool
    iters: int
    rel_resid: float
    history: list


def _givens(a: float, b: float):
    if b == 0.0:
        return 1.0, 0.0
    r = math.hypot(a, b)
    return a / r, b / r


def fgmres(matvec, precond, b, rtol: float, restart: int, max_iter: int, x0=None):
    """Right-preconditioned flexible GMRES(m) with CGS2; returns (x, SolveInfo)."""
    b = np.asarray(b, dtype=np.float64).ravel()
    bnorm = float(np.linalg.norm(b))
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64).ravel().copy()
    if bnorm == 0.0:
        return x * 0.0, SolveInfo(True, 0, 0.0, [0.0])
    r = b - matvec(x) if x0 is not None else b.copy()
    beta = float(np.linalg.norm(r))
    hist = [beta / bnorm]
    iters = 0
    m = restart
    while True:
        if beta / bnorm <= rtol:
            return x, SolveInfo(True, iters, beta / bnorm, hist)
        if iters >= max_iter:
            return x, SolveInfo(False, iters, beta / bnorm, hist)
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        g = np.zeros(m + 1)
        g[0] = beta
        cs = np.zeros(m)
        sn = np.zeros(m)
        k = 0
        for j in range(m):
            z = precond(V[j])
            Z.append(z)
            w = matvec(z)
            Vm = np.stack(V)
            h = Vm @ w
            w = w - Vm.T @ h
            h2 = Vm @ w
            w = w - Vm.T @ h2
            h = h + h2
            hn = float(np.linalg.norm(w))
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            iters += 1
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            est = abs(g[j + 1]) / bnorm
            hist.append(est)
            k = j + 1
            if hn == 0.0 or est <= rtol or iters >= max_iter:
                break
            V.append(w / hn)
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        for i in range(k):
            x = x + y[i] * Z[i]
        r = b - matvec(x)
        beta = float(np.linalg.norm(r))
        hist.append(beta / bnorm)


def stationary(matvec, precond, b, rtol: float, max_iter: int, x0=None):
    """u <- u + P^{-1}(b - A u) until ||b - A u|| <= rtol ||b|| (eq5.1)."""
    b = np.asarray(b, dtype=np.float64).ravel()
    bnorm = float(np.linalg.norm(b))
    u = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64).ravel().copy()
    r = b - matvec(u)
    res = float(np.linalg.norm(r)) / bnorm
    hist = [res]
    iters = 0
    while res > rtol and iters < max_iter:
        u = u + precond(r)
        iters += 1
        r = b - matvec(u)
        res = float(np.linalg.norm(r)) / bnorm
        hist.append(res)
    return u, SolveInfo(res <= rtol, iters, res, hist)
