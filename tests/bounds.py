"""Condition-number bounds of the all-at-once matrix A = B1 (x) I + B2 (x) K.

A solve that stops at relative residual r has relative 2-norm error at most
kappa_2(A) r.  The bounds below follow from the structure of A alone (no
oracle, no library):

* ||A||_2 <= ||B1||_2 + ||B2||_2 ||K||_2 with ||B||_2 <= sum |c_k| for a
  lower-triangular Toeplitz B with first column c, and ||K||_2 <= sum over
  directions of 4 nu / h^2 (the row and column sums of a centred factor with
  cell Peclet number below one).
* A^{-1} is block lower-triangular Toeplitz; ||A^{-1}||_2 is at most the sum of
  the norms of its blocks.  theta-method: the symmetric part of K is positive
  semi-definite, so ||E^{-1}||_2 <= dt for E = I/dt + theta K and the step
  operator is a contraction: ||A^{-1}||_2 <= Nt dt = T.  Implicit leap-frog
  with symmetric K: in K's eigenbasis every mode mu obeys the scalar recursion
  whose impulse response is (dt^2 / c) U_k(1/c), c = 1 + dt^2 mu / 2, U_k the
  Chebyshev polynomial of the second kind; ||A^{-1}||_2 is at most the largest
  sum of |response| over the eigenvalues of K.
"""

import numpy as np


def _knorm(cfg):
    hx = 1.0 / (cfg.nx + 1)
    n = 4.0 * cfg.nu / hx ** 2
    if cfg.dim == 2:
        hy = 1.0 / (cfg.ny + 1)
        n += 4.0 * cfg.nu / hy ** 2
    return n


def _lf_inverse_norm(cfg):
    dt = cfg.dt
    lam = lambda n: (4.0 / (1.0 / (n + 1)) ** 2) * np.sin(np.arange(1, n + 1) * np.pi / (2 * (n + 1))) ** 2
    lx = lam(cfg.nx)
    ly = lam(cfg.ny) if cfg.dim == 2 else np.zeros(1)
    mu = cfg.nu * (lx[:, None] + ly[None, :]).ravel()
    best = 0.0
    k = np.arange(cfg.nt)
    for chunk in np.array_split(mu, max(1, mu.size // 2048)):
        c = 1.0 + 0.5 * dt * dt * chunk
        th = np.arccos(1.0 / c)
        resp = np.abs(np.sin((k[None, :] + 1) * th[:, None]) / np.sin(th)[:, None])
        best = max(best, float(np.max(dt * dt / c * resp.sum(axis=1))))
    return best


def kappa2_bound(cfg):
    """Upper bound of kappa_2(A) for a workload (theta-method or symmetric leap-frog)."""
    K = _knorm(cfg)
    if cfg.scheme in ("be", "tr"):
        return cfg.T * (2.0 / cfg.dt + K)
    if cfg.scheme == "lf":
        if cfg.ax != 0.0 or cfg.ay != 0.0:
            raise ValueError("the leap-frog bound needs a symmetric K")
        return (4.0 / cfg.dt ** 2 + K) * _lf_inverse_norm(cfg)
    raise ValueError(cfg.scheme)


def line_condition(params):
    """2-norm condition number of the worst Step-(b) system of a problem whose
    spatial operator is symmetric (sine basis in x, y lines): in the joint sine
    eigenbasis every system (lambda1_n I + lambda2_n K) is diagonal with
    entries lambda1_n + lambda2_n (t_k + mu_j), so its condition is the ratio
    of the largest to the smallest modulus over j, maximised over the
    frequencies n and x-modes k.  A backward-stable line solve has a forward
    error of order u times this number."""
    from oracle import Problem, operators as ops
    p = Problem.from_kwargs(**params)
    if params.get("ax", 0.0) != 0.0 or params.get("ay", 0.0) != 0.0:
        raise ValueError("line_condition needs a symmetric spatial operator")
    lam1, lam2 = ops.time_symbols(p)

    def eig(n):
        h = 1.0 / (n + 1)
        return 4.0 * params["nu"] / h ** 2 * np.sin(np.arange(1, n + 1) * np.pi / (2 * (n + 1))) ** 2

    tx = eig(params["nx"]) if params["dim"] == 2 else np.zeros(1)
    my = eig(params["ny"] if params["dim"] == 2 else params["nx"])
    worst = 0.0
    for a, b in zip(lam1, lam2):
        ev = np.abs(a + b * (tx[:, None] + my[None, :]))
        worst = max(worst, float(np.max(ev.max(axis=1) / ev.min(axis=1))))
    return worst
