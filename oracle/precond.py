"""z = P_alpha^{-1} r two independent ways (float64).

P_alpha = C1^(alpha) (x) I + C2^(alpha) (x) K (eq1.2) is an exactly defined
linear map, so its oracle is its definition:

* ``assembled``: sparse LU of the assembled block alpha-circulant matrix.
* ``three_steps``: the factorisation of Lemma 1 applied as in eq1.3 / eq2.12,
  with full complex transforms (no Hermitian shortcut):
    Step-(a)  S1 = fft_t(Gamma r)                 (per spatial dof, along time)
    Step-(b)  S2_n = (lambda1_n I + lambda2_n K)^{-1} S1_n, n = 0..Nt-1
    Step-(c)  z = Gamma^{-1} ifft_t(S2)
  with lambda_j = fft(Gamma c_j) and numpy's transform conventions (forward
  sign e^{-2 pi i}, 1/Nt on the inverse).  The paper's Lemma 1 writes the
  unitary Fourier matrix with the opposite sign; any consistent pair gives
  the same P_alpha^{-1}.

Pins: the two routes agree on small inputs; the spectrum of P^{-1} A equals
the closed forms (Thm the3.1 for leap-frog, 1/(1 - alpha r^Nt) for one-step
schemes); see tests/test_oracle_precond.py.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operators import gamma, preconditioner_sparse, spatial_operator, time_symbols
from .problem import Problem


def assembled(p: Problem, r, alpha: float | None = None) -> np.ndarray:
    P = preconditioner_sparse(p, alpha)
    z = spla.spsolve(P, np.asarray(r, dtype=np.float64).reshape(-1))
    return z.reshape(p.nt, p.nspace)


def frequency_solve(p: Problem, n: int, s1: np.ndarray, alpha: float | None = None,
                    K=None) -> np.ndarray:
    """Step-(b) at one frequency n: (lambda1_n I + lambda2_n K)^{-1} s1 (eq2.12).

    K (the complex spatial matrix) may be passed in to skip its assembly."""
    lam1, lam2 = time_symbols(p, alpha)
    if K is None:
        K = spatial_operator(p).astype(np.complex128)
    I = sp.identity(p.nspace, dtype=np.complex128)
    M = (lam1[n] * I + lam2[n] * K).tocsc()
    return spla.splu(M).solve(np.asarray(s1, dtype=np.complex128))


def spectrum_solve(p: Problem, S1: np.ndarray, alpha: float | None = None,
                   freqs=None) -> np.ndarray:
    """Step-(b) on the given frequencies: S2_n = (lambda1_n I + lambda2_n K)^{-1} S1_n."""
    K = spatial_operator(p).astype(np.complex128)
    S2 = np.zeros_like(S1, dtype=np.complex128)
    idx = range(p.nt) if freqs is None else freqs
    for n in idx:
        S2[n] = frequency_solve(p, n, S1[n], alpha, K)
    return S2


def three_steps(p: Problem, r, alpha: float | None = None) -> np.ndarray:
    a = p.alpha if alpha is None else alpha
    R = np.asarray(r, dtype=np.float64).reshape(p.nt, p.nspace)
    g = gamma(p.nt, a)
    S1 = np.fft.fft(g[:, None] * R, axis=0)                 # Step-(a)
    S2 = spectrum_solve(p, S1, a)                           # Step-(b)
    z = (1.0 / g)[:, None] * np.fft.ifft(S2, axis=0)        # Step-(c)
    return z.real


def apply(p: Problem, r, alpha: float | None = None) -> np.ndarray:
    """Default oracle route: the three steps (feasible at every size)."""
    return three_steps(p, r, alpha)
