"""ParaDiag-II for the optimal control of the wave equation (Section 4), float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Optimality system (eq2.2): u_tt - Laplacian u - p / gamma = f, u(0) = u0,
u_t(0) = u1; p_tt - Laplacian p + u = g, p(T) = p_t(T) = 0; homogeneous
Dirichlet data; A = -Laplacian (5-point, nu = 1).  Implicit leap-frog in time,
step dt = T / Nt (reading OC2).  The discrete saddle-point system is

  Ahat [u; p] = ([[B1, -dt^2 Ih / gamma], [dt^2 Ic, B1^T]] (x) I
                 + (dt^2 / 2) blkdiag(B2, B2^T) (x) A) [u; p] = [fh; gh]

with B1 = Toeplitz(1, -2, 1) and B2 = Toeplitz(1, 0, 1) (the matrices of eq3.2b
times dt^2 and 2: reading OC1), Ih = diag(1/2, 1, .., 1), Ic = diag(1, .., 1,
1/2).  Unknowns u = (u(t_1) .. u(t_Nt)) and p = (p(t_0) .. p(t_{Nt-1})):
state row n is the leap-frog equation at t_{n-1} and adjoint row m the one at
t_{m+1}; the first state row and the last adjoint row are halved (ghost
values from u_t(0) = u1 and p_t(T) = 0), which is where Ih and Ic come from
(reading OC3).  So fh = dt^2 times the leap-frog right-hand side of the state
equation (the same rows as ``rhs.build_rhs`` for 'lf'), and gh_m = dt^2
g(t_{m+1}), halved in the last row.

The gamma-similarity gives the system solved here, A [sqrt(gamma) u; p] =
[sqrt(gamma) fh; gh] with the coupling blocks -+ dt^2 Ih / sqrt(gamma),
dt^2 Ic / sqrt(gamma).  The preconditioner P replaces B1, B2 by their
circulants C1, C2 (eq3.3: alpha = 1) and Ih, Ic by I.  With P = Pt
(blkdiag(C2, C2^T) (x) I), Pt is block-diagonalised per frequency (Thm the4):
in the Fourier basis the time part of Pt at frequency n is the 2 x 2 matrix

  G_n = [[a_n, -beta conj(q_n)], [beta q_n, a_n]],  a_n = d1_n / d2_n (real),
  q_n = 1 / d2_n, beta = dt^2 / sqrt(gamma),

with d1, d2 the eigenvalues (Fourier symbols) of C1, C2.  Its eigenvalues
are Sigma_{1,2} = a_n +- i beta |q_n| and its eigenvector matrix
W_n = [[1, 1], [-i E_n, i E_n]], E_n = q_n / |q_n|, is sqrt(2) times a
unitary matrix (Cond_2 = 1).  (The paper's printed V in eq4.4b arranges the
phase blocks differently; this W_n is what G_n gives, reading OC4.)  Hence
P^{-1} r: FFT both fields in time; c1 = (R1 + i conj(E) R2)/2, c2 = (R1 - i
conj(E) R2)/2; solve (Sigma_k I + dt^2/2 A) y_k = c_k; S1 = (y1 + y2)/d2,
S2 = i E (y2 - y1)/conj(d2); inverse FFT.  C2 is singular when 4 divides Nt
(d2 = 0 at n = Nt/4): Nt must not be a multiple of 4 (T2A uses Nt = N + 1).

Pins (tests/test_oracle_ocwave.py): the Theorem the4 route equals a sparse
solve with the assembled P; Cond_2(W_n) = 1; the discrete solution converges
at second order to the exact (u, p) = (e^t sin(pi x) sin(pi y),
(t-T)^2 sin(pi x) sin(pi y)) of the paper's test (readings OC1-OC3);
preconditioned GMRES to 1e-7 takes the iteration counts of Table T2A.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operators import alpha_circulant, spatial_operator, toeplitz_lower
from .problem import Problem


def wave_problem(n: int, nt: int, T: float = 2.0) -> Problem:
    """Space-time grid of mesh width 1/n on (0,1)^2 (n-1 interior points per
    direction), nt time steps of T/nt, A = -Laplacian."""
    return Problem(dim=2, nx=n - 1, ny=n - 1, nt=nt, scheme="lf", T=T, nu=1.0)


def time_matrices(nt: int):
    B1 = toeplitz_lower(np.array([1.0, -2.0, 1.0]), nt)
    B2 = toeplitz_lower(np.array([1.0, 0.0, 1.0]), nt)
    Ih = np.ones(nt)
    Ih[0] = 0.5
    Ic = np.ones(nt)
    Ic[-1] = 0.5
    return B1, B2, Ih, Ic


def assembled(p: Problem, gamma: float, circulant: bool = False) -> sp.csc_matrix:
    """The gamma-scaled system matrix (circulant=False) or P (circulant=True)."""
    nt = p.nt
    dt = p.dt
    A = spatial_operator(p)
    I = sp.identity(p.nspace, format="csr")
    if circulant:
        B1 = alpha_circulant(np.array([1.0, -2.0, 1.0]), nt, 1.0)
        B2 = alpha_circulant(np.array([1.0, 0.0, 1.0]), nt, 1.0)
        Ih = Ic = np.ones(nt)
    else:
        B1, B2, Ih, Ic = time_matrices(nt)
    s = dt * dt / np.sqrt(gamma)
    top = sp.hstack([sp.kron(sp.csr_matrix(B1), I) + 0.5 * dt * dt * sp.kron(sp.csr_matrix(B2), A),
                     -s * sp.kron(sp.diags(Ih), I)])
    bot = sp.hstack([s * sp.kron(sp.diags(Ic), I),
                     sp.kron(sp.csr_matrix(B1.T), I) + 0.5 * dt * dt * sp.kron(sp.csr_matrix(B2.T), A)])
    return sp.vstack([top, bot]).tocsc()


def exact_fields(p: Problem):
    """u(t_1..t_Nt), p(t_0..t_{Nt-1}) of the paper's exact solution, [nt][nspace] each."""
    h = 1.0 / (p.nx + 1)
    x = np.arange(1, p.nx + 1) * h
    y = np.arange(1, p.ny + 1) * h
    s = np.outer(np.sin(np.pi * y), np.sin(np.pi * x)).ravel()
    t = np.arange(p.nt + 1) * p.dt
    u = np.exp(t[1:])[:, None] * s[None]
    q = ((t[:-1] - p.T) ** 2)[:, None] * s[None]
    return u, q


def rhs(p: Problem, gamma: float) -> np.ndarray:
    """[sqrt(gamma) fh; gh] for the paper's data (Section 4), readings OC2-OC3."""
    from .rhs import build_rhs
    dt, T = p.dt, p.T
    h = 1.0 / (p.nx + 1)
    x = np.arange(1, p.nx + 1) * h
    y = np.arange(1, p.ny + 1) * h
    s = np.outer(np.sin(np.pi * y), np.sin(np.pi * x)).ravel()
    t = np.arange(p.nt + 1) * dt
    f = (((1 + 2 * np.pi ** 2) * np.exp(t) - (t - T) ** 2 / gamma))[:, None] * s[None]
    g = (np.exp(t) + 2 + 2 * np.pi ** 2 * (t - T) ** 2)[:, None] * s[None]
    fh = dt * dt * build_rhs(p, s, s, f)          # u0 = u1 = sin sin
    gh = dt * dt * g[1:].copy()
    gh[-1] *= 0.5
    return np.concatenate([np.sqrt(gamma) * fh.ravel(), gh.ravel()])


def symbols(nt: int):
    """d1, d2: Fourier symbols of C1, C2 (numpy's forward transform of their first columns)."""
    c1 = np.zeros(nt)
    c1[:3] = [1.0, -2.0, 1.0]
    c2 = np.zeros(nt)
    c2[[0, 2]] = 1.0
    return np.fft.fft(c1), np.fft.fft(c2)


def block_eigen(nt: int, dt: float, gamma: float):
    """(Sigma1, Sigma2, E) per frequency: G_n = W_n diag(Sigma1, Sigma2) W_n^{-1}."""
    d1, d2 = symbols(nt)
    if np.min(np.abs(d2)) < 1e-12:
        raise ValueError("C2 is singular (4 divides Nt)")
    a = (d1 / d2).real
    q = 1.0 / d2
    beta = dt * dt / np.sqrt(gamma)
    return a + 1j * beta * np.abs(q), a - 1j * beta * np.abs(q), q / np.abs(q)


def preconditioner(p: Problem, gamma: float):
    """P^{-1} as a function (Thm the4): time FFTs, 2 x 2 mixing, shifted spatial
    solves (factorised once per frequency), C2^{-1}, inverse FFTs."""
    nt, S = p.nt, p.nspace
    d1, d2 = symbols(nt)
    s1, s2, E = block_eigen(nt, p.dt, gamma)
    A = spatial_operator(p).astype(np.complex128)
    I = sp.identity(S, dtype=np.complex128, format="csc")
    h = 0.5 * p.dt * p.dt
    lu1 = [spla.splu((s1[n] * I + h * A).tocsc()) for n in range(nt)]
    lu2 = [spla.splu((s2[n] * I + h * A).tocsc()) for n in range(nt)]

    def apply(r):
        R = np.asarray(r, dtype=np.float64).reshape(2, nt, S)
        R1 = np.fft.fft(R[0], axis=0)
        R2 = np.fft.fft(R[1], axis=0)
        c1 = 0.5 * (R1 + 1j * np.conj(E)[:, None] * R2)
        c2 = 0.5 * (R1 - 1j * np.conj(E)[:, None] * R2)
        y1 = np.stack([lu1[n].solve(c1[n]) for n in range(nt)])
        y2 = np.stack([lu2[n].solve(c2[n]) for n in range(nt)])
        S1 = (y1 + y2) / d2[:, None]
        S2 = 1j * E[:, None] * (y2 - y1) / np.conj(d2)[:, None]
        return np.stack([np.fft.ifft(S1, axis=0).real, np.fft.ifft(S2, axis=0).real]).reshape(-1)

    return apply


def apply_P_inverse(p: Problem, gamma: float, r) -> np.ndarray:
    """P^{-1} r by Thm the4 (see ``preconditioner``)."""
    return preconditioner(p, gamma)(r)


def gmres(p: Problem, gamma: float, b, tol: float = 1e-7, maxit: int = 60, precond: bool = True):
    """Right-preconditioned GMRES (no restart, zero start, classical Gram-Schmidt
    twice) on the gamma-scaled system; stops when ||b - A x|| <= tol ||b||.
    Returns (x, iterations, residual history)."""
    A = assembled(p, gamma)
    M = preconditioner(p, gamma) if precond else (lambda v: v)
    b = np.asarray(b, dtype=np.float64)
    beta = np.linalg.norm(b)
    V = [b / beta]
    Z = []
    H = np.zeros((maxit + 1, maxit))
    hist = []
    x = np.zeros_like(b)
    for j in range(maxit):
        z = M(V[j])
        Z.append(z)
        w = A @ z
        for _ in range(2):
            for i in range(j + 1):
                hij = V[i] @ w
                H[i, j] += hij
                w = w - hij * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        e1 = np.zeros(j + 2)
        e1[0] = beta
        y = np.linalg.lstsq(H[: j + 2, : j + 1], e1, rcond=None)[0]
        res = np.linalg.norm(e1 - H[: j + 2, : j + 1] @ y) / beta
        hist.append(res)
        if res <= tol or H[j + 1, j] == 0.0:
            x = sum(yi * zi for yi, zi in zip(y, Z))
            return x, j + 1, hist
        V.append(w / H[j + 1, j])
    x = sum(yi * zi for yi, zi in zip(y, Z))
    return x, maxit, hist


def solve(p: Problem, gamma: float, b) -> np.ndarray:
    """Sparse direct solve of the gamma-scaled system."""
    return spla.spsolve(assembled(p, gamma), np.asarray(b, dtype=np.float64))


def unscale(p: Problem, gamma: float, x):
    """(u, p) from the solution of the gamma-scaled system."""
    X = np.asarray(x).reshape(2, p.nt, p.nspace)
    return X[0] / np.sqrt(gamma), X[1]
