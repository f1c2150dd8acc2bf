"""Seeded input fields evaluated at interior grid points.

Grid: ``n`` interior points per direction on [0, 1] with spacing h = 1/(n+1),
points x_j = j*h, j = 1..n.  Arrays are float64 with x fastest:
``[ny][nx]`` for a spatial field and ``[nt+1][ny][nx]`` for a source sampled
at the time levels t_0 .. t_nt.  Every generator draws from
``numpy.random.default_rng(seed)`` so the same call always returns the same
numbers on every machine.
"""

from __future__ import annotations

import numpy as np

from .configs import Config


def _grid(n: int) -> np.ndarray:
    return np.arange(1, n + 1, dtype=np.float64) / (n + 1)


def _grids(cfg: Config):
    x = _grid(cfg.nx)
    y = _grid(cfg.ny) if cfg.dim == 2 else np.zeros(1)
    return x, y


def _smooth_modes(rng, kmax: int, x: np.ndarray, y: np.ndarray, scale_fn, dim: int):
    """Sum of sin(k pi x) sin(l pi y) modes with coefficients scale_fn(k, l) * N(0,1)."""
    out = np.zeros((y.size, x.size))
    for k in range(1, kmax + 1):
        for l in range(1, kmax + 1) if dim == 2 else [None]:
            c = rng.standard_normal() * scale_fn(k, l)
            sy = np.sin(l * np.pi * y) if dim == 2 else np.ones(1)
            out += c * np.outer(sy, np.sin(k * np.pi * x))
    return out


def initial_state(cfg: Config, seed: int | None = None) -> np.ndarray:
    """U0 of the workload, shape [ny][nx]."""
    seed = cfg.seed if seed is None else seed
    rng = np.random.default_rng(seed)
    x, y = _grids(cfg)
    if cfg.dim == 1:
        # sin(pi x) plus five random sine modes with N(0, 0.1^2) amplitudes and
        # distinct wave numbers drawn from 2..16.
        ks = rng.choice(np.arange(2, 17), size=5, replace=False)
        amps = rng.normal(0.0, 0.1, size=5)
        u = np.sin(np.pi * x)
        for k, a in zip(ks, amps):
            u = u + a * np.sin(k * np.pi * x)
        return u.reshape(1, -1)
    if cfg.scheme == "lf":
        # sum of four Gaussian pulses with random centres, widths and amplitudes
        u = np.zeros((cfg.ny, cfg.nx))
        X, Y = np.meshgrid(x, y)
        for _ in range(4):
            cx, cy = rng.uniform(0.25, 0.75, size=2)
            s = rng.uniform(0.03, 0.06)
            a = rng.standard_normal()
            u += a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * s * s))
        return u
    # Gaussian bump plus low-mode noise (c_kl ~ N(0, 0.01^2))
    X, Y = np.meshgrid(x, y)
    bump = np.exp(-20.0 * ((X - 0.5) ** 2 + (Y - 0.5) ** 2))
    noise = _smooth_modes(rng, 4, x, y, lambda k, l: 0.01, 2)
    return bump + noise


def initial_velocity(cfg: Config) -> np.ndarray:
    """u_t(0) for the wave workload (zero), shape [ny][nx]."""
    return np.zeros((cfg.ny, cfg.nx))


def source_factors(cfg: Config, seed: int):
    """Separable form of a smooth random source.

    f(x, y, t) = sum_{k,l=1..4} sum_{m=0..2} c_klm sin(k pi x) sin(l pi y) cos(m pi t)
    with c_klm ~ N(0,1)/(k^2 + l^2).  Returns (C[k,l,m], SX[k,x], SY[l,y], CT[m,t])
    so that f[t,y,x] = sum C[k,l,m] CT[m,t] SY[l,y] SX[k,x]; time levels t_0..t_nt.
    """
    rng = np.random.default_rng(seed)
    x, y = _grids(cfg)
    t = np.arange(cfg.nt + 1, dtype=np.float64) * cfg.dt
    K = 4
    C = np.zeros((K, K if cfg.dim == 2 else 1, 3))
    for k in range(1, K + 1):
        for l in (range(1, K + 1) if cfg.dim == 2 else [1]):
            for m in range(3):
                C[k - 1, l - 1, m] = rng.standard_normal() / (k * k + (l * l if cfg.dim == 2 else 0))
    SX = np.stack([np.sin(k * np.pi * x) for k in range(1, K + 1)])
    if cfg.dim == 2:
        SY = np.stack([np.sin(l * np.pi * y) for l in range(1, K + 1)])
    else:
        SY = np.ones((1, 1))
    CT = np.stack([np.cos(m * np.pi * t) for m in range(3)])
    return C, SX, SY, CT


def source_term(cfg: Config, seed: int) -> np.ndarray:
    """Dense float64 source [nt+1][ny][nx] (use for sizes that fit host memory)."""
    C, SX, SY, CT = source_factors(cfg, seed)
    return np.einsum("klm,mt,ly,kx->tyx", C, CT, SY, SX, optimize=True)


def source_term_torch(cfg: Config, seed: int, device):
    """The same source built with torch float64 on ``device`` (large workloads)."""
    import torch
    C, SX, SY, CT = (torch.from_numpy(a).to(device) for a in source_factors(cfg, seed))
    # contract k first (smallest intermediate), then l, then m
    a = torch.einsum("klm,kx->lmx", C, SX)
    b = torch.einsum("lmx,ly->myx", a, SY)
    return torch.einsum("myx,mt->tyx", b, CT).contiguous()


def tracking_target(cfg: Config, seed: int = 100) -> np.ndarray:
    """Smooth random target state: sum_{k,l<=3} N(0,1)/(k^2+l^2) sin sin, [ny][nx]."""
    rng = np.random.default_rng(seed)
    x, y = _grids(cfg)
    return _smooth_modes(rng, 3, x, y, lambda k, l: 1.0 / (k * k + (l * l if l else 0)), cfg.dim)


def fd_directions(cfg: Config, count: int = 20, first_seed: int = 200):
    """Normalised Gaussian directions over (U0, f), one per seed first_seed + i."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(first_seed + i)
        d0 = rng.standard_normal((cfg.ny, cfg.nx))
        df = rng.standard_normal((cfg.nt + 1, cfg.ny, cfg.nx))
        nrm = np.sqrt(np.sum(d0 * d0) + np.sum(df * df))
        out.append((d0 / nrm, df / nrm))
    return out


def random_vector(shape, seed: int, low: float = -1.0, high: float = 1.0) -> np.ndarray:
    """Uniform random float64 array used as a generic all-at-once test vector."""
    rng = np.random.default_rng(seed)
    return rng.uniform(low, high, size=shape)


def hybrid_wave_data(cfg: Config):
    """Data of the wave problem of Table Ex2Tab1 on the workload's grid:
    u_tt - Laplacian u = f on (0,1)^2 with u = 0 on the boundary,
    u(0) = 0, u_t(0) = 2 pi phi, phi = x(x-1) y(y-1), and
    f = -4 pi^2 phi sin(2 pi t) - 2 sin(2 pi t) (x(x-1) + y(y-1)).
    Returns (U0 [ny][nx], V0 [ny][nx], f [nt+1][ny][nx] at t_0 .. t_nt)."""
    x, y = _grids(cfg)
    gx, gy = x * (x - 1.0), y * (y - 1.0)
    phi = np.outer(gy, gx)
    lap = np.add.outer(gy, gx)
    t = np.arange(cfg.nt + 1, dtype=np.float64) * cfg.dt
    s = np.sin(2.0 * np.pi * t)
    f = s[:, None, None] * (-4.0 * np.pi ** 2 * phi - 2.0 * lap)[None]
    return np.zeros_like(phi), 2.0 * np.pi * phi, f


def hybrid_wave_exact(cfg: Config) -> np.ndarray:
    """Exact solution x(x-1) y(y-1) sin(2 pi t_n) at t_1 .. t_nt, [nt][ny][nx]."""
    x, y = _grids(cfg)
    phi = np.outer(y * (y - 1.0), x * (x - 1.0))
    t = np.arange(1, cfg.nt + 1, dtype=np.float64) * cfg.dt
    return np.sin(2.0 * np.pi * t)[:, None, None] * phi[None]


def oc_example_data(cfg: Config):
    """Data of the optimal-control example of Section 4 on the workload's grid
    (mesh width 1/(n+1)), whose exact solution is u = e^t S, p = (t - T)^2 S
    with S = sin(pi x) sin(pi y):
    f = ((1 + 2 pi^2) e^t - (t - T)^2 / gamma) S and
    g = (e^t + 2 + 2 pi^2 (t - T)^2) S at t_0 .. t_nt.
    Returns (U0 [ny][nx], u1 [ny][nx], f [nt+1][ny][nx], g [nt+1][ny][nx])."""
    x, y = _grids(cfg)
    S = np.outer(np.sin(np.pi * y), np.sin(np.pi * x))
    t = np.arange(cfg.nt + 1, dtype=np.float64) * cfg.dt
    fa = (1.0 + 2.0 * np.pi ** 2) * np.exp(t) - (t - cfg.T) ** 2 / cfg.gamma
    ga = np.exp(t) + 2.0 + 2.0 * np.pi ** 2 * (t - cfg.T) ** 2
    return S.copy(), S.copy(), fa[:, None, None] * S[None], ga[:, None, None] * S[None]


def oc_example_exact(cfg: Config):
    """Exact (u at t_1 .. t_nt, p at t_0 .. t_{nt-1}) of the example, each [nt][ny][nx]."""
    x, y = _grids(cfg)
    S = np.outer(np.sin(np.pi * y), np.sin(np.pi * x))
    t = np.arange(cfg.nt + 1, dtype=np.float64) * cfg.dt
    return np.exp(t[1:])[:, None, None] * S[None], ((t[:-1] - cfg.T) ** 2)[:, None, None] * S[None]


def parareal_initial(cfg: Config) -> np.ndarray:
    """Initial states of the parareal workload, [batch][nx]: a Gaussian bump at
    a random centre plus 0.1 N(0,1) noise, one per batch entry."""
    x, _ = _grids(cfg)
    rng = np.random.default_rng(cfg.seed)
    c = rng.uniform(0.3, 0.7, cfg.batch)
    return np.exp(-30.0 * (x[None, :] - c[:, None]) ** 2) + 0.1 * rng.standard_normal((cfg.batch, cfg.nx))


def nonlinear_initial(cfg: Config) -> np.ndarray:
    """Initial state of the Allen-Cahn workload, [ny][nx]: 0.9 sin(pi x) sin(pi y)
    + 0.2 sin(pi x) sin(2 pi y) plus smooth random modes of amplitude 0.05."""
    x, y = _grids(cfg)
    rng = np.random.default_rng(cfg.seed)
    u = 0.9 * np.outer(np.sin(np.pi * y), np.sin(np.pi * x)) + 0.2 * np.outer(np.sin(2 * np.pi * y), np.sin(np.pi * x))
    return u + 0.05 * _smooth_modes(rng, 4, x, y, lambda k, l: 1.0 / (k * k + l * l), 2)
