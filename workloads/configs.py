"""Problem parameters of the five reference workloads and of reduced variants.

Every workload is an analytically defined PDE on the unit square (or interval)
with homogeneous Dirichlet data, discretised on ``n`` interior points per
direction.  The values below describe the PDE and the time grid only; each
consumer assembles its own operators from them.

* ``cfg1``  1D advection-diffusion, 64 points, backward Euler, Nt = 64.
* ``cfg2``  2D advection-diffusion, 256^2, trapezoidal rule, Nt = 512.
* ``cfg3``  2D advection-diffusion, 512^2, trapezoidal rule, Nt = 1024,
            a batch of 8 source terms (mixed precision preconditioner).
* ``cfg4``  2D advection-diffusion, 128^2, backward Euler, Nt = 256
            (gradient of a tracking cost through the adjoint solve).
* ``cfg5``  2D wave equation, 512^2, implicit leap-frog, Nt = 2048, T = 2.
* ``oc``    optimal control of the 2D wave equation (Section 4's example):
            255^2 interior points of mesh width 1/256, Nt = 257, T = 2,
            gamma = 1e-4 (the largest size of Table T2A).
* ``par``   parareal variant on 1D advection-diffusion (the coefficients of
            Figure 1.5 on [0, 1]): 1023 points, 64 coarse intervals of
            dT = 1/16, J = 32 backward Euler fine steps each, alpha = 0.1, a
            batch of 64 initial states.
* ``nl``    2D Allen-Cahn u_t = nu Laplacian u + u - u^3, 511^2 points,
            Nt = 256 backward Euler steps, T = 0.5, alpha = 0.05.
* ``hyb``   2D wave equation u_tt = Laplacian u + f on the 511^2 interior
            points of mesh width 1/512, T = 2, Nt = 512, hybrid time
            discretisation solved directly (ParaDiag-I; the problem of Table
            Ex2Tab1, whose exact solution is x(x-1) y(y-1) sin(2 pi t)).
"""

from __future__ import annotations

import dataclasses
from typing import Optional


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    dim: int            # 1 or 2
    nx: int             # interior points along x
    ny: int             # interior points along y (1 when dim == 1)
    nt: int             # number of time steps
    scheme: str         # 'be' (backward Euler), 'tr' (trapezoidal), 'lf' (implicit leap-frog),
                        # 'hyb' / 'hyb2' (hybrid midpoint + backward Euler, first / second order)
    T: float            # final time; dt = T / nt
    nu: float           # diffusion coefficient (c^2 for the wave equation)
    ax: float           # velocity, x component (0 for the wave equation)
    ay: float           # velocity, y component
    alpha: float        # alpha-circulant parameter
    batch: int = 1      # number of right-hand sides solved together
    rtol: float = 1e-8  # relative true-residual target
    prec: str = "fp64"  # 'fp64', 'fp32', 'fp32_bf16gemm'
    seed: int = 0
    with_source: bool = False
    beta: float = 0.0   # control penalty of the tracking cost (cfg4)
    gamma: float = 0.0  # control penalty of the optimality system (oc)
    fine_steps: int = 0  # parareal fine steps per coarse interval (par)
    reaction: tuple = ()  # (k1, k2, k3) of g(u) = k1 u + k2 u^2 + k3 u^3 (nl)

    @property
    def dt(self) -> float:
        return self.T / self.nt

    @property
    def nspace(self) -> int:
        return self.nx * self.ny

    @property
    def unknowns(self) -> int:
        return self.nx * self.ny * self.nt * self.batch

    def problem_kwargs(self) -> dict:
        """The PDE/time-grid parameters as plain keywords."""
        return dict(dim=self.dim, nx=self.nx, ny=self.ny, nt=self.nt, scheme=self.scheme,
                    T=self.T, nu=self.nu, ax=self.ax, ay=self.ay, alpha=self.alpha)

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


CONFIGS = {
    "cfg1": Config("cfg1", 1, 64, 1, 64, "be", 1.0, 1e-2, 1.0, 0.0, 1e-2,
                   rtol=1e-10, prec="fp64"),
    "cfg2": Config("cfg2", 2, 256, 256, 512, "tr", 1.0, 5e-3, 1.0, 0.5, 1e-3,
                   rtol=1e-8, prec="fp64"),
    "cfg3": Config("cfg3", 2, 512, 512, 1024, "tr", 1.0, 5e-3, 1.0, 0.5, 1e-3,
                   batch=8, rtol=1e-8, prec="fp32_bf16gemm", with_source=True),
    "cfg4": Config("cfg4", 2, 128, 128, 256, "be", 1.0, 5e-3, 1.0, 0.5, 1e-3,
                   rtol=1e-12, prec="fp64", with_source=True, beta=1e-4, seed=101),
    "cfg5": Config("cfg5", 2, 512, 512, 2048, "lf", 2.0, 1.0, 0.0, 0.0, 1e-2,
                   rtol=1e-8, prec="fp32"),
    "hyb": Config("hyb", 2, 511, 511, 512, "hyb2", 2.0, 1.0, 0.0, 0.0, 1.0,
                  rtol=1e-8, prec="fp64", with_source=True),
    "oc": Config("oc", 2, 255, 255, 257, "lf", 2.0, 1.0, 0.0, 0.0, 1.0,
                 rtol=1e-7, prec="fp64", with_source=True, gamma=1e-4),
    "par": Config("par", 1, 1023, 1, 64, "be", 4.0, 0.1, 1.0, 0.0, 0.1,
                  batch=64, rtol=1e-10, prec="fp64", seed=7, fine_steps=32),
    "nl": Config("nl", 2, 511, 511, 256, "be", 0.5, 5e-2, 0.0, 0.0, 0.05,
                 rtol=1e-10, prec="fp64", reaction=(-1.0, 0.0, 1.0)),
}


def get_config(name: str) -> Config:
    return CONFIGS[name]


def small_config(name: str, nx: int, ny: Optional[int] = None, nt: Optional[int] = None,
                 batch: Optional[int] = None) -> Config:
    """A reduced copy of a workload: same PDE, coefficients and alpha, fewer points.

    The time step keeps its relation to T (dt = T / nt), so a reduced ``nt``
    keeps the final time of the original workload.
    """
    c = CONFIGS[name]
    if ny is None:
        ny = 1 if c.dim == 1 else nx
    return c.replace(name=f"{name}-small", nx=nx, ny=ny, nt=nt or c.nt,
                     batch=batch or c.batch)
