"""Problem description used by every oracle function."""

from __future__ import annotations

import dataclasses


@dataclasses.dataclass(frozen=True)
class Problem:
    dim: int          # 1 or 2 space dimensions
    nx: int           # interior points along x
    ny: int           # interior points along y (1 for dim == 1)
    nt: int           # time steps
    scheme: str       # 'be' | 'tr' | 'lf'
    T: float          # final time
    nu: float         # diffusion (c^2 for the wave equation)
    ax: float = 0.0   # velocity components
    ay: float = 0.0
    alpha: float = 1e-2
    periodic: bool = False   # periodic boundaries as in eq2.2b (oracle-only option)

    @property
    def dt(self) -> float:
        return self.T / self.nt

    @property
    def nspace(self) -> int:
        return self.nx * self.ny

    @classmethod
    def from_kwargs(cls, **kw) -> "Problem":
        names = {f.name for f in dataclasses.fields(cls)}
        return cls(**{k: v for k, v in kw.items() if k in names})
