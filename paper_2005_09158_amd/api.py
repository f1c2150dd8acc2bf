"""Thin torch binding of the C ABI: same entry points, tensors instead of pointers.

Every call marshals device pointers of float64 CUDA (HIP) tensors and torch's
current stream into the library; all arithmetic runs in the library's HIP
kernels.  The binding refuses CPU tensors and fails loudly when the library is
missing: there is no fallback.
"""

from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional

import torch

from . import _lib


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor], shape=None, name: str = "") -> ctypes.c_void_p:
    if t is None:
        return ctypes.c_void_p(None)
    if not t.is_cuda:
        raise ValueError(f"{name}: expected a GPU tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{name}: expected float64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


@dataclasses.dataclass
class SolveResult:
    status: int
    iters: int
    converged: bool
    rel_resid: float
    iters_per_rhs: list
    resid_per_rhs: list
    history: list


class ParaDiag:
    """A plan (``paradiag_setup``) with its workspace bound (``paradiag_bind_workspace``).

    Shapes: all-at-once vectors [batch, nt, ny, nx]; U0, u1 [batch, ny, nx];
    f [batch, nt+1, ny, nx]; all float64 on the GPU.
    """

    def __init__(self, *, dim: int, nx: int, ny: int, nt: int, scheme: str, T: float, nu: float,
                 ax: float = 0.0, ay: float = 0.0, alpha: float = 1e-2, batch: int = 1,
                 prec: str = "fp64", mode: str = "fgmres", restart: int = 10,
                 device: Optional[torch.device] = None):
        self.lib = _lib.load()
        self.shape = (batch, nt, ny, nx)
        self.field_shape = (batch, ny, nx)
        self.source_shape = (batch, nt + 1, ny, nx)
        self.batch, self.nt, self.ny, self.nx = batch, nt, ny, nx
        self.prob = _lib.Problem(dim=dim, nx=nx, ny=ny, nt=nt, batch=batch,
                                 scheme=_lib.SCHEMES[scheme], prec=_lib.PRECS[prec], reserved=0,
                                 T=T, nu=nu, ax=ax, ay=ay, alpha=alpha)
        h = ctypes.c_void_p()
        _lib.check(self.lib.paradiag_setup(ctypes.byref(self.prob), ctypes.byref(h)), "paradiag_setup")
        self.plan = h
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self._ws = None
        self.bind_workspace(mode, restart)

    # ------------------------------------------------------------ workspace
    def workspace_size(self, mode: str = "fgmres", restart: int = 10) -> int:
        opts = _lib.SolveOpts(mode=_lib.MODES[mode], restart=restart, max_iter=1, use_x0=0, rtol=1.0)
        n = ctypes.c_size_t()
        _lib.check(self.lib.paradiag_workspace_size(self.plan, ctypes.byref(opts), ctypes.byref(n)),
                   "paradiag_workspace_size")
        return int(n.value)

    def bind_workspace(self, mode: str = "fgmres", restart: int = 10) -> None:
        nbytes = self.workspace_size(mode, restart)
        # torch's caching allocator returns 512-byte aligned blocks
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        self._ws = ws
        self._ws_ptr = ws.data_ptr() + off
        _lib.check(self.lib.paradiag_bind_workspace(self.plan, ctypes.c_void_p(self._ws_ptr),
                                                    ctypes.c_size_t(nbytes), _stream()),
                   "paradiag_bind_workspace")
        self.mode, self.restart = mode, restart

    # ----------------------------------------------------------- operations
    def build_rhs(self, U0: torch.Tensor, u1: Optional[torch.Tensor] = None,
                  f: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        b = out if out is not None else torch.empty(self.shape, dtype=torch.float64, device=self.device)
        _lib.check(self.lib.paradiag_build_rhs(self.plan, _ptr(U0, self.field_shape, "U0"),
                                               _ptr(u1, self.field_shape, "u1"),
                                               _ptr(f, self.source_shape, "f"),
                                               _ptr(b, self.shape, "b"), _stream()),
                   "paradiag_build_rhs")
        return b

    def rhs_transpose(self, lam: torch.Tensor):
        gU0 = torch.empty(self.field_shape, dtype=torch.float64, device=self.device)
        gu1 = torch.empty(self.field_shape, dtype=torch.float64, device=self.device)
        gf = torch.empty(self.source_shape, dtype=torch.float64, device=self.device)
        _lib.check(self.lib.paradiag_rhs_transpose(self.plan, _ptr(lam, self.shape, "lam"),
                                                   _ptr(gU0), _ptr(gu1), _ptr(gf), _stream()),
                   "paradiag_rhs_transpose")
        return gU0, gu1, gf

    def matvec(self, u: torch.Tensor, transpose: bool = False,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
        y = out if out is not None else torch.empty(self.shape, dtype=torch.float64, device=self.device)
        _lib.check(self.lib.paradiag_matvec(self.plan, _ptr(u, self.shape, "u"), _ptr(y, self.shape, "y"),
                                            int(bool(transpose)), _stream()), "paradiag_matvec")
        return y

    def apply_precond(self, r: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        z = out if out is not None else torch.empty(self.shape, dtype=torch.float64, device=self.device)
        _lib.check(self.lib.paradiag_apply_precond(self.plan, _ptr(r, self.shape, "r"),
                                                   _ptr(z, self.shape, "z"), _stream()),
                   "paradiag_apply_precond")
        return z

    def apply_precond_static(self, r: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """paradiag_apply_precond_static: the same z = P^{-1} r with the spectral
        buffers in the library's static device array (the call allocates nothing;
        `out` must then be given by a caller that cannot allocate)."""
        z = out if out is not None else torch.empty(self.shape, dtype=torch.float64, device=self.device)
        _lib.check(self.lib.paradiag_apply_precond_static(self.plan, _ptr(r, self.shape, "r"),
                                                          _ptr(z, self.shape, "z"), _stream()),
                   "paradiag_apply_precond_static")
        return z

    def _solve(self, fn, name, b, u, mode, rtol, max_iter, restart, x0):
        if mode is None:
            mode = self.mode
        if restart is None:
            restart = self.restart
        if u is None:
            u = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        if x0 is not None:
            u.copy_(x0)
        opts = _lib.SolveOpts(mode=_lib.MODES[mode], restart=restart, max_iter=max_iter,
                              use_x0=int(x0 is not None), rtol=rtol)
        it = (ctypes.c_int32 * self.batch)()
        rs = (ctypes.c_double * self.batch)()
        cap = max_iter + 64
        hist = (ctypes.c_double * cap)()
        info = _lib.SolveInfo(iters=0, converged=0, rel_resid=0.0, iters_per_rhs=it,
                              resid_per_rhs=rs, history=hist, history_cap=cap, history_len=0)
        st = fn(self.plan, _ptr(b, self.shape, "b"), _ptr(u, self.shape, "u"), ctypes.byref(opts),
                ctypes.byref(info), _stream())
        _lib.check(st, name, allow_not_converged=True)
        res = SolveResult(st, info.iters, bool(info.converged), info.rel_resid, list(it), list(rs),
                          list(hist[: info.history_len]))
        return u, res

    def solve(self, b: torch.Tensor, u: Optional[torch.Tensor] = None, *, mode: Optional[str] = None,
              rtol: float = 1e-8, max_iter: int = 100, restart: Optional[int] = None,
              x0: Optional[torch.Tensor] = None):
        """Solve A u = b; returns (u, SolveResult)."""
        return self._solve(self.lib.paradiag_solve, "paradiag_solve", b, u, mode, rtol, max_iter,
                           restart, x0)

    def adjoint_solve(self, g: torch.Tensor, lam: Optional[torch.Tensor] = None, *,
                      mode: Optional[str] = None, rtol: float = 1e-8, max_iter: int = 100,
                      restart: Optional[int] = None, x0: Optional[torch.Tensor] = None):
        """Solve A^T lam = g; returns (lam, SolveResult)."""
        return self._solve(self.lib.paradiag_adjoint_solve, "paradiag_adjoint_solve", g, lam, mode,
                           rtol, max_iter, restart, x0)

    def parareal(self, U0: torch.Tensor, J: int, u: Optional[torch.Tensor] = None, *,
                 rtol: float = 1e-10, max_iter: int = 50, x0: Optional[torch.Tensor] = None):
        """paradiag_parareal: the ParaDiag-II parareal variant from U0 ([batch, 1, nx]),
        J fine backward Euler steps per coarse interval; returns (u, SolveResult)
        with u [batch, nt, 1, nx] and rel_resid the last relative change."""
        if u is None:
            u = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        if x0 is not None:
            u.copy_(x0)
        opts = _lib.SolveOpts(mode=_lib.MODES["parareal"], restart=1, max_iter=max_iter,
                              use_x0=int(x0 is not None), rtol=rtol)
        it = (ctypes.c_int32 * self.batch)()
        rs = (ctypes.c_double * self.batch)()
        cap = max_iter + 4
        hist = (ctypes.c_double * cap)()
        info = _lib.SolveInfo(iters=0, converged=0, rel_resid=0.0, iters_per_rhs=it,
                              resid_per_rhs=rs, history=hist, history_cap=cap, history_len=0)
        st = self.lib.paradiag_parareal(self.plan, _ptr(U0, self.field_shape, "U0"), int(J),
                                        _ptr(u, self.shape, "u"), ctypes.byref(opts), ctypes.byref(info),
                                        _stream())
        _lib.check(st, "paradiag_parareal", allow_not_converged=True)
        return u, SolveResult(st, info.iters, bool(info.converged), info.rel_resid, list(it), list(rs),
                              list(hist[: info.history_len]))

    def nonlinear_solve(self, U0: torch.Tensor, k1: float = 0.0, k2: float = 0.0, k3: float = 0.0, *,
                        windows: int = 1, u: Optional[torch.Tensor] = None, rtol: float = 1e-10,
                        max_iter: int = 50, x0: Optional[torch.Tensor] = None):
        """paradiag_nonlinear_solve: u' + K u + g(u) = 0 with g(u) = k1 u + k2 u^2 + k3 u^3,
        simplified Newton with the averaged Jacobian over `windows` consecutive
        windows; returns (u [windows, 1, nt, ny, nx], SolveResult)."""
        shape = (windows,) + self.shape
        if u is None:
            u = torch.empty(shape, dtype=torch.float64, device=self.device)
        if x0 is not None:
            u[0].copy_(x0)
        opts = _lib.SolveOpts(mode=_lib.MODES["nonlinear"], restart=1, max_iter=max_iter,
                              use_x0=int(x0 is not None), rtol=rtol)
        it = (ctypes.c_int32 * self.batch)()
        rs = (ctypes.c_double * self.batch)()
        cap = windows * (max_iter + 2) + 4
        hist = (ctypes.c_double * cap)()
        info = _lib.SolveInfo(iters=0, converged=0, rel_resid=0.0, iters_per_rhs=it,
                              resid_per_rhs=rs, history=hist, history_cap=cap, history_len=0)
        gc = _lib.Cubic(k1=k1, k2=k2, k3=k3)
        st = self.lib.paradiag_nonlinear_solve(self.plan, ctypes.byref(gc), _ptr(U0, self.field_shape, "U0"),
                                               int(windows), _ptr(u, shape, "u"), ctypes.byref(opts),
                                               ctypes.byref(info), _stream())
        _lib.check(st, "paradiag_nonlinear_solve", allow_not_converged=True)
        return u, SolveResult(st, info.iters, bool(info.converged), info.rel_resid, list(it), list(rs),
                              list(hist[: info.history_len]))

    # ----------------------------------------------------------- inspection
    def set_timing(self, enable, stages=None) -> None:
        """Turn stage timing on or off; with `stages` (names as in stage_times),
        only those stages are timed."""
        if not enable:
            code = 0
        elif stages is None:
            code = 1
        else:
            code = 0
            for name in stages:
                code |= 1 << (_lib.STAGES.index(name) + 1)
        _lib.check(self.lib.paradiag_set_timing(self.plan, code), "paradiag_set_timing")

    def stage_times(self, reset: bool = True) -> dict:
        """{stage: (ms, launches, algorithmic bytes, flops)} since the last reset."""
        n = len(_lib.STAGES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        by = (ctypes.c_double * n)()
        fl = (ctypes.c_double * n)()
        _lib.check(self.lib.paradiag_get_stage_times(self.plan, ms, cnt, by, fl, int(reset)),
                   "paradiag_get_stage_times")
        return {name: (ms[i], cnt[i], by[i], fl[i]) for i, name in enumerate(_lib.STAGES)}

    def __del__(self):
        try:
            if getattr(self, "plan", None) is not None and self.plan.value:
                self.lib.paradiag_destroy(self.plan)
                self.plan = ctypes.c_void_p()
        except Exception:
            pass


def host_plan(**kw):
    """Create a plan without binding a workspace (host-only calls; no GPU needed)."""
    lib = _lib.load()
    prob = _lib.Problem(dim=kw["dim"], nx=kw["nx"], ny=kw["ny"], nt=kw["nt"], batch=kw.get("batch", 1),
                        scheme=_lib.SCHEMES[kw["scheme"]], prec=_lib.PRECS[kw.get("prec", "fp64")],
                        reserved=0, T=kw["T"], nu=kw["nu"], ax=kw.get("ax", 0.0), ay=kw.get("ay", 0.0),
                        alpha=kw["alpha"])
    h = ctypes.c_void_p()
    st = lib.paradiag_setup(ctypes.byref(prob), ctypes.byref(h))
    return st, h


class ParaDiagSolve(torch.autograd.Function):
    """u = A^{-1} b(U0, f) with a hand-written adjoint.

    forward(pd, U0, f, rtol) -> u; backward uses paradiag_adjoint_solve
    (A^T lam = dL/du) and paradiag_rhs_transpose to return dL/dU0 and dL/df.
    """

    @staticmethod
    def forward(ctx, pd: ParaDiag, U0: torch.Tensor, f: torch.Tensor, rtol: float = 1e-12):
        b = pd.build_rhs(U0.detach().contiguous(), None, f.detach().contiguous())
        u, res = pd.solve(b, rtol=rtol, max_iter=200)
        if not res.converged:
            raise RuntimeError(f"forward solve did not converge: {res}")
        ctx.pd, ctx.rtol = pd, rtol
        return u

    @staticmethod
    def backward(ctx, grad_u: torch.Tensor):
        pd = ctx.pd
        lam, res = pd.adjoint_solve(grad_u.contiguous(), rtol=ctx.rtol, max_iter=200)
        if not res.converged:
            raise RuntimeError(f"adjoint solve did not converge: {res}")
        gU0, _gu1, gf = pd.rhs_transpose(lam)
        return None, gU0, gf, None


class ParaDiagOC(ParaDiag):
    """Plan of the optimal control of the wave equation (``paradiag_oc_setup``,
    Section 4): vectors [2, nt, ny, nx] holding sqrt(gamma) u and p; matvec,
    apply_precond and solve as for ParaDiag, plus ``build_rhs`` from (U0, u1, f, g)."""

    def __init__(self, *, dim: int, nx: int, ny: int, nt: int, T: float, nu: float, gamma: float,
                 prec: str = "fp64", mode: str = "fgmres", restart: int = 30,
                 device: Optional[torch.device] = None):
        self.lib = _lib.load()
        self.shape = (2, nt, ny, nx)
        self.field_shape = (1, ny, nx)
        self.source_shape = (1, nt + 1, ny, nx)
        self.batch, self.nt, self.ny, self.nx = 1, nt, ny, nx
        self.gamma = gamma
        self.prob = _lib.Problem(dim=dim, nx=nx, ny=ny, nt=nt, batch=1, scheme=_lib.SCHEMES["lf"],
                                 prec=_lib.PRECS[prec], reserved=0, T=T, nu=nu, ax=0.0, ay=0.0, alpha=1.0)
        h = ctypes.c_void_p()
        _lib.check(self.lib.paradiag_oc_setup(ctypes.byref(self.prob), ctypes.c_double(gamma), ctypes.byref(h)),
                   "paradiag_oc_setup")
        self.plan = h
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self._ws = None
        self.bind_workspace(mode, restart)

    def build_rhs(self, U0: torch.Tensor, u1: Optional[torch.Tensor] = None,
                  f: Optional[torch.Tensor] = None, g: Optional[torch.Tensor] = None,
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
        b = out if out is not None else torch.empty(self.shape, dtype=torch.float64, device=self.device)
        _lib.check(self.lib.paradiag_oc_build_rhs(self.plan, _ptr(U0, self.field_shape, "U0"),
                                                  _ptr(u1, self.field_shape, "u1"),
                                                  _ptr(f, self.source_shape, "f"),
                                                  _ptr(g, self.source_shape, "g"),
                                                  _ptr(b, self.shape, "b"), _stream()),
                   "paradiag_oc_build_rhs")
        return b

