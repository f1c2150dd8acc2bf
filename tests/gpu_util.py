"""Helpers shared by the GPU tests: build a plan and the matching oracle problem."""

import os
import sys

import numpy as np
import pytest

from oracle import Problem


def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_09158_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        raise RuntimeError("libparadiag.so is missing on a GPU machine: build it first")
    return torch


def announce(msg: str) -> None:
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def make(params: dict, prec: str = "fp64", batch: int = 1, mode: str = "fgmres", restart: int = 10):
    torch = torch_gpu()
    from paper_2005_09158_amd import ParaDiag
    pd = ParaDiag(dim=params["dim"], nx=params["nx"], ny=params["ny"], nt=params["nt"],
                  scheme=params["scheme"], T=params["T"], nu=params["nu"], ax=params.get("ax", 0.0),
                  ay=params.get("ay", 0.0), alpha=params.get("alpha", 1.0), batch=batch, prec=prec,
                  mode=mode, restart=restart)
    prob = Problem.from_kwargs(**params)
    return torch, pd, prob


def to_gpu(torch, a, shape):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).reshape(shape).cuda()


def rel_err(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
