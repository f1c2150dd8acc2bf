"""The allocation-free preconditioner entry point against the ordinary one.

paradiag_apply_precond_static runs the kernels of paradiag_apply_precond with
its spectral buffers in the library's static device array.  Both are called
through the C ABI on the same seeded inputs; the results must agree to the
float64 preconditioner tolerance (they run the same arithmetic, so they are
expected to be identical).  Two calls in a row, the second on a smaller
problem of another precision, check that the shared array carries nothing
from one call into the next; a plan whose spectral buffers exceed the array
is refused.
"""

import ctypes

import numpy as np
import pytest

from tests.gpu_util import announce, make, rel_err, to_gpu

pytestmark = pytest.mark.gpu

CASES = [
    # (problem, precision, batch): larger first, then smaller
    (dict(dim=2, nx=40, ny=36, nt=32, scheme="tr", T=1.0, nu=2e-2, ax=1.0, ay=0.5, alpha=1e-3), "fp64", 3),
    # windowed back-sweep (two 64-mode windows) over two streams
    (dict(dim=2, nx=128, ny=20, nt=8, scheme="tr", T=0.5, nu=0.05, ax=1.0, ay=0.5, alpha=1e-2), "fp32_bf16gemm", 2),
    (dict(dim=2, nx=17, ny=9, nt=8, scheme="lf", T=1.0, nu=1.0, alpha=1e-2), "fp32_bf16gemm", 1),
]


def _both(torch, pd, r):
    z_ref = pd.apply_precond(r)
    z = torch.full_like(r, float("nan"))
    st = pd.lib.paradiag_apply_precond_static(pd.plan, ctypes.c_void_p(r.data_ptr()),
                                              ctypes.c_void_p(z.data_ptr()),
                                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert st == 0, pd.lib.paradiag_last_error()
    return z_ref.cpu().numpy(), z.cpu().numpy()


def test_static_matches_workspace_twice():
    for params, prec, batch in CASES:
        announce(f"static scratch precond {params['nx']}x{params['ny']}x{params['nt']} {prec} batch {batch}")
        torch, pd, prob = make(params, prec, batch=batch)
        rng = np.random.default_rng(params["nx"])
        r = to_gpu(torch, rng.standard_normal(pd.shape), pd.shape)
        z_ref, z = _both(torch, pd, r)
        err = rel_err(z, z_ref)
        print(f"  static vs workspace: {err:.2e} (identical: {np.array_equal(z, z_ref)})")
        tol = 1e-13 if prec == "fp64" else 1e-6
        assert np.all(np.isfinite(z)) and err <= tol


def test_static_in_place():
    announce("static scratch precond in place")
    params, prec, batch = CASES[1]
    torch, pd, prob = make(params, prec, batch=batch)
    r = to_gpu(torch, np.random.default_rng(5).standard_normal(pd.shape), pd.shape)
    z_ref = pd.apply_precond(r).cpu().numpy()
    pd.apply_precond_static(r, out=r)
    torch.cuda.synchronize()
    assert rel_err(r.cpu().numpy(), z_ref) <= 1e-6


def test_static_refuses_oversize():
    announce("static scratch precond: plan larger than the array")
    from paper_2005_09158_amd import _lib
    # 2 x 257 x 256 x 256 complex float64 = 539 MB of spectral buffers > 128 MiB
    params = dict(dim=2, nx=256, ny=256, nt=512, scheme="lf", T=1.0, nu=1.0, alpha=1e-2)
    torch, pd, prob = make(params, "fp64")
    r = torch.zeros(pd.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.ParaDiagError) as e:
        pd.apply_precond_static(r)
    assert e.value.status == _lib.PD_ERR_WORKSPACE
    assert "static scratch" in str(e.value)
