"""GPU parity against the oracle on small shapes (several tiles and ragged tails).

Tolerances (relative, max-abs error over max-abs reference):
* float64 preconditioner: 1e-11.  Step-(a)/(c) are O(log Nt) rounding steps
  and Step-(b) is a backward-stable elimination, amplified by at most
  cond(V) <= 1/alpha (eq2.13) and the spatial condition number.
* float32 preconditioner: 2e-3 (u32 = 6e-8 times 1/alpha = 1e3 times the line
  system condition numbers of these shapes).
* split bf16 x-transform (three bf16 parts, six products): as float32, 2e-3.
* single bf16 x-transform: 5e-2 with the sine basis (u_bf16 = 3.9e-3 in each of the
  two transforms, amplified as above).  With a non-normal x factor the Schur
  basis carries that rounding through the back-substitution, whose coupling
  norm ||T - diag T|| is of the order of ||K_x||, and the error of
  P_alpha^{-1} reached 0.06 - 0.8 on these shapes: setup refuses that
  combination (PD_ERR_UNSUPPORTED), which the tests check.
* matvec, right-hand side and its transpose: 1e-13 (a few float64 operations
  per entry, evaluated in a different order).
* solves: 1e-10 against the sequential time stepper at rtol 1e-12.
"""

import functools

import numpy as np
import pytest

from oracle import Problem, adjoint as o_adj, operators as ops, precond as o_prec, rhs as o_rhs, solve as o_solve
from tests.gpu_util import announce, make, rel_err, to_gpu
from tests.bounds import line_condition

pytestmark = pytest.mark.gpu

CASES = {
    "1d-be": dict(dim=1, nx=64, ny=1, nt=64, scheme="be", T=1.0, nu=1e-2, ax=1.0, alpha=1e-2),
    "1d-tr-ragged": dict(dim=1, nx=37, ny=1, nt=16, scheme="tr", T=1.0, nu=2e-2, ax=-0.7, alpha=1e-3),
    "2d-tr-schur": dict(dim=2, nx=24, ny=20, nt=16, scheme="tr", T=1.0, nu=3e-2, ax=1.0, ay=0.5, alpha=1e-3),
    "2d-be-schur-ragged": dict(dim=2, nx=31, ny=17, nt=8, scheme="be", T=0.5, nu=2e-2, ax=0.8, ay=-0.6, alpha=1e-2),
    "2d-lf-dst": dict(dim=2, nx=30, ny=26, nt=32, scheme="lf", T=1.0, nu=1.0, alpha=1e-2),
    "2d-tr-dst-nt4": dict(dim=2, nx=20, ny=33, nt=4, scheme="tr", T=0.3, nu=5e-2, ay=0.9, alpha=0.1),
    "2d-be-schur-64": dict(dim=2, nx=64, ny=64, nt=32, scheme="be", T=1.0, nu=1e-2, ax=1.0, ay=0.5, alpha=1e-3),
    "2d-tr-schur-mid": dict(dim=2, nx=72, ny=150, nt=8, scheme="tr", T=0.5, nu=1e-2, ax=1.0, ay=-0.5, alpha=1e-3),
    "2d-tr-schur-tall": dict(dim=2, nx=40, ny=300, nt=8, scheme="tr", T=0.5, nu=2e-2, ax=1.0, ay=0.5, alpha=1e-2),
    # x-transform products with K = N = 160 (a multiple of 32, so the split MFMA
    # kernels run) and a ragged last column tile (160 = 128 + 32), 9 x 23 = 207
    # rows (a ragged last row tile)
    "2d-tr-schur-80": dict(dim=2, nx=80, ny=23, nt=16, scheme="tr", T=0.5, nu=2e-2, ax=1.0, ay=-0.4, alpha=1e-2),
}

PREC_TOL = {"fp64": 1e-11, "fp32": 2e-3, "fp32_bf16gemm": 2e-3, "fp32_bf16x1": 5e-2, "fp32_fp16gemm": 2e-3}
UNIT_ROUNDOFF = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24}


def _bf16x1_schur(case, prec):
    c = CASES[case]
    return prec == "fp32_bf16x1" and c["dim"] == 2 and c.get("ax", 0.0) != 0.0


def _shape(prob, batch=1):
    return (batch, prob.nt, prob.ny, prob.nx)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_bf16gemm", "fp32_bf16x1", "fp32_fp16gemm"])
@pytest.mark.parametrize("case", list(CASES))
def test_precond_parity(case, prec):
    announce(f"precond {case} {prec}")
    if _bf16x1_schur(case, prec):
        from paper_2005_09158_amd._lib import PD_ERR_UNSUPPORTED, ParaDiagError
        with pytest.raises(ParaDiagError) as e:
            make(CASES[case], prec)
        assert e.value.status == PD_ERR_UNSUPPORTED
        return
    torch, pd, prob = make(CASES[case], prec)
    r = np.random.default_rng(1).standard_normal((prob.nt, prob.nspace))
    z_ref = o_prec.three_steps(prob, r)
    z = pd.apply_precond(to_gpu(torch, r, pd.shape))
    torch.cuda.synchronize()
    err = rel_err(z.cpu().numpy().reshape(prob.nt, -1), z_ref)
    print(f"  rel err {err:.3e}")
    assert err < PREC_TOL[prec]


# Back-sweep shapes: every line-segment width of the one-wave scan (rows per
# line 3 .. 128 -> 1 .. 32 lanes), a partial last block of modes, and
# x-sizes that are not multiples of 4 (scalar coupling loads).
SWEEP_SHAPES = [(20, 3), (21, 7), (36, 13), (37, 100), (48, 128), (17, 33)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nx,ny", SWEEP_SHAPES)
def test_schur_sweep_shapes(nx, ny, prec):
    announce(f"sweep shape {nx}x{ny} {prec}")
    cfg = dict(dim=2, nx=nx, ny=ny, nt=8, scheme="tr", T=0.5, nu=0.1, ax=1.0, ay=0.5, alpha=1e-2)
    torch, pd, prob = make(cfg, prec)
    r = np.random.default_rng(7).standard_normal((prob.nt, prob.nspace))
    z_ref = o_prec.three_steps(prob, r)
    z = pd.apply_precond(to_gpu(torch, r, pd.shape))
    torch.cuda.synchronize()
    err = rel_err(z.cpu().numpy().reshape(prob.nt, -1), z_ref)
    print(f"  rel err {err:.3e}")
    assert err < PREC_TOL[prec]


# Windowed back-sweep (split-bf16 and split-fp16 modes, x-sizes that are
# multiples of 64): the coupling of each 64-mode window to the later ones is
# one row-scaled split-fp16 product over all slices before the window is swept.  Rows per line from 20 to 300 (1 .. 64
# lanes; 150 and 256 rows give the coupling waves row ranges that are not a
# multiple of their 32-row passes), two to four windows.  The error against
# the oracle must stay at the float32 level of the same plan in plain float32
# (whose sweep is not windowed): within 4x of it, plus 1e-6.
WINDOW_SHAPES = [(128, 20), (192, 37), (256, 64), (192, 150), (128, 256), (128, 300)]


@pytest.mark.parametrize("nx,ny", WINDOW_SHAPES)
def test_windowed_sweep_shapes(nx, ny):
    announce(f"windowed sweep {nx}x{ny}")
    cfg = dict(dim=2, nx=nx, ny=ny, nt=8, scheme="tr", T=0.5, nu=0.05, ax=1.0, ay=0.5, alpha=1e-2)
    r = np.random.default_rng(11).standard_normal((cfg["nt"], nx * ny))
    errs = {}
    for prec in ("fp32", "fp32_bf16gemm", "fp32_fp16gemm"):
        torch, pd, prob = make(cfg, prec)
        z = pd.apply_precond(to_gpu(torch, r, pd.shape))
        torch.cuda.synchronize()
        if prec == "fp32":
            z_ref = o_prec.three_steps(prob, r)
        errs[prec] = rel_err(z.cpu().numpy().reshape(prob.nt, -1), z_ref)
    print(f"  rel err fp32 {errs['fp32']:.3e}, windowed split bf16 {errs['fp32_bf16gemm']:.3e}, "
          f"split fp16 x-transform {errs['fp32_fp16gemm']:.3e}")
    assert errs["fp32_bf16gemm"] <= 4 * errs["fp32"] + 1e-6
    assert errs["fp32_fp16gemm"] <= 4 * errs["fp32"] + 1e-6


# The far product's fp16 operands are scaled per row by the largest solved
# mode of that row: a batch with a zero entry and entries scaled by 1e30 and
# 1e-30 must give each entry's own result (linearity: c r -> c z), with no
# overflow or flush to zero on the way.  Five entries: the sweep runs the
# first two and the last three on two streams.
@pytest.mark.parametrize("prec", ["fp32_bf16gemm", "fp32_fp16gemm"])
def test_windowed_sweep_scaled_batch(prec):
    announce(f"windowed sweep scaled batch {prec}")
    cfg = dict(dim=2, nx=128, ny=20, nt=8, scheme="tr", T=0.5, nu=0.05, ax=1.0, ay=0.5, alpha=1e-2)
    r = np.random.default_rng(5).standard_normal((cfg["nt"], 128 * 20))
    scales = [1.0, 0.0, 1e30, 1e-30, -2.5]
    torch, pd, prob = make(cfg, prec, batch=len(scales))
    z_ref = o_prec.three_steps(prob, r)
    rb = np.stack([c * r for c in scales])
    z = pd.apply_precond(to_gpu(torch, rb, pd.shape)).cpu().numpy().reshape(len(scales), prob.nt, -1)
    assert np.all(np.isfinite(z))
    assert np.all(z[1] == 0.0)
    for b, c in enumerate(scales):
        if c == 0.0:
            continue
        err = rel_err(z[b] / c, z_ref)
        print(f"  scale {c:g}: rel err {err:.3e}")
        assert err < PREC_TOL[prec]


# Sine-basis x-transform by FFT (nx + 1 a power of two: a DST-I as one complex
# FFT of length 2 (nx + 1) per spectral row, both halves at once): FFT lengths
# 16 .. 1024, odd and even row counts, every precision.  Same tolerances as
# the dense product it replaces.
DST_SHAPES = [(7, 9), (15, 40), (63, 17), (255, 12), (511, 9)]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_bf16gemm"])
@pytest.mark.parametrize("nx,ny", DST_SHAPES)
def test_dst_xform_shapes(nx, ny, prec):
    announce(f"DST x-transform {nx}x{ny} {prec}")
    cfg = dict(dim=2, nx=nx, ny=ny, nt=8, scheme="tr", T=0.5, nu=0.05, ay=0.7, alpha=1e-2)
    torch, pd, prob = make(cfg, prec)
    r = np.random.default_rng(nx + ny).standard_normal((prob.nt, prob.nspace))
    z_ref = o_prec.three_steps(prob, r)
    z = pd.apply_precond(to_gpu(torch, r, pd.shape))
    torch.cuda.synchronize()
    err = rel_err(z.cpu().numpy().reshape(prob.nt, -1), z_ref)
    print(f"  rel err {err:.3e}")
    assert err < PREC_TOL[prec]


# Line-solver shapes (sine basis): lines of 256 .. 512 rows take 8 rows per
# lane (32 or 64 lanes per line), 1024 and 2048 rows take 16 and 32 rows per
# lane (tiles of 4 modes; 135 KiB of LDS at 2048 rows in float64), a ragged
# length pads the last lane, and an x-size that is not a multiple of 4 takes
# the element-wise tile copies.
LINE_SHAPES = [(8, 256), (6, 300), (4, 512), (5, 129), (4, 1024), (3, 2048), (5, 1500)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nx,ny", LINE_SHAPES)
def test_line_solver_shapes(nx, ny, prec):
    announce(f"line shape {nx}x{ny} {prec}")
    cfg = dict(dim=2, nx=nx, ny=ny, nt=8, scheme="lf", T=1.0, nu=1.0, alpha=1e-2)
    torch, pd, prob = make(cfg, prec)
    r = np.random.default_rng(13).standard_normal((prob.nt, prob.nspace))
    z_ref = o_prec.three_steps(prob, r)
    z = pd.apply_precond(to_gpu(torch, r, pd.shape))
    torch.cuda.synchronize()
    err = rel_err(z.cpu().numpy().reshape(prob.nt, -1), z_ref)
    # long lines are ill-conditioned (the condition grows as ny^2): a
    # backward-stable elimination leaves an error of order u times it
    tol = max(PREC_TOL[prec], 4 * UNIT_ROUNDOFF[prec] * line_condition(cfg))
    print(f"  rel err {err:.3e} tol {tol:.2e}")
    assert err < tol


# Time-FFT shapes: on a 16 x 8 grid (sine basis) these Nt select the
# four-step kernels with pencil lengths 4 .. 32 and tiles of 32, 16 and 8
# columns (Nt = 2048 in float32, and Nt = 512 and 1024 in float64, take the
# 512-thread workgroups), and the Stockham kernel below them and above them
# (Nt = 4096, and Nt = 2048 in float64: one complex column per workgroup,
# 98 KiB of LDS at Nt = 4096 in float64).
FFT_NT = {"fp32": [16, 64, 128, 256, 512, 2048, 4096], "fp64": [16, 64, 256, 512, 1024, 2048, 4096]}


@pytest.mark.parametrize("prec,nt", [(p, n) for p, ns in FFT_NT.items() for n in ns])
def test_time_fft_shapes(prec, nt):
    announce(f"fft shape nt={nt} {prec}")
    cfg = dict(dim=2, nx=16, ny=8, nt=nt, scheme="tr", T=1.0, nu=0.05, alpha=1e-2)
    torch, pd, prob = make(cfg, prec)
    r = np.random.default_rng(11).standard_normal((prob.nt, prob.nspace))
    z_ref = o_prec.three_steps(prob, r)
    z = pd.apply_precond(to_gpu(torch, r, pd.shape))
    torch.cuda.synchronize()
    err = rel_err(z.cpu().numpy().reshape(prob.nt, -1), z_ref)
    print(f"  rel err {err:.3e}")
    assert err < PREC_TOL[prec]


# The time FFTs over many tiles: 66 x 61 points (4026 = 251 x 16 + 10: a
# ragged last tile of the 16-column tiles) in a batch of 8 at Nt = 512, several
# thousand workgroups.  Batch entry b is (b + 1) r, so its result must be
# (b + 1) z: a tile read from or written to the wrong entry shows as a wrong
# scale.
_MANY_TILES = dict(dim=2, nx=66, ny=61, nt=512, scheme="tr", T=1.0, nu=0.05, ax=0.7, alpha=1e-2)


@functools.lru_cache(maxsize=1)
def _many_tiles_oracle():
    prob = Problem.from_kwargs(**_MANY_TILES)
    r = np.random.default_rng(21).standard_normal((prob.nt, prob.nspace))
    return r, o_prec.three_steps(prob, r)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_time_fft_many_tiles_batch(prec):
    announce(f"fft tiles 66x61 nt=512 batch 8 {prec}")
    torch, pd, prob = make(_MANY_TILES, prec, batch=8)
    r, z_ref = _many_tiles_oracle()
    rb = np.stack([(b + 1) * r for b in range(8)])
    z = pd.apply_precond(to_gpu(torch, rb, pd.shape)).cpu().numpy().reshape(8, prob.nt, -1)
    errs = [rel_err(z[b] / (b + 1), z_ref) for b in range(8)]
    print(f"  rel err max {max(errs):.3e}")
    assert max(errs) < PREC_TOL[prec]


def test_adjoint_solve_long_time():
    announce("adjoint nt=256 (time-reversed four-step transforms)")
    cfg = dict(dim=2, nx=16, ny=8, nt=256, scheme="be", T=1.0, nu=0.05, ax=0.5, ay=0.3, alpha=1e-2)
    torch, pd, prob = make(cfg, "fp64")
    g = np.random.default_rng(12).standard_normal((prob.nt, prob.nspace))
    lam, res = pd.adjoint_solve(to_gpu(torch, g, pd.shape), rtol=1e-12, max_iter=60)
    assert res.converged
    ref = o_adj.sequential_transpose(prob, g)
    assert rel_err(lam.cpu().numpy().reshape(prob.nt, -1), ref) < 1e-10


@pytest.mark.parametrize("case", ["1d-be", "2d-tr-schur", "2d-lf-dst", "2d-be-schur-ragged"])
def test_precond_in_place_and_batch(case):
    announce(f"precond batch/in-place {case}")
    torch, pd, prob = make(CASES[case], "fp64", batch=3)
    r = np.random.default_rng(2).standard_normal((3, prob.nt, prob.nspace))
    rg = to_gpu(torch, r, pd.shape)
    z = pd.apply_precond(rg)
    z_np = z.cpu().numpy().reshape(3, prob.nt, -1)
    for i in range(3):
        assert rel_err(z_np[i], o_prec.three_steps(prob, r[i])) < 1e-11
    pd.apply_precond(rg, out=rg)      # z == r allowed
    assert torch.equal(rg, z)


@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("case", list(CASES))
def test_matvec_parity(case, transpose):
    announce(f"matvec {case} T={transpose}")
    torch, pd, prob = make(CASES[case], "fp64")
    u = np.random.default_rng(3).standard_normal((prob.nt, prob.nspace))
    y = pd.matvec(to_gpu(torch, u, pd.shape), transpose=transpose).cpu().numpy().reshape(prob.nt, -1)
    ref = ops.apply_AT(prob, u) if transpose else ops.apply_A(prob, u)
    assert rel_err(y, ref) < 1e-13


@pytest.mark.parametrize("case", list(CASES))
def test_rhs_and_transpose_parity(case):
    announce(f"rhs {case}")
    torch, pd, prob = make(CASES[case], "fp64")
    rng = np.random.default_rng(4)
    S = prob.nspace
    U0, u1 = rng.standard_normal(S), rng.standard_normal(S)
    f = rng.standard_normal((prob.nt + 1, S))
    fs = (1, prob.ny, prob.nx)
    b = pd.build_rhs(to_gpu(torch, U0, fs), to_gpu(torch, u1, fs), to_gpu(torch, f, pd.source_shape))
    use_u1 = u1 if prob.scheme == "lf" else None
    assert rel_err(b.cpu().numpy().reshape(prob.nt, -1), o_rhs.build_rhs(prob, U0, use_u1, f)) < 1e-13
    lam = rng.standard_normal((prob.nt, S))
    gU0, gu1, gf = pd.rhs_transpose(to_gpu(torch, lam, pd.shape))
    rU0, ru1, rf = o_rhs.rhs_transpose(prob, lam)
    assert rel_err(gU0.cpu().numpy().ravel(), rU0) < 1e-13
    assert rel_err(gf.cpu().numpy().reshape(prob.nt + 1, -1), rf) < 1e-13
    if prob.scheme == "lf":
        assert rel_err(gu1.cpu().numpy().ravel(), ru1) < 1e-13


@pytest.mark.parametrize("case", list(CASES))
def test_fgmres_fp64_matches_sequential(case):
    announce(f"fgmres fp64 {case}")
    torch, pd, prob = make(CASES[case], "fp64")
    b = np.random.default_rng(5).standard_normal((prob.nt, prob.nspace))
    u, res = pd.solve(to_gpu(torch, b, pd.shape), rtol=1e-12, max_iter=60)
    assert res.converged, res
    ref = o_solve.sequential(prob, b)
    err = rel_err(u.cpu().numpy().reshape(prob.nt, -1), ref)
    print(f"  iters {res.iters} resid {res.rel_resid:.2e} err {err:.2e}")
    assert err < 1e-10
    assert res.rel_resid <= 1e-12


@pytest.mark.parametrize("prec", ["fp32", "fp32_bf16gemm", "fp32_bf16x1"])
@pytest.mark.parametrize("case", ["1d-be", "2d-tr-schur", "2d-lf-dst", "2d-be-schur-64"])
def test_fgmres_mixed_reaches_fp64_residual(case, prec):
    announce(f"fgmres {prec} {case}")
    if _bf16x1_schur(case, prec):
        pytest.skip("single-bf16 x-transform is refused with a Schur basis (see test_precond_parity)")
    torch, pd, prob = make(CASES[case], prec)
    b = np.random.default_rng(6).standard_normal((prob.nt, prob.nspace))
    u, res = pd.solve(to_gpu(torch, b, pd.shape), rtol=1e-10, max_iter=60)
    assert res.converged, res
    un = u.cpu().numpy().reshape(prob.nt, -1)
    true_res = np.linalg.norm(b - ops.apply_A(prob, un)) / np.linalg.norm(b)
    err = rel_err(un, o_solve.sequential(prob, b))
    print(f"  iters {res.iters} resid {res.rel_resid:.2e} true {true_res:.2e} err {err:.2e}")
    assert true_res <= 1.01e-10


@pytest.mark.parametrize("case", ["1d-be", "2d-tr-schur", "2d-lf-dst"])
def test_stationary_and_direct(case):
    announce(f"stationary/direct {case}")
    torch, pd, prob = make(CASES[case], "fp64", mode="stationary")
    b = np.random.default_rng(7).standard_normal((prob.nt, prob.nspace))
    bg = to_gpu(torch, b, pd.shape)
    u, res = pd.solve(bg, mode="stationary", rtol=1e-12, max_iter=50)
    assert res.converged
    assert rel_err(u.cpu().numpy().reshape(prob.nt, -1), o_solve.sequential(prob, b)) < 1e-10
    # linear convergence at about alpha/(1-alpha) per step (eq5.4)
    a = prob.alpha
    print(f"  stationary iters {res.iters} history {res.history}")
    assert res.iters <= 2 * int(np.ceil(np.log(1e-12) / np.log(a / (1 - a)))) + 2
    z, res_d = pd.solve(bg, mode="direct", rtol=1.0, max_iter=1)
    assert rel_err(z.cpu().numpy().reshape(prob.nt, -1), o_prec.three_steps(prob, b)) < 1e-11


@pytest.mark.parametrize("case", ["1d-be", "2d-tr-schur", "2d-lf-dst", "2d-be-schur-ragged"])
def test_adjoint_solve_matches_oracle(case):
    announce(f"adjoint {case}")
    torch, pd, prob = make(CASES[case], "fp64")
    g = np.random.default_rng(8).standard_normal((prob.nt, prob.nspace))
    lam, res = pd.adjoint_solve(to_gpu(torch, g, pd.shape), rtol=1e-12, max_iter=60)
    assert res.converged
    ref = o_adj.sequential_transpose(prob, g)
    assert rel_err(lam.cpu().numpy().reshape(prob.nt, -1), ref) < 1e-10


def test_batch_matches_single_solves():
    announce("batch independence")
    params = CASES["2d-tr-schur"]
    torch, pd3, prob = make(params, "fp64", batch=3)
    b = np.random.default_rng(9).standard_normal((3, prob.nt, prob.nspace))
    b[1] *= 1e-3   # different scales converge at different steps
    u3, r3 = pd3.solve(to_gpu(torch, b, pd3.shape), rtol=1e-12, max_iter=60)
    _, pd1, _ = make(params, "fp64", batch=1)
    for i in range(3):
        u1, r1 = pd1.solve(to_gpu(torch, b[i], pd1.shape), rtol=1e-12, max_iter=60)
        assert rel_err(u3[i].cpu().numpy(), u1[0].cpu().numpy()) < 1e-13
        assert r3.iters_per_rhs[i] == r1.iters


def test_batch_with_zero_rhs():
    # ||b|| of a zero-guess solve comes out of its first Arnoldi step: a zero
    # right-hand side in a batch must stay inactive (zero solution, no
    # iterations) while the others converge as when solved alone
    announce("batch with a zero right-hand side")
    params = CASES["2d-tr-schur"]
    torch, pd3, prob = make(params, "fp64", batch=3)
    b = np.random.default_rng(12).standard_normal((3, prob.nt, prob.nspace))
    b[1] = 0.0
    u3, r3 = pd3.solve(to_gpu(torch, b, pd3.shape), rtol=1e-12, max_iter=60)
    assert r3.converged
    assert float(u3[1].abs().max()) == 0.0
    assert r3.iters_per_rhs[1] == 0 and r3.resid_per_rhs[1] == 0.0
    assert r3.history[0] == 1.0
    _, pd1, _ = make(params, "fp64", batch=1)
    for i in (0, 2):
        u1, r1 = pd1.solve(to_gpu(torch, b[i], pd1.shape), rtol=1e-12, max_iter=60)
        assert rel_err(u3[i].cpu().numpy(), u1[0].cpu().numpy()) < 1e-13
        assert r3.iters_per_rhs[i] == r1.iters
        ref = o_solve.sequential(prob, b[i])
        assert rel_err(u3[i].cpu().numpy().reshape(prob.nt, -1), ref) < 1e-9


@pytest.mark.parametrize("adjoint", [False, True])
def test_mixed_batch_with_zero_rhs(adjoint):
    # the deferred right-hand-side norm in mixed precision, for A and A^T:
    # right-hand sides of very different scales and a zero one in one batch
    announce(f"mixed batch with a zero right-hand side, adjoint={adjoint}")
    torch, pd3, prob = make(CASES["2d-tr-schur"], "fp32_bf16gemm", batch=3)
    b = np.random.default_rng(14).standard_normal((3, prob.nt, prob.nspace))
    b[0] *= 1e4
    b[1] = 0.0
    b[2] *= 1e-4
    bg = to_gpu(torch, b, pd3.shape)
    solve = pd3.adjoint_solve if adjoint else pd3.solve
    u, res = solve(bg, rtol=1e-10, max_iter=60)
    assert res.converged, res
    assert float(u[1].abs().max()) == 0.0 and res.iters_per_rhs[1] == 0
    apply = ops.apply_AT if adjoint else ops.apply_A
    for i in (0, 2):
        un = u[i].cpu().numpy().reshape(prob.nt, -1)
        true_res = np.linalg.norm(b[i] - apply(prob, un)) / np.linalg.norm(b[i])
        print(f"  rhs {i}: iters {res.iters_per_rhs[i]} true residual {true_res:.2e}")
        assert true_res <= 1.01e-10


def test_zero_guess_start_variants():
    # the start from a zero guess has three forms: ||b|| deferred into the
    # first Arnoldi step (the usual one), a separate norm pass (rtol >= 1,
    # where the solve ends before any step) and an explicit zero x0 (the
    # restart path): they must agree
    announce("zero-guess start variants")
    params = CASES["2d-tr-schur"]
    torch, pd3, prob = make(params, "fp64", batch=3)
    b = np.random.default_rng(13).standard_normal((3, prob.nt, prob.nspace))
    b[2] = 0.0
    bg = to_gpu(torch, b, pd3.shape)
    u, res = pd3.solve(bg, rtol=1.5)
    assert res.converged and res.iters == 0 and float(u.abs().max()) == 0.0
    assert res.history[:1] == [1.0]
    ua, ra = pd3.solve(bg, rtol=1e-12, max_iter=60, restart=1)
    ub, rb = pd3.solve(bg, rtol=1e-12, max_iter=60, restart=1, x0=torch.zeros_like(bg))
    assert ra.converged and rb.converged
    assert ra.iters_per_rhs[2] == 0 and float(ua[2].abs().max()) == 0.0
    for i in (0, 1):
        assert rel_err(ua[i].cpu().numpy(), ub[i].cpu().numpy()) < 1e-10
        assert ra.iters_per_rhs[i] == rb.iters_per_rhs[i]
        ref = o_solve.sequential(prob, b[i])
        assert rel_err(ua[i].cpu().numpy().reshape(prob.nt, -1), ref) < 1e-9


def test_error_paths():
    announce("error paths")
    torch, pd, prob = make(CASES["2d-tr-schur"], "fp64")
    from paper_2005_09158_amd import ParaDiagError
    b = torch.zeros(pd.shape, dtype=torch.float64, device="cuda")
    b[0, 0, 0, 0] = float("nan")
    with pytest.raises(ParaDiagError) as e:
        pd.solve(b, rtol=1e-8)
    assert e.value.status == -5
    b = torch.randn(pd.shape, dtype=torch.float64, device="cuda")
    u, res = pd.solve(b, rtol=1e-14, max_iter=1)
    assert res.status == 1 and not res.converged and res.iters == 1
    assert np.isfinite(u.cpu().numpy()).all()
    # zero right-hand side: zero solution, converged without iterations
    u, res = pd.solve(torch.zeros_like(b), rtol=1e-8)
    assert res.converged and float(u.abs().max()) == 0.0
    assert res.iters == 0 and res.history[:1] == [0.0] and res.rel_resid == 0.0
    # workspace too small for a longer restart than bound
    with pytest.raises(ParaDiagError) as e:
        pd.solve(b, rtol=1e-8, restart=30)
    assert e.value.status == -3


def test_gradient_autograd_matches_oracle():
    announce("autograd gradient")
    params = dict(dim=2, nx=12, ny=10, nt=16, scheme="be", T=1.0, nu=5e-2, ax=1.0, ay=0.5, alpha=1e-3)
    torch, pd, prob = make(params, "fp64")
    from paper_2005_09158_amd import ParaDiagSolve
    rng = np.random.default_rng(10)
    S = prob.nspace
    U0 = rng.standard_normal(S)
    f = rng.standard_normal((prob.nt + 1, S))
    target = rng.standard_normal(S)
    beta = 1e-4
    U0g = to_gpu(torch, U0, pd.field_shape).requires_grad_(True)
    fg = to_gpu(torch, f, pd.source_shape).requires_grad_(True)
    tg = to_gpu(torch, target, pd.field_shape)
    u = ParaDiagSolve.apply(pd, U0g, fg, 1e-13)
    J = 0.5 * ((u[:, -1] - tg) ** 2).sum() + 0.5 * beta * (fg ** 2).sum()
    J.backward()
    Jr, gU0r, gfr = o_adj.gradient(prob, U0, f, target, beta)
    assert abs(J.item() - Jr) <= 1e-10 * abs(Jr)
    assert rel_err(U0g.grad.cpu().numpy().ravel(), gU0r) < 1e-9
    assert rel_err(fg.grad.cpu().numpy().reshape(prob.nt + 1, -1), gfr) < 1e-9


def test_initial_guess_and_restarts():
    """A warm start (use_x0) and a restart length that forces several cycles
    both reach the oracle's solution; the first cycle from a zero guess
    starts from V_0 = b without writing u until its first update."""
    announce("initial guess and restarts")
    torch, pd, prob = make(CASES["2d-tr-schur"], "fp32", restart=2)
    b = np.random.default_rng(11).standard_normal((prob.nt, prob.nspace))
    bg = to_gpu(torch, b, pd.shape)
    ref = o_solve.sequential(prob, b)
    u, res = pd.solve(bg, rtol=1e-10, max_iter=60, restart=2)
    assert res.converged
    assert rel_err(u.cpu().numpy().reshape(prob.nt, -1), ref) < 1e-8
    # warm start from a perturbed solution: converges, and to the same answer
    x0 = u + 1e-3 * torch.randn_like(u)
    u2, res2 = pd.solve(bg, rtol=1e-10, max_iter=60, restart=2, x0=x0)
    assert res2.converged
    assert rel_err(u2.cpu().numpy().reshape(prob.nt, -1), ref) < 1e-8
    # warm start from the solution itself: no iteration needed
    u3, res3 = pd.solve(bg, rtol=1e-8, max_iter=60, restart=2, x0=u)
    assert res3.converged and res3.iters == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32_bf16gemm"])
@pytest.mark.parametrize("m", [1, 2, 5, 8, 11])
def test_solution_update_lengths(m, prec):
    """One FGMRES cycle of exactly m iterations (the solution update then sums
    m preconditioned vectors: the vectorised kernel up to 8, the generic one
    beyond).  The true residual of the returned u, evaluated by the oracle,
    must equal the cycle's least-squares residual estimate (exact in exact
    arithmetic for flexible GMRES, whose relation A Z = V H holds for the
    stored Z of either precision) down to a float64 rounding floor, and the
    residual the solver reports.  alpha = 0.5 (a weaker preconditioner) keeps
    the first iterations' residuals above that floor."""
    announce(f"solution update m={m} {prec}")
    params = dict(CASES["2d-tr-schur"], alpha=0.5)
    torch, pd, prob = make(params, prec, restart=m)
    b = np.random.default_rng(12).standard_normal((prob.nt, prob.nspace))
    u, res = pd.solve(to_gpu(torch, b, pd.shape), rtol=1e-30, max_iter=m, restart=m)
    assert not res.converged and res.iters == m
    un = u.cpu().numpy().reshape(prob.nt, -1)
    true_res = np.linalg.norm(b - ops.apply_A(prob, un)) / np.linalg.norm(b)
    est = res.history[m]            # estimate after the m-th iteration
    print(f"  est {est:.6e} true {true_res:.6e} reported {res.rel_resid:.6e}")
    assert abs(true_res - est) <= 1e-7 * est + 1e-12
    assert abs(res.rel_resid - true_res) <= 1e-9 * true_res + 1e-14


def test_stage_timing_selection():
    announce("stage timing selection")
    torch, pd, prob = make(CASES["2d-tr-schur"], "fp32")
    r = torch.randn(pd.shape, dtype=torch.float64, device="cuda")
    pd.set_timing(True, stages=["fft_fwd", "line_solve"])
    pd.stage_times(reset=True)
    pd.apply_precond(r)
    st = pd.stage_times(reset=True)
    assert st["fft_fwd"][1] == 1 and st["line_solve"][1] == 1
    assert all(v[1] == 0 for k, v in st.items() if k not in ("fft_fwd", "line_solve"))
    pd.set_timing(True)
    pd.apply_precond(r)
    st = pd.stage_times(reset=True)
    assert all(st[k][1] == 1 for k in ("fft_fwd", "xform_fwd", "line_solve", "xform_inv", "fft_inv"))
    pd.set_timing(False)
    pd.apply_precond(r)
    assert all(v[1] == 0 for v in pd.stage_times(reset=True).values())
    # a selector with bits past the last stage is rejected
    assert pd.lib.paradiag_set_timing(pd.plan, 1 << 12) == -1
