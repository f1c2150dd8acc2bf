/*
 * paradiag.h - C ABI of the ParaDiag-II all-at-once solver for gfx950.
 *
 * Problem (Gander, Liu, Wu, Yue, Zhou, "ParaDiag: parallel-in-time algorithms
 * based on the diagonalization technique", Section 1, eq1.1): solve
 *
 *     A u = b,   A = B1 (x) I + B2 (x) K,
 *
 * for all Nt time steps at once, where K is the finite-difference spatial
 * operator of a linear advection-diffusion equation (eq2.2b, homogeneous
 * Dirichlet data on [0,1]^d, d = 1 or 2) or of the wave equation (eq3.1), and
 * B1, B2 are the lower-triangular Toeplitz time matrices of backward Euler,
 * the trapezoidal rule (eq2.5b) or implicit leap-frog (eq3.2b).
 *
 * Method: the alpha-circulant preconditioner P_alpha = C1 (x) I + C2 (x) K
 * (eq1.2, eq2.11b, eq3.4) is applied by the three steps of eq1.3 / eq2.12:
 * a scaled FFT along time (Step-(a)), independent complex shifted spatial
 * solves per frequency (Step-(b)) and the inverse scaled FFT (Step-(c)).  It
 * is used inside flexible GMRES, as a stationary iteration (eq5.1) and as a
 * one-shot solve; the transposed system A^T lam = g is solved by the same
 * machinery on time-reversed data with K^T.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layout.  All-at-once vectors are device float64 arrays [batch][nt][ny][nx]
 *   (x fastest) holding U_1 .. U_Nt.  Spatial fields (U0, u1) are
 *   [batch][ny][nx]; a source f is [batch][nt+1][ny][nx] sampled at t_0..t_Nt.
 *   ny = 1 for one space dimension.  Pointers must be 8-byte aligned.
 * Ownership.  The caller owns every vector and the workspace (device memory
 *   obtained from any allocator, e.g. PyTorch's).  A plan owns host tables
 *   and, from its first solve on, a small pinned host buffer for the solvers'
 *   per-step scalars (freed by paradiag_destroy); its device tables live
 *   inside the bound workspace.  The library allocates no device memory at
 *   run time; its code object holds one static array per device, used only by
 *   paradiag_apply_precond_static.  A
 *   plan is not thread-safe, and two solves with one plan must not overlap
 *   in time, even on different streams (they share that buffer).
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  Every
 *   call is ordered on that stream.  matvec, apply_precond and build_rhs only
 *   enqueue work; solve and adjoint_solve synchronise the stream once per
 *   Krylov step and return after `info` is filled.
 * Aliasing.  Inputs and outputs must not overlap, except apply_precond which
 *   allows z == r.
 * Errors.  No C++ exception crosses the ABI.  A negative status means the
 *   outputs are undefined; paradiag_last_error() returns a message for the
 *   last non-OK status of the calling thread.
 */
#ifndef PARADIAG_H
#define PARADIAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct paradiag_plan_s* paradiag_plan;

typedef enum {
  PD_OK = 0,
  PD_NOT_CONVERGED = 1,     /* outputs valid: best iterate and its residual */
  PD_ERR_INVALID = -1,      /* bad argument (sizes, alpha outside (0,1], NULL, aliasing) */
  PD_ERR_UNSUPPORTED = -2,  /* valid problem outside the implemented range */
  PD_ERR_WORKSPACE = -3,    /* no workspace bound, or too small for the request */
  PD_ERR_HIP = -4,          /* a HIP runtime call failed */
  PD_ERR_NONFINITE = -5,    /* NaN/Inf in the right-hand side or in Krylov scalars */
  PD_ERR_BREAKDOWN = -6     /* singular pivot in setup or a Krylov breakdown */
} paradiag_status;

/* PD_HYBRID, PD_HYBRID_WAVE: ParaDiag-I with the hybrid time discretisation
 * of Section 2.1.2 (explicit midpoint for the first Nt - 1 steps, backward
 * Euler for the last, neq2.9a).  The all-at-once matrix is A = B (x) I + I (x) K
 * (neq2.9b, B of neq2.9c) for u' + K u = f, and A = B^2 (x) I + I (x) K
 * (neq2.15) for the second-order problem u'' + K u = f with the velocity
 * eliminated.  B = V D V^{-1} in closed form (Thm thmCondU), so
 * paradiag_apply_precond computes A^{-1} r exactly (up to rounding): Step-(a)
 * and Step-(c) are dense float64 products with V^{-1} and V on MFMA instead of
 * FFTs, Step-(b) solves (d_n I + K) per eigenvalue d_n of B (or B^2).  alpha
 * is unused; nt must be even (any even value in [4, 4096]).  Supported: matvec
 * (and its transpose), build_rhs, apply_precond, solve in PD_MODE_DIRECT and
 * PD_MODE_STATIONARY (iterative refinement; one step suffices in float64);
 * PD_MODE_FGMRES, adjoint_solve and rhs_transpose return PD_ERR_UNSUPPORTED. */
typedef enum { PD_BE = 0, PD_TR = 1, PD_LEAPFROG = 2, PD_HYBRID = 3, PD_HYBRID_WAVE = 4 } paradiag_scheme;

/* Arithmetic of the preconditioner.  The all-at-once residual, the matvec,
 * the Krylov vectors, the Arnoldi process and the alpha-scaling tables are
 * float64 in every mode. */
typedef enum {
  PD_PREC_FP64 = 0,           /* FFT, x-transform and line solves in float64 */
  PD_PREC_FP32 = 1,           /* FFT, x-transform and line solves in float32 */
  PD_PREC_FP32_BF16GEMM = 2,  /* as FP32; x-transform on bf16 MFMA with fp32 accumulation,
                                 operands split into three bf16 parts (six products:
                                 float32-level accuracy at bf16 instruction rate) */
  PD_PREC_FP32_BF16X1 = 3     /* as FP32; x-transform as one bf16 product (fastest, least
                                 accurate).  Symmetric K_x only (sine basis): with a
                                 non-normal K_x setup returns PD_ERR_UNSUPPORTED, since
                                 the back-substitution over the Schur factor carries the
                                 bf16 rounding into an error of order one */,
  PD_PREC_FP32_FP16GEMM = 4   /* as FP32; x-transform on fp16 MFMA with fp32 accumulation:
                                 each row scaled by a power of two (its largest entry
                                 near 2^14), both operands split into two fp16 parts,
                                 three products (about 22 significant bits) */
} paradiag_prec;

typedef enum {
  PD_MODE_FGMRES = 0,      /* flexible GMRES(restart) preconditioned by P_alpha */
  PD_MODE_STATIONARY = 1,  /* u <- u + P_alpha^{-1}(b - A u)  (eq5.1) */
  PD_MODE_DIRECT = 2,      /* u = P_alpha^{-1} b once (solution of the alpha-circulant system) */
  PD_MODE_PARAREAL = 3,    /* workspace sizing of paradiag_parareal (not a paradiag_solve mode) */
  PD_MODE_NONLINEAR = 4    /* workspace sizing of paradiag_nonlinear_solve (not a paradiag_solve mode) */
} paradiag_mode;

typedef struct {
  int32_t dim;        /* 1 or 2 */
  int32_t nx, ny;     /* interior points per direction; ny = 1 when dim = 1; nx, ny in [1, 2048]
                       (nx <= 1024 when ax != 0: host Schur cost) */
  int32_t nt;         /* time steps: a power of two in [4, 4096] (hybrid schemes: even, [4, 4096]) */
  int32_t batch;      /* independent right-hand sides, 1..64 */
  int32_t scheme;     /* paradiag_scheme */
  int32_t prec;       /* paradiag_prec */
  int32_t reserved;   /* must be 0 */
  double T;           /* final time; dt = T / nt */
  double nu;          /* diffusion coefficient (c^2 for the wave equation), > 0 */
  double ax, ay;      /* velocity (0 for the wave equation); |a| h / (2 nu) < 1 required */
  double alpha;       /* alpha-circulant parameter in (0, 1] */
} paradiag_problem;

typedef struct {
  int32_t mode;       /* paradiag_mode */
  int32_t restart;    /* FGMRES cycle length m, 1..32 (ignored otherwise) */
  int32_t max_iter;   /* total preconditioner applications allowed, >= 1 */
  int32_t use_x0;     /* 1: u holds the initial guess on entry; 0: start from zero */
  double rtol;        /* target ||b - A u||_2 / ||b||_2 per right-hand side, > 0 */
} paradiag_solve_opts;

typedef struct {
  int32_t iters;          /* preconditioner applications performed */
  int32_t converged;      /* 1 if every right-hand side met rtol */
  double rel_resid;       /* max over the batch of the final true relative residual */
  int32_t* iters_per_rhs; /* optional, caller-owned arrays of length batch (may be NULL) */
  double* resid_per_rhs;
  double* history;        /* optional caller-owned array: max relative residual estimate per step */
  int32_t history_cap;    /* capacity of history */
  int32_t history_len;    /* entries written */
} paradiag_solve_info;

/* Validate the problem and build host tables: the time symbols
 * lambda_j = fft(Gamma_alpha c_j) of Lemma 1, the Gamma_alpha table
 * (alpha^{n/Nt}), FFT twiddles, and the x-direction basis of K_x: the sine
 * basis when K_x is symmetric, otherwise a unitary complex Schur form
 * K_x = Q T Q^H computed on the host in float64.  Host only: no device call.
 * Returns PD_ERR_INVALID / PD_ERR_UNSUPPORTED for a problem outside the
 * stated ranges; *out is NULL then. */
paradiag_status paradiag_setup(const paradiag_problem* prob, paradiag_plan* out);

/* Bytes of device workspace needed for calls with `opts` (opts may be NULL:
 * enough for matvec, apply_precond, build_rhs and rhs_transpose; solves need
 * the size for their mode and restart).  Host only. */
paradiag_status paradiag_workspace_size(paradiag_plan plan, const paradiag_solve_opts* opts,
                                        size_t* bytes);

/* Hand the plan a device workspace of `bytes` bytes (256-byte aligned) and
 * upload the device tables into it on `stream`.  The caller keeps ownership
 * and must keep it alive until the plan is destroyed or rebound. */
paradiag_status paradiag_bind_workspace(paradiag_plan plan, void* workspace, size_t bytes,
                                        void* stream);

/* b = all-at-once right-hand side from U0, the initial velocity u1 (leap-frog
 * and PD_HYBRID_WAVE only; NULL = 0) and the source f (NULL = 0).
 * theta-method: b_1 = (I/dt - (1-theta)K)U0 + theta f_1 + (1-theta) f_0,
 * b_n = theta f_n + (1-theta) f_{n-1} (eq2.5 with a source); leap-frog: first
 * two rows from the scheme at t_0 with a central ghost value (eq3.2).
 * PD_HYBRID: b_n = f_n, plus U0/(2 dt) in row 1 (neq2.9c); PD_HYBRID_WAVE:
 * b_n = f_n, plus u1/(2 dt) in row 1 and -U0/(4 dt^2) in row 2 (the first-order
 * system neq2.14b with the velocity eliminated). */
paradiag_status paradiag_build_rhs(paradiag_plan plan, const double* U0, const double* u1,
                                   const double* f, double* b, void* stream);

/* Transpose of the map (U0, u1, f) -> b applied to lam [batch][nt][ny][nx]:
 * gU0 [batch][ny][nx], gu1 [batch][ny][nx] (may be NULL), gf
 * [batch][nt+1][ny][nx] (may be NULL).  Used for gradients. */
paradiag_status paradiag_rhs_transpose(paradiag_plan plan, const double* lam, double* gU0,
                                       double* gu1, double* gf, void* stream);

/* y = A u (eq1.1), float64.  transpose != 0 gives y = A^T u. */
paradiag_status paradiag_matvec(paradiag_plan plan, const double* u, double* y, int32_t transpose,
                                void* stream);

/* z = P_alpha^{-1} r by Step-(a), (b), (c) of eq2.12, in the plan's
 * preconditioner precision (input and output float64).  z == r allowed. */
paradiag_status paradiag_apply_precond(paradiag_plan plan, const double* r, double* z,
                                       void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): z =
 * P_alpha^{-1} r computed exactly as by paradiag_apply_precond (same kernels,
 * same arithmetic), but with the two spectral buffers of Step-(a)..(c) in a
 * static device array of PD_STATIC_SCRATCH_BYTES per device instead of the
 * bound workspace.  The call allocates nothing (no hipMalloc, hipFree or
 * event creation) and records no stage timing.  The plan must still be bound
 * (its tables live in the workspace).  Limit: twice the plan's spectral buffer
 * (batch * (nt/2+1) * nx * ny complex values in the preconditioner precision,
 * 256-byte aligned) must fit in PD_STATIC_SCRATCH_BYTES, else
 * PD_ERR_WORKSPACE.  The array is shared by every call on one GPU and keeps
 * the last call's contents (no call relies on it starting at zero): calls that
 * overlap in time on one GPU, with any plans and on any streams, race.
 * z == r allowed. */
#define PD_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
paradiag_status paradiag_apply_precond_static(paradiag_plan plan, const double* r, double* z,
                                              void* stream);

/* Solve A u = b per opts->mode.  u: in = initial guess if opts->use_x0,
 * out = solution.  Returns PD_NOT_CONVERGED (u = last iterate) when max_iter
 * is reached first.  b is read throughout the solve (from a zero guess the
 * first Krylov vector is b itself); u overlapping b is PD_ERR_INVALID. */
paradiag_status paradiag_solve(paradiag_plan plan, const double* b, double* u,
                               const paradiag_solve_opts* opts, paradiag_solve_info* info,
                               void* stream);

/* ParaDiag-II parareal variant (Section 2.2.2, eq2.15): parareal for
 * u' + K u = 0, u(0) = U0, on the plan's coarse grid of nt intervals of
 * dT = T / nt, with the fine propagator F = J backward Euler steps of dT / J
 * and the coarse-grid correction applied to the alpha-periodic problem
 * u(0) = alpha u(T) (Thm the1.3: the same contraction as classical parareal
 * for alpha below about 0.3).  Iteration k: Ut_n = F(U^{k-1}_{n-1}) for all n at
 * once (U^{k-1}_0 = U0), then
 *   (C1^(alpha) (x) I + I (x) K) u^k = b^k,
 *   b^k_n = (I/dT + K) Ut_n - (n == 1 ? alpha U^{k-1}_nt : U^{k-1}_{n-1}) / dT,
 * whose matrix is P_alpha of backward Euler, solved by the three steps of
 * eq2.12.  The plan must use PD_BE in one space dimension (others:
 * PD_ERR_UNSUPPORTED) and be bound with a workspace sized for
 * PD_MODE_PARAREAL; opts->mode must be PD_MODE_PARAREAL.
 * U0: [batch][nx] device float64.  u: [batch][nt][nx]; in = the initial
 * iterate when opts->use_x0 (else zero), out = the last iterate, approximating
 * the fine solution at t_1 .. t_nt.  Iterates until the relative change
 * ||u^k - u^{k-1}||_2 / ||u^k||_2 <= opts->rtol for every right-hand side or
 * opts->max_iter iterations (PD_NOT_CONVERGED); info->rel_resid and
 * info->history report that relative change.  J in [1, 65536]. */
paradiag_status paradiag_parareal(paradiag_plan plan, const double* U0, int32_t J, double* u,
                                  const paradiag_solve_opts* opts, paradiag_solve_info* info,
                                  void* stream);

/* Optimal control of the wave equation (Section 4).  Setup of the plan of
 * the gamma-scaled optimality system
 *   A x = b,  x = [sqrt(gamma) u; p],
 *   A = [[B1, -s Ih], [s Ic, B1^T]] (x) I + (dt^2/2) blkdiag(B2, B2^T) (x) K,
 * B1 = Toeplitz(1, -2, 1), B2 = Toeplitz(1, 0, 1) (implicit leap-frog, dt = T/nt),
 * Ih = diag(1/2, 1, .., 1), Ic = diag(1, .., 1, 1/2), s = dt^2 / sqrt(gamma), K the
 * spatial operator of `prob` (nu times the negative Laplacian; prob->scheme
 * must be PD_LEAPFROG, ax = ay = 0, batch 1), u = u(t_1 .. t_nt) the state and
 * p = p(t_0 .. t_{nt-1}) the adjoint.  The plan's vectors are [2][nt][ny][nx]
 * (x1 = sqrt(gamma) u, then x2 = p).  Its preconditioner (apply_precond, and
 * inside paradiag_solve) is the block circulant P of Section 4 (B1, B2 replaced
 * by their circulants, Ih, Ic by I), applied as in Thm the4: DFTs of both
 * fields along time (dense float64 products on MFMA: nt need not be a power
 * of two), a 2 x 2 mixing per frequency with perfectly conditioned
 * eigenvectors, 2 (nt/2 + 1) shifted solves (Sigma_n I + dt^2/2 K), the
 * unmixing with C2^{-1}, and the inverse DFTs.  nt must not be divisible by 4
 * (C2 is singular then), 3 <= nt <= 4096.  Supported afterwards:
 * workspace_size, bind_workspace, matvec (not the transpose), apply_precond
 * (and _static), solve in every mode, oc_build_rhs; build_rhs, rhs_transpose
 * and adjoint_solve return PD_ERR_UNSUPPORTED. */
paradiag_status paradiag_oc_setup(const paradiag_problem* prob, double gamma, paradiag_plan* out);

/* b = [sqrt(gamma) fh; gh] of the optimal-control plan from the data of
 * Section 4: fh = dt^2 times the implicit leap-frog rows of the state
 * equation with u(0) = U0, u_t(0) = u1 (NULL = 0) and source f
 * ([nt+1][ny][nx] at t_0..t_nt, NULL = 0), as paradiag_build_rhs builds them for
 * PD_LEAPFROG; gh_m = dt^2 g(t_{m+1}) with the last row halved (g [nt+1][ny][nx],
 * NULL = 0).  b: [2][nt][ny][nx]. */
paradiag_status paradiag_oc_build_rhs(paradiag_plan plan, const double* U0, const double* u1,
                                      const double* f, const double* g, double* b, void* stream);

/* Pointwise cubic reaction g(u) = k1 u + k2 u^2 + k3 u^3 of paradiag_nonlinear_solve
 * (Allen-Cahn: k1 = -1/eps^2, k2 = 0, k3 = 1/eps^2). */
typedef struct { double k1, k2, k3; } paradiag_cubic;

/* Nonlinear ParaDiag (eq1.4, eq1.5) with windowing: u' + K u + g(u) = 0,
 * u(0) = U0, theta-method (PD_BE or PD_TR), so the all-at-once system of one
 * window is (B1 (x) I) u + (B2 (x) I) F(u) = b with F(U) = K U + g(U) and
 * b_1 = U0/dt - (1-theta) F(U0).  Each window runs the simplified Newton
 * iteration u <- u + P_alpha(u)^{-1} R(u), R(u) = b - (B1 (x) I) u - (B2 (x) I) F(u),
 * P_alpha(u) = C1^(alpha) (x) I + C2^(alpha) (x) (K + cbar I), where cbar is the
 * mean of g'(U_n) over every time step and grid point (the averaged Jacobian,
 * averaged over space too so that Step-(b) stays a shifted solve: lambda1_n
 * becomes lambda1_n + cbar lambda2_n), starting from U_n = U0 for every n.  It
 * stops when ||R(u)||_2 <= opts->rtol ||b||_2 or after opts->max_iter
 * corrections.  Window w starts from the last state of window w-1 (windowing
 * as at the end of Section 1).  batch must be 1; opts->mode must be
 * PD_MODE_NONLINEAR (workspace sizing); opts->use_x0: window 0 starts from u
 * instead of U0.  U0: [1][ny][nx]; u: [windows][1][nt][ny][nx].  info->iters =
 * corrections over all windows, info->rel_resid = the largest final relative
 * residual, info->history = the relative residual before every correction and
 * at the end of each window.  The plan's time symbols (and line factors) are
 * restored before returning.  Returns PD_NOT_CONVERGED when a window misses
 * rtol (later windows still run). */
paradiag_status paradiag_nonlinear_solve(paradiag_plan plan, const paradiag_cubic* g, const double* U0,
                                         int32_t windows, double* u, const paradiag_solve_opts* opts,
                                         paradiag_solve_info* info, void* stream);

/* Solve A^T lam = g.  Uses A^T = (J (x) I)(B1 (x) I + B2 (x) K^T)(J (x) I) with J
 * the time reversal (Toeplitz and alpha-circulant matrices are persymmetric),
 * so the same preconditioned iteration runs on reversed data with K^T. */
paradiag_status paradiag_adjoint_solve(paradiag_plan plan, const double* g, double* lam,
                                       const paradiag_solve_opts* opts,
                                       paradiag_solve_info* info, void* stream);

/* Copy the host x-basis of the plan: q and t receive nx*nx complex float64
 * values (interleaved re, im; row-major) with K_x = Q T Q^H (adjoint != 0:
 * the basis of K_x^T).  Host only; for inspection and tests. */
paradiag_status paradiag_get_xbasis(paradiag_plan plan, int32_t adjoint, double* q, double* t);

/* Copy the host time symbols lambda_1, lambda_2 for n = 0..nt/2 (interleaved
 * complex float64, nt/2+1 values each).  Hybrid schemes: the nt/2 eigenvalues
 * d_n of B (or B^2) with Re(x_n) > 0 in lambda_1 (the others are their
 * conjugates) and 1 in lambda_2.  Host only. */
paradiag_status paradiag_get_symbols(paradiag_plan plan, double* lam1, double* lam2);

/* Stage timing.  When enabled, every later call records HIP events around
 * each kernel launch of the selected stages on the call's own stream.
 * paradiag_set_timing: enable = 0 turns timing off, 1 times every stage,
 * and a value >= 2 is a stage mask shifted left by one (bit s + 1 selects
 * PD_STAGE s), so that a single stage can be timed with the fewest events;
 * values with bits beyond the last stage return PD_ERR_INVALID.
 * paradiag_get_stage_times
 * returns, per stage (PD_STAGE_*), the summed milliseconds, the launch count
 * and the algorithmic work of those launches since the last reset: bytes
 * that must cross HBM at least once (inputs read once, outputs written once)
 * and floating-point operations.  It synchronises on the recorded events.
 * Any output pointer may be NULL. */
enum {
  PD_STAGE_FFT_FWD = 0,    /* Step-(a): scaled real-to-complex FFT along time */
  PD_STAGE_XFORM_FWD = 1,  /* Step-(b): x-transform GEMM into the x basis */
  PD_STAGE_LINE_SOLVE = 2, /* Step-(b): y line solves (or the Schur back-sweep) */
  PD_STAGE_XFORM_INV = 3,  /* Step-(b): x-transform GEMM back */
  PD_STAGE_FFT_INV = 4,    /* Step-(c): complex-to-real FFT along time, scaled */
  PD_STAGE_MATVEC = 5,     /* all-at-once matvec (optionally fused b - A u) */
  PD_STAGE_DOT = 6,        /* Krylov multi-dot products */
  PD_STAGE_UPDATE = 7,     /* Krylov vector updates (fused with the next dots) */
  PD_STAGE_OTHER = 8,      /* reductions of partial sums, solution update, copies */
  PD_STAGE_FINE = 9,       /* parareal: the J fine steps of every coarse interval */
  PD_STAGE_REACTION = 10,  /* nonlinear solve: reaction term, residual norm, mean slope */
  PD_NUM_STAGES = 11
};
paradiag_status paradiag_set_timing(paradiag_plan plan, int32_t enable);
paradiag_status paradiag_get_stage_times(paradiag_plan plan, double* ms, int64_t* counts,
                                         double* bytes, double* flops, int32_t reset);

void paradiag_destroy(paradiag_plan plan);
const char* paradiag_last_error(void);
const char* paradiag_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PARADIAG_H */
