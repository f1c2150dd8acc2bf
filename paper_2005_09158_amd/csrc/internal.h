// Internal declarations of the ParaDiag-II library (not part of the ABI).
#pragma once

#include <complex>
#include <map>
#include <mutex>
#include <utility>
#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/paradiag.h"

namespace pd {

// Raises a kernel's dynamic-LDS limit to `bytes` on the current device.  The
// runtime call is made once per (device, kernel) and size, not per launch: on
// a drained queue its cost shows up as idle time before the kernel.
inline void lds_limit(const void* fn, size_t bytes) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, size_t> done;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lock(mu);
  size_t& cur = done[{dev, fn}];
  if (bytes > cur) {
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    cur = bytes;
  }
}


using cd = std::complex<double>;

bool complex_schur(int n, std::vector<cd>& h, std::vector<cd>& q);

// Eigendecomposition of the hybrid time matrix B (or B^2 for order 2) on the
// half set of eigenvalues Re x > 0 (the others are their conjugates):
//   d[n]            eigenvalue of B (order 1) or B^2 (order 2), n < nt/2
//   wf[(2n+c)][l]   real (c = 0) and imaginary (c = 1) parts of V^{-1}[n][l]
//   wi[l][(2n+c)]   2 Re V[l][n] (c = 0) and -2 Im V[l][n] (c = 1), so that
//                   sum_c wi[l][2n+c] (S_n)_c = 2 Re(V[l][n] S_n)
//   band[r][k+2]    entry (r, r+k) of B or B^2, |k| <= 2
struct HybridTables {
  std::vector<cd> d;
  std::vector<double> wf, wi, band;
  double inverse_error = 0.0;
};
bool hybrid_eigen(int nt, double dt, int order, HybridTables& out, std::string& err);

// Workgroup order for the chip's 8 XCDs.  The dispatcher deals consecutive
// workgroup ids round-robin to the XCDs, each with its own L2; renumbering
// id -> (id mod 8) * share + id / 8 hands every XCD one contiguous range of
// tiles, so workgroups that read or write neighbouring pieces of the same
// cache lines (adjacent columns of a row, the rows of a stencil) share an L2
// while they run.  A bijection of [0, total) for every total.
__device__ __forceinline__ unsigned xcd_order(unsigned id, unsigned total) {
  const unsigned q = total >> 3, rem = total & 7, x = id & 7, i = id >> 3;
  return x < rem ? x * (q + 1) + i : rem * (q + 1) + (x - rem) * q + i;
}

// This workgroup's (x, y, z) grid position after xcd_order.
struct BlockPos { int x, y, z; };
__device__ __forceinline__ BlockPos xcd_block() {
  const unsigned gx = gridDim.x, gy = gridDim.y;
  const unsigned id = xcd_order(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
  return BlockPos{(int)(id % gx), (int)((id / gx) % gy), (int)(id / (gx * gy))};
}

// Numeric formats of the preconditioner.
// BF16: operands split into three bf16 parts (six bf16 MFMAs per product);
// BF16X1: single bf16 product.
enum class Prec { F64 = 0, F32 = 1, BF16 = 2, BF16X1 = 3, F16 = 4 };
// PD_PREC_FP32_FP16GEMM: the x-transform matrices are stored times this power
// of two (their entries are at most 1 in magnitude) before the fp16 split
constexpr float F16_BSCALE = 16384.0f;

// Geometry of the spectral buffer [batch][F][sy][2][sx]: F = nt/2 + 1
// frequencies, each slice a sy x sx complex field stored row-planar (a row
// of sx real parts followed by sx imaginary parts).  In 2D (sy, sx) =
// (ny, nx); in 1D the single line of nx points is stored as (sy, sx) =
// (nx, 1) so that Step-(b) always solves along the "y" index.
struct Geom {
  int B, nt, F;
  int nx, ny;     // physical grid
  int sx, sy;     // spectral slice shape
  int64_t S;      // nx * ny
  int64_t N1;     // nt * S: one right-hand side
  int64_t NA;     // B * N1
  int64_t spec_elems;  // B * F * sy * 2 * sx
};

// Tables of one spatial operator (K, or K^T for the adjoint).
struct SpaceOp {
  // 5-point stencil of K at a point: K u = sxl u[x-1] + sxu u[x+1] + syl u[y-1] + syu u[y+1] + sd u
  double sxl, sxu, syl, syu, sd;
  // line operator solved in Step-(b) along the spectral y index: tridiag(lo, di, up)
  double lo, di, up;
  // x-direction basis (2D): per-mode shift t_k (complex), GEMM matrices stored
  // transposed ([N][K], K contiguous) in the compute format, upper part of T.
  const double2* tk = nullptr;
  const void* g_fwd = nullptr;  // S -> S * conj(Q)
  const void* g_inv = nullptr;  // W -> W * Q^T
  const void* tup = nullptr;    // Schur T (planar re/im, [2][nx][nx], compute format); null if diagonal
  void* lu = nullptr;           // Schur path: inverse LU pivots of every line, [F][nx][ny] complex
  // windowed back-sweep: the real block form of T for the far-coupling product,
  // times the power of two tfar_scale, as two fp16 parts (hi, lo),
  // [2][2 nx][2 nx] (see sweep_windowed); tfar_inv = 1 / tfar_scale
  const void* tfar = nullptr;
  float tfar_inv = 1.f;
  // host copies
  std::vector<cd> Q, Tm;        // nx*nx complex (row-major): K_x = Q T Q^H
};

struct Workspace;

struct StageTimer {
  bool enabled = false;
  unsigned mask = 0;   // stages timed while enabled (bit = stage)
  struct Rec { int stage; hipEvent_t a, b; };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  double ms[PD_NUM_STAGES] = {0};
  int64_t count[PD_NUM_STAGES] = {0};
  double bytes[PD_NUM_STAGES] = {0};
  double flops[PD_NUM_STAGES] = {0};
};

struct Plan {
  paradiag_problem p;
  Geom g;
  Prec prec;
  bool schur = false;     // non-normal x factor: Schur back-sweep in Step-(b)
  // sine basis with nx + 1 a power of two: the x-transform is a DST-I computed
  // by an FFT of length 2 (nx + 1) instead of the dense product
  bool dst = false;
  void* d_dtw = nullptr;  // exp(-2 pi i k / (2 (nx + 1))), k < nx + 1, compute precision
  float* d_rowscale = nullptr;  // PD_PREC_FP32_FP16GEMM: power-of-two scale of every x-transform row
  float* d_rmax = nullptr;      // windowed back-sweep: running maximum of every spectral row's solved modes
  // windowed back-sweep with a batch of two or more: the second half of the
  // batch runs on a stream of its own (default priority), forked from and
  // joined to the caller's stream by events
  hipStream_t sweep_side = nullptr;
  hipEvent_t sweep_fork = nullptr, sweep_join = nullptr;
  int L = 2;              // bands of the time stencil
  double c1[3] = {0, 0, 0}, c2[3] = {0, 0, 0};
  double theta = 1.0;
  std::vector<cd> lam1, lam2;      // nt/2+1 time symbols
  std::vector<double> gam, invgam; // alpha^{n/nt} and alpha^{-n/nt}/nt
  SpaceOp op[2];                   // [0] = K, [1] = K^T

  // device (carved from the bound workspace)
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool bound = false;
  size_t ws_solver_bytes = 0;      // part of the workspace usable by the solvers
  // tables
  double* d_gam = nullptr;
  double* d_invgam = nullptr;
  double2* d_tw64 = nullptr;
  float2* d_tw32 = nullptr;
  double2* d_lam = nullptr;        // [2][F]
  // hybrid discretisation (ParaDiag-I): F = nt/2 eigenvalue pairs, time
  // transforms by dense products (tables in MFMA fragment order), banded rows
  // of the time matrix and of its transpose for the matvec
  bool hybrid = false;
  int order = 1;
  // optimal control of the wave equation (Section 4): Fh = nt/2 + 1 frequencies
  // per field, g.F = 2 Fh spectral slices (Sigma1 block, then Sigma2 block),
  // vectors of 2 nt S values; per-frequency mixing coefficients conj(E),
  // 1/d2 and i E / conj(d2) (double2 each, d_ocmix: [3][Fh])
  bool oc = false;
  int oc_fh = 0;
  double oc_gamma = 0.0, oc_beta = 0.0;
  std::vector<double2> ocmix;
  double2* d_ocmix = nullptr;
  std::vector<double> wf_frag, wi_frag, band, band_t;
  // host staging of the shifted time symbols of the nonlinear solver (kept
  // alive until the plan is destroyed: an asynchronous copy reads it)
  std::vector<double2> lam_stage;
  double* d_wf = nullptr;
  double* d_wi = nullptr;
  double* d_band = nullptr;
  double* d_band_t = nullptr;
  // spectral buffers
  void* spec_a = nullptr;
  void* spec_b = nullptr;
  // solver scratch (start of the solver region)
  char* solver_base = nullptr;
  int num_cu = 256;                // compute units of the bound device (persistent grids)
  StageTimer timer;
  // pinned host staging of the solvers' small transfers (Krylov scalars, norms)
  double* pin = nullptr;
  size_t pin_n = 0;
  int seq = 0;   // last value of the host-visible completion word (see wait_host)
};

size_t spec_elem_bytes(Prec p);          // 8 (double) or 4 (float)
size_t tables_bytes(const Plan& pl);     // device tables + spectral buffers
size_t solver_bytes(const Plan& pl, const paradiag_solve_opts* o);
void set_error(const std::string& msg);
// z = P_alpha^{-1} r (paradiag_apply_precond) with caller-supplied spectral
// buffers of spec_bytes each in place of the bound workspace's; no stage timing.
paradiag_status apply_precond_into(paradiag_plan plan, const double* r, double* z, void* spec_a,
                                   void* spec_b, size_t spec_bytes, hipStream_t s);

// ---------------------------------------------------------------- kernels
struct Launch { hipStream_t stream; };

// Step-(a): spec = rfft_t(Gamma * scale_b * x) ; x float64 [B][nt][S].
// reverse != 0 reads x with time reversed (adjoint).
void fft_time_forward(const Plan& pl, const double* x, const double* bscale, int bstride, void* spec,
                      int reverse, hipStream_t s);
// Step-(c): z = Gamma^{-1} irfft_t(spec) (float64 or float32 output), optional accumulate.
void fft_time_inverse(const Plan& pl, const void* spec, void* z, bool z_is_f32, int accumulate,
                      int reverse, hipStream_t s);
// ParaDiag-I time transforms (hybrid discretisation): forward spec = V^{-1} x
// (x float64 [B][nt][S]), inverse z (+)= V spec (z float64 or float32).
void time_transform(const Plan& pl, bool forward, const void* in, void* out, bool out_f32,
                    int accumulate, hipStream_t s);
// Dense time products C[b] = W X[b] on MFMA (float64): forward reads real data
// [batch][nt][S] and writes m spectral rows (2 per frequency, F frequencies per
// batch entry, planar layout); the inverse reads k = 2F' spectral rows and
// writes (or adds to, accumulate) m = nt real rows.  `table` holds W (m x k) in
// the fragment order of time_gemm_fragments.
void time_gemm(const Plan& pl, bool forward, const double* table, const void* in, void* out, bool spec_f32,
               bool out_f32, int accumulate, int batch, int nt, int F, int m, int k, hipStream_t s,
               const double* cscale = nullptr);
std::vector<double> time_gemm_fragments(const std::vector<double>& W, int m, int k);
size_t time_gemm_fragment_elems(int m, int k);
// Step-(b) pieces
// the x-transform of a sine-basis plan with pl.dst set (forward = inverse)
void dst_transform(const Plan& pl, const void* in, void* out, hipStream_t s);
void xform(const Plan& pl, const SpaceOp& op, bool forward, const void* in, void* out,
           hipStream_t s);
void line_solve(const Plan& pl, const SpaceOp& op, void* spec, hipStream_t s);
void schur_sweep(const Plan& pl, const SpaceOp& op, void* spec, hipStream_t s);
size_t schur_sweep_lds(const Plan& pl);   // dynamic LDS bytes of the back-sweep
// true where the back-sweep runs in windows of SWEEP_WINDOW modes, their
// coupling to later windows as one split-fp16 MFMA product (op.tfar needed)
constexpr int SWEEP_WINDOW = 64;
bool sweep_windowed(const Plan& pl);
void schur_line_lu(const Plan& pl, const SpaceOp& op, hipStream_t s);  // fills op.lu
// all-at-once operator
// y = A u (or b - A u).  With nv > 0 also the partial dots of y with the
// vectors Vk + i vstride (i < nv; vector 0 at V0 instead when V0 is given),
// and with sq the partial sums of y . y (slot nv), one per workgroup
// (matvec_chunks per right-hand side, layout as multi_dot's partial sums).
// y may be null with sq: only the norm is formed.  v0sq (nv >= 1): also
// V_0 . V_0, in the slot after y . y (or after the dots without sq).
void matvec(const Plan& pl, const SpaceOp& op, const void* u, bool u_is_f32, const double* b,
            double* y, int transpose, hipStream_t s, const double* Vk = nullptr,
            int64_t vstride = 0, int nv = 0, double* partial = nullptr, int sq = 0,
            const double* V0 = nullptr, int v0sq = 0);
int matvec_chunks(const Plan& pl);
void build_rhs(const Plan& pl, const double* U0, const double* u1, const double* f, double* b,
               hipStream_t s);
void rhs_transpose(const Plan& pl, const double* lam, double* gU0, double* gu1, double* gf,
                   hipStream_t s);
// Krylov helpers (float64).  Vectors of one batch entry are N1 long and the
// batch stride of every vector is N1.
int dot_chunks(const Plan& pl);
// slot0: first partial-sum slot written (dots land in slots slot0 .. slot0 + nv - 1)
void multi_dot(const Plan& pl, const double* V, int64_t vstride, int nv, const double* w,
               double* partial, hipStream_t s, int slot0 = 0);
// y = A u (or b - A u) of one field of nt * S values with the plan's Toeplitz
// columns and stencil, no dots (transpose: A^T)
void matvec_plain(const Plan& pl, const SpaceOp& op, const void* u, bool u_is_f32, const double* b,
                  double* y, int transpose, hipStream_t s);
// Optimal control of the wave equation (vectors [2][nt][S]: sqrt(gamma) u, p):
// y = A u (or b - A u) with the Krylov dots of matvec's interface, and
// z (+)= P^{-1} r (Thm the4) with the spectral buffers sa, sb
void oc_matvec(const Plan& pl, const void* u, bool u_is_f32, const double* b, double* y, hipStream_t s,
               const double* Vk, int64_t vstride, int nv, double* partial, int sq, const double* V0,
               int v0sq);
// Step-(a) of the optimal-control preconditioner: DFT of both fields into
// tmp, then the 2 x 2 mixing into out (the spectral layout Step-(b) reads)
void oc_time_forward(const Plan& pl, const double* in, const double* scale, void* out, void* tmp,
                     hipStream_t s);
// Step-(c): the unmixing into tmp, then the inverse DFT of both fields into out
void oc_time_inverse(const Plan& pl, const void* in, void* out, bool out_f32, int accumulate, void* tmp,
                     hipStream_t s);
void oc_build_rhs(const Plan& pl, const double* U0, const double* u1, const double* f, const double* gsrc,
                  double* b, hipStream_t s);
// h[b][i] = t s, coef[b][i] = t s^2 with t the reduced dot and s = sigma[b][i]
// for i < nscaled (else 1): dots against unnormalised Krylov vectors.
// chunks: partial sums per right-hand side (<= 0: dot_chunks).  hhost
// (pinned host memory, same layout as h) also receives h when given.
void reduce_partials(const Plan& pl, const double* partial, int nv, const double* sigma,
                     int nscaled, double* h, double* coef, hipStream_t s, int chunks = 0,
                     double* hhost = nullptr);
// dst[0..n) = src[0..n) with src in pinned host memory (one small kernel).
void fetch_host(const double* src, double* dst, int n, hipStream_t s);
// *word = v (word in pinned host memory) once the work queued before it on s
// has finished: the host polls it instead of synchronising the stream.
void signal_host(int* word, int v, hipStream_t s);
// w -= sum_i coef_i V_i (i < nv; V_0 at V0 instead when V0 is given), with
// the partial dots of the result when want_dots; a no-op when skip is given
// and *skip is set on the device.
void update_dot(const Plan& pl, const double* V, int64_t vstride, int nv, const double* coef,
                double* w, double* partial, int want_dots, hipStream_t s,
                const int* skip = nullptr, const double* V0 = nullptr);
// Device-side test whether Arnoldi step j ends its cycle without the update
// (*flag = 1): h = first-pass coefficients plus w . w in slot j+1, giv = per
// right-hand side [threshold, g_j, c_0..c_{j-1}, s_0..s_{j-1}] with stride gs.
// first: step 0 of a cycle started from the unnormalised V_0 = b, whose h
// carries b . b in slot 2; the kernel then also sets sigma[b][0] = 1/||b|| and
// scales c1[b][0] by its square (see k_arnoldi_skip).
void arnoldi_skip(const Plan& pl, const double* h, const double* giv, int gs, int j, bool force,
                  int* flag, hipStream_t s, int* flag_host = nullptr, bool first = false,
                  double* c1 = nullptr, double* sigma = nullptr, double rtol = 0.0);
void x_update(const Plan& pl, const void* Z, bool z_is_f32, int64_t zstride, int nz,
              const double* y, double* x, bool overwrite, hipStream_t s);
void copy_vec(const double* src, double* dst, int64_t n, hipStream_t s);
// partial[b][chunk][0..1] = sums of (u - v)^2 and u^2 over chunk `chunk` of right-hand side b
void diff_norms(const Plan& pl, const double* u, const double* v, double* partial, int chunks,
                hipStream_t s);
// Nonlinear problems (eq1.4, g(u) = gk[0] u + gk[1] u^2 + gk[2] u^3): r -= (B2 (x) I) g(u) with
// partial sums [b][chunk] of r^2 (slot 0) and g'(u) (slot 1); b_1 -= (1-theta) g(U0);
// u_n = U0 for all n; dst[b] = src[b][nt-1].
void nl_residual(const Plan& pl, const double* u, double* r, const double* gk, double* partial, int chunks,
                 hipStream_t s);
void nl_rhs_fix(const Plan& pl, const double* U0, double* b, const double* gk, hipStream_t s);
void bcast_rows(const Plan& pl, const double* U0, double* u, hipStream_t s);
void last_rows(const Plan& pl, const double* src, double* dst, hipStream_t s);
// Parareal (1D): b = right-hand side of the alpha-periodic coarse-grid
// correction after J fine backward Euler steps from U0 / the iterate uprev.
void parareal_fine(const Plan& pl, const double* U0, const double* uprev, double* b, int J, double alpha,
                   hipStream_t s);
void fill_zero(double* dst, int64_t n, hipStream_t s);

}  // namespace pd
