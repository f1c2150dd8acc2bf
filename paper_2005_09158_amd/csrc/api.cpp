// C ABI of the ParaDiag-II library: plan setup (host tables), workspace
// binding, and the drivers of the three solve modes.  See include/paradiag.h.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <type_traits>

#include "internal.h"

namespace pd {

namespace {
thread_local std::string g_last_error;
constexpr int MAXV = 33;   // Krylov slots per right-hand side (restart <= 32)
// Second Gram-Schmidt pass (see the Arnoldi step): components along the
// Krylov basis left by the first pass, relative to the vector's norm (eta),
// never need it below kReorthTol and always do above kReorthMax; in between
// they do when eta times the residual estimate before the step exceeds
// kReorthRel rtol (the error a skipped pass leaves in the residual estimate
// is about that product).
constexpr double kReorthTol = 1e-12, kReorthMax = 1e-6, kReorthRel = 1e-2;
constexpr size_t ALIGN = 256;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

size_t compute_elem_bytes(Prec p) { return p == Prec::F64 ? 8 : (p == Prec::F32 ? 4 : 2); }
// bytes of one x-transform matrix of `elems` entries in the compute format
// (split bf16 keeps hi, mid and lo parts plus a float32 copy for ragged sizes)
size_t gemm_matrix_bytes(Prec p, size_t elems) {
  if (p == Prec::BF16) return elems * (2 + 2 + 2 + 4);   // three bf16 parts and a float32 copy
  if (p == Prec::F16) return elems * (2 + 2 + 4);        // two fp16 parts and a float32 copy
  return elems * compute_elem_bytes(p);
}
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }
size_t spec_elem_bytes(Prec p) { return p == Prec::F64 ? 8 : 4; }

// ------------------------------------------------------------------ tables

namespace {

void time_columns(int scheme, double dt, double* c1, double* c2, int* L, double* theta) {
  c1[0] = c1[1] = c1[2] = 0;
  c2[0] = c2[1] = c2[2] = 0;
  if (scheme == PD_LEAPFROG) {
    // implicit leap-frog (eq3.2b): B1 = tridiag-Toeplitz (1,-2,1)/dt^2, B2 = (1/2, 0, 1/2)
    c1[0] = 1.0 / (dt * dt); c1[1] = -2.0 / (dt * dt); c1[2] = 1.0 / (dt * dt);
    c2[0] = 0.5; c2[1] = 0.0; c2[2] = 0.5;
    *L = 3;
    *theta = 0.5;
  } else {
    // theta-method with uniform step (eq2.5b): B1 = (1, -1)/dt, B2 = (theta, 1 - theta)
    double th = (scheme == PD_BE) ? 1.0 : 0.5;
    c1[0] = 1.0 / dt; c1[1] = -1.0 / dt;
    c2[0] = th; c2[1] = 1.0 - th;
    *L = 2;
    *theta = th;
  }
}

// 1D factor -nu d2 + a d on n Dirichlet points: tridiag(lo, di, up)
void factor_1d(int n, double nu, double a, double* lo, double* di, double* up) {
  double h = 1.0 / (n + 1);
  *lo = -nu / (h * h) - a / (2 * h);
  *di = 2 * nu / (h * h);
  *up = -nu / (h * h) + a / (2 * h);
}

}  // namespace

// oc_gamma > 0: the plan of the optimal-control system of the wave equation
// (Section 4) with that regularisation parameter.
static paradiag_status build_plan(const paradiag_problem* pr, Plan*& out, double oc_gamma = 0.0) {
  out = nullptr;
  if (!pr) { set_error("problem is NULL"); return PD_ERR_INVALID; }
  const paradiag_problem& p = *pr;
  if (p.dim != 1 && p.dim != 2) { set_error("dim must be 1 or 2"); return PD_ERR_INVALID; }
  if (p.nx < 1 || p.ny < 1 || p.nt < 1 || p.batch < 1) { set_error("sizes must be positive"); return PD_ERR_INVALID; }
  if (p.dim == 1 && p.ny != 1) { set_error("ny must be 1 in one dimension"); return PD_ERR_INVALID; }
  if (p.batch > 64) { set_error("batch must be <= 64"); return PD_ERR_INVALID; }
  if (!(p.alpha > 0.0 && p.alpha <= 1.0)) { set_error("alpha must lie in (0, 1]"); return PD_ERR_INVALID; }
  if (!(p.T > 0.0) || !(p.nu > 0.0) || !std::isfinite(p.T) || !std::isfinite(p.nu) ||
      !std::isfinite(p.ax) || !std::isfinite(p.ay)) {
    set_error("T and nu must be positive and finite"); return PD_ERR_INVALID;
  }
  if (p.scheme < 0 || p.scheme > 4) { set_error("unknown scheme"); return PD_ERR_INVALID; }
  const bool hybrid = p.scheme == PD_HYBRID || p.scheme == PD_HYBRID_WAVE;
  if (p.prec < 0 || p.prec > 4) { set_error("unknown precision"); return PD_ERR_INVALID; }
  if (p.reserved != 0) { set_error("reserved must be 0"); return PD_ERR_INVALID; }
  const bool oc = oc_gamma > 0.0;
  if (oc) {
    if (p.scheme != PD_LEAPFROG || p.ax != 0.0 || p.ay != 0.0 || p.batch != 1) {
      set_error("optimal control: implicit leap-frog, zero velocity and batch 1 required"); return PD_ERR_UNSUPPORTED;
    }
    if (p.nt % 4 == 0 || p.nt < 3 || p.nt > 4096) {
      // C2 (the circulant of (1, 0, 1)) is singular when 4 divides nt
      set_error("optimal control needs nt in [3, 4096] not divisible by 4"); return PD_ERR_UNSUPPORTED;
    }
    if (!std::isfinite(oc_gamma)) { set_error("gamma must be finite"); return PD_ERR_INVALID; }
  } else if (hybrid) {
    if ((p.nt & 1) || p.nt < 4 || p.nt > 4096) {
      set_error("hybrid schemes need an even nt in [4, 4096]"); return PD_ERR_UNSUPPORTED;
    }
  } else if (!is_pow2(p.nt) || p.nt < 4 || p.nt > 4096) {
    set_error("nt must be a power of two in [4, 4096]"); return PD_ERR_UNSUPPORTED;
  }
  if (p.dim == 1 && p.nx > 2048) { set_error("nx > 2048 unsupported in 1D"); return PD_ERR_UNSUPPORTED; }
  if (p.dim == 2 && (p.ny > 2048 || p.nx > 2048)) { set_error("nx, ny > 2048 unsupported"); return PD_ERR_UNSUPPORTED; }
  if (p.dim == 2 && p.ax != 0.0 && p.prec == PD_PREC_FP32_BF16X1) {
    // one bf16 rounding (2^-9) of the x-transform operands, carried through the
    // back-substitution over the non-normal Schur factor, leaves the
    // preconditioner error of order one: no stated accuracy can be met
    set_error("single-bf16 x-transform needs a symmetric x factor (use PD_PREC_FP32_BF16GEMM)");
    return PD_ERR_UNSUPPORTED;
  }
  if (p.dim == 2 && p.ax != 0.0 && p.nx > 1024) {
    set_error("non-symmetric x factor with nx > 1024 unsupported (host Schur cost)"); return PD_ERR_UNSUPPORTED;
  }
  double hx = 1.0 / (p.nx + 1), hy = 1.0 / (p.ny + 1);
  if (std::fabs(p.ax) * hx / (2 * p.nu) >= 1.0 || (p.dim == 2 && std::fabs(p.ay) * hy / (2 * p.nu) >= 1.0)) {
    set_error("cell Peclet number |a| h / (2 nu) must be < 1"); return PD_ERR_UNSUPPORTED;
  }

  std::unique_ptr<Plan> pl(new (std::nothrow) Plan());
  if (!pl) { set_error("out of host memory"); return PD_ERR_INVALID; }
  pl->p = p;
  pl->prec = static_cast<Prec>(p.prec);
  Geom& g = pl->g;
  g.B = p.batch; g.nt = p.nt; g.F = hybrid ? p.nt / 2 : p.nt / 2 + 1;
  if (oc) g.F = 2 * (p.nt / 2 + 1);   // Sigma1 and Sigma2 slices of both fields' half spectra
  g.nx = p.nx; g.ny = p.ny;
  if (p.dim == 2) { g.sx = p.nx; g.sy = p.ny; } else { g.sx = 1; g.sy = p.nx; }
  g.S = (int64_t)p.nx * p.ny;
  g.N1 = g.S * p.nt * (oc ? 2 : 1);
  g.NA = g.N1 * p.batch;
  g.spec_elems = (int64_t)g.B * g.F * g.sy * 2 * g.sx;

  const double dt = p.T / p.nt;
  const double PI = 3.14159265358979323846;
  if (oc) {
    // Section 4: Fourier symbols of the circulants of (1, -2, 1) and (1, 0, 1),
    // the per-frequency eigenvalues Sigma = a +- i beta |q| of Thm the4 and the
    // mixing coefficients; DFT tables of length nt (no power of two)
    pl->oc = true;
    pl->oc_gamma = oc_gamma;
    pl->oc_beta = dt * dt / std::sqrt(oc_gamma);
    const int Fh = p.nt / 2 + 1;
    pl->oc_fh = Fh;
    pl->c1[0] = 1.0; pl->c1[1] = -2.0; pl->c1[2] = 1.0;
    pl->c2[0] = 0.5 * dt * dt; pl->c2[1] = 0.0; pl->c2[2] = 0.5 * dt * dt;
    pl->L = 3;
    pl->theta = 0.5;
    pl->lam1.resize(2 * Fh);
    pl->lam2.assign(2 * Fh, cd(0.5 * dt * dt, 0.0));
    pl->ocmix.resize(3 * (size_t)Fh);
    for (int n = 0; n < Fh; ++n) {
      const cd w = std::polar(1.0, -2.0 * PI * n / p.nt);
      const cd d1 = 1.0 - 2.0 * w + w * w, d2 = 1.0 + w * w;
      const double a = (d1 / d2).real(), aq = 1.0 / std::abs(d2);
      const cd E = (1.0 / d2) * std::abs(d2);   // q / |q|
      pl->lam1[n] = cd(a, pl->oc_beta * aq);
      pl->lam1[Fh + n] = cd(a, -pl->oc_beta * aq);
      const cd inv1 = 1.0 / d2, inv2 = cd(0.0, 1.0) * E / std::conj(d2);
      pl->ocmix[n] = double2{E.real(), -E.imag()};
      pl->ocmix[Fh + n] = double2{inv1.real(), inv1.imag()};
      pl->ocmix[2 * Fh + n] = double2{inv2.real(), inv2.imag()};
    }
    std::vector<double> wf((size_t)2 * Fh * p.nt), wi((size_t)p.nt * 2 * Fh);
    for (int n = 0; n < Fh; ++n) {
      const double wgt = (n == 0 || 2 * n == p.nt) ? 1.0 : 2.0;
      for (int m = 0; m < p.nt; ++m) {
        const double ang = 2.0 * PI * (double)(((int64_t)n * m) % p.nt) / p.nt;
        wf[(size_t)(2 * n) * p.nt + m] = std::cos(ang);
        wf[(size_t)(2 * n + 1) * p.nt + m] = -std::sin(ang);
        wi[(size_t)m * 2 * Fh + 2 * n] = wgt / p.nt * std::cos(ang);
        wi[(size_t)m * 2 * Fh + 2 * n + 1] = -wgt / p.nt * std::sin(ang);
      }
    }
    pl->wf_frag = time_gemm_fragments(wf, 2 * Fh, p.nt);
    pl->wi_frag = time_gemm_fragments(wi, p.nt, 2 * Fh);
  } else if (hybrid) {
    // ParaDiag-I: the closed-form eigendecomposition of B (Thm thmCondU)
    pl->hybrid = true;
    pl->order = p.scheme == PD_HYBRID ? 1 : 2;
    HybridTables ht;
    std::string err;
    if (!hybrid_eigen(p.nt, dt, pl->order, ht, err)) { set_error(err); return PD_ERR_BREAKDOWN; }
    pl->lam1 = ht.d;
    pl->lam2.assign(g.F, cd(1.0, 0.0));
    pl->wf_frag = time_gemm_fragments(ht.wf, p.nt, p.nt);
    pl->wi_frag = time_gemm_fragments(ht.wi, p.nt, p.nt);
    pl->band = ht.band;
    pl->band_t.assign(ht.band.size(), 0.0);   // rows of the transpose: (B^T)[r][r+k] = B[r+k][r]
    for (int r = 0; r < p.nt; ++r)
      for (int k = -2; k <= 2; ++k)
        if (r + k >= 0 && r + k < p.nt) pl->band_t[(size_t)r * 5 + k + 2] = ht.band[(size_t)(r + k) * 5 - k + 2];
    pl->L = 1;
    pl->theta = 1.0;
  } else {
  time_columns(p.scheme, dt, pl->c1, pl->c2, &pl->L, &pl->theta);

  // time symbols lambda_j(n) = sum_k c_jk z_n^k, z_n = alpha^{1/Nt} e^{-2 pi i n/Nt}
  // (the Fourier transform of Gamma_alpha c_j, Lemma 1)
  double r = std::pow(p.alpha, 1.0 / p.nt);
  pl->lam1.resize(g.F);
  pl->lam2.resize(g.F);
  for (int n = 0; n < g.F; ++n) {
    double ang = -2.0 * PI * n / p.nt;
    cd z = std::polar(r, ang), zk = 1.0, s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < pl->L; ++k) {
      s1 += pl->c1[k] * zk;
      s2 += pl->c2[k] * zk;
      zk *= z;
    }
    pl->lam1[n] = s1;
    pl->lam2[n] = s2;
  }
  }  // not hybrid
  pl->gam.resize(p.nt);
  pl->invgam.resize(p.nt);
  double la = std::log(p.alpha);
  for (int n = 0; n < p.nt; ++n) {
    pl->gam[n] = std::exp(la * n / p.nt);
    pl->invgam[n] = std::exp(-la * n / p.nt) / p.nt;
  }

  // spatial operator and its transpose
  double lx, dx, ux, ly = 0, dy = 0, uy = 0;
  factor_1d(p.nx, p.nu, p.ax, &lx, &dx, &ux);
  if (p.dim == 2) factor_1d(p.ny, p.nu, p.ay, &ly, &dy, &uy);
  for (int v = 0; v < 2; ++v) {
    SpaceOp& op = pl->op[v];
    double lxv = v ? ux : lx, uxv = v ? lx : ux, lyv = v ? uy : ly, uyv = v ? ly : uy;
    op.sxl = lxv; op.sxu = uxv; op.syl = lyv; op.syu = uyv; op.sd = dx + dy;
    if (p.dim == 1) { op.lo = lxv; op.di = dx; op.up = uxv; }
    else { op.lo = lyv; op.di = dy; op.up = uyv; }
  }
  if (p.dim == 2) {
    const int n = p.nx;
    pl->schur = (p.ax != 0.0);
    std::vector<cd> Q((size_t)n * n), T((size_t)n * n, cd(0.0));
    if (!pl->schur) {
      // symmetric factor: sine basis, eigenvalues di + 2 lo cos(k pi/(n+1))
      double s = std::sqrt(2.0 / (n + 1));
      for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) Q[(size_t)j * n + k] = s * std::sin((j + 1.0) * (k + 1.0) * PI / (n + 1));
      for (int k = 0; k < n; ++k) T[(size_t)k * n + k] = dx + 2 * lx * std::cos((k + 1.0) * PI / (n + 1));
    } else {
      std::vector<cd> H((size_t)n * n, cd(0.0));
      for (int i = 0; i < n; ++i) {
        H[(size_t)i * n + i] = dx;
        if (i > 0) H[(size_t)i * n + i - 1] = lx;
        if (i + 1 < n) H[(size_t)i * n + i + 1] = ux;
      }
      if (!complex_schur(n, H, Q)) { set_error("Schur iteration did not converge"); return PD_ERR_BREAKDOWN; }
      T = H;
    }
    // DST-I by FFT: lengths 2 (nx + 1) = 8 .. 4096, a power of two
    pl->dst = !pl->schur && n >= 3 && ((n + 1) & n) == 0 && 2 * (n + 1) <= 4096;
    pl->op[0].Q = Q;
    pl->op[0].Tm = T;
    // K_x^T = conj(Q) T^T Q^T = (conj(Q) J)(J T^T J)(J Q^T): Schur form of the transpose
    std::vector<cd> Qa((size_t)n * n), Ta((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) {
        Qa[(size_t)i * n + k] = std::conj(Q[(size_t)i * n + (n - 1 - k)]);
        Ta[(size_t)i * n + k] = T[(size_t)(n - 1 - k) * n + (n - 1 - i)];
      }
    if (!pl->schur) { Qa = Q; Ta = T; }
    pl->op[1].Q = Qa;
    pl->op[1].Tm = Ta;
    if (pl->schur && (p.ny > 512 || schur_sweep_lds(*pl) > 160 * 1024)) {
      set_error("non-symmetric x factor with ny > 512 unsupported (back-sweep tile exceeds LDS)");
      return PD_ERR_UNSUPPORTED;
    }
  }
  out = pl.release();
  return PD_OK;
}

size_t tables_bytes(const Plan& pl) {
  const Geom& g = pl.g;
  size_t b = 0;
  b += align_up(sizeof(double) * g.nt) * 2;          // gam, invgam
  b += align_up(sizeof(double2) * g.nt);              // twiddles f64
  b += align_up(sizeof(float2) * g.nt);               // twiddles f32
  b += align_up(sizeof(double2) * 2 * g.F);           // lam
  if (pl.dst) b += align_up(spec_elem_bytes(pl.prec) * 2 * (g.nx + 1));   // DST twiddles
  if (pl.prec == Prec::F16 && pl.p.dim == 2)
    b += align_up(sizeof(float) * 2 * (size_t)g.B * g.F * g.sy);   // x-transform row scales
  if (sweep_windowed(pl)) b += align_up(sizeof(float) * (size_t)g.B * g.F * g.sy);   // row maxima of the sweep
  if (pl.hybrid) {
    b += 2 * align_up(sizeof(double) * time_gemm_fragment_elems(g.nt, g.nt));   // V^{-1}, V (fragment order)
    b += 2 * align_up(sizeof(double) * 5 * g.nt);                         // banded rows of B, B^T
  }
  if (pl.oc) {
    b += align_up(sizeof(double) * time_gemm_fragment_elems(2 * pl.oc_fh, g.nt));   // DFT
    b += align_up(sizeof(double) * time_gemm_fragment_elems(g.nt, 2 * pl.oc_fh));   // inverse DFT
    b += align_up(sizeof(double2) * 3 * pl.oc_fh);                                  // mixing
  }
  if (pl.p.dim == 2) {
    const size_t n = g.nx;
    size_t gm = pl.schur ? (2 * n) * (2 * n) : n * n;
    for (int v = 0; v < 2; ++v) {
      b += align_up(sizeof(double2) * n);                             // tk
      b += 2 * align_up(gemm_matrix_bytes(pl.prec, gm));              // g_fwd, g_inv
      if (pl.schur) b += align_up(2 * n * n * spec_elem_bytes(pl.prec));  // T (line precision)
      if (pl.schur) b += align_up((size_t)2 * g.F * n * g.sy * spec_elem_bytes(pl.prec));  // line LU
      if (sweep_windowed(pl)) b += align_up((size_t)2 * 4 * n * n * 2);   // far-coupling B^T, fp16 parts
    }
  }
  b += 2 * align_up((size_t)g.spec_elems * spec_elem_bytes(pl.prec));
  return b;
}

// partial-sum slots per right-hand side: the Krylov kernels' chunks or the
// matvec's workgroups, whichever is more
static size_t partial_chunks(const Plan& pl) {
  return (size_t)std::max(2048, matvec_chunks(pl));
}

size_t solver_bytes(const Plan& pl, const paradiag_solve_opts* o) {
  if (!o) return 0;
  const Geom& g = pl.g;
  size_t small = align_up(sizeof(double) * g.B * partial_chunks(pl) * MAXV) + 12 * align_up(sizeof(double) * g.B * MAXV);
  size_t zb = (pl.prec == Prec::F64) ? 8 : 4;
  if (o->mode == PD_MODE_FGMRES) {
    int m = std::max(1, std::min(o->restart, 32));
    return small + align_up(sizeof(double) * (size_t)g.NA) * (m + 1) + align_up(zb * (size_t)g.NA) * m;
  }
  // stationary: the residual vector; direct: only the norm of its residual
  if (o->mode == PD_MODE_DIRECT) return small;
  // parareal: the previous iterate and the coarse right-hand side
  if (o->mode == PD_MODE_PARAREAL) return small + 2 * align_up(sizeof(double) * (size_t)g.NA);
  // nonlinear: residual, right-hand side, the next window's initial state
  if (o->mode == PD_MODE_NONLINEAR)
    return small + 2 * align_up(sizeof(double) * (size_t)g.NA) + align_up(sizeof(double) * (size_t)g.B * g.S);
  return small + align_up(sizeof(double) * (size_t)g.NA);
}

// ------------------------------------------------------------------ timing

struct Timed {
  Plan& pl;
  int stage;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  Timed(Plan& p, int st, hipStream_t str, double bytes = 0, double flops = 0)
      : pl(p), stage(st), s(str) {
    if (!pl.timer.enabled || !((pl.timer.mask >> stage) & 1u)) return;
    pl.timer.bytes[stage] += bytes;
    pl.timer.flops[stage] += flops;
    a = take();
    b = take();
    hipEventRecord(a, s);
  }
  hipEvent_t take() {
    if (!pl.timer.pool.empty()) { hipEvent_t e = pl.timer.pool.back(); pl.timer.pool.pop_back(); return e; }
    hipEvent_t e;
    hipEventCreate(&e);
    return e;
  }
  ~Timed() {
    if (!a) return;
    hipEventRecord(b, s);
    pl.timer.pending.push_back({stage, a, b});
  }
};

static void drain_timer(Plan& pl) {
  for (auto& r : pl.timer.pending) {
    hipEventSynchronize(r.b);
    float ms = 0;
    hipEventElapsedTime(&ms, r.a, r.b);
    pl.timer.ms[r.stage] += ms;
    pl.timer.count[r.stage] += 1;
    pl.timer.pool.push_back(r.a);
    pl.timer.pool.push_back(r.b);
  }
  pl.timer.pending.clear();
}

// Removes the most recent record of `stage` (a launch that returned without
// doing its work) and the work it was credited with.
static void untime_last(Plan& pl, int stage, double bytes, double flops) {
  auto& pend = pl.timer.pending;
  for (size_t k = pend.size(); k-- > 0;) {
    if (pend[k].stage != stage) continue;
    hipEventSynchronize(pend[k].b);
    pl.timer.pool.push_back(pend[k].a);
    pl.timer.pool.push_back(pend[k].b);
    pend.erase(pend.begin() + (ptrdiff_t)k);
    pl.timer.bytes[stage] -= bytes;
    pl.timer.flops[stage] -= flops;
    return;
  }
}

// ------------------------------------------------------------ operations

// Algorithmic work of one launch of each kernel (bytes that must cross HBM
// once, floating-point operations), used by the stage accounting.
static double spec_bytes(const Plan& pl) {
  return (double)pl.g.spec_elems * spec_elem_bytes(pl.prec);
}
static double fft_flops(const Plan& pl) {
  // complex FFT of length Nt on NA/2 packed pairs: 5 (Nt/2... ) -> 5 N log2 N per complex column
  double lg = std::log2((double)pl.g.nt);
  return 5.0 * pl.g.nt * lg * (pl.g.NA / (double)pl.g.nt) * 0.5;
}
static double time_flops(const Plan& pl) {
  if (pl.hybrid) return 2.0 * pl.g.nt * (double)pl.g.NA;   // two dense nt x nt products per point
  if (pl.oc) return 2.0 * 2.0 * pl.oc_fh * (double)pl.g.NA;   // (2 Fh) x nt products, both fields
  return fft_flops(pl);
}
static double xform_flops(const Plan& pl) {
  const Geom& g = pl.g;
  double rows = (double)g.B * g.F * g.sy;
  if (pl.dst) {   // one complex FFT of length 2 (nx + 1) per row (both halves)
    const double n2 = 2.0 * (g.sx + 1);
    return rows * 5.0 * n2 * std::log2(n2);
  }
  return pl.schur ? 2.0 * rows * (2.0 * g.sx) * (2.0 * g.sx) : 2.0 * (2.0 * rows) * g.sx * g.sx;
}
static double sweep_flops(const Plan& pl) {
  // complex multiply-adds of the coupling sum_{j>k} T_kj w_j: 8 flops each
  const Geom& g = pl.g;
  return 8.0 * g.B * g.F * g.sy * 0.5 * (double)g.sx * (g.sx - 1);
}

// bscale: per right-hand side factor on the input (entry b * bstride), or null.
// buf_a, buf_b: the two spectral buffers (null: the plan's, in the bound workspace).
static void apply_prec(Plan& pl, int variant, const double* in, const double* bscale, int bstride,
                       void* out, bool out_f32, int accumulate, hipStream_t s,
                       void* buf_a = nullptr, void* buf_b = nullptr) {
  const SpaceOp& op = pl.op[variant];
  void* const spec_a = buf_a ? buf_a : pl.spec_a;
  void* const spec_b = buf_b ? buf_b : pl.spec_b;
  const double vin = 8.0 * pl.g.NA, sb = spec_bytes(pl);
  const double vout = (out_f32 ? 4.0 : 8.0) * pl.g.NA * (accumulate ? 2.0 : 1.0);
  {
    Timed t(pl, PD_STAGE_FFT_FWD, s, vin + sb, time_flops(pl));
    if (pl.oc) oc_time_forward(pl, in, bscale, spec_a, spec_b, s);
    else if (pl.hybrid) time_transform(pl, true, in, spec_a, false, 0, s);
    else fft_time_forward(pl, in, bscale, bstride, spec_a, variant, s);
  }
  if (pl.p.dim == 2) {
    { Timed t(pl, PD_STAGE_XFORM_FWD, s, 2 * sb, xform_flops(pl)); xform(pl, op, true, spec_a, spec_b, s); }
    {
      Timed t(pl, PD_STAGE_LINE_SOLVE, s, 2 * sb, pl.schur ? sweep_flops(pl) : 0.0);
      if (pl.schur) schur_sweep(pl, op, spec_b, s);
      else line_solve(pl, op, spec_b, s);
    }
    { Timed t(pl, PD_STAGE_XFORM_INV, s, 2 * sb, xform_flops(pl)); xform(pl, op, false, spec_b, spec_a, s); }
  } else {
    Timed t(pl, PD_STAGE_LINE_SOLVE, s, 2 * sb, 0.0);
    line_solve(pl, op, spec_a, s);
  }
  {
    Timed t(pl, PD_STAGE_FFT_INV, s, sb + vout, time_flops(pl));
    if (pl.oc) oc_time_inverse(pl, spec_a, out, out_f32, accumulate, spec_b, s);
    else if (pl.hybrid) time_transform(pl, false, spec_a, out, out_f32, accumulate, s);
    else fft_time_inverse(pl, spec_a, out, out_f32, accumulate, variant, s);
  }
}

// y = b - A u (A u without b); with `sq`, also the partial sums of y . y, one
// per matvec workgroup (reduced with matvec_chunks); y null: the norm only
static void apply_A(Plan& pl, int variant, const void* u, bool u_f32, const double* b, double* y,
                    hipStream_t s, double* sq = nullptr) {
  const double n = (double)pl.g.NA;
  Timed t(pl, PD_STAGE_MATVEC, s, n * ((u_f32 ? 4.0 : 8.0) + (y ? 8.0 : 0.0) + (b ? 8.0 : 0.0)),
          n * ((pl.L == 3 ? 22.0 : 18.0) + (sq ? 2.0 : 0.0)));
  matvec(pl, pl.op[variant], u, u_f32, b, y, variant, s, nullptr, 0, 0, sq, sq ? 1 : 0);
}

namespace {

struct Small {
  double* partial;
  double* h1;
  double* c1;
  double* h2;
  double* c2;
  double* sigma;
  double* y;
  double* nrm;
  double* giv;   // B x GIVS: Givens state for k_arnoldi_skip
  int* skip;     // its decision
};
constexpr int GIVS = 3 * MAXV;   // per right-hand side: >= 2 + 2 (m - 1) entries for restart m <= 32

Small carve_small(Plan& pl, char*& p) {
  const Geom& g = pl.g;
  Small sm;
  sm.partial = (double*)p; p += align_up(sizeof(double) * g.B * partial_chunks(pl) * MAXV);
  // slots of B * MAXV doubles (rounded up to ALIGN); h1, h2 and the skip flag
  // are adjacent (one copy to the host per Arnoldi step), and so are sigma and
  // the Givens state (one copy to the device)
  const size_t slot = align_up(sizeof(double) * g.B * MAXV);
  auto take = [&](size_t nslots) { double* q = (double*)p; p += nslots * slot; return q; };
  sm.h1 = take(1);
  sm.h2 = take(1);
  sm.skip = (int*)take(1);
  sm.c1 = take(1);
  sm.c2 = take(1);
  sm.sigma = take(1);
  sm.giv = take(3);
  sm.y = take(1);
  sm.nrm = take(1);
  take(1);
  return sm;
}

}  // namespace
static void timed_dot(Plan& pl, const double* V, int64_t vs, int nv, const double* w, double* part,
                      hipStream_t s) {
  const double n = (double)pl.g.NA;
  Timed t(pl, PD_STAGE_DOT, s, n * 8.0 * (nv + (V == w ? 0 : 1)), 2.0 * n * nv);
  multi_dot(pl, V, vs, nv, w, part, s);
}
static void timed_update(Plan& pl, const double* V, int64_t vs, int nv, const double* coef, double* w,
                         double* part, int dots, hipStream_t s, const int* skip = nullptr,
                         const double* V0 = nullptr) {
  const double n = (double)pl.g.NA;
  Timed t(pl, PD_STAGE_UPDATE, s, n * 8.0 * (nv + 2), n * (2.0 * nv + (dots ? 2.0 * nv + 2.0 : 0.0)));
  update_dot(pl, V, vs, nv, coef, w, part, dots, s, skip, V0);
}
static void timed_reduce(Plan& pl, const double* part, int nv, const double* sigma, int nscaled,
                         double* h, double* coef, hipStream_t s, int chunks = 0,
                         double* hhost = nullptr) {
  Timed t(pl, PD_STAGE_OTHER, s);
  reduce_partials(pl, part, nv, sigma, nscaled, h, coef, s, chunks, hhost);
}
namespace {
// Pinned (coherent) host staging of the solvers' small transfers, in slots of
// pin_slot doubles laid out like the device's: [norms | h1 h2 skip | sigma,
// Givens state (3 slots) | y].  The reduction kernels write the norms, the
// Hessenberg columns and the skip flag straight into it, and a one-block
// kernel fetches the scales, Givens state and y from it (no copy engine on
// the per-step round trip).  A region is rewritten by the host only after a
// wait (wait_host) that follows its last use by a kernel (every Arnoldi step
// and every norm ends with one).
size_t pin_slot(const Plan& pl) { return align_up(sizeof(double) * pl.g.B * MAXV) / sizeof(double); }

double* pinned(Plan& pl) {
  const size_t n = 9 * pin_slot(pl) + 8;   // + the completion word (wait_host)
  if (pl.pin_n < n) {
    if (pl.pin) hipHostFree(pl.pin);
    pl.pin = nullptr;
    pl.pin_n = 0;
    if (hipHostMalloc((void**)&pl.pin, sizeof(double) * n, hipHostMallocCoherent) != hipSuccess) {
      pl.pin = nullptr;
      return nullptr;
    }
    pl.pin_n = n;
    std::memset(pl.pin, 0, sizeof(double) * n);
  }
  return pl.pin;
}

// Waits for the work queued on s so far by polling a completion word in the
// pinned buffer (written by k_signal behind that work), which wakes the host
// sooner than a stream synchronisation.  k_signal makes every earlier write
// of the stream visible at system scope before it stores the word (release),
// and the host reads the word with acquire ordering before it reads the
// pinned results.  After about a second of polling it falls back to the
// synchronisation.  Returns PD_OK, or PD_ERR_HIP (message set) when a launch
// failed or the stream reports an error: the caller must then return at once,
// without reading the pinned buffer.
paradiag_status wait_host(Plan& pl, hipStream_t s) {
  int* word = reinterpret_cast<int*>(pl.pin + 9 * pin_slot(pl));
  const int v = pl.seq = pl.seq % 0x3fffffff + 1;   // never 0
  __atomic_store_n(word, 0, __ATOMIC_RELEASE);       // whatever an earlier solve left there
  signal_host(word, v, s);
  auto failed = [](const char* what, hipError_t e) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return PD_ERR_HIP;
  };
  // a launch that failed (this one or one before it) never signals
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return failed("kernel launch", e);
  const auto t0 = std::chrono::steady_clock::now();
  for (long it = 0;; ++it) {
    if (__atomic_load_n(word, __ATOMIC_ACQUIRE) == v) break;
    if ((it & 1023) == 1023 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(1)) {
      e = hipStreamSynchronize(s);
      if (e != hipSuccess) return failed("stream synchronisation", e);
      break;
    }
  }
  e = hipGetLastError();
  if (e != hipSuccess) return failed("solver step", e);
  return PD_OK;
}

// chunks: partial sums per right-hand side in sm.partial (<= 0: dot_chunks)
paradiag_status norms_from(Plan& pl, Small& sm, std::vector<double>& out, hipStream_t s,
                           int chunks = 0) {
  double* tmp = pl.pin;   // norms region, written by the reduction kernel
  timed_reduce(pl, sm.partial, 1, nullptr, 0, sm.nrm, nullptr, s, chunks, tmp);
  paradiag_status st = wait_host(pl, s);
  if (st != PD_OK) return st;
  out.resize(pl.g.B);
  // |.| keeps a NaN visible (std::max(0, NaN) would hide it)
  for (int b = 0; b < pl.g.B; ++b) out[b] = std::sqrt(std::fabs(tmp[(size_t)b * MAXV]));
  return PD_OK;
}


}  // namespace


static paradiag_status check_hip(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return PD_ERR_HIP;
  }
  return PD_OK;
}

static paradiag_status solve_impl(Plan& pl, int variant, const double* b, double* u,
                                  const paradiag_solve_opts* o, paradiag_solve_info* info,
                                  hipStream_t s) {
  const Geom& g = pl.g;
  const int B = g.B;
  char* p = pl.solver_base;
  size_t need = solver_bytes(pl, o);
  if ((size_t)(pl.ws + pl.ws_bytes - pl.solver_base) < need) {
    set_error("workspace too small for this solve (see paradiag_workspace_size)");
    return PD_ERR_WORKSPACE;
  }
  const bool zf32 = pl.prec != Prec::F64;
  const size_t zb = zf32 ? 4 : 8;
  Small sm = carve_small(pl, p);
  if (!pinned(pl)) { set_error("pinned host staging allocation failed"); return PD_ERR_HIP; }
  // FGMRES from a zero guess takes V_0 = b: the first cycle reads it in place
  const bool fused_start = o->mode == PD_MODE_FGMRES && !o->use_x0;
  // ... and, when it cannot end before its first Arnoldi step, starts that
  // step from the unnormalised b: ||b|| then comes from the step's own matvec
  // (which reads b for its first dot anyway) instead of a pass of its own, and
  // the step's scalars are rescaled once it is known
  const bool defer_norm = fused_start && o->rtol < 1.0 && o->max_iter >= 1;
  std::vector<double> bn(B, 1.0);   // placeholders while defer_norm
  if (!defer_norm) {
    timed_dot(pl, b, 0, 1, b, sm.partial, s);
    if (paradiag_status st = norms_from(pl, sm, bn, s); st != PD_OK) return st;
    for (int i = 0; i < B; ++i)
      if (!std::isfinite(bn[i])) { set_error("right-hand side contains NaN or Inf"); return PD_ERR_NONFINITE; }
  }
  std::vector<int> it_rhs(B, 0);
  std::vector<double> res(B, 0.0);
  int iters = 0;
  int hist_len = 0;
  // false while u is implicitly zero (FGMRES from a zero guess has not yet
  // written it): the first solution update then overwrites instead of adding
  bool u_valid = true;
  auto push_hist = [&](double v) {
    if (info && info->history && hist_len < info->history_cap) info->history[hist_len] = v;
    ++hist_len;
  };
  auto finish = [&](bool conv) -> paradiag_status {
    if (!u_valid) { fill_zero(u, g.NA, s); u_valid = true; }
    double mx = 0;
    for (int i = 0; i < B; ++i) mx = std::max(mx, res[i]);
    if (info) {
      info->iters = iters;
      info->converged = conv ? 1 : 0;
      info->rel_resid = mx;
      info->history_len = std::min(hist_len, info->history ? info->history_cap : 0);
      for (int i = 0; i < B; ++i) {
        if (info->iters_per_rhs) info->iters_per_rhs[i] = it_rhs[i];
        if (info->resid_per_rhs) info->resid_per_rhs[i] = res[i];
      }
    }
    paradiag_status st = check_hip("solve");
    if (st != PD_OK) return st;
    return conv ? PD_OK : PD_NOT_CONVERGED;
  };
  auto rel = [&](const std::vector<double>& nr) {
    bool all = true;
    for (int i = 0; i < B; ++i) {
      res[i] = bn[i] > 0 ? nr[i] / bn[i] : 0.0;
      if (res[i] > o->rtol) all = false;
    }
    return all;
  };

  if (o->mode == PD_MODE_DIRECT) {
    apply_prec(pl, variant, b, nullptr, 0, u, false, 0, s);
    iters = 1;
    for (int i = 0; i < B; ++i) it_rhs[i] = 1;
    // residual of the result with respect to A (reported, not iterated; its
    // norm only)
    std::vector<double> nr;
    apply_A(pl, variant, u, false, b, nullptr, s, sm.partial);
    if (paradiag_status st = norms_from(pl, sm, nr, s, matvec_chunks(pl)); st != PD_OK) return st;
    rel(nr);
    push_hist(*std::max_element(res.begin(), res.end()));
    return finish(true);
  }

  if (o->mode == PD_MODE_STATIONARY) {
    double* r = (double*)p;
    if (!o->use_x0) fill_zero(u, g.NA, s);
    std::vector<double> nr;
    while (true) {
      apply_A(pl, variant, u, false, b, r, s, sm.partial);
      if (paradiag_status st = norms_from(pl, sm, nr, s, matvec_chunks(pl)); st != PD_OK) return st;
      bool all = rel(nr);
      for (int i = 0; i < B; ++i)
        if (!std::isfinite(res[i])) { set_error("non-finite residual"); return PD_ERR_NONFINITE; }
      push_hist(*std::max_element(res.begin(), res.end()));
      if (all) return finish(true);
      if (iters >= o->max_iter) return finish(false);
      apply_prec(pl, variant, r, nullptr, 0, u, false, 1, s);
      ++iters;
      for (int i = 0; i < B; ++i)
        if (res[i] > o->rtol) it_rhs[i] = iters;
    }
  }

  // ---------------------------------------------------------------- FGMRES
  const int m = std::max(1, std::min(o->restart, 32));
  double* V = (double*)p;
  const int64_t vs = (int64_t)(align_up(sizeof(double) * (size_t)g.NA) / sizeof(double));
  p += align_up(sizeof(double) * (size_t)g.NA) * (m + 1);
  char* Z = p;
  const int64_t zs = (int64_t)(align_up(zb * (size_t)g.NA) / zb);
  auto Vj = [&](int j) { return V + (int64_t)j * vs; };
  auto Zj = [&](int j) { return (void*)(Z + (size_t)j * zs * zb); };

  if (!o->use_x0) u_valid = false;
  std::vector<double> H((size_t)B * (m + 1) * m), gv((size_t)B * (m + 1)), cs((size_t)B * m),
      sn((size_t)B * m);
  // pinned staging (see pinned): Hessenberg columns, Krylov scales, LSQ solution
  const size_t ps = pin_slot(pl);
  double* hbuf = pl.pin + ps;            // h1, then h2 at + ps, then the skip flag
  double* h2buf = hbuf + ps;
  int* skiph = reinterpret_cast<int*>(hbuf + 2 * ps);
  double* sig = pl.pin + 4 * ps;         // sigma, then the Givens state at + ps
  double* givh = sig + ps;
  double* yv = pl.pin + 8 * ps;
  std::vector<double> nr;
  bool first = true;
  while (true) {
    // residual of the current iterate into V_0 (from a zero guess V_0 = b,
    // read where it is: V0x, in place of the basis slot, for the kernels that
    // read V_0)
    const double* V0x = nullptr;
    if (first && fused_start) {
      nr = bn;
      V0x = b;
    } else {
      // the norm first; the residual itself is stored (as V_0) only when
      // another cycle follows
      if (!u_valid) { fill_zero(u, g.NA, s); u_valid = true; }
      apply_A(pl, variant, u, false, b, nullptr, s, sm.partial);
      if (paradiag_status st = norms_from(pl, sm, nr, s, matvec_chunks(pl)); st != PD_OK) return st;
    }
    const bool restart_cycle = !(first && fused_start);
    // this cycle's step 0 runs on the unnormalised b (scale 1 until known)
    const bool defer = first && defer_norm;
    first = false;
    bool all = rel(nr);
    for (int i = 0; i < B; ++i)
      if (!std::isfinite(res[i])) { set_error("non-finite residual"); return PD_ERR_NONFINITE; }
    push_hist(*std::max_element(res.begin(), res.end()));
    if (all) return finish(true);
    if (iters >= o->max_iter) return finish(false);
    if (restart_cycle) apply_A(pl, variant, u, false, b, Vj(0), s);
    std::vector<char> active(B);
    for (int i = 0; i < B; ++i) active[i] = res[i] > o->rtol && nr[i] > 0;
    std::fill(sig, sig + (size_t)B * MAXV, 0.0);
    for (int i = 0; i < B; ++i) {
      if (active[i]) sig[(size_t)i * MAXV] = 1.0 / nr[i];
      gv[(size_t)i * (m + 1)] = nr[i];
    }
    std::vector<int> kk(B, 0);   // columns used per right-hand side
    std::vector<char> live = active;
    bool second = true, skipped = false;
    // Givens state of step jj for k_arnoldi_skip, per right-hand side:
    // [rtol ||b|| (negative when not live), g_jj, c_0..c_{jj-1}, s_0..s_{jj-1}],
    // copied with the scales (the host rewrites the pinned area only after the
    // step's synchronisation)
    auto stage_givens = [&](int jj) {
      for (int i = 0; i < B; ++i) {
        double* G = givh + (size_t)i * GIVS;
        G[0] = live[i] ? o->rtol * bn[i] : -1.0;
        G[1] = gv[(size_t)i * (m + 1) + jj];
        for (int q = 0; q < jj; ++q) {
          G[2 + q] = cs[(size_t)i * m + q];
          G[2 + jj + q] = sn[(size_t)i * m + q];
        }
      }
    };
    // the step's scales and Givens state, one copy
    auto send_scales = [&]() { fetch_host(sig, sm.sigma, (int)(ps + (size_t)B * GIVS), s); };
    stage_givens(0);
    send_scales();
    int j = 0;
    for (; j < m; ++j) {
      // z_j = P^{-1} v_j  (v_j = sigma_j V_j, the scale fused into Step-(a) and
      // read from the device copy of the scales, entry i * MAXV + j)
      apply_prec(pl, variant, (j == 0 && V0x) ? V0x : Vj(j), sm.sigma + j, MAXV, Zj(j), zf32, 0, s);
      {
        double* w = Vj(j + 1);
        // w = A z_j with the first pass's dots V_q . w (q <= j) from the same kernel
        {
          const double n = (double)g.NA;
          Timed t(pl, PD_STAGE_MATVEC, s, n * ((zf32 ? 4.0 : 8.0) + 8.0 + 8.0 * (j + 1)),
                  n * ((pl.L == 3 ? 22.0 : 18.0) + 2.0 * (j + 1)));
          matvec(pl, pl.op[variant], Zj(j), zf32, nullptr, w, variant, s, V, vs, j + 1, sm.partial, 1, V0x,
                 (defer && j == 0) ? 1 : 0);
        }
        // classical Gram-Schmidt, two passes; the first pass's dots (and w . w)
        // come from the matvec kernel, the second pass's from the first pass's
        // update kernel, the final norm by Pythagoras.  The second update is
        // applied only when some live right-hand side keeps a component along
        // the basis that matters (kReorthTol, kReorthMax, kReorthRel):
        // otherwise the vector is kept as it is.
        {
          Timed t(pl, PD_STAGE_OTHER, s);
          reduce_partials(pl, sm.partial, j + ((defer && j == 0) ? 3 : 2), sm.sigma, j + 1, sm.h1, sm.c1, s,
                          matvec_chunks(pl), hbuf);
        }
        // A step that ends its cycle (every live residual estimate within
        // rtol, or the restart length or iteration limit reached) needs no
        // orthogonalised w: its subdiagonal entry follows from w . w and the
        // first pass by Pythagoras.  The device decides before the update,
        // which then returns at once (the Givens state it needs was staged
        // with the step's scales).
        {
          Timed t(pl, PD_STAGE_OTHER, s);
          const bool force = j + 1 == m || iters + 1 >= o->max_iter;
          arnoldi_skip(pl, sm.h1, sm.giv, GIVS, j, force, sm.skip, s, skiph, defer && j == 0, sm.c1,
                       sm.sigma, o->rtol);
        }
        const double upd_bytes = (double)g.NA * 8.0 * (j + 3);
        const double upd_flops = (double)g.NA * (4.0 * (j + 1) + 2.0);
        timed_update(pl, V, vs, j + 1, sm.c1, w, sm.partial, 1, s, sm.skip, V0x);
        timed_reduce(pl, sm.partial, j + 2, sm.sigma, j + 1, sm.h2, sm.c2, s, 0, h2buf);
        // h1, h2 and the flag are in pinned memory
        if (paradiag_status st = wait_host(pl, s); st != PD_OK) return st;
        skipped = *skiph != 0;
        if (defer && j == 0) {
          // beta = ||b|| from slot 2; V_0 = b and z_0, w carry the factor
          // beta against the unit-norm basis: h1 (dots taken with scale 1)
          // and w . w scale by 1/beta^2, the second pass's dots (taken with
          // the device's scale 1/beta) by 1/beta
          bool any = false;
          for (int i = 0; i < B; ++i) {
            double* h1 = hbuf + (size_t)i * MAXV;
            double* h2 = h2buf + (size_t)i * MAXV;
            const double beta = std::sqrt(h1[2]);
            if (!std::isfinite(beta)) { set_error("right-hand side contains NaN or Inf"); return PD_ERR_NONFINITE; }
            bn[i] = beta;
            nr[i] = beta;
            gv[(size_t)i * (m + 1)] = beta;
            active[i] = live[i] = beta > 0.0;
            any = any || beta > 0.0;
            const double r1 = beta > 0.0 ? 1.0 / beta : 0.0;
            sig[(size_t)i * MAXV] = r1;
            h1[0] *= r1 * r1;
            h1[1] *= r1 * r1;
            h2[0] *= r1;
            h2[1] *= r1 * r1;
            res[i] = beta > 0.0 ? 1.0 : 0.0;
          }
          if (!any) {   // b = 0: u = 0, nothing iterated
            if (info && info->history && info->history_cap > 0) info->history[0] = 0.0;
            return finish(true);
          }
        }
        second = false;
        if (skipped) {
          untime_last(pl, PD_STAGE_UPDATE, upd_bytes, upd_flops);   // it did not run
        } else {
          for (int i = 0; i < B; ++i) {
            if (!live[i]) continue;
            const double* h2 = h2buf + (size_t)i * MAXV;
            double mx = 0;
            for (int q = 0; q <= j; ++q) mx = std::max(mx, h2[q] * h2[q]);
            const double eta = std::sqrt(mx / h2[j + 1]);   // NaN when h2[j+1] <= 0: second pass
            const double est_prev = std::fabs(gv[(size_t)i * (m + 1) + j]) / bn[i];
            if (!(eta <= kReorthTol) && (!(eta <= kReorthMax) || !(eta * est_prev <= kReorthRel * o->rtol)))
              second = true;
          }
          if (second) timed_update(pl, V, vs, j + 1, sm.c2, w, sm.partial, 0, s, nullptr, V0x);
        }
      }
      ++iters;
      double est_max = 0;
      bool any_live = false;
      for (int i = 0; i < B; ++i) {
        const double* h1 = hbuf + (size_t)i * MAXV;
        const double* h2 = h2buf + (size_t)i * MAXV;
        double* Hc = H.data() + (size_t)i * (m + 1) * m;   // column-major (m+1) x m
        for (int q = 0; q <= j; ++q) {
          double v = h1[q] + (second ? h2[q] : 0.0);
          if (!std::isfinite(v)) { set_error("non-finite Krylov scalar"); return PD_ERR_NONFINITE; }
          Hc[(size_t)j * (m + 1) + q] = v;
        }
        double nn = h2[j + 1];
        if (second)
          for (int q = 0; q <= j; ++q) nn -= h2[q] * h2[q];
        if (skipped) {   // w . w minus the first pass (see k_arnoldi_skip)
          nn = h1[j + 1];
          for (int q = 0; q <= j; ++q) nn -= h1[q] * h1[q];
        }
        double hn = nn > 0 ? std::sqrt(nn) : 0.0;
        Hc[(size_t)j * (m + 1) + j + 1] = hn;
        if (!live[i]) { sig[(size_t)i * MAXV + j + 1] = 0.0; continue; }
        // Givens rotations
        double* col = Hc + (size_t)j * (m + 1);
        double* c_ = cs.data() + (size_t)i * m;
        double* s_ = sn.data() + (size_t)i * m;
        double* gg = gv.data() + (size_t)i * (m + 1);
        for (int q = 0; q < j; ++q) {
          double t = c_[q] * col[q] + s_[q] * col[q + 1];
          col[q + 1] = -s_[q] * col[q] + c_[q] * col[q + 1];
          col[q] = t;
        }
        double a = col[j], bb = col[j + 1];
        double cc = 1, ss = 0;
        if (bb != 0.0) { double rr = std::hypot(a, bb); cc = a / rr; ss = bb / rr; }
        c_[j] = cc; s_[j] = ss;
        col[j] = cc * a + ss * bb;
        col[j + 1] = 0.0;
        gg[j + 1] = -ss * gg[j];
        gg[j] = cc * gg[j];
        kk[i] = j + 1;
        it_rhs[i] += 1;
        double est = std::fabs(gg[j + 1]) / bn[i];
        est_max = std::max(est_max, est);
        if (est <= o->rtol || hn == 0.0) live[i] = 0;
        else any_live = true;
        // (the stored V_1 of a deferred step 0 carries the factor beta too)
        const double vscale = (defer && j == 0) ? sig[(size_t)i * MAXV] : 1.0;
        sig[(size_t)i * MAXV + j + 1] = (hn > 0 && live[i]) ? vscale / hn : 0.0;
      }
      push_hist(est_max);
      // a skipped update ends the cycle whatever the host's estimate says (w
      // was not orthogonalised); the true residual decides what follows
      if (skipped || !any_live || iters >= o->max_iter || j + 1 == m) { ++j; break; }
      stage_givens(j + 1);
      send_scales();
    }
    // solve the triangular systems and update x
    std::fill(yv, yv + (size_t)B * MAXV, 0.0);
    int kmax = 0;
    for (int i = 0; i < B; ++i) {
      int k = kk[i];
      kmax = std::max(kmax, k);
      const double* Hc = H.data() + (size_t)i * (m + 1) * m;
      const double* gg = gv.data() + (size_t)i * (m + 1);
      double* y = yv + (size_t)i * MAXV;
      for (int q = k - 1; q >= 0; --q) {
        double acc = gg[q];
        for (int c = q + 1; c < k; ++c) acc -= Hc[(size_t)c * (m + 1) + q] * y[c];
        double d = Hc[(size_t)q * (m + 1) + q];
        y[q] = d != 0.0 ? acc / d : 0.0;
      }
      // Z_0 of a deferred step 0 is beta z_0
      if (defer && k > 0 && bn[i] > 0.0) y[0] /= bn[i];
    }
    if (kmax > 0) {
      fetch_host(yv, sm.y, B * MAXV, s);
      Timed t(pl, PD_STAGE_OTHER, s, (double)g.NA * (16.0 + kmax * (double)zb), 2.0 * g.NA * kmax);
      x_update(pl, Z, zf32, zs, kmax, sm.y, u, !u_valid, s);
      u_valid = true;
    }
  }
}

}  // namespace pd

// ====================================================================== ABI

using namespace pd;

// bf16 storage: float rounded to nearest even, upper 16 bits kept
struct Bf16Bits { uint16_t v; };
static uint16_t to_bf16_bits(double x) {
  float f = (float)x;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <typename T>
static void store_compute(void* dst, const std::vector<double>& v, hipStream_t s,
                          std::vector<std::vector<char>>& keep) {
  std::vector<char> buf(v.size() * sizeof(T));
  T* t = reinterpret_cast<T*>(buf.data());
  for (size_t i = 0; i < v.size(); ++i) {
    if constexpr (std::is_same<T, Bf16Bits>::value) t[i].v = to_bf16_bits(v[i]);
    else t[i] = (T)v[i];
  }
  hipMemcpyAsync(dst, buf.data(), buf.size(), hipMemcpyHostToDevice, s);
  keep.push_back(std::move(buf));
}

extern "C" {

const char* paradiag_last_error(void) { return g_last_error.c_str(); }
const char* paradiag_version(void) { return "paradiag-gfx950 0.1"; }

paradiag_status paradiag_oc_setup(const paradiag_problem* prob, double gamma, paradiag_plan* out) {
  if (!out) { set_error("out is NULL"); return PD_ERR_INVALID; }
  *out = nullptr;
  if (!(gamma > 0.0)) { set_error("gamma must be positive"); return PD_ERR_INVALID; }
  try {
    Plan* pl = nullptr;
    paradiag_status st = build_plan(prob, pl, gamma);
    if (st != PD_OK) return st;
    *out = reinterpret_cast<paradiag_plan>(pl);
    return PD_OK;
  } catch (...) {
    set_error("out of host memory");
    return PD_ERR_INVALID;
  }
}

paradiag_status paradiag_setup(const paradiag_problem* prob, paradiag_plan* out) {
  if (!out) { set_error("out is NULL"); return PD_ERR_INVALID; }
  *out = nullptr;
  try {
    Plan* pl = nullptr;
    paradiag_status st = build_plan(prob, pl);
    if (st != PD_OK) return st;
    *out = reinterpret_cast<paradiag_plan>(pl);
    return PD_OK;
  } catch (...) {
    set_error("setup failed (host allocation)");
    return PD_ERR_INVALID;
  }
}

void paradiag_destroy(paradiag_plan plan) {
  Plan* pl = reinterpret_cast<Plan*>(plan);
  if (!pl) return;
  for (auto& r : pl->timer.pending) { hipEventDestroy(r.a); hipEventDestroy(r.b); }
  for (auto e : pl->timer.pool) hipEventDestroy(e);
  if (pl->sweep_fork) hipEventDestroy(pl->sweep_fork);
  if (pl->sweep_join) hipEventDestroy(pl->sweep_join);
  if (pl->sweep_side) hipStreamDestroy(pl->sweep_side);
  if (pl->pin) hipHostFree(pl->pin);
  delete pl;
}

paradiag_status paradiag_workspace_size(paradiag_plan plan, const paradiag_solve_opts* opts,
                                        size_t* bytes) {
  Plan* pl = reinterpret_cast<Plan*>(plan);
  if (!pl || !bytes) { set_error("NULL argument"); return PD_ERR_INVALID; }
  if (opts && (opts->mode < 0 || opts->mode > 4)) { set_error("unknown mode"); return PD_ERR_INVALID; }
  *bytes = tables_bytes(*pl) + solver_bytes(*pl, opts);
  return PD_OK;
}



paradiag_status paradiag_bind_workspace(paradiag_plan plan, void* workspace, size_t bytes,
                                        void* stream) {
  Plan* pl = reinterpret_cast<Plan*>(plan);
  if (!pl || !workspace) { set_error("NULL argument"); return PD_ERR_INVALID; }
  if (reinterpret_cast<uintptr_t>(workspace) % ALIGN) { set_error("workspace must be 256-byte aligned"); return PD_ERR_INVALID; }
  size_t need = tables_bytes(*pl);
  if (bytes < need) { set_error("workspace smaller than the device tables"); return PD_ERR_WORKSPACE; }
  hipStream_t s = (hipStream_t)stream;
  const Geom& g = pl->g;
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
      pl->num_cu = ncu;
  }
  char* p = (char*)workspace;
  auto take = [&](size_t n) { char* r = p; p += align_up(n); return r; };
  std::vector<std::vector<char>> keep;
  auto up = [&](void* dst, const void* src, size_t n) {
    std::vector<char> buf((const char*)src, (const char*)src + n);
    hipMemcpyAsync(dst, buf.data(), n, hipMemcpyHostToDevice, s);
    keep.push_back(std::move(buf));
  };
  pl->d_gam = (double*)take(sizeof(double) * g.nt);
  pl->d_invgam = (double*)take(sizeof(double) * g.nt);
  pl->d_tw64 = (double2*)take(sizeof(double2) * g.nt);
  pl->d_tw32 = (float2*)take(sizeof(float2) * g.nt);
  pl->d_lam = (double2*)take(sizeof(double2) * 2 * g.F);
  if (pl->dst) pl->d_dtw = take(spec_elem_bytes(pl->prec) * 2 * (g.nx + 1));
  if (pl->prec == Prec::F16 && pl->p.dim == 2)
    pl->d_rowscale = (float*)take(sizeof(float) * 2 * (size_t)g.B * g.F * g.sy);
  if (sweep_windowed(*pl)) pl->d_rmax = (float*)take(sizeof(float) * (size_t)g.B * g.F * g.sy);
  if (sweep_windowed(*pl) && g.B >= 2 && !pl->sweep_side) {
    if (hipStreamCreateWithFlags(&pl->sweep_side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&pl->sweep_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&pl->sweep_join, hipEventDisableTiming) != hipSuccess) {
      set_error("creating the back-sweep's second stream");
      return PD_ERR_HIP;
    }
  }
  up(pl->d_gam, pl->gam.data(), sizeof(double) * g.nt);
  up(pl->d_invgam, pl->invgam.data(), sizeof(double) * g.nt);
  {
    const double PI = 3.14159265358979323846;
    std::vector<double2> t64(g.nt);
    std::vector<float2> t32(g.nt);
    for (int k = 0; k < g.nt; ++k) {
      double a = -2.0 * PI * k / g.nt;
      t64[k] = double2{std::cos(a), std::sin(a)};
      t32[k] = float2{(float)std::cos(a), (float)std::sin(a)};
    }
    up(pl->d_tw64, t64.data(), sizeof(double2) * g.nt);
    up(pl->d_tw32, t32.data(), sizeof(float2) * g.nt);
    if (pl->dst) {   // first half of the length-2(nx+1) table, in the compute precision
      const int h = g.nx + 1;
      std::vector<double2> d64(h);
      std::vector<float2> d32(h);
      for (int k = 0; k < h; ++k) {
        const double a = -PI * k / h;
        d64[k] = double2{std::cos(a), std::sin(a)};
        d32[k] = float2{(float)std::cos(a), (float)std::sin(a)};
      }
      if (pl->prec == Prec::F64) up(pl->d_dtw, d64.data(), sizeof(double2) * h);
      else up(pl->d_dtw, d32.data(), sizeof(float2) * h);
    }
    std::vector<double2> lam(2 * g.F);
    for (int n = 0; n < g.F; ++n) {
      lam[n] = double2{pl->lam1[n].real(), pl->lam1[n].imag()};
      lam[g.F + n] = double2{pl->lam2[n].real(), pl->lam2[n].imag()};
    }
    up(pl->d_lam, lam.data(), sizeof(double2) * 2 * g.F);
  }
  if (pl->oc) {
    const size_t f1 = time_gemm_fragment_elems(2 * pl->oc_fh, g.nt), f2 = time_gemm_fragment_elems(g.nt, 2 * pl->oc_fh);
    pl->d_wf = (double*)take(sizeof(double) * f1);
    pl->d_wi = (double*)take(sizeof(double) * f2);
    pl->d_ocmix = (double2*)take(sizeof(double2) * 3 * pl->oc_fh);
    up(pl->d_wf, pl->wf_frag.data(), sizeof(double) * f1);
    up(pl->d_wi, pl->wi_frag.data(), sizeof(double) * f2);
    up(pl->d_ocmix, pl->ocmix.data(), sizeof(double2) * 3 * pl->oc_fh);
  }
  if (pl->hybrid) {
    const size_t fe = time_gemm_fragment_elems(g.nt, g.nt);
    pl->d_wf = (double*)take(sizeof(double) * fe);
    pl->d_wi = (double*)take(sizeof(double) * fe);
    pl->d_band = (double*)take(sizeof(double) * 5 * g.nt);
    pl->d_band_t = (double*)take(sizeof(double) * 5 * g.nt);
    up(pl->d_wf, pl->wf_frag.data(), sizeof(double) * fe);
    up(pl->d_wi, pl->wi_frag.data(), sizeof(double) * fe);
    up(pl->d_band, pl->band.data(), sizeof(double) * 5 * g.nt);
    up(pl->d_band_t, pl->band_t.data(), sizeof(double) * 5 * g.nt);
  }
  if (pl->p.dim == 2) {
    const int n = g.nx;
    for (int v = 0; v < 2; ++v) {
      SpaceOp& op = pl->op[v];
      std::vector<double2> tk(n);
      for (int k = 0; k < n; ++k) tk[k] = double2{op.Tm[(size_t)k * n + k].real(), op.Tm[(size_t)k * n + k].imag()};
      op.tk = (const double2*)take(sizeof(double2) * n);
      up((void*)op.tk, tk.data(), sizeof(double2) * n);
      // GEMM matrices: out = in * G, stored Bt[col][k]
      std::vector<double> gf, gi;
      const size_t ce = compute_elem_bytes(pl->prec);
      if (!pl->schur) {
        gf.resize((size_t)n * n);
        gi.resize((size_t)n * n);
        for (int c = 0; c < n; ++c)
          for (int k = 0; k < n; ++k) {
            gf[(size_t)c * n + k] = op.Q[(size_t)k * n + c].real();          // G = conj(Q) = Q
            gi[(size_t)c * n + k] = op.Q[(size_t)c * n + k].real();          // G = Q^T
          }
      } else {
        const int n2 = 2 * n;
        gf.resize((size_t)n2 * n2);
        gi.resize((size_t)n2 * n2);
        auto fill = [&](std::vector<double>& Bt, auto G) {
          // real block matrix M = [[Gr, Gi], [-Gi, Gr]] (row index k, column j); Bt[j][k] = M[k][j]
          for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j) {
              cd v = G(k, j);
              Bt[(size_t)j * n2 + k] = v.real();
              Bt[(size_t)(j + n) * n2 + k] = v.imag();
              Bt[(size_t)j * n2 + (k + n)] = -v.imag();
              Bt[(size_t)(j + n) * n2 + (k + n)] = v.real();
            }
        };
        fill(gf, [&](int k, int j) { return std::conj(op.Q[(size_t)k * n + j]); });
        fill(gi, [&](int k, int j) { return op.Q[(size_t)j * n + k]; });
      }
      (void)ce;
      op.g_fwd = take(gemm_matrix_bytes(pl->prec, gf.size()));
      op.g_inv = take(gemm_matrix_bytes(pl->prec, gi.size()));
      for (int w = 0; w < 2; ++w) {
        void* dst = (void*)(w ? op.g_inv : op.g_fwd);
        const std::vector<double>& src = w ? gi : gf;
        if (pl->prec == Prec::F64) store_compute<double>(dst, src, s, keep);
        else if (pl->prec == Prec::F32) store_compute<float>(dst, src, s, keep);
        else if (pl->prec == Prec::BF16X1) store_compute<Bf16Bits>(dst, src, s, keep);
        else if (pl->prec == Prec::F16) {
          // two fp16 parts of the entry times F16_BSCALE (the residual after the
          // first is exact in float32), then a float32 copy
          std::vector<uint16_t> part[2];
          for (auto& v : part) v.resize(src.size());
          for (size_t i = 0; i < src.size(); ++i) {
            const float x = (float)src[i] * F16_BSCALE;
            const _Float16 h = (_Float16)x;
            const _Float16 l = (_Float16)(x - (float)h);
            std::memcpy(&part[0][i], &h, 2);
            std::memcpy(&part[1][i], &l, 2);
          }
          for (int a = 0; a < 2; ++a) {
            std::vector<char> buf((const char*)part[a].data(), (const char*)part[a].data() + 2 * src.size());
            hipMemcpyAsync((char*)dst + 2 * a * src.size(), buf.data(), buf.size(), hipMemcpyHostToDevice, s);
            keep.push_back(std::move(buf));
          }
          store_compute<float>((char*)dst + 4 * src.size(), src, s, keep);
        } else {
          // three bf16 parts of the float32 value (hi, then the rounded
          // residuals mid and lo; the float32 subtractions are exact), then
          // a float32 copy
          std::vector<double> part[3];
          for (auto& v : part) v.resize(src.size());
          for (size_t i = 0; i < src.size(); ++i) {
            float rest = (float)src[i];
            for (int a = 0; a < 3; ++a) {
              uint32_t u = (uint32_t)to_bf16_bits(rest) << 16;
              float h;
              std::memcpy(&h, &u, 4);
              part[a][i] = h;
              rest -= h;
            }
          }
          for (int a = 0; a < 3; ++a) store_compute<Bf16Bits>((char*)dst + 2 * a * src.size(), part[a], s, keep);
          store_compute<float>((char*)dst + 6 * src.size(), src, s, keep);
        }
      }
      if (pl->schur) {
        std::vector<double> tp(2 * (size_t)n * n);
        for (size_t i = 0; i < (size_t)n * n; ++i) { tp[i] = op.Tm[i].real(); tp[(size_t)n * n + i] = op.Tm[i].imag(); }
        op.tup = take(tp.size() * spec_elem_bytes(pl->prec));
        if (pl->prec == Prec::F64) store_compute<double>((void*)op.tup, tp, s, keep);
        else store_compute<float>((void*)op.tup, tp, s, keep);
        op.lu = take((size_t)2 * g.F * n * g.sy * spec_elem_bytes(pl->prec));
        op.tfar = nullptr;
        if (sweep_windowed(*pl)) {
          // the windowed sweep's far-coupling product: B^T[m][k] with m < n the
          // real and m >= n the imaginary part of mode q = m mod n, and k < n
          // the real, k >= n the imaginary part of the solved mode:
          // [[Tr, -Ti], [Ti, Tr]] row-wise, times the power of two that brings
          // its largest entry into [2^13, 2^14), as two fp16 parts (hi, lo)
          const size_t n2 = 2 * (size_t)n;
          double tmax = 0.0;
          for (const cd& t : op.Tm) tmax = std::max({tmax, std::fabs(t.real()), std::fabs(t.imag())});
          int e2 = 0;
          (void)std::frexp(tmax, &e2);
          const float tsc = tmax > 0.0 ? std::ldexp(1.0f, 14 - e2) : 1.0f;
          op.tfar_inv = 1.0f / tsc;
          std::vector<_Float16> part[2];
          for (auto& v : part) v.assign(n2 * n2, (_Float16)0.0f);
          for (int q = 0; q < n; ++q)
            for (int j = 0; j < n; ++j) {
              const cd t = op.Tm[(size_t)q * n + j];
              const double e[4] = {t.real(), -t.imag(), t.imag(), t.real()};
              const size_t at[4] = {q * n2 + j, q * n2 + n + j, (n + q) * n2 + j, (n + q) * n2 + n + j};
              for (int c = 0; c < 4; ++c) {
                const float x = (float)e[c] * tsc;   // exact: a power of two
                const _Float16 h = (_Float16)x;
                part[0][at[c]] = h;
                part[1][at[c]] = (_Float16)(x - (float)h);
              }
            }
          op.tfar = take(2 * n2 * n2 * 2);
          for (int a = 0; a < 2; ++a) {
            std::vector<char> buf((const char*)part[a].data(), (const char*)part[a].data() + 2 * n2 * n2);
            hipMemcpyAsync((char*)op.tfar + 2 * a * n2 * n2, buf.data(), buf.size(), hipMemcpyHostToDevice, s);
            keep.push_back(std::move(buf));
          }
        }
      } else {
        op.tfar = nullptr;
        op.tup = nullptr;
        op.lu = nullptr;
      }
    }
  }
  // line factorisations of the back-sweep (both operators), once per binding
  if (pl->p.dim == 2 && pl->schur)
    for (int v = 0; v < 2; ++v) schur_line_lu(*pl, pl->op[v], s);
  pl->spec_a = take((size_t)g.spec_elems * spec_elem_bytes(pl->prec));
  pl->spec_b = take((size_t)g.spec_elems * spec_elem_bytes(pl->prec));
  pl->solver_base = p;
  pl->ws = (char*)workspace;
  pl->ws_bytes = bytes;
  pl->bound = true;
  hipError_t e = hipStreamSynchronize(s);   // host staging buffers must outlive the copies
  if (e != hipSuccess) { set_error(std::string("bind: ") + hipGetErrorString(e)); return PD_ERR_HIP; }
  return PD_OK;
}

static Plan* ready(paradiag_plan plan) {
  Plan* pl = reinterpret_cast<Plan*>(plan);
  if (!pl) { set_error("plan is NULL"); return nullptr; }
  if (!pl->bound) { set_error("no workspace bound"); return nullptr; }
  return pl;
}

static bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return a && b && x < y + nb && y < x + na;
}

paradiag_status paradiag_build_rhs(paradiag_plan plan, const double* U0, const double* u1,
                                   const double* f, double* b, void* stream) {
  Plan* pl = ready(plan);
  if (!pl) return plan ? PD_ERR_WORKSPACE : PD_ERR_INVALID;
  if (!U0 || !b) { set_error("U0 and b are required"); return PD_ERR_INVALID; }
  if (pl->oc) { set_error("optimal-control plans build their right-hand side with paradiag_oc_build_rhs"); return PD_ERR_UNSUPPORTED; }
  build_rhs(*pl, U0, (pl->p.scheme == PD_LEAPFROG || pl->p.scheme == PD_HYBRID_WAVE) ? u1 : nullptr, f, b, (hipStream_t)stream);
  return check_hip("build_rhs");
}

paradiag_status paradiag_oc_build_rhs(paradiag_plan plan, const double* U0, const double* u1,
                                      const double* f, const double* g, double* b, void* stream) {
  Plan* pl = ready(plan);
  if (!pl) return plan ? PD_ERR_WORKSPACE : PD_ERR_INVALID;
  if (!pl->oc) { set_error("not an optimal-control plan"); return PD_ERR_INVALID; }
  if (!U0 || !b) { set_error("U0 and b are required"); return PD_ERR_INVALID; }
  oc_build_rhs(*pl, U0, u1, f, g, b, (hipStream_t)stream);
  return check_hip("oc_build_rhs");
}

paradiag_status paradiag_rhs_transpose(paradiag_plan plan, const double* lam, double* gU0,
                                       double* gu1, double* gf, void* stream) {
  Plan* pl = ready(plan);
  if (!pl) return plan ? PD_ERR_WORKSPACE : PD_ERR_INVALID;
  if (!lam || !gU0) { set_error("lam and gU0 are required"); return PD_ERR_INVALID; }
  if (pl->hybrid || pl->oc) { set_error("rhs_transpose is not provided for this plan"); return PD_ERR_UNSUPPORTED; }
  rhs_transpose(*pl, lam, gU0, gu1, gf, (hipStream_t)stream);
  return check_hip("rhs_transpose");
}

paradiag_status paradiag_matvec(paradiag_plan plan, const double* u, double* y, int32_t transpose,
                                void* stream) {
  Plan* pl = ready(plan);
  if (!pl) return plan ? PD_ERR_WORKSPACE : PD_ERR_INVALID;
  if (!u || !y) { set_error("NULL vector"); return PD_ERR_INVALID; }
  size_t nb = sizeof(double) * (size_t)pl->g.NA;
  if (overlap(u, nb, y, nb)) { set_error("u and y overlap"); return PD_ERR_INVALID; }
  if (pl->oc && transpose) { set_error("the transpose of the optimal-control operator is not provided"); return PD_ERR_UNSUPPORTED; }
  apply_A(*pl, transpose ? 1 : 0, u, false, nullptr, y, (hipStream_t)stream);
  return check_hip("matvec");
}

paradiag_status paradiag_apply_precond(paradiag_plan plan, const double* r, double* z,
                                       void* stream) {
  Plan* pl = ready(plan);
  if (!pl) return plan ? PD_ERR_WORKSPACE : PD_ERR_INVALID;
  if (!r || !z) { set_error("NULL vector"); return PD_ERR_INVALID; }
  size_t nb = sizeof(double) * (size_t)pl->g.NA;
  if (r != z && overlap(r, nb, z, nb)) { set_error("r and z partially overlap"); return PD_ERR_INVALID; }
  apply_prec(*pl, 0, r, nullptr, 0, z, false, 0, (hipStream_t)stream);
  return check_hip("apply_precond");
}

static paradiag_status solve_entry(paradiag_plan plan, int variant, const double* b, double* u,
                                   const paradiag_solve_opts* opts, paradiag_solve_info* info,
                                   void* stream) {
  Plan* pl = ready(plan);
  if (!pl) return plan ? PD_ERR_WORKSPACE : PD_ERR_INVALID;
  if (!b || !u || !opts) { set_error("NULL argument"); return PD_ERR_INVALID; }
  if (opts->mode < 0 || opts->mode > 2) { set_error("unknown mode (parareal has its own entry point)"); return PD_ERR_INVALID; }
  if (opts->mode == PD_MODE_FGMRES && (opts->restart < 1 || opts->restart > 32)) {
    set_error("restart must be in [1, 32]"); return PD_ERR_INVALID;
  }
  if (opts->max_iter < 1 || !(opts->rtol > 0)) { set_error("max_iter >= 1 and rtol > 0 required"); return PD_ERR_INVALID; }
  if (pl->oc && variant != 0) { set_error("no adjoint solve for optimal-control plans"); return PD_ERR_UNSUPPORTED; }
  if (pl->hybrid && (variant != 0 || opts->mode == PD_MODE_FGMRES)) {
    set_error("hybrid schemes (ParaDiag-I) solve in the direct and stationary modes only");
    return PD_ERR_UNSUPPORTED;
  }
  size_t nb = sizeof(double) * (size_t)pl->g.NA;
  if (overlap(b, nb, u, nb)) { set_error("b and u overlap"); return PD_ERR_INVALID; }
  try {
    return solve_impl(*pl, variant, b, u, opts, info, (hipStream_t)stream);
  } catch (...) {
    set_error("solve failed (host allocation)");
    return PD_ERR_INVALID;
  }
}

paradiag_status paradiag_parareal(paradiag_plan plan, const double* U0, int32_t J, double* u,
                                  const paradiag_solve_opts* o, paradiag_solve_info* info,
                                  void* stream) {
  Plan* pl = ready(plan);
  if (!pl) return plan ? PD_ERR_WORKSPACE : PD_ERR_INVALID;
  if (!U0 || !u || !o) { set_error("NULL argument"); return PD_ERR_INVALID; }
  if (o->mode != PD_MODE_PARAREAL) { set_error("opts->mode must be PD_MODE_PARAREAL"); return PD_ERR_INVALID; }
  if (J < 1 || J > 65536) { set_error("J must lie in [1, 65536]"); return PD_ERR_INVALID; }
  if (o->max_iter < 1 || !(o->rtol > 0)) { set_error("max_iter >= 1 and rtol > 0 required"); return PD_ERR_INVALID; }
  if (pl->p.scheme != PD_BE || pl->p.dim != 1) {
    set_error("parareal needs a backward Euler plan in one space dimension");
    return PD_ERR_UNSUPPORTED;
  }
  const Geom& g = pl->g;
  const size_t nb = sizeof(double) * (size_t)g.NA;
  if (overlap(U0, sizeof(double) * (size_t)g.B * g.S, u, nb)) { set_error("U0 and u overlap"); return PD_ERR_INVALID; }
  if ((size_t)(pl->ws + pl->ws_bytes - pl->solver_base) < solver_bytes(*pl, o)) {
    set_error("workspace too small for parareal (see paradiag_workspace_size with PD_MODE_PARAREAL)");
    return PD_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  char* p = pl->solver_base;
  Small sm = carve_small(*pl, p);
  double* uprev = (double*)p;
  p += align_up(nb);
  double* bvec = (double*)p;
  if (!pinned(*pl)) { set_error("pinned host staging allocation failed"); return PD_ERR_HIP; }
  if (!o->use_x0) fill_zero(u, g.NA, s);
  const int chunks = std::max(1, std::min(512, (int)(g.N1 / (256 * 16))));
  std::vector<double> rel(g.B, 0.0);
  int iters = 0, hist = 0;
  bool conv = false;
  while (iters < o->max_iter) {
    copy_vec(u, uprev, g.NA, s);
    {
      // J tridiagonal solves per interval: 8 flops per row (Thomas elimination
      // and substitution) plus 3 for the right-hand side; uprev read, b written
      Timed t(*pl, PD_STAGE_FINE, s, 2.0 * nb, 11.0 * J * (double)g.NA);
      parareal_fine(*pl, U0, uprev, bvec, J, pl->p.alpha, s);
    }
    apply_prec(*pl, 0, bvec, nullptr, 0, u, false, 0, s);
    diff_norms(*pl, u, uprev, sm.partial, chunks, s);
    timed_reduce(*pl, sm.partial, 2, nullptr, 0, sm.nrm, nullptr, s, chunks, pl->pin);
    if (paradiag_status st = wait_host(*pl, s); st != PD_OK) return st;
    ++iters;
    double mx = 0.0;
    for (int b = 0; b < g.B; ++b) {
      const double dd = pl->pin[(size_t)b * MAXV], uu = pl->pin[(size_t)b * MAXV + 1];
      rel[b] = uu > 0 ? std::sqrt(dd / uu) : (dd > 0 ? INFINITY : 0.0);
      if (!std::isfinite(rel[b])) { set_error("non-finite parareal iterate"); return PD_ERR_NONFINITE; }
      mx = std::max(mx, rel[b]);
    }
    if (info && info->history && hist < info->history_cap) info->history[hist] = mx;
    ++hist;
    if (mx <= o->rtol) { conv = true; break; }
  }
  if (info) {
    double mx = 0.0;
    for (int b = 0; b < g.B; ++b) {
      mx = std::max(mx, rel[b]);
      if (info->iters_per_rhs) info->iters_per_rhs[b] = iters;
      if (info->resid_per_rhs) info->resid_per_rhs[b] = rel[b];
    }
    info->iters = iters;
    info->converged = conv ? 1 : 0;
    info->rel_resid = mx;
    info->history_len = std::min(hist, info->history ? info->history_cap : 0);
  }
  if (paradiag_status st = check_hip("parareal"); st != PD_OK) return st;
  return conv ? PD_OK : PD_NOT_CONVERGED;
}

// Uploads lambda1_n + shift lambda2_n (and lambda2) to the device table and
// refactors the back-sweep's lines; shift 0 restores the plan's own symbols.
static void shift_symbols(Plan& pl, double shift, bool both_ops, hipStream_t s) {
  const int F = pl.g.F;
  pl.lam_stage.resize(2 * (size_t)F);
  for (int n = 0; n < F; ++n) {
    const cd l1 = pl.lam1[n] + shift * pl.lam2[n];
    pl.lam_stage[n] = double2{l1.real(), l1.imag()};
    pl.lam_stage[F + n] = double2{pl.lam2[n].real(), pl.lam2[n].imag()};
  }
  hipMemcpyAsync(pl.d_lam, pl.lam_stage.data(), sizeof(double2) * 2 * F, hipMemcpyHostToDevice, s);
  if (pl.p.dim == 2 && pl.schur) {
    schur_line_lu(pl, pl.op[0], s);
    if (both_ops) schur_line_lu(pl, pl.op[1], s);
  }
}

paradiag_status paradiag_nonlinear_solve(paradiag_plan plan, const paradiag_cubic* gc, const double* U0,
                                         int32_t windows, double* u, const paradiag_solve_opts* o,
                                         paradiag_solve_info* info, void* stream) {
  Plan* pl = ready(plan);
  if (!pl) return plan ? PD_ERR_WORKSPACE : PD_ERR_INVALID;
  if (!gc || !U0 || !u || !o) { set_error("NULL argument"); return PD_ERR_INVALID; }
  if (o->mode != PD_MODE_NONLINEAR) { set_error("opts->mode must be PD_MODE_NONLINEAR"); return PD_ERR_INVALID; }
  if (windows < 1 || o->max_iter < 1 || !(o->rtol > 0)) {
    set_error("windows >= 1, max_iter >= 1 and rtol > 0 required"); return PD_ERR_INVALID;
  }
  if (!std::isfinite(gc->k1) || !std::isfinite(gc->k2) || !std::isfinite(gc->k3)) {
    set_error("non-finite reaction coefficients"); return PD_ERR_INVALID;
  }
  if (pl->hybrid || (pl->p.scheme != PD_BE && pl->p.scheme != PD_TR) || pl->g.B != 1) {
    set_error("nonlinear solves need a theta-method plan (PD_BE, PD_TR) with batch 1");
    return PD_ERR_UNSUPPORTED;
  }
  const Geom& g = pl->g;
  const size_t nb = sizeof(double) * (size_t)g.NA;
  if (overlap(U0, sizeof(double) * (size_t)g.S, u, nb * (size_t)windows)) { set_error("U0 and u overlap"); return PD_ERR_INVALID; }
  if ((size_t)(pl->ws + pl->ws_bytes - pl->solver_base) < solver_bytes(*pl, o)) {
    set_error("workspace too small for the nonlinear solver (see paradiag_workspace_size with PD_MODE_NONLINEAR)");
    return PD_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  char* p = pl->solver_base;
  Small sm = carve_small(*pl, p);
  double* r = (double*)p;
  p += align_up(nb);
  double* bvec = (double*)p;
  p += align_up(nb);
  double* u0buf = (double*)p;
  if (!pinned(*pl)) { set_error("pinned host staging allocation failed"); return PD_ERR_HIP; }
  const double gk[3] = {gc->k1, gc->k2, gc->k3};
  const int chunks = std::max(1, std::min(512, (int)(g.N1 / (256 * 16))));
  int iters = 0, hist = 0;
  bool all_conv = true;
  double worst = 0.0;
  auto record = [&](double v) {
    if (info && info->history && hist < info->history_cap) info->history[hist] = v;
    ++hist;
  };
  paradiag_status st = PD_OK;
  for (int w = 0; w < windows && st == PD_OK; ++w) {
    double* uw = u + (size_t)w * g.NA;
    const double* U0w = U0;
    if (w > 0) {
      last_rows(*pl, uw - g.NA, u0buf, s);
      U0w = u0buf;
    }
    build_rhs(*pl, U0w, nullptr, nullptr, bvec, s);
    nl_rhs_fix(*pl, U0w, bvec, gk, s);
    std::vector<double> bn;
    timed_dot(*pl, bvec, 0, 1, bvec, sm.partial, s);
    if ((st = norms_from(*pl, sm, bn, s)) != PD_OK) break;
    if (!(w == 0 && o->use_x0)) bcast_rows(*pl, U0w, uw, s);
    double rel = 0.0;
    bool conv = false;
    for (int it = 0;; ++it) {
      apply_A(*pl, 0, uw, false, bvec, r, s);          // r = b - (B1 (x) I + B2 (x) K) u
      {
        Timed t(*pl, PD_STAGE_REACTION, s, 3.0 * nb, 8.0 * (double)g.NA);
        nl_residual(*pl, uw, r, gk, sm.partial, chunks, s);
      }
      timed_reduce(*pl, sm.partial, 2, nullptr, 0, sm.nrm, nullptr, s, chunks, pl->pin);
      if ((st = wait_host(*pl, s)) != PD_OK) break;
      const double rr = pl->pin[0], gsum = pl->pin[1];
      rel = bn[0] > 0 ? std::sqrt(std::fabs(rr)) / bn[0] : std::sqrt(std::fabs(rr));
      if (!std::isfinite(rel) || !std::isfinite(gsum)) { set_error("non-finite nonlinear residual"); st = PD_ERR_NONFINITE; break; }
      record(rel);
      if (rel <= o->rtol) { conv = true; break; }
      if (it >= o->max_iter) break;
      shift_symbols(*pl, gsum / (double)g.NA, false, s);   // P_alpha(u) with the averaged slope
      apply_prec(*pl, 0, r, nullptr, 0, uw, false, 1, s);  // u += P_alpha(u)^{-1} R(u)
      ++iters;
    }
    worst = std::max(worst, rel);
    all_conv = all_conv && conv;
  }
  shift_symbols(*pl, 0.0, true, s);   // the plan's own symbols and line factors again
  if (st == PD_OK) st = check_hip("nonlinear solve");
  if (info) {
    info->iters = iters;
    info->converged = all_conv && st == PD_OK ? 1 : 0;
    info->rel_resid = worst;
    info->history_len = std::min(hist, info->history ? info->history_cap : 0);
    if (info->iters_per_rhs) info->iters_per_rhs[0] = iters;
    if (info->resid_per_rhs) info->resid_per_rhs[0] = worst;
  }
  if (st != PD_OK) return st;
  hipError_t e = hipStreamSynchronize(s);   // the restored symbols are in place on return
  if (e != hipSuccess) { set_error(std::string("nonlinear solve: ") + hipGetErrorString(e)); return PD_ERR_HIP; }
  return all_conv ? PD_OK : PD_NOT_CONVERGED;
}

paradiag_status paradiag_solve(paradiag_plan plan, const double* b, double* u,
                               const paradiag_solve_opts* opts, paradiag_solve_info* info,
                               void* stream) {
  return solve_entry(plan, 0, b, u, opts, info, stream);
}

paradiag_status paradiag_adjoint_solve(paradiag_plan plan, const double* g, double* lam,
                                       const paradiag_solve_opts* opts,
                                       paradiag_solve_info* info, void* stream) {
  return solve_entry(plan, 1, g, lam, opts, info, stream);
}

paradiag_status paradiag_get_xbasis(paradiag_plan plan, int32_t adjoint, double* q, double* t) {
  Plan* pl = reinterpret_cast<Plan*>(plan);
  if (!pl || !q || !t) { set_error("NULL argument"); return PD_ERR_INVALID; }
  if (pl->p.dim != 2) { set_error("the x basis exists only in two dimensions"); return PD_ERR_INVALID; }
  const SpaceOp& op = pl->op[adjoint ? 1 : 0];
  for (size_t i = 0; i < op.Q.size(); ++i) {
    q[2 * i] = op.Q[i].real(); q[2 * i + 1] = op.Q[i].imag();
    t[2 * i] = op.Tm[i].real(); t[2 * i + 1] = op.Tm[i].imag();
  }
  return PD_OK;
}

paradiag_status paradiag_get_symbols(paradiag_plan plan, double* lam1, double* lam2) {
  Plan* pl = reinterpret_cast<Plan*>(plan);
  if (!pl || !lam1 || !lam2) { set_error("NULL argument"); return PD_ERR_INVALID; }
  for (int n = 0; n < pl->g.F; ++n) {
    lam1[2 * n] = pl->lam1[n].real(); lam1[2 * n + 1] = pl->lam1[n].imag();
    lam2[2 * n] = pl->lam2[n].real(); lam2[2 * n + 1] = pl->lam2[n].imag();
  }
  return PD_OK;
}

paradiag_status paradiag_set_timing(paradiag_plan plan, int32_t enable) {
  Plan* pl = reinterpret_cast<Plan*>(plan);
  if (!pl) { set_error("plan is NULL"); return PD_ERR_INVALID; }
  if (enable < 0 || enable >= (2 << PD_NUM_STAGES)) { set_error("timing selector out of range"); return PD_ERR_INVALID; }
  pl->timer.enabled = enable != 0;
  pl->timer.mask = enable == 1 ? (1u << PD_NUM_STAGES) - 1 : (unsigned)enable >> 1;
  return PD_OK;
}

paradiag_status paradiag_get_stage_times(paradiag_plan plan, double* ms, int64_t* counts,
                                         double* bytes, double* flops, int32_t reset) {
  Plan* pl = reinterpret_cast<Plan*>(plan);
  if (!pl) { set_error("plan is NULL"); return PD_ERR_INVALID; }
  drain_timer(*pl);
  for (int i = 0; i < PD_NUM_STAGES; ++i) {
    if (ms) ms[i] = pl->timer.ms[i];
    if (counts) counts[i] = pl->timer.count[i];
    if (bytes) bytes[i] = pl->timer.bytes[i];
    if (flops) flops[i] = pl->timer.flops[i];
    if (reset) { pl->timer.ms[i] = 0; pl->timer.count[i] = 0; pl->timer.bytes[i] = 0; pl->timer.flops[i] = 0; }
  }
  return check_hip("stage times");
}

}  // extern "C"

// z = P_alpha^{-1} r with the spectral buffers at spec_a, spec_b (each spec_bytes
// long) instead of the bound workspace's; used by the allocation-free entry point.
paradiag_status pd::apply_precond_into(paradiag_plan plan, const double* r, double* z, void* spec_a,
                                   void* spec_b, size_t spec_bytes, hipStream_t s) {
  Plan* pl = ready(plan);
  if (!pl) return plan ? PD_ERR_WORKSPACE : PD_ERR_INVALID;
  if (!r || !z) { set_error("NULL vector"); return PD_ERR_INVALID; }
  size_t nb = sizeof(double) * (size_t)pl->g.NA;
  if (r != z && overlap(r, nb, z, nb)) { set_error("r and z partially overlap"); return PD_ERR_INVALID; }
  const size_t need = align_up((size_t)pl->g.spec_elems * spec_elem_bytes(pl->prec));
  if (spec_bytes < need) {
    set_error("spectral buffers of this plan (" + std::to_string(2 * need) +
              " bytes) exceed the static scratch (" + std::to_string(2 * spec_bytes) + " bytes)");
    return PD_ERR_WORKSPACE;
  }
  // no stage timing here: recording events may create them
  const bool timing = pl->timer.enabled;
  pl->timer.enabled = false;
  apply_prec(*pl, 0, r, nullptr, 0, z, false, 0, s, spec_a, spec_b);
  pl->timer.enabled = timing;
  return check_hip("apply_precond_static");
}
