// Optimal control of the wave equation (Section 4): the operator of the
// gamma-scaled optimality system and its block-circulant preconditioner.
//
// Vectors hold two fields one after the other, [2][nt][ny][nx]: x1 = sqrt(gamma) u
// (u at t_1 .. t_Nt) and x2 = p (p at t_0 .. t_{Nt-1}).  With the implicit
// leap-frog Toeplitz columns B1 = (1, -2, 1), B2 = (dt^2/2) (1, 0, 1) and
// s = dt^2 / sqrt(gamma):
//
//   y1 = (B1 (x) I + B2 (x) A) x1 - s Ih x2,     Ih = diag(1/2, 1, .., 1)
//   y2 = s Ic x1 + (B1^T (x) I + B2^T (x) A) x2, Ic = diag(1, .., 1, 1/2)
//
// The preconditioner P uses the circulants of B1, B2 and drops Ih, Ic.  With
// Fourier symbols d1, d2 of the circulants, P = Pt (blkdiag(C2, C2^T) (x) I)
// and Pt's time part at frequency n is [[a, -beta conj(q)], [beta q, a]]
// (a = d1/d2 real, q = 1/d2, beta = s), diagonalised by
// W = [[1, 1], [-i E, i E]], E = q/|q|, with eigenvalues a +- i beta |q| (Thm the4).
// So P^{-1} r: time DFT of both fields (dense product on MFMA: Nt is not a
// power of two here, since C2 is singular when 4 divides Nt), the mixing
// c1 = (R1 + i conj(E) R2)/2, c2 = (R1 - i conj(E) R2)/2 into 2 Fh spectral
// slices (oc_time_forward), the plan's Step-(b) (x-transform, line solves with
// lambda1 = Sigma, lambda2 = dt^2/2, x-transform back), the unmixing
// S1 = (y1 + y2)/d2, S2 = i E (y2 - y1)/conj(d2), and the inverse DFT of both
// fields (oc_time_inverse).

#include "internal.h"

namespace pd {
namespace {

constexpr int NT = 256;

// in: [2][Fh][sy][2][sx] (field, frequency); out: [2 Fh][sy][2][sx] with the
// c1 slices first.  One thread per (frequency, point).
template <typename T>
__global__ __launch_bounds__(NT) void k_oc_mix(const T* __restrict__ in, T* __restrict__ out,
                                               const double2* __restrict__ cE, int Fh, int64_t S, int sx) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= (int64_t)Fh * S) return;
  const int n = (int)(e / S);
  const int j = (int)(e - (int64_t)n * S);
  const int y = j / sx, x = j - y * sx;
  const int64_t off = (int64_t)n * 2 * S + (int64_t)y * 2 * sx + x;   // real part; imag at + sx
  const int64_t fstride = (int64_t)Fh * 2 * S;
  const double r1r = in[off], r1i = in[off + sx];
  const double r2r = in[fstride + off], r2i = in[fstride + off + sx];
  const double er = cE[n].x, ei = -cE[n].y;   // E (the table holds conj(E))
  // i conj(E) R2 = (-er r2i + ei r2r) + i (er r2r + ei r2i)
  const double tr = -er * r2i + ei * r2r, ti = er * r2r + ei * r2i;
  out[off] = (T)(0.5 * (r1r + tr));
  out[off + sx] = (T)(0.5 * (r1i + ti));
  out[fstride + off] = (T)(0.5 * (r1r - tr));
  out[fstride + off + sx] = (T)(0.5 * (r1i - ti));
}

// in: [2 Fh][...] (y1 slices, then y2); out: [2][Fh][...]:
// S1 = (y1 + y2) / d2, S2 = i E (y2 - y1) / conj(d2)
template <typename T>
__global__ __launch_bounds__(NT) void k_oc_unmix(const T* __restrict__ in, T* __restrict__ out,
                                                 const double2* __restrict__ c1t,
                                                 const double2* __restrict__ c2t, int Fh, int64_t S, int sx) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= (int64_t)Fh * S) return;
  const int n = (int)(e / S);
  const int j = (int)(e - (int64_t)n * S);
  const int y = j / sx, x = j - y * sx;
  const int64_t off = (int64_t)n * 2 * S + (int64_t)y * 2 * sx + x;
  const int64_t fstride = (int64_t)Fh * 2 * S;
  const double y1r = in[off], y1i = in[off + sx];
  const double y2r = in[fstride + off], y2i = in[fstride + off + sx];
  const double2 a = c1t[n], b = c2t[n];
  const double pr = y1r + y2r, pi = y1i + y2i, mr = y2r - y1r, mi = y2i - y1i;
  out[off] = (T)(a.x * pr - a.y * pi);
  out[off + sx] = (T)(a.x * pi + a.y * pr);
  out[fstride + off] = (T)(b.x * mr - b.y * mi);
  out[fstride + off + sx] = (T)(b.x * mi + b.y * mr);
}

// coupling of the two fields: y1 += sgn (-s Ih x2), y2 += sgn (s Ic x1)
// (sgn = -1 when y holds b - A x)
template <typename Tin>
__global__ __launch_bounds__(NT) void k_oc_couple(const Tin* __restrict__ x, double* __restrict__ y, int nt,
                                                  int64_t S, double s, double sgn) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t N = (int64_t)nt * S;
  if (e >= N) return;
  const int n = (int)(e / S);
  const double wh = n == 0 ? 0.5 : 1.0, wc = n == nt - 1 ? 0.5 : 1.0;
  y[e] -= sgn * s * wh * (double)x[N + e];
  y[N + e] += sgn * s * wc * (double)x[e];
}

// b1 = scale1 b1 (the leap-frog rows already built there), b2_m = dt^2 g(t_{m+1})
// with the last row halved
__global__ __launch_bounds__(NT) void k_oc_rhs(double* __restrict__ b, const double* __restrict__ g, int nt,
                                               int64_t S, double scale1, double dt2) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t N = (int64_t)nt * S;
  if (e >= N) return;
  const int m = (int)(e / S);
  b[e] *= scale1;
  b[N + e] = g ? dt2 * (m == nt - 1 ? 0.5 : 1.0) * g[e + S] : 0.0;
}

unsigned blocks(int64_t n) { return (unsigned)((n + NT - 1) / NT); }

}  // namespace

void oc_matvec(const Plan& pl, const void* u, bool u_is_f32, const double* b, double* y, hipStream_t s,
               const double* Vk, int64_t vstride, int nv, double* partial, int sq, const double* V0,
               int v0sq) {
  const Geom& g = pl.g;
  const int64_t N = (int64_t)g.nt * g.S;
  const size_t eb = u_is_f32 ? 4 : 8;
  const char* u2 = (const char*)u + N * eb;
  // y == null asks for the norm of b - A u only; the coupling of the two fields
  // needs the values, so they go to the spectral buffers (at least 16 nt S
  // bytes between them, free while no preconditioner runs)
  if (!y) y = (double*)pl.spec_a;
  matvec_plain(pl, pl.op[0], u, u_is_f32, b, y, 0, s);
  matvec_plain(pl, pl.op[1], u2, u_is_f32, b ? b + N : nullptr, y + N, 1, s);
  const double sgn = b ? -1.0 : 1.0;
  if (u_is_f32) k_oc_couple<float><<<blocks(N), NT, 0, s>>>((const float*)u, y, g.nt, g.S, pl.oc_beta, sgn);
  else k_oc_couple<double><<<blocks(N), NT, 0, s>>>((const double*)u, y, g.nt, g.S, pl.oc_beta, sgn);
  if (!partial) return;
  // the dots matvec fuses elsewhere, here as separate passes in the same
  // partial-sum layout (matvec_chunks == dot_chunks for this operator)
  int slot = 0;
  if (nv > 0) {
    if (V0) {
      multi_dot(pl, V0, 0, 1, y, partial, s, 0);
      if (nv > 1) multi_dot(pl, Vk + vstride, vstride, nv - 1, y, partial, s, 1);
    } else {
      multi_dot(pl, Vk, vstride, nv, y, partial, s, 0);
    }
    slot = nv;
  }
  if (sq) multi_dot(pl, y, 0, 1, y, partial, s, slot++);
  if (v0sq) {
    const double* v0 = V0 ? V0 : Vk;
    multi_dot(pl, v0, 0, 1, v0, partial, s, slot);
  }
}

void oc_time_forward(const Plan& pl, const double* in, const double* scale, void* out, void* tmp,
                     hipStream_t s) {
  const Geom& g = pl.g;
  const int Fh = pl.oc_fh;
  const bool f32 = pl.prec != Prec::F64;
  // time DFT of both fields: tmp = [2][Fh][...]
  time_gemm(pl, true, pl.d_wf, in, tmp, f32, false, 0, 2, g.nt, Fh, 2 * Fh, g.nt, s, scale);
  const int64_t n = (int64_t)Fh * g.S;
  if (f32) k_oc_mix<float><<<blocks(n), NT, 0, s>>>((const float*)tmp, (float*)out, pl.d_ocmix, Fh, g.S, g.sx);
  else k_oc_mix<double><<<blocks(n), NT, 0, s>>>((const double*)tmp, (double*)out, pl.d_ocmix, Fh, g.S, g.sx);
}

void oc_time_inverse(const Plan& pl, const void* in, void* out, bool out_f32, int accumulate, void* tmp,
                     hipStream_t s) {
  const Geom& g = pl.g;
  const int Fh = pl.oc_fh;
  const bool f32 = pl.prec != Prec::F64;
  const int64_t n = (int64_t)Fh * g.S;
  const double2* c1t = pl.d_ocmix + Fh;
  const double2* c2t = pl.d_ocmix + 2 * Fh;
  if (f32) k_oc_unmix<float><<<blocks(n), NT, 0, s>>>((const float*)in, (float*)tmp, c1t, c2t, Fh, g.S, g.sx);
  else k_oc_unmix<double><<<blocks(n), NT, 0, s>>>((const double*)in, (double*)tmp, c1t, c2t, Fh, g.S, g.sx);
  time_gemm(pl, false, pl.d_wi, tmp, out, f32, out_f32, accumulate, 2, g.nt, Fh, g.nt, 2 * Fh, s);
}

void oc_build_rhs(const Plan& pl, const double* U0, const double* u1, const double* f, const double* gsrc,
                  double* b, hipStream_t s) {
  const Geom& g = pl.g;
  const int64_t N = (int64_t)g.nt * g.S;
  build_rhs(pl, U0, u1, f, b, s);   // leap-frog rows of the state equation (the plan's scheme)
  const double dt = pl.p.T / g.nt;
  k_oc_rhs<<<blocks(N), NT, 0, s>>>(b, gsrc, g.nt, g.S, std::sqrt(pl.oc_gamma) * dt * dt, dt * dt);
}

}  // namespace pd
