// Step-(a) and Step-(c) of the ParaDiag-II preconditioner (eq1.3, eq2.12):
// the alpha-scaled discrete Fourier transform along the time axis, applied
// independently to every spatial unknown.
//
//   Step-(a):  S_k = sum_n alpha^{n/Nt} r_n e^{-2 pi i k n / Nt}, k = 0..Nt/2
//   Step-(c):  z_n = alpha^{-n/Nt} (1/Nt) sum_k S_k e^{+2 pi i k n / Nt}
//
// Data is real and the time symbols are real-coefficient polynomials, so the
// spectrum is Hermitian (S_{Nt-k} = conj S_k) and only Nt/2+1 frequencies are
// stored and solved.
//
// Kernel design (gfx950): one workgroup owns TX consecutive spatial unknowns
// and all Nt time samples.  The time columns are read with coalesced rows of
// TX doubles, scaled by Gamma in float64, rounded to the working precision and
// packed pairwise into TX/2 complex columns in LDS (two real transforms for
// the price of one complex transform).  A self-sorting Stockham FFT
// (radix-4 passes, one radix-2 pass when log2 Nt is odd) runs in place in
// LDS; each pass holds all of a thread's butterfly inputs in registers
// between the read barrier and the write barrier.  The pair is then split
// into the two half spectra, X_a = (Z_k + conj Z_{Nt-k})/2 and
// X_b = (Z_k - conj Z_{Nt-k})/(2i), and written row-planar.  The inverse runs
// the same steps backwards, using ifft(Z) = conj(fft(conj Z))/Nt.

#include "internal.h"

namespace pd {
namespace {

template <typename T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };

template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
// multiply by -i
template <typename C> __device__ __forceinline__ C cmi(C a) { return C{a.y, -a.x}; }

constexpr int NT = 256;

// In-place forward Stockham FFT of `ncol` columns of length Nt (column stride
// ld) in LDS.  EPT = complex values held per thread in a pass (>= ncol*Nt/NT).
template <typename T, int EPT>
__device__ void fft_columns(typename V2<T>::t* sm, int ncol, int ld, int Nt, int logNt,
                            const typename V2<T>::t* __restrict__ tw) {
  using C = typename V2<T>::t;
  int Ns = 1;
  int bits = logNt;
  if (bits & 1) {  // one radix-2 pass
    const int nb = Nt >> 1, lognb = logNt - 1, total = ncol * nb;
    C v[EPT];
#pragma unroll
    for (int i = 0; i < EPT / 2; ++i) {
      int bf = threadIdx.x + i * NT;
      if (bf < total) {
        int col = bf >> lognb, j = bf & (nb - 1);
        const C* src = sm + col * ld + j;
        v[2 * i] = src[0];
        v[2 * i + 1] = src[nb];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT / 2; ++i) {
      int bf = threadIdx.x + i * NT;
      if (bf < total) {
        int col = bf >> lognb, j = bf & (nb - 1);
        // Ns == 1: no twiddle
        C* dst = sm + col * ld + (j << 1);
        dst[0] = cadd(v[2 * i], v[2 * i + 1]);
        dst[1] = csub(v[2 * i], v[2 * i + 1]);
      }
    }
    __syncthreads();
    Ns = 2;
    bits -= 1;
  }
  while (bits > 0) {  // radix-4 passes
    const int nb = Nt >> 2, lognb = logNt - 2, total = ncol * nb;
    const int step = Nt / (Ns << 2);
    C v[EPT];
#pragma unroll
    for (int i = 0; i < EPT / 4; ++i) {
      int bf = threadIdx.x + i * NT;
      if (bf < total) {
        int col = bf >> lognb, j = bf & (nb - 1);
        const C* src = sm + col * ld + j;
        v[4 * i] = src[0];
        v[4 * i + 1] = src[nb];
        v[4 * i + 2] = src[2 * nb];
        v[4 * i + 3] = src[3 * nb];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT / 4; ++i) {
      int bf = threadIdx.x + i * NT;
      if (bf < total) {
        int col = bf >> lognb, j = bf & (nb - 1);
        int k = j & (Ns - 1);
        C v0 = v[4 * i], v1 = v[4 * i + 1], v2 = v[4 * i + 2], v3 = v[4 * i + 3];
        if (k) {
          v1 = cmul(v1, tw[k * step]);
          v2 = cmul(v2, tw[2 * k * step]);
          v3 = cmul(v3, tw[3 * k * step]);
        }
        C t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = cmi(csub(v1, v3));
        C* dst = sm + col * ld + ((j - k) << 2) + k;
        dst[0] = cadd(t0, t2);
        dst[Ns] = cadd(t1, t3);
        dst[2 * Ns] = csub(t0, t2);
        dst[3 * Ns] = csub(t1, t3);
      }
    }
    __syncthreads();
    Ns <<= 2;
    bits -= 2;
  }
}

template <typename T, int EPT>
__global__ __launch_bounds__(NT) void k_fft_fwd(const double* __restrict__ x, T* __restrict__ spec,
                                                const double* __restrict__ gam,
                                                const double* __restrict__ bscale,
                                                const typename V2<T>::t* __restrict__ tw, int Nt,
                                                int logNt, int S, int sx, int sy, int logTX,
                                                int reverse) {
  using C = typename V2<T>::t;
  extern __shared__ __align__(16) unsigned char smraw[];
  C* sm = reinterpret_cast<C*>(smraw);
  T* smT = reinterpret_cast<T*>(smraw);
  const int TX = 1 << logTX, ld = Nt + 1, F = (Nt >> 1) + 1;
  const int b = blockIdx.y;
  const int s0 = blockIdx.x * TX;
  const double* xb = x + (int64_t)b * Nt * S;
  const double sc = bscale ? bscale[b] : 1.0;
  for (int e = threadIdx.x; e < (Nt << logTX); e += NT) {
    int n = e >> logTX, c = e & (TX - 1);
    int s = s0 + c;
    int nsrc = reverse ? (Nt - 1 - n) : n;
    double v = 0.0;
    if (s < S) v = xb[(int64_t)nsrc * S + s] * (gam[n] * sc);
    smT[2 * ((c >> 1) * ld + n) + (c & 1)] = (T)v;
  }
  __syncthreads();
  fft_columns<T, EPT>(sm, TX >> 1, ld, Nt, logNt, tw);
  T* specb = spec + (int64_t)b * F * sy * 2 * sx;
  for (int e = threadIdx.x; e < (F << logTX); e += NT) {
    int k = e >> logTX, c = e & (TX - 1);
    int s = s0 + c;
    if (s >= S) continue;
    const C* col = sm + (c >> 1) * ld;
    C zk = col[k], zm = col[(Nt - k) & (Nt - 1)];
    T re, im;
    if ((c & 1) == 0) {
      re = (T)0.5 * (zk.x + zm.x);
      im = (T)0.5 * (zk.y - zm.y);
    } else {
      re = (T)0.5 * (zk.y + zm.y);
      im = (T)0.5 * (zm.x - zk.x);
    }
    int y = s / sx, xx = s - y * sx;
    T* dst = specb + ((int64_t)k * sy + y) * 2 * sx + xx;
    dst[0] = re;
    dst[sx] = im;
  }
}

template <typename T, int EPT, typename Tout>
__global__ __launch_bounds__(NT) void k_fft_inv(const T* __restrict__ spec, Tout* __restrict__ z,
                                                const double* __restrict__ invgam,
                                                const typename V2<T>::t* __restrict__ tw, int Nt,
                                                int logNt, int S, int sx, int sy, int logTX,
                                                int accumulate, int reverse) {
  using C = typename V2<T>::t;
  extern __shared__ __align__(16) unsigned char smraw[];
  C* sm = reinterpret_cast<C*>(smraw);
  T* smT = reinterpret_cast<T*>(smraw);
  const int TX = 1 << logTX, ld = Nt + 1, F = (Nt >> 1) + 1, half = Nt >> 1;
  const int b = blockIdx.y;
  const int s0 = blockIdx.x * TX;
  const T* specb = spec + (int64_t)b * F * sy * 2 * sx;
  // 1. load half spectra: X_a[k] -> slot k, X_b[k] -> slot Nt-k; DC and
  //    Nyquist keep only their real parts (they are real for real data).
  for (int e = threadIdx.x; e < (F << logTX); e += NT) {
    int k = e >> logTX, c = e & (TX - 1);
    int s = s0 + c;
    T re = 0, im = 0;
    if (s < S) {
      int y = s / sx, xx = s - y * sx;
      const T* src = specb + ((int64_t)k * sy + y) * 2 * sx + xx;
      re = src[0];
      im = src[sx];
    }
    int cc = c >> 1;
    if (k == 0 || k == half) {
      smT[2 * (cc * ld + k) + (c & 1)] = re;
    } else if ((c & 1) == 0) {
      sm[cc * ld + k] = C{re, im};
    } else {
      sm[cc * ld + Nt - k] = C{re, im};
    }
  }
  __syncthreads();
  // 2. Z = X_a + i X_b on the full circle, stored conjugated
  const int ncol = TX >> 1;
  for (int e = threadIdx.x; e < (ncol << (logNt - 1)); e += NT) {
    int cc = e >> (logNt - 1), k = e & (half - 1);
    C* col = sm + cc * ld;
    if (k == 0) {
      C z0 = col[0], zh = col[half];
      col[0] = C{z0.x, -z0.y};
      col[half] = C{zh.x, -zh.y};
    } else {
      C A = col[k], Bv = col[Nt - k];
      col[k] = C{A.x - Bv.y, -(A.y + Bv.x)};
      col[Nt - k] = C{A.x + Bv.y, -(Bv.x - A.y)};
    }
  }
  __syncthreads();
  fft_columns<T, EPT>(sm, ncol, ld, Nt, logNt, tw);
  // 3. z = conj(fft(conj Z)) / Nt, split into the two real columns, Gamma^{-1}
  Tout* zb = z + (int64_t)b * Nt * S;
  for (int e = threadIdx.x; e < (Nt << logTX); e += NT) {
    int n = e >> logTX, c = e & (TX - 1);
    int s = s0 + c;
    if (s >= S) continue;
    C yv = sm[(c >> 1) * ld + n];
    double v = ((c & 1) ? -(double)yv.y : (double)yv.x) * invgam[n];
    int nd = reverse ? (Nt - 1 - n) : n;
    Tout* dst = zb + (int64_t)nd * S + s;
    if (accumulate) *dst = (Tout)((double)*dst + v);
    else *dst = (Tout)v;
  }
}

struct FftShape { int logTX; int ept; size_t lds; };

FftShape choose_shape(const Plan& pl) {
  const Geom& g = pl.g;
  const size_t csize = (pl.prec == Prec::F64) ? 16 : 8;
  const size_t budget = 66 * 1024;
  int logTX = 4;  // TX = 16
  while (logTX > 1 && (size_t)((1 << logTX) / 2) * (g.nt + 1) * csize > budget) --logTX;
  // do not tile wider than the spatial extent needs
  while (logTX > 1 && (1 << (logTX - 1)) >= g.S) --logTX;
  int ncol = (1 << logTX) / 2;
  int need = (ncol * g.nt + NT - 1) / NT;
  int ept = 4;
  while (ept < need) ept <<= 1;
  FftShape sh{logTX, ept, (size_t)ncol * (g.nt + 1) * csize};
  return sh;
}

template <typename T>
void launch_fwd(const Plan& pl, const double* x, const double* bscale, T* spec, int reverse,
                hipStream_t s, const typename V2<T>::t* tw) {
  const Geom& g = pl.g;
  FftShape sh = choose_shape(pl);
  int logNt = 0;
  while ((1 << logNt) < g.nt) ++logNt;
  dim3 grid((g.S + (1 << sh.logTX) - 1) >> sh.logTX, g.B);
#define PD_FWD(E)                                                                          \
  case E:                                                                                  \
    hipFuncSetAttribute((const void*)k_fft_fwd<T, E>,                                      \
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds);          \
    k_fft_fwd<T, E><<<grid, NT, sh.lds, s>>>(x, spec, pl.d_gam, bscale, tw, g.nt, logNt,   \
                                             (int)g.S, g.sx, g.sy, sh.logTX, reverse);     \
    break;
  switch (sh.ept) {
    PD_FWD(4) PD_FWD(8) PD_FWD(16) PD_FWD(32)
    default: break;
  }
#undef PD_FWD
}

template <typename T, typename Tout>
void launch_inv(const Plan& pl, const T* spec, Tout* z, int accumulate, int reverse,
                hipStream_t s, const typename V2<T>::t* tw) {
  const Geom& g = pl.g;
  FftShape sh = choose_shape(pl);
  int logNt = 0;
  while ((1 << logNt) < g.nt) ++logNt;
  dim3 grid((g.S + (1 << sh.logTX) - 1) >> sh.logTX, g.B);
#define PD_INV(E)                                                                          \
  case E:                                                                                  \
    hipFuncSetAttribute((const void*)k_fft_inv<T, E, Tout>,                                \
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds);          \
    k_fft_inv<T, E, Tout><<<grid, NT, sh.lds, s>>>(spec, z, pl.d_invgam, tw, g.nt, logNt,  \
                                                   (int)g.S, g.sx, g.sy, sh.logTX,         \
                                                   accumulate, reverse);                   \
    break;
  switch (sh.ept) {
    PD_INV(4) PD_INV(8) PD_INV(16) PD_INV(32)
    default: break;
  }
#undef PD_INV
}

}  // namespace

void fft_time_forward(const Plan& pl, const double* x, const double* bscale, void* spec,
                      int reverse, hipStream_t s) {
  if (pl.prec == Prec::F64)
    launch_fwd<double>(pl, x, bscale, (double*)spec, reverse, s, pl.d_tw64);
  else
    launch_fwd<float>(pl, x, bscale, (float*)spec, reverse, s, pl.d_tw32);
}

void fft_time_inverse(const Plan& pl, const void* spec, void* z, bool z_is_f32, int accumulate,
                      int reverse, hipStream_t s) {
  if (pl.prec == Prec::F64) {
    if (z_is_f32)
      launch_inv<double, float>(pl, (const double*)spec, (float*)z, accumulate, reverse, s, pl.d_tw64);
    else
      launch_inv<double, double>(pl, (const double*)spec, (double*)z, accumulate, reverse, s, pl.d_tw64);
  } else {
    if (z_is_f32)
      launch_inv<float, float>(pl, (const float*)spec, (float*)z, accumulate, reverse, s, pl.d_tw32);
    else
      launch_inv<float, double>(pl, (const float*)spec, (double*)z, accumulate, reverse, s, pl.d_tw32);
  }
}

}  // namespace pd
