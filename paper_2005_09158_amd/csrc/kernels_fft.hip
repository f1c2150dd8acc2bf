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
__device__ __forceinline__ void fft_columns(typename V2<T>::t* sm, int ncol, int ld, int Nt, int logNt,
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

// Tile width TX (spatial unknowns per workgroup) and the per-thread register
// budget of one FFT pass; see choose_shape.
template <typename T> struct FftTraits;
template <> struct FftTraits<float> { static constexpr int EPT = 32; };
template <> struct FftTraits<double> { static constexpr int EPT = 16; };


// Copies the Nt-entry twiddle table into LDS behind the data columns.
template <typename C>
__device__ __forceinline__ void stage_twiddles(C* smtw, const C* __restrict__ tw, int Nt) {
  for (int i = threadIdx.x; i < Nt; i += NT) smtw[i] = tw[i];
}

// Reads the pair of real time samples (s, s+1) at one time row; columns past
// the spatial extent read as zero.  `vec` is set when the row start is
// 16-byte aligned for every row (S even), which allows one double2 load.
__device__ __forceinline__ double2 load_pair(const double* __restrict__ row, int s, int S, bool vec) {
  if (vec && s + 1 < S) return *reinterpret_cast<const double2*>(row + s);
  double2 v{0.0, 0.0};
  if (s < S) v.x = row[s];
  if (s + 1 < S) v.y = row[s + 1];
  return v;
}

template <typename T, int TX>
__global__ __launch_bounds__(NT, 2) void k_fft_fwd(const double* __restrict__ x, T* __restrict__ spec,
                                                   const double* __restrict__ gam,
                                                   const double* __restrict__ bscale,
                                                   const typename V2<T>::t* __restrict__ tw, int Nt,
                                                   int logNt, int S, int sx, int sy, int reverse,
                                                   int gam_lds) {
  using C = typename V2<T>::t;
  constexpr int EPT = FftTraits<T>::EPT;
  constexpr int NCOL = TX / 2;           // complex columns: one per pair of real columns
  constexpr int RPI = NT / NCOL;         // time rows per load sweep
  extern __shared__ __align__(16) unsigned char smraw[];
  C* sm = reinterpret_cast<C*>(smraw);
  const int ld = Nt + 1, F = (Nt >> 1) + 1;
  C* smtw = sm + NCOL * ld;
  const int b = blockIdx.y;
  const int s0 = blockIdx.x * TX;
  const double* xb = x + (int64_t)b * Nt * S;
  const double sc = bscale ? bscale[b] : 1.0;
  const bool vec = (S & 1) == 0;
  double* smg = reinterpret_cast<double*>(smtw + Nt);   // Gamma
  // 1. stage: lane j of a row reads real columns (2j, 2j+1) with one 16-byte
  //    load and stores them as the complex value r_2j + i r_2j+1 of column j.
  //    A tile's loads fit one batch ((TX/2) Nt <= EPT NT), all issued before
  //    the first is consumed.
  {
    const int j = threadIdx.x % NCOL, r = threadIdx.x / NCOL;
    const int s = s0 + 2 * j;
    double2 v[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int n = r + u * RPI;
      if (n < Nt) {
        const int nsrc = reverse ? (Nt - 1 - n) : n;
        v[u] = load_pair(xb + (int64_t)nsrc * S, s, S, vec);
      }
    }
    stage_twiddles(smtw, tw, Nt);
    if (gam_lds)
      for (int i = threadIdx.x; i < Nt; i += NT) smg[i] = gam[i];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int n = r + u * RPI;
      if (n < Nt) {
        const double g = (gam_lds ? smg[n] : gam[n]) * sc;
        sm[j * ld + n] = C{(T)(v[u].x * g), (T)(v[u].y * g)};
      }
    }
  }
  __syncthreads();
  fft_columns<T, EPT>(sm, NCOL, ld, Nt, logNt, smtw);
  // 2. Hermitian split of column j into the half spectra of real columns 2j
  //    and 2j+1, written as (re, re) and (im, im) pairs of adjacent x.
  T* specb = spec + (int64_t)b * F * sy * 2 * sx;
  const bool vout = (sx & 1) == 0;
  const int j = threadIdx.x % NCOL, r = threadIdx.x / NCOL;
  const int s = s0 + 2 * j;
  if (s >= S) return;
  const int y = s / sx, xx = s - y * sx;
  const int y1 = (s + 1) / sx, xx1 = (s + 1) - y1 * sx;
  for (int k = r; k < F; k += RPI) {
    const C* col = sm + j * ld;
    C zk = col[k], zm = col[(Nt - k) & (Nt - 1)];
    const T ar = (T)0.5 * (zk.x + zm.x), ai = (T)0.5 * (zk.y - zm.y);
    const T br = (T)0.5 * (zk.y + zm.y), bi = (T)0.5 * (zm.x - zk.x);
    T* dst = specb + ((int64_t)k * sy + y) * 2 * sx + xx;
    if (vout && s + 1 < S) {
      *reinterpret_cast<C*>(dst) = C{ar, br};
      *reinterpret_cast<C*>(dst + sx) = C{ai, bi};
    } else {
      dst[0] = ar;
      dst[sx] = ai;
      if (s + 1 < S) {
        T* d1 = specb + ((int64_t)k * sy + y1) * 2 * sx + xx1;
        d1[0] = br;
        d1[sx] = bi;
      }
    }
  }
}

template <typename Tout> struct Out2;
template <> struct Out2<float> { using t = float2; };
template <> struct Out2<double> { using t = double2; };

template <typename T, int TX, typename Tout>
__global__ __launch_bounds__(NT, 2) void k_fft_inv(const T* __restrict__ spec, Tout* __restrict__ z,
                                                   const double* __restrict__ invgam,
                                                   const typename V2<T>::t* __restrict__ tw, int Nt,
                                                   int logNt, int S, int sx, int sy, int accumulate,
                                                   int reverse) {
  using C = typename V2<T>::t;
  using O2 = typename Out2<Tout>::t;
  constexpr int EPT = FftTraits<T>::EPT;
  constexpr int NCOL = TX / 2;
  constexpr int RPI = NT / NCOL;
  extern __shared__ __align__(16) unsigned char smraw[];
  C* sm = reinterpret_cast<C*>(smraw);
  const int ld = Nt + 1, F = (Nt >> 1) + 1, half = Nt >> 1;
  C* smtw = sm + NCOL * ld;
  const int b = blockIdx.y;
  const int s0 = blockIdx.x * TX;
  const T* specb = spec + (int64_t)b * F * sy * 2 * sx;
  stage_twiddles(smtw, tw, Nt);
  const int j = threadIdx.x % NCOL, r = threadIdx.x / NCOL;
  const int s = s0 + 2 * j;
  const bool vin = (sx & 1) == 0;
  // 1. merge the half spectra X_a (column 2j) and X_b (column 2j+1) into the
  //    full circle of Z = X_a + i X_b, stored conjugated for the forward
  //    kernel: ifft(Z) = conj(fft(conj Z)) / Nt.  DC and Nyquist keep only
  //    the real parts (real data).
  {
    const int y = s / sx, xx = s - y * sx;
    const int y1 = (s + 1) / sx, xx1 = (s + 1) - y1 * sx;
    C* col = sm + j * ld;
    constexpr int KU = EPT / 2 + 1;   // F <= KU * RPI: one batch
    {
      C a[KU], bb[KU];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int k = r + u * RPI;
        a[u] = C{0, 0};
        bb[u] = C{0, 0};
        if (k < F && s < S) {
          const T* src = specb + ((int64_t)k * sy + y) * 2 * sx + xx;
          if (vin && s + 1 < S) {
            C re = *reinterpret_cast<const C*>(src), im = *reinterpret_cast<const C*>(src + sx);
            a[u] = C{re.x, im.x};
            bb[u] = C{re.y, im.y};
          } else {
            a[u] = C{src[0], src[sx]};
            if (s + 1 < S) {
              const T* s1 = specb + ((int64_t)k * sy + y1) * 2 * sx + xx1;
              bb[u] = C{s1[0], s1[sx]};
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int k = r + u * RPI;
        if (k < F) {
          const C A = a[u], Bv = bb[u];
          if (k == 0 || k == half) {
            col[k] = C{A.x, -Bv.x};
          } else {
            col[k] = C{A.x - Bv.y, -(A.y + Bv.x)};
            col[Nt - k] = C{A.x + Bv.y, A.y - Bv.x};
          }
        }
      }
    }
  }
  __syncthreads();
  fft_columns<T, EPT>(sm, NCOL, ld, Nt, logNt, smtw);
  // 2. z = conj(fft(conj Z)) / Nt: real column 2j is Re, column 2j+1 is -Im;
  //    Gamma^{-1} (with the 1/Nt) in float64.
  if (s >= S) return;
  Tout* zb = z + (int64_t)b * Nt * S;
  const bool vec = (S & 1) == 0 && s + 1 < S;
  for (int n = r; n < Nt; n += RPI) {
    const C yv = sm[j * ld + n];
    const double ig = invgam[n];
    const double v0 = (double)yv.x * ig, v1 = -(double)yv.y * ig;
    const int nd = reverse ? (Nt - 1 - n) : n;
    Tout* dst = zb + (int64_t)nd * S + s;
    if (vec) {
      O2* d2 = reinterpret_cast<O2*>(dst);
      if (accumulate) {
        const O2 o = *d2;
        *d2 = O2{(Tout)((double)o.x + v0), (Tout)((double)o.y + v1)};
      } else {
        *d2 = O2{(Tout)v0, (Tout)v1};
      }
    } else {
      if (accumulate) dst[0] = (Tout)((double)dst[0] + v0);
      else dst[0] = (Tout)v0;
      if (s + 1 < S) {
        if (accumulate) dst[1] = (Tout)((double)dst[1] + v1);
        else dst[1] = (Tout)v1;
      }
    }
  }
}

struct FftShape { int TX; size_t lds; bool gam_lds; };

// Widest tile (TX <= 32 spatial unknowns) whose LDS image -- TX/2 complex
// columns of Nt+1 entries plus the twiddle table -- lets two workgroups share
// a CU, and whose FFT pass fits the per-thread register budget.
FftShape choose_shape(const Plan& pl) {
  const Geom& g = pl.g;
  const bool f64 = pl.prec == Prec::F64;
  const size_t csize = f64 ? 16 : 8;
  const int ept = f64 ? FftTraits<double>::EPT : FftTraits<float>::EPT;
  const size_t budget = 79 * 1024;
  int TX = 32;
  // columns and twiddles; the forward kernel adds the Gamma table when it
  // fits beside them without narrowing the tile
  auto lds = [&](int tx) { return (size_t)(tx / 2) * (g.nt + 1) * csize + (size_t)g.nt * csize; };
  while (TX > 2 && (lds(TX) > budget || (int64_t)(TX / 2) * g.nt > (int64_t)ept * NT)) TX >>= 1;
  while (TX > 2 && TX / 2 >= g.S) TX >>= 1;  // no wider than the spatial extent needs
  const size_t with_gam = lds(TX) + (size_t)g.nt * sizeof(double);
  const bool gam_lds = with_gam <= budget;
  return FftShape{TX, gam_lds ? with_gam : lds(TX), gam_lds};
}

template <typename T>
void launch_fwd(const Plan& pl, const double* x, const double* bscale, T* spec, int reverse,
                hipStream_t s, const typename V2<T>::t* tw) {
  const Geom& g = pl.g;
  FftShape sh = choose_shape(pl);
  int logNt = 0;
  while ((1 << logNt) < g.nt) ++logNt;
  dim3 grid((unsigned)((g.S + sh.TX - 1) / sh.TX), g.B);
#define PD_FWD(W)                                                                          \
  case W:                                                                                  \
    hipFuncSetAttribute((const void*)k_fft_fwd<T, W>,                                      \
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds);          \
    k_fft_fwd<T, W><<<grid, NT, sh.lds, s>>>(x, spec, pl.d_gam, bscale, tw, g.nt, logNt,   \
                                             (int)g.S, g.sx, g.sy, reverse, sh.gam_lds);   \
    break;
  switch (sh.TX) {
    PD_FWD(2) PD_FWD(4) PD_FWD(8) PD_FWD(16) PD_FWD(32)
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
  dim3 grid((unsigned)((g.S + sh.TX - 1) / sh.TX), g.B);
#define PD_INV(W)                                                                          \
  case W:                                                                                  \
    hipFuncSetAttribute((const void*)k_fft_inv<T, W, Tout>,                                \
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds);          \
    k_fft_inv<T, W, Tout><<<grid, NT, sh.lds, s>>>(spec, z, pl.d_invgam, tw, g.nt, logNt,  \
                                                   (int)g.S, g.sx, g.sy, accumulate,       \
                                                   reverse);                               \
    break;
  switch (sh.TX) {
    PD_INV(2) PD_INV(4) PD_INV(8) PD_INV(16) PD_INV(32)
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
