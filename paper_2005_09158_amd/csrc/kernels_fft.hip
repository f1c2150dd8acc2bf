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
// the same steps backwards, using ifft(Z) = conj(fft(conj Z))/Nt.  Where Nt
// splits as N1 x (threads per column), the four-step kernels further down
// transform each thread's loaded pencil in registers first and leave only the
// remaining passes to LDS.  Workgroups are renumbered so that each XCD owns a
// range of tiles at a time (fft_block): neighbouring tiles share cache lines.

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

// Twiddle W^m (0 <= m < 2 half) from a table of its first half, W^k for
// k < half: W^{k + half} = -W^k.  Halving the table keeps it in LDS beside
// the widest tiles.
template <typename C> __device__ __forceinline__ C twid(const C* t, int m, int half) {
  const C w = t[m & (half - 1)];
  return (m & half) ? C{-w.x, -w.y} : w;
}

constexpr int NT = 256;

// Column bases in LDS: a uniform stride, or the sub-columns of the four-step
// kernels (column c = N1 j + q at j cstr + q ldc).
struct ColUniform {
  int ld;
  __device__ __forceinline__ int base(int c) const { return c * ld; }
};
template <int LOGN1> struct ColSub {
  int ldc, cstr;
  __device__ __forceinline__ int base(int c) const {
    return (c >> LOGN1) * cstr + (c & ((1 << LOGN1) - 1)) * ldc;
  }
};

// In-place forward Stockham FFT of `ncol` columns of length Nt in LDS, column
// c at sm + cm.base(c).  EPT = complex values held per thread in a pass
// (>= ncol*Nt/NT).  tw[k * tws] = exp(-2 pi i k / Nt) for k * tws below half
// the table (see twid).
template <typename T, int EPT, typename CM, int NTH = NT>
__device__ __forceinline__ void fft_columns(typename V2<T>::t* sm, int ncol, CM cm, int Nt, int logNt,
                                            const typename V2<T>::t* __restrict__ tw, int tws = 1) {
  using C = typename V2<T>::t;
  int Ns = 1;
  int bits = logNt;
  if (bits & 1) {  // one radix-2 pass
    const int nb = Nt >> 1, lognb = logNt - 1, total = ncol * nb;
    C v[EPT];
#pragma unroll
    for (int i = 0; i < EPT / 2; ++i) {
      int bf = threadIdx.x + i * NTH;
      if (bf < total) {
        int col = bf >> lognb, j = bf & (nb - 1);
        const C* src = sm + cm.base(col) + j;
        v[2 * i] = src[0];
        v[2 * i + 1] = src[nb];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT / 2; ++i) {
      int bf = threadIdx.x + i * NTH;
      if (bf < total) {
        int col = bf >> lognb, j = bf & (nb - 1);
        // Ns == 1: no twiddle
        C* dst = sm + cm.base(col) + (j << 1);
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
    const int step = Nt / (Ns << 2), half = (Nt * tws) >> 1;
    C v[EPT];
#pragma unroll
    for (int i = 0; i < EPT / 4; ++i) {
      int bf = threadIdx.x + i * NTH;
      if (bf < total) {
        int col = bf >> lognb, j = bf & (nb - 1);
        const C* src = sm + cm.base(col) + j;
        v[4 * i] = src[0];
        v[4 * i + 1] = src[nb];
        v[4 * i + 2] = src[2 * nb];
        v[4 * i + 3] = src[3 * nb];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT / 4; ++i) {
      int bf = threadIdx.x + i * NTH;
      if (bf < total) {
        int col = bf >> lognb, j = bf & (nb - 1);
        int k = j & (Ns - 1);
        C v0 = v[4 * i], v1 = v[4 * i + 1], v2 = v[4 * i + 2], v3 = v[4 * i + 3];
        if (k) {
          v1 = cmul(v1, twid(tw, k * step * tws, half));
          v2 = cmul(v2, twid(tw, 2 * k * step * tws, half));
          v3 = cmul(v3, twid(tw, 3 * k * step * tws, half));
        }
        C t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = cmi(csub(v1, v3));
        C* dst = sm + cm.base(col) + ((j - k) << 2) + k;
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


// Copies the first half of the Nt-entry twiddle table into LDS behind the
// data columns (twid supplies the second half).
template <typename C>
__device__ __forceinline__ void stage_twiddles(C* smtw, const C* __restrict__ tw, int Nt) {
  for (int i = threadIdx.x; i < (Nt >> 1); i += blockDim.x) smtw[i] = tw[i];
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

// Tile order of the time transforms: workgroup i runs on XCD i % 8
// (round-robin dispatch); XCD x takes chunks x, x + 8, x + 16, ... of C = 128
// consecutive tiles, so the eight XCDs work on neighbouring chunks of one
// right-hand side at a time (with xcd_block each XCD works in its own), while
// the tiles of a chunk, whose 64-byte output rows share cache lines, stay on
// one XCD.  At 512^2 x 1024 x 8 this took the inverse transform from 7.35 to
// 6.75 ms and the forward one from 8.12 to 7.93 ms.  Tiles past the last
// whole group of 8 C keep dispatch order.
__device__ __forceinline__ BlockPos fft_block() {
  constexpr unsigned C = 128;
  const unsigned gx = gridDim.x, gy = gridDim.y, total = gx * gy;
  const unsigned i = blockIdx.x + gx * blockIdx.y;
  unsigned id = i;
  if (i < total / (8 * C) * (8 * C)) {
    const unsigned x = i & 7, li = i >> 3;
    id = ((li / C) * 8 + x) * C + li % C;
  }
  return BlockPos{(int)(id % gx), (int)(id / gx), 0};
}

template <typename T, int TX>
__global__ __launch_bounds__(NT, 2) void k_fft_fwd(const double* __restrict__ x, T* __restrict__ spec,
                                                   const double* __restrict__ gam,
                                                   const double* __restrict__ bscale, int bstride,
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
  const BlockPos bp = fft_block();
  const int b = bp.y;
  const int s0 = bp.x * TX;
  const double* xb = x + (int64_t)b * Nt * S;
  const double sc = bscale ? bscale[(int64_t)b * bstride] : 1.0;
  const bool vec = (S & 1) == 0;
  double* smg = reinterpret_cast<double*>(smtw + (Nt >> 1));   // Gamma
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
  fft_columns<T, EPT>(sm, NCOL, ColUniform{ld}, Nt, logNt, smtw);
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
  const BlockPos bp = fft_block();
  const int b = bp.y;
  const int s0 = bp.x * TX;
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
  fft_columns<T, EPT>(sm, NCOL, ColUniform{ld}, Nt, logNt, smtw);
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

// ---------------------------------------------------------------------------
// Four-step form (Nt = N1 * TPC, TPC = NT / NCOL threads per column): thread
// r of column j holds the samples n = r + TPC u (u < N1) -- exactly its global
// loads -- and transforms them in registers,
//   X_r[q] = sum_u x[r + TPC u] W_N1^{u q},  then  X_r[q] *= W_Nt^{r q};
// the TPC-point transforms over r of every (j, q) then run as Stockham passes
// in LDS, and Z[q + N1 p] is their output p.  Two LDS passes replace five at
// Nt = 512 (three replace six at Nt = 2048).

// In-register radix-2 decimation-in-frequency transform of N values; the
// result is in bit-reversed order.  tw[k * tws] = exp(-2 pi i k / N).
template <int N, typename C>
__device__ __forceinline__ void reg_fft(C (&c)[N], const C* tw, int tws) {
#pragma unroll
  for (int len = N; len >= 2; len >>= 1) {
    const int h = len >> 1;
#pragma unroll
    for (int i0 = 0; i0 < N; i0 += len)
#pragma unroll
      for (int t = 0; t < h; ++t) {
        const C a = c[i0 + t], b = c[i0 + t + h];
        c[i0 + t] = cadd(a, b);
        const C d = csub(a, b);
        const int e = t * (N / len);   // W_len^t = W_N^e
        if (e == 0) c[i0 + t + h] = d;
        else if (4 * e == N) c[i0 + t + h] = cmi(d);
        else c[i0 + t + h] = cmul(d, tw[e * tws]);
      }
  }
}

template <int N> __device__ __forceinline__ constexpr int brev(int q) {
  int r = 0;
  for (int b = 1; b < N; b <<= 1) r = (r << 1) | ((q & b) ? 1 : 0);
  return r;
}

template <int V> struct Log2 { static constexpr int v = 1 + Log2<V / 2>::v; };
template <> struct Log2<1> { static constexpr int v = 0; };

// Pass 1 of the four-step form on this thread's pencil c (natural order in
// u), twiddle, and store to the sub-column layout: (j, q) position r.
template <typename T, int N1, int TPC>
__device__ __forceinline__ void fourstep_pass1(typename V2<T>::t (&c)[N1], typename V2<T>::t* sm,
                                               const typename V2<T>::t* smtw, int Nt, int j, int r,
                                               int ldc, int cstr) {
  using C = typename V2<T>::t;
  reg_fft<N1>(c, smtw, Nt / N1);
#pragma unroll
  for (int q = 0; q < N1; ++q) {
    C xq = c[brev<N1>(q)];
    if (q) xq = cmul(xq, twid(smtw, (r * q) & (Nt - 1), Nt >> 1));
    sm[j * cstr + q * ldc + r] = xq;
  }
}

template <typename T, int TX, int N1, int NTH = NT>
__global__ __launch_bounds__(NTH, NTH / 128) void k_fft4_fwd(const double* __restrict__ x, T* __restrict__ spec,
                                                    const double* __restrict__ gam,
                                                    const double* __restrict__ bscale, int bstride,
                                                    const typename V2<T>::t* __restrict__ tw, int Nt,
                                                    int S, int sx, int sy, int reverse, int gam_lds,
                                                    int tw_lds) {
  using C = typename V2<T>::t;
  constexpr int NCOL = TX / 2, TPC = NTH / NCOL, LOGN1 = Log2<N1>::v, LOGTPC = Log2<TPC>::v;
  constexpr int LDC = TPC + 1;           // sub-column stride
  extern __shared__ __align__(16) unsigned char smraw[];
  C* sm = reinterpret_cast<C*>(smraw);
  const int cstr = N1 * LDC + 1;         // column stride (odd: columns fall in different banks)
  const int F = (Nt >> 1) + 1;
  C* smtw = sm + NCOL * cstr;
  double* smg = reinterpret_cast<double*>(smtw + (tw_lds ? (Nt >> 1) : 0));
  const C* twp = tw_lds ? smtw : tw;     // twiddles in LDS, or through the caches
  const BlockPos bp = fft_block();
  const int b = bp.y, s0 = bp.x * TX;
  const double* xb = x + (int64_t)b * Nt * S;
  const double sc = bscale ? bscale[(int64_t)b * bstride] : 1.0;
  const bool vec = (S & 1) == 0;
  const int j = threadIdx.x % NCOL, r = threadIdx.x / NCOL;
  const int s = s0 + 2 * j;
  double2 v[N1];
#pragma unroll
  for (int u = 0; u < N1; ++u) {
    const int n = r + TPC * u;
    const int nsrc = reverse ? (Nt - 1 - n) : n;
    v[u] = load_pair(xb + (int64_t)nsrc * S, s, S, vec);
  }
  if (tw_lds) stage_twiddles(smtw, tw, Nt);
  if (gam_lds)
    for (int i = threadIdx.x; i < Nt; i += NTH) smg[i] = gam[i];
  __syncthreads();
  C c[N1];
#pragma unroll
  for (int u = 0; u < N1; ++u) {
    const int n = r + TPC * u;
    const double g = (gam_lds ? smg[n] : gam[n]) * sc;
    c[u] = C{(T)(v[u].x * g), (T)(v[u].y * g)};
  }
  fourstep_pass1<T, N1, TPC>(c, sm, twp, Nt, j, r, LDC, cstr);
  __syncthreads();
  fft_columns<T, N1, ColSub<LOGN1>, NTH>(sm, NCOL * N1, ColSub<LOGN1>{LDC, cstr}, TPC, LOGTPC, twp, N1);
  // Hermitian split (as k_fft_fwd), Z[k] at (j, k mod N1) position k / N1
  if (s >= S) return;
  T* specb = spec + (int64_t)b * F * sy * 2 * sx;
  const bool vout = (sx & 1) == 0;
  const int y = s / sx, xx = s - y * sx;
  const int y1 = (s + 1) / sx, xx1 = (s + 1) - y1 * sx;
  const C* colj = sm + j * cstr;
  for (int k = r; k < F; k += TPC) {
    const int km = (Nt - k) & (Nt - 1);
    const C zk = colj[(k & (N1 - 1)) * LDC + (k >> LOGN1)];
    const C zm = colj[(km & (N1 - 1)) * LDC + (km >> LOGN1)];
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

template <typename T, int TX, int N1, typename Tout, int NTH = NT>
__global__ __launch_bounds__(NTH, NTH / 128) void k_fft4_inv(const T* __restrict__ spec, Tout* __restrict__ z,
                                                    const double* __restrict__ invgam,
                                                    const typename V2<T>::t* __restrict__ tw, int Nt,
                                                    int S, int sx, int sy, int accumulate, int reverse,
                                                    int tw_lds) {
  using C = typename V2<T>::t;
  using O2 = typename Out2<Tout>::t;
  constexpr int NCOL = TX / 2, TPC = NTH / NCOL, LOGN1 = Log2<N1>::v, LOGTPC = Log2<TPC>::v;
  constexpr int LDC = TPC + 1;
  constexpr int KU = N1 / 2 + 1;         // spectrum rows k = r + TPC u < F
  extern __shared__ __align__(16) unsigned char smraw[];
  C* sm = reinterpret_cast<C*>(smraw);
  const int cstr = N1 * LDC + 1;
  const int F = (Nt >> 1) + 1, half = Nt >> 1;
  C* smtw = sm + NCOL * cstr;
  const C* twp = tw_lds ? smtw : tw;
  const BlockPos bp = fft_block();
  const int b = bp.y, s0 = bp.x * TX;
  const T* specb = spec + (int64_t)b * F * sy * 2 * sx;
  const int j = threadIdx.x % NCOL, r = threadIdx.x / NCOL;
  const int s = s0 + 2 * j;
  const bool vin = (sx & 1) == 0;
  C a[KU], bb[KU];
  {
    const int y = s / sx, xx = s - y * sx;
    const int y1 = (s + 1) / sx, xx1 = (s + 1) - y1 * sx;
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int k = r + TPC * u;
      a[u] = C{0, 0};
      bb[u] = C{0, 0};
      if (k < F && s < S) {
        const T* src = specb + ((int64_t)k * sy + y) * 2 * sx + xx;
        if (vin && s + 1 < S) {
          const C re = *reinterpret_cast<const C*>(src), im = *reinterpret_cast<const C*>(src + sx);
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
  }
  if (tw_lds) stage_twiddles(smtw, tw, Nt);
  // 1. conj Z on the full circle in natural order (column j at j cstr)
  C* colj = sm + j * cstr;
#pragma unroll
  for (int u = 0; u < KU; ++u) {
    const int k = r + TPC * u;
    if (k < F) {
      const C A = a[u], Bv = bb[u];
      if (k == 0 || k == half) {
        colj[k] = C{A.x, -Bv.x};
      } else {
        colj[k] = C{A.x - Bv.y, -(A.y + Bv.x)};
        colj[Nt - k] = C{A.x + Bv.y, A.y - Bv.x};
      }
    }
  }
  __syncthreads();
  // 2. pencils, pass 1 in registers, sub-columns, TPC-point passes
  C c[N1];
#pragma unroll
  for (int u = 0; u < N1; ++u) c[u] = colj[r + TPC * u];
  __syncthreads();
  fourstep_pass1<T, N1, TPC>(c, sm, twp, Nt, j, r, LDC, cstr);
  __syncthreads();
  fft_columns<T, N1, ColSub<LOGN1>, NTH>(sm, NCOL * N1, ColSub<LOGN1>{LDC, cstr}, TPC, LOGTPC, twp, N1);
  // 3. z = conj(fft(conj Z)) / Nt with Gamma^{-1}; sample n at (j, n mod N1) position n / N1
  if (s >= S) return;
  Tout* zb = z + (int64_t)b * Nt * S;
  const bool vec = (S & 1) == 0 && s + 1 < S;
  for (int n = r; n < Nt; n += TPC) {
    const C yv = colj[(n & (N1 - 1)) * LDC + (n >> LOGN1)];
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

// LDS bytes of the four-step kernels' columns (stride N1 (TPC + 1) + 1);
// the twiddle and Gamma tables follow when they fit.
inline size_t fourstep_cols(int tx, int nt, size_t csize, int nth = NT) {
  const int ncol = tx / 2, tpc = nth / ncol, n1 = nt / tpc;
  return (size_t)ncol * ((size_t)n1 * (tpc + 1) + 1) * csize;
}

// n1 > 0: four-step kernels; lds_inv: bytes of the inverse (no Gamma table)
struct FftShape { int TX; size_t lds; bool gam_lds; int n1; bool tw_lds; size_t lds_inv; int nth; };

// Tile shape: the four-step form where an instantiated (TX, N1, threads)
// fits (see the preference order below), else the widest Stockham tile
// (TX <= 32 spatial unknowns) whose LDS image -- TX/2 complex columns of
// Nt+1 entries plus half the twiddle table -- lets two workgroups share a
// CU, and whose FFT pass fits the per-thread register budget.
FftShape choose_shape(const Plan& pl) {
  const Geom& g = pl.g;
  const bool f64 = pl.prec == Prec::F64;
  const size_t csize = f64 ? 16 : 8;
  const int ept = f64 ? FftTraits<double>::EPT : FftTraits<float>::EPT;
  const size_t budget = 79 * 1024;
  int TX = 32;
  // columns and twiddles; the forward kernel adds the Gamma table when it
  // fits beside them without narrowing the tile
  auto lds = [&](int tx) { return (size_t)(tx / 2) * (g.nt + 1) * csize + (size_t)(g.nt / 2) * csize; };
  while (TX > 2 && (lds(TX) > budget || (int64_t)(TX / 2) * g.nt > (int64_t)ept * NT)) TX >>= 1;
  while (TX > 2 && TX / 2 >= g.S) TX >>= 1;  // no wider than the spatial extent needs
  // four-step form when the pencil length N1 = Nt / TPC is 4 .. EPT and the
  // tile is one of the instantiated widths
  // (the twiddle table in LDS only when it fits beside the columns, else it
  // is read through the caches)
  // Preference: a tile of 16 or 32 columns (rows of 128 B or more) that
  // lets four, else three workgroups share a CU (float32 only: the float64
  // pencils need more than a quarter of the registers), else the widest
  // valid tile at two per CU.
  const size_t twb = (size_t)(g.nt / 2) * csize, gb = (size_t)g.nt * sizeof(double);
  const size_t tiers[3] = {f64 ? 0 : (size_t)39 * 1024, (size_t)53 * 1024, budget};
  // At every tier a 512-thread workgroup (half the pencil per thread, twice
  // the waves) is tried first where it is instantiated: measured faster at
  // Nt = 2048 (two per CU) and at Nt = 512 (four per CU: 113 / 102 us against
  // 121 / 109 us for the forward / inverse transform at 256^2 x 512).
  for (int pass = 0; pass < 3; ++pass) {
    const size_t lim = tiers[pass];
    for (int tx4 = 32; tx4 >= (pass < 2 ? 16 : 8); tx4 >>= 1)
      for (int nth = 2 * NT; nth >= NT; nth >>= 1) {
        const int ncol = tx4 / 2, tpc = nth / ncol, n1 = g.nt / tpc;
        if (tx4 / 2 >= g.S && tx4 > 8) continue;
        if (n1 < 4 || n1 > ept || n1 * tpc != g.nt) continue;
        if (nth > NT && (tx4 > 16 || n1 < 8 || n1 > 16)) continue;   // instantiated shapes
        const size_t cols = fourstep_cols(tx4, g.nt, csize, nth);
        if (cols > lim) continue;
        const bool twl = cols + twb <= lim;
        const size_t inv = cols + (twl ? twb : 0);
        const bool gl = inv + gb <= lim;
        return FftShape{tx4, inv + (gl ? gb : 0), gl, n1, twl, inv, nth};
      }
  }
  const size_t with_gam = lds(TX) + gb;
  const bool gam_lds = with_gam <= budget;
  return FftShape{TX, gam_lds ? with_gam : lds(TX), gam_lds, 0, true, lds(TX), NT};
}

template <typename T>
void launch_fwd(const Plan& pl, const double* x, const double* bscale, int bstride, T* spec, int reverse,
                hipStream_t s, const typename V2<T>::t* tw) {
  const Geom& g = pl.g;
  FftShape sh = choose_shape(pl);
  int logNt = 0;
  while ((1 << logNt) < g.nt) ++logNt;
  dim3 grid((unsigned)((g.S + sh.TX - 1) / sh.TX), g.B);
  if (sh.n1 > 0) {
#define PD_FWD4T(W, N, H)                                                                  \
  if (sh.TX == W && sh.n1 == N && sh.nth == H) {                                           \
    lds_limit((const void*)k_fft4_fwd<T, W, N, H>, sh.lds);                                \
    k_fft4_fwd<T, W, N, H><<<grid, H, sh.lds, s>>>(x, spec, pl.d_gam, bscale, bstride, tw, g.nt, \
                                                   (int)g.S, g.sx, g.sy, reverse,          \
                                                   sh.gam_lds, sh.tw_lds);                 \
    return;                                                                                \
  }
#define PD_FWD4(W, N) PD_FWD4T(W, N, NT)
    PD_FWD4(8, 4) PD_FWD4(8, 8) PD_FWD4(8, 16) PD_FWD4(16, 4) PD_FWD4(16, 8) PD_FWD4(16, 16)
    PD_FWD4(32, 4) PD_FWD4(32, 8) PD_FWD4(32, 16)
    if constexpr (FftTraits<T>::EPT >= 32) {
      PD_FWD4(8, 32) PD_FWD4(16, 32) PD_FWD4(32, 32)
    }
    PD_FWD4T(8, 8, 512) PD_FWD4T(8, 16, 512) PD_FWD4T(16, 8, 512) PD_FWD4T(16, 16, 512)
#undef PD_FWD4
#undef PD_FWD4T
  }
#define PD_FWD(W)                                                                          \
  case W:                                                                                  \
    lds_limit((const void*)k_fft_fwd<T, W>, sh.lds);                                       \
    k_fft_fwd<T, W><<<grid, NT, sh.lds, s>>>(x, spec, pl.d_gam, bscale, bstride, tw, g.nt, logNt, \
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
  if (sh.n1 > 0) {
    const size_t lds4 = sh.lds_inv;
#define PD_INV4T(W, N, H)                                                                  \
  if (sh.TX == W && sh.n1 == N && sh.nth == H) {                                           \
    lds_limit((const void*)k_fft4_inv<T, W, N, Tout, H>, lds4);                            \
    k_fft4_inv<T, W, N, Tout, H><<<grid, H, lds4, s>>>(spec, z, pl.d_invgam, tw, g.nt,     \
                                                       (int)g.S, g.sx, g.sy, accumulate,   \
                                                       reverse, sh.tw_lds);                \
    return;                                                                                \
  }
#define PD_INV4(W, N) PD_INV4T(W, N, NT)
    PD_INV4(8, 4) PD_INV4(8, 8) PD_INV4(8, 16) PD_INV4(16, 4) PD_INV4(16, 8) PD_INV4(16, 16)
    PD_INV4(32, 4) PD_INV4(32, 8) PD_INV4(32, 16)
    if constexpr (FftTraits<T>::EPT >= 32) {
      PD_INV4(8, 32) PD_INV4(16, 32) PD_INV4(32, 32)
    }
    PD_INV4T(8, 8, 512) PD_INV4T(8, 16, 512) PD_INV4T(16, 8, 512) PD_INV4T(16, 16, 512)
#undef PD_INV4
#undef PD_INV4T
  }
#define PD_INV(W)                                                                          \
  case W:                                                                                  \
    lds_limit((const void*)k_fft_inv<T, W, Tout>, sh.lds);                                 \
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

// Step-(b) x-transform of a sine basis by FFT (nx + 1 a power of two).  For
// a real row x_1 .. x_n, the DST-I S_k = sum_j x_j sin(pi j k / (n+1)),
// k = 1..n, is -Im(Z_k) / 2 for the FFT Z of the odd extension
// z = (0, x_1 .. x_n, 0, -x_n .. -x_1) of length N2 = 2 (n+1).  The real and
// imaginary halves of a spectral row go in as the real and imaginary parts
// of one z: both extensions are odd, so each transform is purely imaginary and
// Z_k = -2i S_k(x_re) + 2 S_k(x_im) keeps them apart.  The basis is
// sqrt(2/(n+1)) sin(pi j k/(n+1)) (orthonormal and symmetric), so the
// forward and the inverse x-transform are this same map.  ncol rows per
// workgroup, ncol N2 <= EPT NT / 2 (four workgroups per CU), columns in LDS
// with an odd stride.
template <typename T>
__global__ __launch_bounds__(NT, 2) void k_dst(const T* __restrict__ in, T* __restrict__ out, int64_t rows, int n,
                                               int logN2, int ncol, T scale,
                                               const typename V2<T>::t* __restrict__ tw) {
  using C = typename V2<T>::t;
  constexpr int EPT = FftTraits<T>::EPT;
  extern __shared__ __align__(16) unsigned char smraw[];
  C* sm = reinterpret_cast<C*>(smraw);
  const int N2 = 1 << logN2, ld = N2 + 1;
  C* smtw = sm + ncol * ld;
  stage_twiddles(smtw, tw, N2);
  const int64_t r0 = (int64_t)blockIdx.x * ncol;
  const int64_t rs = 2 * (int64_t)n;   // row length of the buffer: n real, then n imaginary parts
  // the odd extensions: each input value read once, stored at j and N2 - j.
  // All of a thread's loads (at most EPT / 2 pairs, since ncol N2 <= EPT NT)
  // are issued before the first store; out-of-range ones read a valid
  // address and are dropped, so they carry no branches.
  constexpr int MAXE = EPT / 2;
  const int tot = ncol * n;
  C v[MAXE];
#pragma unroll
  for (int u = 0; u < MAXE; ++u) {
    const int e = min((int)threadIdx.x + u * NT, tot - 1);
    const int c = e / n, i = e - c * n;
    const int64_t r = min(r0 + c, rows - 1);
    const T* row = in + r * rs;
    v[u] = C{row[i], row[n + i]};
  }
#pragma unroll
  for (int u = 0; u < MAXE; ++u) {
    const int e = (int)threadIdx.x + u * NT;
    if (e < tot) {
      const int c = e / n, i = e - c * n;
      const C w = (r0 + c < rows) ? v[u] : C{0, 0};
      sm[c * ld + i + 1] = w;
      sm[c * ld + N2 - 1 - i] = C{-w.x, -w.y};
    }
  }
  for (int c = threadIdx.x; c < ncol; c += NT) {
    sm[c * ld] = C{0, 0};
    sm[c * ld + n + 1] = C{0, 0};
  }
  __syncthreads();
  fft_columns<T, EPT>(sm, ncol, ColUniform{ld}, N2, logN2, smtw);
  for (int e = threadIdx.x; e < ncol * 2 * n; e += NT) {
    const int c = e / (2 * n), q = e - c * 2 * n;
    const int64_t r = r0 + c;
    if (r >= rows) continue;
    const bool imag = q >= n;
    const C z = sm[c * ld + (imag ? q - n : q) + 1];
    out[r * rs + q] = imag ? scale * z.x : -scale * z.y;
  }
}

}  // namespace

void fft_time_forward(const Plan& pl, const double* x, const double* bscale, int bstride, void* spec,
                      int reverse, hipStream_t s) {
  if (pl.prec == Prec::F64)
    launch_fwd<double>(pl, x, bscale, bstride, (double*)spec, reverse, s, pl.d_tw64);
  else
    launch_fwd<float>(pl, x, bscale, bstride, (float*)spec, reverse, s, pl.d_tw32);
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

void dst_transform(const Plan& pl, const void* in, void* out, hipStream_t s) {
  const Geom& g = pl.g;
  const int n = g.sx, N2 = 2 * (n + 1);
  int logN2 = 0;
  while ((1 << logN2) < N2) ++logN2;
  const int64_t rows = (int64_t)g.B * g.F * g.sy;
  const double scale = 0.5 * std::sqrt(2.0 / (n + 1));
  if (pl.prec == Prec::F64) {
    const int ncol = std::max(1, FftTraits<double>::EPT * NT / (2 * N2));   // half the pass capacity: four workgroups per CU
    const size_t lds = sizeof(double2) * ((size_t)ncol * (N2 + 1) + N2 / 2);
    lds_limit((const void*)k_dst<double>, lds);
    k_dst<double><<<(unsigned)((rows + ncol - 1) / ncol), NT, lds, s>>>(
        (const double*)in, (double*)out, rows, n, logN2, ncol, scale, (const double2*)pl.d_dtw);
  } else {
    const int ncol = std::max(1, FftTraits<float>::EPT * NT / (2 * N2));   // half the pass capacity: four workgroups per CU
    const size_t lds = sizeof(float2) * ((size_t)ncol * (N2 + 1) + N2 / 2);
    lds_limit((const void*)k_dst<float>, lds);
    k_dst<float><<<(unsigned)((rows + ncol - 1) / ncol), NT, lds, s>>>(
        (const float*)in, (float*)out, rows, n, logN2, ncol, (float)scale, (const float2*)pl.d_dtw);
  }
}

}  // namespace pd
