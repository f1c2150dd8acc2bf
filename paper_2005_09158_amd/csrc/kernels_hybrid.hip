// Time transforms of ParaDiag-I with the hybrid discretisation (Section
// 2.1.2): Step-(a) S = (V^{-1} (x) I) r and Step-(c) z = (V (x) I) S, where
// B = V D V^{-1} has the closed-form eigenvectors of Thm thmCondU.  B is real,
// so its eigenpairs come in conjugate pairs and only the half set n < Nt/2
// is transformed: S_n for the kept eigenvalues, and z = sum_n 2 Re(V[:, n] S_n).
// Both are one dense real product per right-hand side,
//
//   C[m][j] = sum_k W[m][k] X[k][j],   m, k < Nt,  j < S = nx * ny,
//
// with W the Nt x Nt real table of the transform (rows 2n, 2n+1 of the
// forward one: Re and Im of row n of V^{-1}; columns 2n, 2n+1 of the inverse
// one: 2 Re V[:, n] and -2 Im V[:, n]) and X, C the data.  The spectral side
// uses the planar layout of the spectral buffer [F][sy][2][sx] (F = Nt/2):
// row 2n + c, point j = (y, x) sits at n (2S) + c sx + y (2 sx) + x.  The time
// side is [Nt][S].
//
// These are compute-bound contractions (2 Nt flops per byte of X at Nt >= 256
// rows per workgroup), run in float64 on MFMA (v_mfma_f64_16x16x4f64): the
// roundoff of ParaDiag-I grows with Cond_2(V) = O(Nt^2), so the transforms
// keep float64 whatever the precision of Step-(b).
//
// Kernel: 256 threads = 4 waves; a workgroup owns BM = 64 FM rows (wave w
// the 16 FM rows from 16 FM w) and BN = 64 points.  The X tile (16 time rows
// x 64 points) is staged through LDS, double-buffered, with the next tile
// prefetched into registers; W is read straight from global memory as MFMA
// fragments (the host stores it in fragment order, so one fragment is one
// coalesced 512-byte load, and the table stays in L2).  Workgroups are
// numbered so that the row tiles of one point range run on one XCD (the
// second read of the X tile comes from that XCD's L2).
// Fragment layout (16x16x4 float64 MFMA): lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; accumulator v of lane l is C[l / 16 + 4 v][l % 16].

#include "internal.h"

namespace pd {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int NT = 256;
constexpr int BN = 64, BK = 16, LDB = BN + 2;

__device__ __forceinline__ int64_t spec_off(int row, int j, int sx, int64_t S) {
  const int y = j / sx, x = j - y * sx;
  return (int64_t)(row >> 1) * (2 * S) + (row & 1) * sx + (int64_t)y * 2 * sx + x;
}

// FWD: X = real data [Nt][S] (double), C = spectral (Tc).  INV: X = spectral
// (Tx), C = real data [Nt][S] (Tc), accumulated into when acc != 0.
template <typename Tx, typename Tc, int FM, bool FWD>
__global__ __launch_bounds__(NT) void k_time_gemm(const double* __restrict__ Wf, const Tx* __restrict__ X,
                                                  Tc* __restrict__ C, int M, int K, int Kpad, int64_t S,
                                                  int sx, int64_t xbatch, int64_t cbatch, int ntm,
                                                  int ntn, int acc_out, const double* __restrict__ cscale) {
  constexpr int BM = 64 * FM;
  __shared__ __align__(16) double Xs[2][BK * LDB];
  const unsigned total = (unsigned)(ntm * ntn) * gridDim.y;
  const unsigned id = xcd_order(blockIdx.x + gridDim.x * blockIdx.y, total);
  const int tm = (int)(id % ntm);
  const int tn = (int)((id / ntm) % ntn);
  const int bz = (int)(id / ((unsigned)ntm * ntn));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t j0 = (int64_t)tn * BN;
  const Tx* Xb = X + (int64_t)bz * xbatch;
  Tc* Cb = C + (int64_t)bz * cbatch;

  // X tile loader: thread t owns row t / 16 and points 4 (t % 16) .. + 3
  const int lrow = threadIdx.x >> 4, lcol = (threadIdx.x & 15) * 4;
  double pre[4];
  auto load_tile = [&](int k0) {
    const int k = k0 + lrow;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t j = j0 + lcol + q;
      double v = 0.0;
      if (k < K && j < S) {
        if constexpr (FWD) v = (double)Xb[(int64_t)k * S + j];
        else v = (double)Xb[spec_off(k, (int)j, sx, S)];
      }
      pre[q] = v;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) Xs[buf][lrow * LDB + lcol + q] = pre[q];
  };

  d4 acc[FM][4];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[i][c] = d4{0.0, 0.0, 0.0, 0.0};

  // fragment rows of this wave: row blocks rb = tm * 4 FM + wave FM + i
  const int kq = Kpad / 4;   // 4-wide k steps per row block
  const double* Wrow = Wf + ((int64_t)(tm * 4 * FM + wave * FM) * kq) * 64 + lane;

  // A fragments of one X tile (4 k steps), prefetched one tile ahead like X
  double acur[FM][BK / 4], anext[FM][BK / 4];
  auto load_a = [&](int k0, double (&a)[FM][BK / 4]) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int ks = 0; ks < BK / 4; ++ks) a[i][ks] = Wrow[((int64_t)i * kq + k0 / 4 + ks) * 64];
  };
  load_a(0, acur);
  load_tile(0);
  store_tile(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < Kpad; k0 += BK) {
    const bool more = k0 + BK < Kpad;
    if (more) {
      load_tile(k0 + BK);
      load_a(k0 + BK, anext);
    }
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      double bfr[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) bfr[c] = Xs[buf][(ks * 4 + lk) * LDB + c * 16 + lr];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[i][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(acur[i][ks], bfr[c], acc[i][c], 0, 0, 0);
    }
    if (more) {
      store_tile(buf ^ 1);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) acur[i][ks] = anext[i][ks];
      __syncthreads();
      buf ^= 1;
    }
  }
  // epilogue: C[m][j], m = row of this lane, j = point of this lane (times
  // *cscale when given: the Krylov scale of the input vector)
  const double sc = cscale ? *cscale : 1.0;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t j = j0 + c * 16 + lr;
      if (j >= S) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = tm * BM + (wave * FM + i) * 16 + lk + 4 * v;
        if (m >= M) continue;
        if constexpr (FWD) {
          Cb[spec_off(m, (int)j, sx, S)] = (Tc)(sc * acc[i][c][v]);
        } else {
          Tc* dst = Cb + (int64_t)m * S + j;
          const double prev = acc_out ? (double)*dst : 0.0;
          *dst = (Tc)(prev + sc * acc[i][c][v]);
        }
      }
    }
}

}  // namespace

// Row tile of the time product: 256 rows (each data tile feeds four times the
// MFMA work) unless padding m to a multiple of 256 wastes more than a tenth
// beyond what 64-row tiles pad (m = 258: 512 against 320 rows)
int time_gemm_rows(int m) {
  const int p256 = 256 * ((m + 255) / 256), p64 = 64 * ((m + 63) / 64);
  return (m >= 256 && 10 * p256 <= 11 * p64) ? 256 : 64;
}

// W (m x k, row-major) in MFMA fragment order for workgroups of
// time_gemm_rows(m) rows: frag[(rb * (Kpad/4) + ks) * 64 + lane] =
// W[16 rb + lane % 16][4 ks + lane / 16], zero outside the matrix;
// Mpad = rows * ceil(m / rows), Kpad = 16 ceil(k / 16).
std::vector<double> time_gemm_fragments(const std::vector<double>& W, int m, int k) {
  const int rows = time_gemm_rows(m);
  const int Mpad = rows * ((m + rows - 1) / rows), Kpad = BK * ((k + BK - 1) / BK);
  std::vector<double> f((size_t)Mpad * Kpad, 0.0);
  const int kq = Kpad / 4;
  for (int rb = 0; rb < Mpad / 16; ++rb)
    for (int ks = 0; ks < kq; ++ks)
      for (int l = 0; l < 64; ++l) {
        const int r = 16 * rb + (l & 15), c = 4 * ks + (l >> 4);
        if (r < m && c < k) f[((size_t)rb * kq + ks) * 64 + l] = W[(size_t)r * k + c];
      }
  return f;
}

size_t time_gemm_fragment_elems(int m, int k) {
  const int rows = time_gemm_rows(m);
  return (size_t)(rows * ((m + rows - 1) / rows)) * (BK * ((k + BK - 1) / BK));
}

void time_gemm(const Plan& pl, bool forward, const double* table, const void* in, void* out, bool spec_f32,
               bool out_f32, int accumulate, int batch, int nt, int F, int m, int k, hipStream_t s,
               const double* cscale) {
  const Geom& g = pl.g;
  const int rows = time_gemm_rows(m);
  const int Kpad = BK * ((k + BK - 1) / BK);
  const int ntm = (m + rows - 1) / rows;
  const int ntn = (int)((g.S + BN - 1) / BN);
  const int64_t tb = (int64_t)nt * g.S, sb = (int64_t)F * 2 * g.S;
  dim3 grid((unsigned)(ntm * ntn), batch);
#define PD_TG(TX, TC, FM, FW)                                                                       \
  k_time_gemm<TX, TC, FM, FW><<<grid, NT, 0, s>>>(table, (const TX*)in, (TC*)out, m, k, Kpad, g.S, g.sx, \
                                                  FW ? tb : sb, FW ? sb : tb, ntm, ntn, accumulate, cscale)
#define PD_TG_FM(TX, TC, FW) \
  if (rows == 256) PD_TG(TX, TC, 4, FW); else PD_TG(TX, TC, 1, FW);
  if (forward) {
    if (!spec_f32) { PD_TG_FM(double, double, true) }
    else { PD_TG_FM(double, float, true) }
  } else {
    if (!spec_f32) {
      if (out_f32) { PD_TG_FM(double, float, false) } else { PD_TG_FM(double, double, false) }
    } else {
      if (out_f32) { PD_TG_FM(float, float, false) } else { PD_TG_FM(float, double, false) }
    }
  }
#undef PD_TG_FM
#undef PD_TG
}

void time_transform(const Plan& pl, bool forward, const void* in, void* out, bool out_f32,
                    int accumulate, hipStream_t s) {
  const Geom& g = pl.g;
  time_gemm(pl, forward, forward ? pl.d_wf : pl.d_wi, in, out, pl.prec != Prec::F64, out_f32, accumulate,
            g.B, g.nt, g.F, g.nt, g.nt, s);
}

}  // namespace pd
