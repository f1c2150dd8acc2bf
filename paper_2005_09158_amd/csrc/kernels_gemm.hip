// x-direction transform of Step-(b) on MFMA.
//
// With the basis K_x = Q T Q^H, the 2D shifted system of frequency n,
// lambda1 U + lambda2 (U K_x^T + K_y U) = R (U stored as an ny x nx matrix),
// becomes lambda1 W + lambda2 (W T^T + K_y W) = R conj(Q) for W = U conj(Q),
// and U = W Q^T afterwards.  Both transforms are one GEMM over all
// (right-hand side, frequency, y) rows of the spectral buffer.
//
// Rows are stored row-planar (nx real parts, then nx imaginary parts), so a
// complex row times a complex matrix is one real GEMM with the 2nx x 2nx
// block matrix [[Re M, Im M], [-Im M, Re M]]; for the real sine basis the
// real and imaginary halves are independent rows times the nx x nx matrix.
// The host prepares the real matrix transposed (Bt[n][k], k contiguous) in
// the compute format, so both operands are read along k.
//
//   C[m][n] = sum_k A[m][k] * Bt[n][k]
//
// Kernel: 256 threads = 2 x 2 waves, block tile BM x BN x BK staged in LDS,
// each wave a (BM/2) x (BN/2) tile of 16 x 16 MFMA blocks:
//   float64  v_mfma_f64_16x16x4f64   (64 x 64 x 16 tiles)
//   float32  v_mfma_f32_16x16x4f32   (64 x 64 x 16 tiles)
//   bf16     v_mfma_f32_16x16x32_bf16 with float32 accumulation (128 x 128 x 32 tiles);
//            float32 rows are rounded to bf16 (nearest even) on the way into LDS.
// Fragment layout (16x16xK MFMA): lane l supplies A[l % 16][k-slice l / 16]
// and B[k-slice l / 16][l % 16]; accumulator v of lane l is C[4 (l / 16) + v][l % 16]
// for the float32 and bf16 instructions and C[l / 16 + 4 v][l % 16] for the
// float64 one (checked on gfx950 with a single-wave product).

#include "internal.h"

namespace pd {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int NT = 256;

template <typename Tc> struct Mfma;

template <> struct Mfma<double> {
  static constexpr int KI = 4;      // k per instruction
  static constexpr int KL = 1;      // k values per lane
  using acc_t = d4;
  using frag_t = double;
  static __device__ __forceinline__ acc_t run(frag_t a, frag_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <> struct Mfma<float> {
  static constexpr int KI = 4;
  static constexpr int KL = 1;
  using acc_t = f4;
  using frag_t = float;
  static __device__ __forceinline__ acc_t run(frag_t a, frag_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};
template <> struct Mfma<__bf16> {
  static constexpr int KI = 32;
  static constexpr int KL = 8;
  using acc_t = f4;
  using frag_t = bf8;
  static __device__ __forceinline__ acc_t run(frag_t a, frag_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};

template <typename Tc> __device__ __forceinline__ Tc to_c(float v);
template <> __device__ __forceinline__ double to_c<double>(float v) { return v; }
template <> __device__ __forceinline__ float to_c<float>(float v) { return v; }
template <> __device__ __forceinline__ __bf16 to_c<__bf16>(float v) { return (__bf16)v; }

template <typename Ts, typename Tc> __device__ __forceinline__ Tc conv(Ts v) { return (Tc)v; }
template <> __device__ __forceinline__ __bf16 conv<float, __bf16>(float v) { return (__bf16)v; }

template <typename Ts, typename Tc, int BM, int BN, int BK>
__global__ __launch_bounds__(NT) void k_gemm(const Ts* __restrict__ A, const Tc* __restrict__ Bt,
                                             Ts* __restrict__ C, int64_t M, int N, int K,
                                             int ntn) {
  using MF = Mfma<Tc>;
  constexpr int PAD = (sizeof(Tc) == 2) ? 8 : (sizeof(Tc) == 4 ? 4 : 2);
  constexpr int LDK = BK + PAD;
  constexpr int WM = BM / 2, WN = BN / 2;       // wave tile
  constexpr int FM = WM / 16, FN = WN / 16;     // MFMA blocks per wave
  __shared__ __align__(16) Tc As[BM * LDK];
  __shared__ __align__(16) Tc Bs[BN * LDK];

  const int bid = blockIdx.x;
  const int tn = bid % ntn;
  const int64_t tm = bid / ntn;
  const int64_t m0 = tm * BM;
  const int n0 = tn * BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;
  const int lr = lane & 15, lk = lane >> 4;

  typename MF::acc_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;

  for (int k0 = 0; k0 < K; k0 += BK) {
    // stage A (BM x BK) and Bt (BN x BK)
    for (int e = threadIdx.x; e < BM * BK; e += NT) {
      int r = e / BK, kk = e - r * BK;
      int64_t gm = m0 + r;
      int gk = k0 + kk;
      Ts v = 0;
      if (gm < M && gk < K) v = A[gm * K + gk];
      As[r * LDK + kk] = conv<Ts, Tc>(v);
    }
    for (int e = threadIdx.x; e < BN * BK; e += NT) {
      int r = e / BK, kk = e - r * BK;
      int gn = n0 + r, gk = k0 + kk;
      Tc v = (gn < N && gk < K) ? Bt[(int64_t)gn * K + gk] : to_c<Tc>(0.0f);
      Bs[r * LDK + kk] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += MF::KI) {
      typename MF::frag_t af[FM], bf[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const Tc* src = &As[(wm0 + i * 16 + lr) * LDK + ks + lk * MF::KL];
        if constexpr (MF::KL == 1) af[i] = src[0];
        else {
#pragma unroll
          for (int q = 0; q < MF::KL; ++q) af[i][q] = src[q];
        }
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const Tc* src = &Bs[(wn0 + j * 16 + lr) * LDK + ks + lk * MF::KL];
        if constexpr (MF::KL == 1) bf[j] = src[0];
        else {
#pragma unroll
          for (int q = 0; q < MF::KL; ++q) bf[j][q] = src[q];
        }
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = MF::run(af[i], bf[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int64_t gm = m0 + wm0 + i * 16 + MF::row(lk, v);
        int gn = n0 + wn0 + j * 16 + lr;
        if (gm < M && gn < N) C[gm * N + gn] = (Ts)acc[i][j][v];
      }
}

template <typename Ts, typename Tc, int BM, int BN, int BK>
void launch_gemm(const Ts* A, const Tc* Bt, Ts* C, int64_t M, int N, int K, hipStream_t s) {
  int ntn = (N + BN - 1) / BN;
  int64_t ntm = (M + BM - 1) / BM;
  int64_t blocks = ntm * ntn;
  k_gemm<Ts, Tc, BM, BN, BK><<<dim3((unsigned)blocks), NT, 0, s>>>(A, Bt, C, M, N, K, ntn);
}

}  // namespace

void xform(const Plan& pl, const SpaceOp& op, bool forward, const void* in, void* out,
           hipStream_t s) {
  const Geom& g = pl.g;
  const void* Bt = forward ? op.g_fwd : op.g_inv;
  int64_t rows = (int64_t)g.B * g.F * g.sy;   // complex rows of length sx
  int64_t M;
  int N, K;
  if (pl.schur) {
    M = rows;
    N = K = 2 * g.sx;
  } else {
    M = 2 * rows;
    N = K = g.sx;
  }
  switch (pl.prec) {
    case Prec::F64:
      launch_gemm<double, double, 64, 64, 16>((const double*)in, (const double*)Bt, (double*)out, M, N, K, s);
      break;
    case Prec::F32:
      launch_gemm<float, float, 64, 64, 16>((const float*)in, (const float*)Bt, (float*)out, M, N, K, s);
      break;
    case Prec::BF16:
      launch_gemm<float, __bf16, 128, 128, 32>((const float*)in, (const __bf16*)Bt, (float*)out, M, N, K, s);
      break;
  }
}

}  // namespace pd
