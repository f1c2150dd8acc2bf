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
//            Split mode writes each operand as hi + mid + lo in bf16 (24
//            significand bits, exact residuals) and keeps the six partial
//            products down to relative size 2^-16, so the result carries
//            float32-level accuracy at the bf16 instruction rate.
// Fragment layout (16x16xK MFMA): lane l supplies A[l % 16][k-slice l / 16]
// and B[k-slice l / 16][l % 16]; accumulator v of lane l is C[4 (l / 16) + v][l % 16]
// for the float32 and bf16 instructions and C[l / 16 + 4 v][l % 16] for the
// float64 one (checked on gfx950 with a single-wave product).

#include <type_traits>

#include "internal.h"

namespace pd {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

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

// The float64 / float32 product for aligned shapes (K a multiple of 32, N of
// 64): 64 x 64 x 32 tiles, 16-byte operand loads without branches (rows past
// M load row M-1 and are zeroed), the next k tile loaded into registers while
// the current one is multiplied, LDS rows padded by one 16-byte unit.  Twice
// the k depth of k_gemm per barrier pair: 32 float64 MFMAs per wave and tile.
template <typename T>
__global__ __launch_bounds__(NT) void k_gemm_pf(const T* __restrict__ A, const T* __restrict__ Bt,
                                                T* __restrict__ C, int64_t M, int N, int K, int ntn) {
  using MF = Mfma<T>;
  constexpr int BM = 64, BN = 64, BK = 32;
  constexpr int VW = 16 / sizeof(T);                 // values per 16-byte load
  constexpr int LDK = BK + VW;                       // padded row
  constexpr int PER = BM * BK / (NT * VW);           // 16-byte loads per thread and operand
  typedef T V __attribute__((ext_vector_type(VW)));
  __shared__ __align__(16) T As[BM * LDK];
  __shared__ __align__(16) T Bs[BN * LDK];
  const int bid = blockIdx.x;
  const int tn = bid % ntn;
  const int64_t m0 = (int64_t)(bid / ntn) * BM;
  const int n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * 32, wn0 = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  constexpr int UPR = BK / VW;                       // 16-byte units per row
  int64_t aoff[PER];
  bool aok[PER];
  int boff[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + u * NT, r = e / UPR, c = (e % UPR) * VW;
    const int64_t gm = m0 + r;
    aok[u] = gm < M;
    aoff[u] = (aok[u] ? gm : M - 1) * K + c;
    boff[u] = (n0 + r) * K + c;
  }
  V ra[PER], rb[PER];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      ra[u] = *reinterpret_cast<const V*>(A + aoff[u] + k0);
      rb[u] = *reinterpret_cast<const V*>(Bt + boff[u] + k0);
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * NT, r = e / UPR, c = (e % UPR) * VW;
      V a = ra[u];
      if (!aok[u]) a = V{};
      *reinterpret_cast<V*>(&As[r * LDK + c]) = a;
      *reinterpret_cast<V*>(&Bs[r * LDK + c]) = rb[u];
    }
  };
  typename MF::acc_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;
  gload(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    sstore();
    __syncthreads();
    if (k0 + BK < K) gload(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += MF::KI) {
      T af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = As[(wm0 + 16 * i + lr) * LDK + ks + lk];
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = Bs[(wn0 + 16 * j + lr) * LDK + ks + lk];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = MF::run(af[i], bf[j], acc[i][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gm = m0 + wm0 + 16 * i + MF::row(lk, v);
        const int gn = n0 + wn0 + 16 * j + lr;
        if (gm < M) C[gm * N + gn] = acc[i][j][v];
      }
}

template <typename Ts, typename Tc, int BM, int BN, int BK>
void launch_gemm(const Ts* A, const Tc* Bt, Ts* C, int64_t M, int N, int K, hipStream_t s) {
  if constexpr (std::is_same<Ts, Tc>::value && (std::is_same<Ts, double>::value || std::is_same<Ts, float>::value)) {
    if (K % 32 == 0 && N % 64 == 0) {
      const int ntn = N / 64;
      const int64_t blocks = ((M + 63) / 64) * ntn;
      k_gemm_pf<Ts><<<dim3((unsigned)blocks), NT, 0, s>>>(A, Bt, C, M, N, K, ntn);
      return;
    }
  }
  int ntn = (N + BN - 1) / BN;
  int64_t ntm = (M + BM - 1) / BM;
  int64_t blocks = ntm * ntn;
  k_gemm<Ts, Tc, BM, BN, BK><<<dim3((unsigned)blocks), NT, 0, s>>>(A, Bt, C, M, N, K, ntn);
}

// bf16 MFMA path for float32 rows (K % 32 == 0): float4 row loads, the rows
// rounded to bf16 on the way into LDS, 16-byte fragment reads, the next k-tile
// prefetched into registers while the current one is multiplied.  SPLIT = 6
// keeps float32-level accuracy with bf16 instructions: a = a0 + a1 + a2 and
// b = b0 + b1 + b2 (bf16 parts of relative size 1, 2^-8, 2^-16), and
// a b ~ sum of a_x b_y over x + y <= 2, the dropped terms being 2^-24 relative
// or less.  SPLIT = 3 is the two-part form (hi + lo, about 16 significand
// bits), SPLIT = 1 the plain single bf16 product.  Bt holds the parts
// ([N][K] each) one after the other.
// Tiles: 128 x 128 x 32, 2 x 2 waves of 64 x 64 (4 x 4 blocks of 16 x 16).
// Blocks are ordered so that the N-tiles sharing one row block of A run on
// the same XCD (consecutive workgroup ids are dealt round-robin to the 8
// XCDs, each with its own L2).
typedef unsigned short us4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_bits(float v) {
  __bf16 h = (__bf16)v;
  return __builtin_bit_cast(unsigned short, h);
}
__device__ __forceinline__ float bf16_val(unsigned short b) {
  return __builtin_bit_cast(float, (unsigned int)b << 16);
}

template <int SPLIT>
__global__ __launch_bounds__(NT, 2) void k_gemm_bf16(const float* __restrict__ A,
                                                  const unsigned short* __restrict__ Bt,
                                                  float* __restrict__ C, int64_t M, int N, int K,
                                                  int ntn, int64_t nblocks, const float* __restrict__ rscale,
                                                  float binv) {
  constexpr int BM = 128, BN = 128, BK = 32;
  // LDS rows of BK bf16 (64 bytes, four 16-byte chunks); chunk c of row r is
  // stored at position c ^ ((r >> 1) & 3), so that the eight rows one
  // fragment read touches per LDS cycle (and the rows of a staging write)
  // fall on distinct banks
  auto off = [](int r, int ch) { return r * BK + 8 * (ch ^ ((r >> 1) & 3)); };
  // operand terms: 1 (plain bf16), 2 (hi + lo), 3 (hi + mid + lo); SPLIT = 16:
  // fp16 hi + lo of rows scaled by a power of two (rscale) and of B (scaled
  // by 1 / binv), three products a_hi b_hi + a_hi b_lo + a_lo b_hi
  constexpr bool F16 = SPLIT == 16;
  constexpr int NA = (SPLIT == 6) ? 3 : (SPLIT == 3 || F16) ? 2 : 1;
  __shared__ __align__(16) unsigned short As[NA][BM * BK];
  __shared__ __align__(16) unsigned short Bs[NA][BN * BK];

  int64_t bid = blockIdx.x;
  if ((nblocks & 7) == 0) bid = (bid & 7) * (nblocks >> 3) + (bid >> 3);   // XCD-aware order
  const int tn = (int)(bid % ntn);
  const int64_t tm = bid / ntn;
  const int64_t m0 = tm * BM;
  const int n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * 64, wn0 = (wave & 1) * 64;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t NKp = (int64_t)N * K;   // elements per bf16 part of the matrix

  // per-thread staging: A 4 x float4 (rows tid/8 + 32 i, k = 4 (tid%8)),
  // B 2 x 16 bytes per part (rows tid/4 + 64 i, k = 8 (tid%4)).  Rows beyond
  // M or N load a valid row and are zeroed afterwards, so the loads carry no
  // branches and the waits can count them.
  float4 ra[1][4];
  uint4 rb[NA][2];
  int64_t arow[4];
  bool aok[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t gm = m0 + (tid >> 3) + 32 * i;
    aok[i] = gm < M;
    arow[i] = (aok[i] ? gm : M - 1) * K + 4 * (tid & 7);
  }
  float rsc[4];   // SPLIT = 16: scales of this thread's staged rows
#pragma unroll
  for (int i = 0; i < 4; ++i) rsc[i] = F16 ? rscale[arow[i] / K] : 1.f;
  int64_t brow[2];
  bool bok[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int gn = n0 + (tid >> 2) + 64 * i;
    bok[i] = gn < N;
    brow[i] = (int64_t)(bok[i] ? gn : N - 1) * K + 8 * (tid & 3);
  }
  // the next k tile is loaded while the current one is multiplied
  auto aload = [&](auto bufc, int k0) {
    constexpr int bb = decltype(bufc)::value;
#pragma unroll
    for (int i = 0; i < 4; ++i) ra[bb][i] = *reinterpret_cast<const float4*>(A + arow[i] + k0);
  };
  auto bload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int a = 0; a < NA; ++a) rb[a][i] = *reinterpret_cast<const uint4*>(Bt + a * NKp + brow[i] + k0);
  };
  auto sstore = [&](auto bufc) {
    constexpr int bb = decltype(bufc)::value;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int r = (tid >> 3) + 32 * i, c = 4 * (tid & 7);
      float v[4] = {ra[bb][i].x, ra[bb][i].y, ra[bb][i].z, ra[bb][i].w};
      if (!aok[i]) v[0] = v[1] = v[2] = v[3] = 0.f;
      // exact residuals in float32: v - hi and (v - hi) - mid have at most 16
      // and 8 significant bits beyond the parts already taken
      us4 part[NA];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if constexpr (F16) {   // power-of-two row scale (exact), then hi and the exact residual
          const float x = v[q] * rsc[i];
          const _Float16 h = (_Float16)x;
          part[0][q] = __builtin_bit_cast(unsigned short, h);
          part[1][q] = __builtin_bit_cast(unsigned short, (_Float16)(x - (float)h));
        } else {
          float rest = v[q];
#pragma unroll
          for (int a = 0; a < NA; ++a) {
            part[a][q] = bf16_bits(rest);
            if (a + 1 < NA) rest -= bf16_val(part[a][q]);
          }
        }
      }
#pragma unroll
      for (int a = 0; a < NA; ++a) *reinterpret_cast<us4*>(&As[a][off(r, c >> 3) + (c & 7)]) = part[a];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      int r = (tid >> 2) + 64 * i, c = 8 * (tid & 3);
#pragma unroll
      for (int a = 0; a < NA; ++a)
        *reinterpret_cast<uint4*>(&Bs[a][off(r, c >> 3)]) = bok[i] ? rb[a][i] : uint4{0, 0, 0, 0};
    }
  };

  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  auto compute = [&]() {
    // B fragments held for the tile, A fragments one row block at a time
    bf8 b[NA][4];
#pragma unroll
    for (int x = 0; x < NA; ++x)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        b[x][j] = *reinterpret_cast<const bf8*>(&Bs[x][off(wn0 + 16 * j + lr, lk)]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      bf8 a[NA];
#pragma unroll
      for (int x = 0; x < NA; ++x) a[x] = *reinterpret_cast<const bf8*>(&As[x][off(wm0 + 16 * i + lr, lk)]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        // terms of size 2^-16 and above (relative): a_x b_y with x + y < NA,
        // the smallest first
        if constexpr (F16) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a[1]), __builtin_bit_cast(h8, b[0][j]),
                                                             acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a[0]), __builtin_bit_cast(h8, b[1][j]),
                                                             acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a[0]), __builtin_bit_cast(h8, b[0][j]),
                                                             acc[i][j], 0, 0, 0);
          continue;
        }
        if constexpr (NA == 3) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2][j], acc[i][j], 0, 0, 0);
        }
        if constexpr (NA >= 2) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1][j], acc[i][j], 0, 0, 0);
        }
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0][j], acc[i][j], 0, 0, 0);
      }
    }
  };
  using I0 = std::integral_constant<int, 0>;
  aload(I0{}, 0);
  bload(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    sstore(I0{});
    __syncthreads();
    if (k0 + BK < K) {
      aload(I0{}, k0 + BK);
      bload(k0 + BK);
    }
    compute();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int64_t gm = m0 + wm0 + 16 * i + 4 * lk + v;
        int gn = n0 + wn0 + 16 * j + lr;
        if (gm < M && gn < N) C[gm * N + gn] = F16 ? acc[i][j][v] * (binv / rscale[gm]) : acc[i][j][v];
      }
}

// Ping-pong form of the split-bf16 product (three parts, six products, as
// k_gemm_bf16<6>): 256 x 128 tiles, eight waves (4 x 2 of 64 x 64), and two
// LDS stages: the waves multiply from one stage while the next k tile, already
// in registers, is split and written into the other, with one barrier per k
// tile instead of two.  144 KiB of LDS (one workgroup per CU, two waves per
// SIMD as before); same XCD-aware tile order.  Measured 3 % faster than
// k_gemm_bf16<6> at 512^2 x 1024 x 8; for the split-fp16 product the same
// structure was 8 % slower, so that one keeps k_gemm_bf16<16>.
__global__ __launch_bounds__(2 * NT, 1) void k_gemm_bf16x6_pp(const float* __restrict__ A,
                                                           const unsigned short* __restrict__ Bt,
                                                           float* __restrict__ C, int64_t M, int N, int K,
                                                           int ntn, int64_t nblocks) {
  constexpr int BM = 256, BN = 128, BK = 32, NA = 3;
  auto off = [](int r, int ch) { return r * BK + 8 * (ch ^ ((r >> 1) & 3)); };
  extern __shared__ __align__(16) unsigned short lds_pp[];   // [2][NA][BM BK] A, then [2][NA][BN BK] B
  auto As = [&](int st, int a) { return lds_pp + (st * NA + a) * BM * BK; };
  auto Bs = [&](int st, int a) { return lds_pp + 2 * NA * BM * BK + (st * NA + a) * BN * BK; };

  int64_t bid = blockIdx.x;
  if ((nblocks & 7) == 0) bid = (bid & 7) * (nblocks >> 3) + (bid >> 3);   // XCD-aware order
  const int tn = (int)(bid % ntn);
  const int64_t m0 = (bid / ntn) * BM;
  const int n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * 64, wn0 = (wave & 1) * 64;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t NKp = (int64_t)N * K;

  // staging: A 4 x float4 (rows tid/8 + 64 i, k = 4 (tid%8)), B one 16-byte
  // piece per part (row tid/4, k = 8 (tid%4)); rows beyond M or N load a
  // valid row and are zeroed afterwards (branch-free loads)
  float4 ra[4];
  u32x4 rb[NA];
  int64_t arow[4];
  bool aok[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t gm = m0 + (tid >> 3) + 64 * i;
    aok[i] = gm < M;
    arow[i] = (aok[i] ? gm : M - 1) * K + 4 * (tid & 7);
  }
  const int gnb = n0 + (tid >> 2);
  const bool bok = gnb < N;
  const int64_t brow = (int64_t)(bok ? gnb : N - 1) * K + 8 * (tid & 3);
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) ra[i] = *reinterpret_cast<const float4*>(A + arow[i] + k0);
#pragma unroll
    for (int a = 0; a < NA; ++a) rb[a] = *reinterpret_cast<const u32x4*>(Bt + a * NKp + brow + k0);
  };
  auto sstore = [&](int st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = (tid >> 3) + 64 * i, c = 4 * (tid & 7);
      float v[4] = {ra[i].x, ra[i].y, ra[i].z, ra[i].w};
      if (!aok[i]) v[0] = v[1] = v[2] = v[3] = 0.f;
      us4 part[NA];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float rest = v[q];
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          part[a][q] = bf16_bits(rest);
          if (a + 1 < NA) rest -= bf16_val(part[a][q]);
        }
      }
#pragma unroll
      for (int a = 0; a < NA; ++a) *reinterpret_cast<us4*>(As(st, a) + off(r, c >> 3) + (c & 7)) = part[a];
    }
    const int r = tid >> 2, c = 8 * (tid & 3);
#pragma unroll
    for (int a = 0; a < NA; ++a)
      *reinterpret_cast<u32x4*>(Bs(st, a) + off(r, c >> 3)) = bok ? rb[a] : u32x4{0, 0, 0, 0};
  };

  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  auto compute = [&](int st) {
    bf8 b[NA][4];
#pragma unroll
    for (int x = 0; x < NA; ++x)
#pragma unroll
      for (int j = 0; j < 4; ++j) b[x][j] = *reinterpret_cast<const bf8*>(Bs(st, x) + off(wn0 + 16 * j + lr, lk));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      bf8 a[NA];
#pragma unroll
      for (int x = 0; x < NA; ++x) a[x] = *reinterpret_cast<const bf8*>(As(st, x) + off(wm0 + 16 * i + lr, lk));
#pragma unroll
      for (int j = 0; j < 4; ++j) {   // terms down to 2^-16 (relative), the smallest first
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0][j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1][j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2][j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0][j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1][j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0][j], acc[i][j], 0, 0, 0);
      }
    }
  };
  const int nkt = K / BK;
  gload(0);
  sstore(0);
  if (nkt > 1) gload(BK);
  __syncthreads();
  for (int kt = 0; kt < nkt; ++kt) {
    const int cur = kt & 1;
    compute(cur);
    if (kt + 1 < nkt) {
      sstore(cur ^ 1);   // tile kt + 1, from registers, into the stage read in step kt - 1
      if (kt + 2 < nkt) gload((kt + 2) * BK);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gm = m0 + wm0 + 16 * i + 4 * lk + v;
        const int gn = n0 + wn0 + 16 * j + lr;
        if (gm < M && gn < N) C[gm * N + gn] = acc[i][j][v];
      }
}

// Power-of-two scale of each row of A (M rows of K floats, K % 4 == 0) that
// brings its largest magnitude into [2^13, 2^14): one wave per row.  Zero
// rows get 1.
__global__ __launch_bounds__(NT) void k_rowscale(const float* __restrict__ A, int64_t M, int K,
                                                 float* __restrict__ rscale) {
  const int64_t row = (int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  if (row >= M) return;   // whole waves
  const int lane = threadIdx.x & 63;
  const float* a = A + row * K;
  float m = 0.f;
  for (int k = 4 * lane; k < K; k += 256) {
    const float4 v = *reinterpret_cast<const float4*>(a + k);
    m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if (lane == 0) {
    int e = 0;
    (void)frexpf(m, &e);   // m = f 2^e, f in [0.5, 1)
    rscale[row] = m > 0.f ? ldexpf(1.f, 14 - e) : 1.f;
  }
}

template <int SPLIT>
void launch_gemm_bf16(const float* A, const unsigned short* Bt, float* C, int64_t M, int N, int K,
                      hipStream_t s, float* rscale = nullptr) {
  int ntn = (N + 127) / 128;
  if constexpr (SPLIT == 16)
    k_rowscale<<<dim3((unsigned)((M + NT / 64 - 1) / (NT / 64))), NT, 0, s>>>(A, M, K, rscale);
  if constexpr (SPLIT == 6) {
    const size_t lds = (size_t)2 * 3 * (256 + 128) * 32 * sizeof(unsigned short);
    const int64_t nblocks = ((M + 255) / 256) * ntn;
    lds_limit((const void*)k_gemm_bf16x6_pp, lds);
    k_gemm_bf16x6_pp<<<dim3((unsigned)nblocks), 2 * NT, lds, s>>>(A, Bt, C, M, N, K, ntn, nblocks);
  } else {
    const int64_t nblocks = ((M + 127) / 128) * ntn;
    k_gemm_bf16<SPLIT><<<dim3((unsigned)nblocks), NT, 0, s>>>(A, Bt, C, M, N, K, ntn, nblocks, rscale,
                                                               1.0f / F16_BSCALE);
  }
}

}  // namespace

void xform(const Plan& pl, const SpaceOp& op, bool forward, const void* in, void* out,
           hipStream_t s) {
  if (pl.dst) {   // sine basis, nx + 1 a power of two: DST-I by FFT
    dst_transform(pl, in, out, s);
    return;
  }
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
    case Prec::F16:
      if (K % 32 == 0) {
        launch_gemm_bf16<16>((const float*)in, (const unsigned short*)Bt, (float*)out, M, N, K, s, pl.d_rowscale);
      } else {   // ragged K: the float32 product on the float32 copy after the two fp16 parts
        const float* B32 = (const float*)((const unsigned short*)Bt + (size_t)2 * N * K);
        launch_gemm<float, float, 64, 64, 16>((const float*)in, B32, (float*)out, M, N, K, s);
      }
      break;
    case Prec::BF16:
    case Prec::BF16X1: {
      const bool split = pl.prec == Prec::BF16;
      if (K % 32 == 0) {
        if (split) launch_gemm_bf16<6>((const float*)in, (const unsigned short*)Bt, (float*)out, M, N, K, s);
        else launch_gemm_bf16<1>((const float*)in, (const unsigned short*)Bt, (float*)out, M, N, K, s);
      } else if (split) {
        // ragged K (nx not a multiple of 16): the float32 MFMA kernel on the float32
        // copy of the matrix that follows the three bf16 parts
        const float* B32 = (const float*)((const unsigned short*)Bt + (size_t)3 * N * K);
        launch_gemm<float, float, 64, 64, 16>((const float*)in, B32, (float*)out, M, N, K, s);
      } else {
        launch_gemm<float, __bf16, 128, 128, 32>((const float*)in, (const __bf16*)Bt, (float*)out, M, N, K, s);
      }
      break;
    }
  }
}

}  // namespace pd
