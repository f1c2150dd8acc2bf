// Step-(b) with a non-normal x factor: back-substitution over the x-modes of
// the Schur basis (Bartels-Stewart), one workgroup per (right-hand side,
// frequency) slice.
//
// For the slice of frequency n the modes are solved from the last to the first:
//
//   [(lambda1 + lambda2 T_kk) I + lambda2 K_y] w_k = r_k - lambda2 sum_{j>k} T_kj w_j,
//
// in blocks of NB consecutive modes (left-looking):
//   1. coupling of the block to every solved mode j >= end of block, as one
//      product over all ny rows of the slice on MFMA:
//        C[y][q] = sum_j W[y][j] T[k0+q][j]   (complex; real block form
//        [Wr | Wi] x [[Tr^T, Ti^T], [-Ti^T, Tr^T]]),
//      with W read row-wise from HBM through LDS and T from the table;
//   2. r_q -= lambda2 C[:, q] in the LDS tile of the block;
//   3. one wave solves the NB tridiagonal lines of the block in order,
//      each followed by the rank-1 update of the remaining block columns;
//   4. the block is written back and becomes part of W for later blocks.
//
// Occupancy: the register budget is capped at two waves per SIMD (two
// workgroups per CU; the LDS footprint stays under 80 KiB) so that all
// Nt/2 + 1 slices of a 256-CU launch are resident at once and one
// workgroup's sequential phase overlaps the other's products.  Chunks are
// staged global -> LDS in batches of 8 loads per thread rather than
// prefetched whole into registers.

#include "tri_device.h"

namespace pd {
namespace {

using namespace tri;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct SweepMfma;
template <> struct SweepMfma<float> {
  using acc_t = f4;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};
template <> struct SweepMfma<double> {
  using acc_t = d4;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};

// NB: modes per block; BK: k-chunk of the coupling product; RB: 16-row MFMA
// blocks per wave (the four waves cover 64 RB rows >= ny).
template <typename T, int R, int P, int NB, int BK, int RB>
__global__ __launch_bounds__(NT, 2) void k_schur_sweep(T* __restrict__ spec, const double2* __restrict__ lam,
                                                    const double2* __restrict__ tk,
                                                    const T* __restrict__ tup, double lo, double di,
                                                    double up, int F, int sx, int sy, int ldy) {
  static_assert(2 * NB <= BK + 1, "the product staging area also holds C");
  static_assert((2 * NB) % 16 == 0, "MFMA column blocks");
  static_assert((BK & (BK - 1)) == 0, "BK is a power of two");
  using MF = SweepMfma<T>;
  constexpr int NCB = 2 * NB / 16;       // MFMA column blocks (real and imaginary parts)
  constexpr int NYP = 64 * RB;           // rows covered by the MFMA tiles
  constexpr int LDA = BK + 1;
  extern __shared__ __align__(16) unsigned char smraw[];
  T* sre = reinterpret_cast<T*>(smraw);
  T* sim = sre + NB * ldy;
  T* As = sim + NB * ldy;                // [NYP][LDA]; after the K loop: C[NYP][LDA]
  T* Bs = As + NYP * LDA;                // [2 NB][LDA]
  T* Tb = Bs + 2 * NB * LDA;             // block of T: [2][NB][NB] (re, im)
  T* Sb = Tb + 2 * NB * NB;              // per-mode diagonal coefficient b_q: [2][NB]

  const int n = blockIdx.x, b = blockIdx.y;
  T* slice = spec + ((int64_t)b * F + n) * sy * 2 * sx;
  const T* tre = tup;
  const T* tim = tup + (int64_t)sx * sx;
  const double2 l1 = lam[n], l2 = lam[F + n];
  const T l2r = (T)l2.x, l2i = (T)l2.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int p = lane % P, seg = lane / P;
  const int nblk = (sx + NB - 1) / NB;

  for (int kb = nblk - 1; kb >= 0; --kb) {
    const int k0 = kb * NB, nk = min(NB, sx - k0), kend = k0 + nk;
    const int J = sx - kend, K2 = 2 * J;
    __syncthreads();
    tile_load(slice, sre, sim, k0, nk, NB, sx, sy, ldy, R);
    // T block and the line diagonals of the block's modes
    for (int e = tid; e < NB * NB; e += NT) {
      int qq = e / NB, q = e - qq * NB;
      bool ok = qq < nk && q < nk;
      Tb[e] = ok ? tre[(int64_t)(k0 + qq) * sx + k0 + q] : (T)0;
      Tb[NB * NB + e] = ok ? tim[(int64_t)(k0 + qq) * sx + k0 + q] : (T)0;
    }
    if (tid < NB) {
      double2 t = (tid < nk) ? tk[k0 + tid] : double2{0.0, 0.0};
      double shr = t.x + di, shi = t.y;
      Sb[tid] = (T)(l1.x + l2.x * shr - l2.y * shi);
      Sb[NB + tid] = (T)(l1.y + l2.x * shi + l2.y * shr);
    }
    if (J > 0) {
      typename MF::acc_t acc[RB][NCB];
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < NCB; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;
      auto stage = [&](int kc) {
        // A chunk (W rows) and B chunk (real block form of T^T), batched global -> LDS
        for (int base = 0; base < NYP * BK; base += 8 * NT) {
          T v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            int e = base + u * NT + tid;
            int r = e / BK, kap = kc + (e & (BK - 1));
            T x = 0;
            if (e < NYP * BK && r < sy && kap < K2) {
              int sg = kap >= J;
              x = slice[(int64_t)r * 2 * sx + sg * sx + kend + kap - sg * J];
            }
            v[u] = x;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            int e = base + u * NT + tid;
            if (e < NYP * BK) As[(e / BK) * LDA + (e & (BK - 1))] = v[u];
          }
        }
        for (int e = tid; e < 2 * NB * BK; e += NT) {
          int nn = e / BK, kap = kc + (e & (BK - 1));
          int q = nn % NB, part = nn / NB;
          T x = 0;
          if (q < nk && kap < K2) {
            int sg = kap >= J;
            int j = kend + kap - sg * J;
            T tr = tre[(int64_t)(k0 + q) * sx + j], ti = tim[(int64_t)(k0 + q) * sx + j];
            x = sg == 0 ? (part == 0 ? tr : ti) : (part == 0 ? -ti : tr);
          }
          Bs[nn * LDA + (e & (BK - 1))] = x;
        }
      };
      for (int kc = 0; kc < K2; kc += BK) {
        stage(kc);
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
          T af[RB], bf[NCB];
#pragma unroll
          for (int i = 0; i < RB; ++i) af[i] = As[(wave * RB * 16 + i * 16 + lr) * LDA + ks + lk];
#pragma unroll
          for (int j = 0; j < NCB; ++j) bf[j] = Bs[(j * 16 + lr) * LDA + ks + lk];
#pragma unroll
          for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int j = 0; j < NCB; ++j) acc[i][j] = MF::run(af[i], bf[j], acc[i][j]);
        }
        __syncthreads();
      }
      // C -> LDS (reusing the A staging area), then r -= lambda2 C in the tile
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < NCB; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            As[(wave * RB * 16 + i * 16 + MF::row(lk, v)) * LDA + j * 16 + lr] = acc[i][j][v];
      __syncthreads();
      for (int e = tid; e < sy * nk; e += NT) {
        int y = e / nk, q = e - y * nk;
        T cr = As[y * LDA + q], ci = As[y * LDA + NB + q];
        int idx = lidx(q, y, ldy, R);
        sre[idx] -= l2r * cr - l2i * ci;
        sim[idx] -= l2r * ci + l2i * cr;
      }
    }
    __syncthreads();
    if (wave == 0) {
      const bool active = (seg == 0);
      const Cx<T> ca = active ? Cx<T>{(T)(l2.x * lo), (T)(l2.y * lo)} : cz<T>();
      const Cx<T> cc = active ? Cx<T>{(T)(l2.x * up), (T)(l2.y * up)} : cz<T>();
      for (int q = nk - 1; q >= 0; --q) {
        Cx<T> cb = active ? Cx<T>{Sb[q], Sb[NB + q]} : c1<T>();
        Cx<T> d[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
          int idx = q * ldy + p * (R + 1) + i;
          d[i] = active ? Cx<T>{sre[idx], sim[idx]} : cz<T>();
        }
        tri_wave<T, R, P>(d, ca, cb, cc, sy, p);
        if (active) {
#pragma unroll
          for (int i = 0; i < R; ++i) {
            int idx = q * ldy + p * (R + 1) + i;
            sre[idx] = d[i].x;
            sim[idx] = d[i].y;
          }
          // columns q' < q of the block: r_q' -= lambda2 T[k0+q'][k0+q] w_q
          for (int qq = 0; qq < q; ++qq) {
            T tr = Tb[qq * NB + q], ti = Tb[NB * NB + qq * NB + q];
            T cr = l2r * tr - l2i * ti, ci = l2r * ti + l2i * tr;
#pragma unroll
            for (int i = 0; i < R; ++i) {
              int idx = qq * ldy + p * (R + 1) + i;
              sre[idx] -= cr * d[i].x - ci * d[i].y;
              sim[idx] -= cr * d[i].y + ci * d[i].x;
            }
          }
        }
      }
    }
    __syncthreads();
    tile_store(slice, sre, sim, k0, nk, NB, sx, sy, ldy, R);
    __threadfence_block();
  }
}

struct SweepShape { int R, P, RB, ldy; size_t lds; };

template <typename T, int NB, int BK>
SweepShape sweep_shape(const Plan& pl) {
  const Geom& g = pl.g;
  int R = 4;
  while (R * 64 < g.sy) R <<= 1;
  int P = 1;
  while (P * R < g.sy) P <<= 1;
  int ldy = P * (R + 1);
  if ((ldy & 1) == 0) ldy += 1;
  int RB = 1;
  while (64 * RB < g.sy) RB <<= 1;
  size_t lds = sizeof(T) * ((size_t)2 * NB * ldy + (size_t)64 * RB * (BK + 1) + (size_t)2 * NB * (BK + 1) +
                            (size_t)2 * NB * NB + (size_t)2 * NB);
  return SweepShape{R, P, RB, ldy, lds};
}

template <typename T, int R, int P, int NB, int BK, int RB>
void launch_one(const Plan& pl, const SpaceOp& op, T* spec, hipStream_t s) {
  const Geom& g = pl.g;
  SweepShape sh = sweep_shape<T, NB, BK>(pl);
  auto kfn = k_schur_sweep<T, R, P, NB, BK, RB>;
  hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds);
  kfn<<<dim3(g.F, g.B), NT, sh.lds, s>>>(spec, pl.d_lam, op.tk, (const T*)op.tup, op.lo, op.di,
                                         op.up, g.F, g.sx, g.sy, sh.ldy);
}

// (NB, BK) per precision and row count: wide blocks while the A staging fits
// in registers, narrower ones for 512 rows.
template <typename T> struct SweepCfg;
template <> struct SweepCfg<float> { static constexpr int NB = 16, BK = 32, NB8 = 8, BK8 = 16; };
template <> struct SweepCfg<double> { static constexpr int NB = 8, BK = 16, NB8 = 8, BK8 = 16; };

template <typename T>
void launch(const Plan& pl, const SpaceOp& op, T* spec, hipStream_t s) {
  using C = SweepCfg<T>;
  SweepShape sh = sweep_shape<T, C::NB, C::BK>(pl);
#define PD_SWEEP(RR, PP, BB)                                                              \
  if (sh.R == RR && sh.P == PP && sh.RB == BB) {                                          \
    launch_one<T, RR, PP, C::NB, C::BK, BB>(pl, op, spec, s);                             \
    return;                                                                               \
  }
  PD_SWEEP(4, 1, 1) PD_SWEEP(4, 2, 1) PD_SWEEP(4, 4, 1) PD_SWEEP(4, 8, 1) PD_SWEEP(4, 16, 1)
  PD_SWEEP(4, 32, 2) PD_SWEEP(4, 64, 4)
#undef PD_SWEEP
  if (sh.R == 8 && sh.P == 64 && sh.RB == 8) launch_one<T, 8, 64, C::NB8, C::BK8, 8>(pl, op, spec, s);
}

}  // namespace

size_t schur_sweep_lds(const Plan& pl) {
  if (pl.prec == Prec::F64) {
    SweepShape a = sweep_shape<double, 8, 16>(pl);
    return a.RB == 8 ? sweep_shape<double, SweepCfg<double>::NB8, SweepCfg<double>::BK8>(pl).lds : a.lds;
  }
  SweepShape a = sweep_shape<float, 16, 32>(pl);
  return a.RB == 8 ? sweep_shape<float, SweepCfg<float>::NB8, SweepCfg<float>::BK8>(pl).lds : a.lds;
}

void schur_sweep(const Plan& pl, const SpaceOp& op, void* spec, hipStream_t s) {
  if (pl.prec == Prec::F64) launch<double>(pl, op, (double*)spec, s);
  else launch<float>(pl, op, (float*)spec, s);
}

}  // namespace pd
