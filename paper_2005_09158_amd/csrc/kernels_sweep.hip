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

#include <type_traits>

#include "tri_device.h"

namespace pd {
namespace {

using namespace tri;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short us4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_bits(float v) {
  __bf16 h = (__bf16)v;
  return __builtin_bit_cast(unsigned short, h);
}
__device__ __forceinline__ float bf16_val(unsigned short b) {
  return __builtin_bit_cast(float, (unsigned int)b << 16);
}

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
template <typename T> struct V4;
template <> struct V4<float> { using t = float4; };
template <> struct V4<double> { using t = double4; };

// Load unit of the pipelined kernel's pivot staging: four values where the
// pivot blocks are 16-byte aligned (sx % 4 == 0), else two.
template <typename T, bool VEC> struct PivUnit {
  static constexpr int n = VEC ? 4 : 2;
  typedef T t __attribute__((ext_vector_type(VEC ? 4 : 2)));
};

// Coupling product with fragments loaded straight from global memory
// (sx % 4 == 0).  Within each block of 16 consecutive solved modes j, lane
// group g = lane/16 owns j0 + 4g .. j0 + 4g + 3 and feeds element s of its
// four-vector to MFMA step s: the k order inside the block is permuted, the
// same way for A (W rows) and B (T rows), which leaves the sum unchanged.
// Each wave covers its own RB x 16 rows; T rows are shared through the cache.
template <typename T> __device__ __forceinline__ typename V4<T>::t load4(const T* ptr, int j, int sx, bool vec) {
  using Q4 = typename V4<T>::t;
  if (vec) return *reinterpret_cast<const Q4*>(ptr + j);
  Q4 v{};
  v.x = ptr[j];
  if (j + 1 < sx) v.y = ptr[j + 1];
  if (j + 2 < sx) v.z = ptr[j + 2];
  if (j + 3 < sx) v.w = ptr[j + 3];
  return v;
}

template <typename T, int NB, int RB, bool VEC = true>
__device__ __forceinline__ void coupling_direct(const T* slice, const T* tre, const T* tim, int sx,
                                                int sy, int k0, int nk, int kend, int wave, int lr,
                                                int lk, typename SweepMfma<T>::acc_t (&acc)[RB][2 * NB / 16]) {
  using MF = SweepMfma<T>;
  using Q4 = typename V4<T>::t;
  constexpr int NCB = 2 * NB / 16;
  const int q = (NCB == 2) ? lr : (lr & 7);          // mode of this lane's output column
  const int part = (NCB == 2) ? 0 : (lr >> 3);       // NB = 8: lanes 8..15 hold imaginary parts
  const bool qok = q < nk;
  const T* trow = tre + (int64_t)(k0 + q) * sx;
  const T* irow = tim + (int64_t)(k0 + q) * sx;
  const int r0 = wave * RB * 16 + lr;
  for (int j0 = kend; j0 < sx; j0 += 16) {
    const int j = j0 + 4 * lk;
    const bool jok = j < sx;
    Q4 tr{}, ti{};
    if (qok && jok) {
      tr = load4(trow, j, sx, VEC);
      ti = load4(irow, j, sx, VEC);
    }
    Q4 ar[RB], ai[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int r = r0 + 16 * i;
      if (jok && r < sy) {
        const T* row = slice + (int64_t)r * 2 * sx;
        ar[i] = load4(row, j, sx, VEC);
        ai[i] = load4(row + sx, j, sx, VEC);
      } else {
        ar[i] = Q4{};
        ai[i] = Q4{};
      }
    }
    const T trv[4] = {tr.x, tr.y, tr.z, tr.w}, tiv[4] = {ti.x, ti.y, ti.z, ti.w};
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      // real block form: out_re += Wr Tr - Wi Ti ; out_im += Wr Ti + Wi Tr
      T b_re_r, b_re_i, b_im_r, b_im_i;   // B for (re input, im input) x (re out, im out)
      b_re_r = trv[st]; b_re_i = -tiv[st]; b_im_r = tiv[st]; b_im_i = trv[st];
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const T av_r = (st == 0) ? ar[i].x : (st == 1) ? ar[i].y : (st == 2) ? ar[i].z : ar[i].w;
        const T av_i = (st == 0) ? ai[i].x : (st == 1) ? ai[i].y : (st == 2) ? ai[i].z : ai[i].w;
        if constexpr (NCB == 2) {
          acc[i][0] = MF::run(av_r, b_re_r, acc[i][0]);
          acc[i][0] = MF::run(av_i, b_re_i, acc[i][0]);
          acc[i][1] = MF::run(av_r, b_im_r, acc[i][1]);
          acc[i][1] = MF::run(av_i, b_im_i, acc[i][1]);
        } else {
          acc[i][0] = MF::run(av_r, part ? b_im_r : b_re_r, acc[i][0]);
          acc[i][0] = MF::run(av_i, part ? b_im_i : b_re_i, acc[i][0]);
        }
      }
    }
  }
}

// Fragments of one 16-mode step of the coupling product: the T rows of this
// lane's output column for each of NTB blocks of output modes, and RB rows of
// solved lines (real, imaginary parts).
template <typename T, int RB, int NTB> struct CouplingFrag {
  typename V4<T>::t tr[NTB], ti[NTB], ar[RB], ai[RB];
};

// Loads modes j .. j+3 (those below je) of the fragment.
template <typename T, int RB, int NTB, bool VEC>
__device__ __forceinline__ void load_frag(CouplingFrag<T, RB, NTB>& f, const T* slice,
                                          const T* const (&trow)[NTB], const T* const (&irow)[NTB],
                                          const bool (&tok)[NTB], int sx, int sy, int j, int je, int r0) {
  using Q4 = typename V4<T>::t;
  const bool jok = j < je;
#pragma unroll
  for (int tb = 0; tb < NTB; ++tb) {
    f.tr[tb] = Q4{};
    f.ti[tb] = Q4{};
    if (tok[tb] && jok) {
      f.tr[tb] = load4(trow[tb], j, je, VEC);
      f.ti[tb] = load4(irow[tb], j, je, VEC);
    }
  }
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    const int r = r0 + 16 * i;
    if (jok && r < sy) {
      const T* row = slice + (int64_t)r * 2 * sx;
      f.ar[i] = load4(row, j, je, VEC);
      f.ai[i] = load4(row + sx, j, je, VEC);
    } else {
      f.ar[i] = Q4{};
      f.ai[i] = Q4{};
    }
  }
}

template <typename T, int NB, int RB, int NTB>
__device__ __forceinline__ void mma_frag(const CouplingFrag<T, RB, NTB>& f, int part,
                                         typename SweepMfma<T>::acc_t (&acc)[NTB][RB][2 * NB / 16]) {
  using MF = SweepMfma<T>;
  constexpr int NCB = 2 * NB / 16;
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    T b_re_r[NTB], b_re_i[NTB], b_im_r[NTB], b_im_i[NTB];
#pragma unroll
    for (int tb = 0; tb < NTB; ++tb) {
      const T tr = (st == 0) ? f.tr[tb].x : (st == 1) ? f.tr[tb].y : (st == 2) ? f.tr[tb].z : f.tr[tb].w;
      const T ti = (st == 0) ? f.ti[tb].x : (st == 1) ? f.ti[tb].y : (st == 2) ? f.ti[tb].z : f.ti[tb].w;
      b_re_r[tb] = tr; b_re_i[tb] = -ti; b_im_r[tb] = ti; b_im_i[tb] = tr;
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const T av_r = (st == 0) ? f.ar[i].x : (st == 1) ? f.ar[i].y : (st == 2) ? f.ar[i].z : f.ar[i].w;
      const T av_i = (st == 0) ? f.ai[i].x : (st == 1) ? f.ai[i].y : (st == 2) ? f.ai[i].z : f.ai[i].w;
#pragma unroll
      for (int tb = 0; tb < NTB; ++tb) {
        if constexpr (NCB == 2) {
          acc[tb][i][0] = MF::run(av_r, b_re_r[tb], acc[tb][i][0]);
          acc[tb][i][0] = MF::run(av_i, b_re_i[tb], acc[tb][i][0]);
          acc[tb][i][1] = MF::run(av_r, b_im_r[tb], acc[tb][i][1]);
          acc[tb][i][1] = MF::run(av_i, b_im_i[tb], acc[tb][i][1]);
        } else {
          acc[tb][i][0] = MF::run(av_r, part ? b_im_r[tb] : b_re_r[tb], acc[tb][i][0]);
          acc[tb][i][0] = MF::run(av_i, part ? b_im_i[tb] : b_re_i[tb], acc[tb][i][0]);
        }
      }
    }
  }
}

// Coupling of NTB blocks of output modes (block tb: rows k0t[tb] .. of T,
// skipped where tok[tb] is false) to the solved modes jb <= j < je, with W
// read from global memory and the fragments of the next 16 modes loaded while
// the current ones multiply.  With NTB = 2 every W fragment feeds both blocks.
template <typename T, int NB, int RB, int NTB, bool VEC>
__device__ __forceinline__ void coupling_far(const T* slice, const T* tre, const T* tim, int sx, int sy,
                                             const int (&k0t)[NTB], const bool (&tok)[NTB], int jb,
                                             int je, int y0, int lr, int lk,
                                             typename SweepMfma<T>::acc_t (&acc)[NTB][RB][2 * NB / 16]) {
  constexpr int NCB = 2 * NB / 16;
  const int q = (NCB == 2) ? lr : (lr & 7);
  const int part = (NCB == 2) ? 0 : (lr >> 3);
  const T* trow[NTB];
  const T* irow[NTB];
#pragma unroll
  for (int tb = 0; tb < NTB; ++tb) {
    const int64_t off = tok[tb] ? (int64_t)(k0t[tb] + q) * sx : 0;
    trow[tb] = tre + off;
    irow[tb] = tim + off;
  }
  const int r0 = y0 + lr;
  if (jb >= je) return;
  CouplingFrag<T, RB, NTB> fa, fb;
  load_frag<T, RB, NTB, VEC>(fa, slice, trow, irow, tok, sx, sy, jb + 4 * lk, je, r0);
#pragma unroll 1
  for (int j0 = jb; j0 < je; j0 += 32) {
    const bool more = j0 + 16 < je;
    if (more) load_frag<T, RB, NTB, VEC>(fb, slice, trow, irow, tok, sx, sy, j0 + 16 + 4 * lk, je, r0);
    mma_frag<T, NB, RB, NTB>(fa, part, acc);
    if (!more) break;
    if (j0 + 32 < je) load_frag<T, RB, NTB, VEC>(fa, slice, trow, irow, tok, sx, sy, j0 + 32 + 4 * lk, je, r0);
    mma_frag<T, NB, RB, NTB>(fb, part, acc);
  }
}

// Coupling of the next block to the block just solved, with the solved lines
// read from the LDS tile (lane group lk owns tile columns 4 lk .. 4 lk + 3,
// the same permuted k order as coupling_direct).  NB <= 16: one 16-column
// step.  The T entries (rows of the next block, columns of the solved block)
// are loaded ahead by near_t.
template <typename T, int NB>
__device__ __forceinline__ void near_t(T (&trv)[4], T (&tiv)[4], const T* tre, const T* tim, int sx,
                                       int k0n, int k0, int nk, int lr, int lk) {
  constexpr int NCB = 2 * NB / 16;
  const int q = (NCB == 2) ? lr : (lr & 7);
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int jj = 4 * lk + st;
    const bool ok = jj < nk;
    trv[st] = ok ? tre[(int64_t)(k0n + q) * sx + k0 + jj] : (T)0;
    tiv[st] = ok ? tim[(int64_t)(k0n + q) * sx + k0 + jj] : (T)0;
  }
}

template <typename T, int NB, int RB, int R>
__device__ __forceinline__ void coupling_lds(const T* sre, const T* sim, const T (&trv)[4],
                                             const T (&tiv)[4], int sy, int ldy, int nk, int cw,
                                             int lr, int lk,
                                             typename SweepMfma<T>::acc_t (&acc)[RB][2 * NB / 16]) {
  static_assert(NB <= 16, "one 16-column step");
  using MF = SweepMfma<T>;
  constexpr int NCB = 2 * NB / 16;
  const int part = (NCB == 2) ? 0 : (lr >> 3);
  const int r0 = cw * RB * 16 + lr;
  T av_r[RB][4], av_i[RB][4];
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int jj = 4 * lk + st;
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int y = r0 + 16 * i;
      const bool rok = jj < nk && y < sy;
      av_r[i][st] = rok ? sre[lidx(jj, y, ldy, R)] : (T)0;
      av_i[i][st] = rok ? sim[lidx(jj, y, ldy, R)] : (T)0;
    }
  }
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const T b_re_r = trv[st], b_re_i = -tiv[st], b_im_r = tiv[st], b_im_i = trv[st];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      if constexpr (NCB == 2) {
        acc[i][0] = MF::run(av_r[i][st], b_re_r, acc[i][0]);
        acc[i][0] = MF::run(av_i[i][st], b_re_i, acc[i][0]);
        acc[i][1] = MF::run(av_r[i][st], b_im_r, acc[i][1]);
        acc[i][1] = MF::run(av_i[i][st], b_im_i, acc[i][1]);
      } else {
        acc[i][0] = MF::run(av_r[i][st], part ? b_im_r : b_re_r, acc[i][0]);
        acc[i][0] = MF::run(av_i[i][st], part ? b_im_i : b_re_i, acc[i][0]);
      }
    }
  }
}

// One wave copies rows [y0, y1) of a full tile of NB modes (k0 .. k0+NB-1)
// into LDS: 16-byte vectors of consecutive modes when VEC (sx % 4 == 0), all
// loads issued before the LDS stores.  MAXR bounds y1 - y0.
template <typename T, int NB, int MAXR, bool VEC>
__device__ __forceinline__ void tile_rows_load(const T* slice, T* sre, T* sim, int k0, int sx, int y0,
                                               int y1, int ldy, int R, int lane) {
  if constexpr (VEC) {
    using V = typename Vec16<T>::t;
    constexpr int MV = Vec16<T>::n, NV = NB / MV;
    constexpr int MAXU = (MAXR * 2 * NV + 63) / 64;
    const int total = (y1 - y0) * 2 * NV;
    V v[MAXU];
#pragma unroll
    for (int u = 0; u < MAXU; ++u) {
      const int e = lane + 64 * u;
      if (e < total) {
        const int kv = e % NV, comp = (e / NV) & 1, y = y0 + e / (2 * NV);
        // read once before the block is solved: non-temporal (see load_inv)
        typedef T NV4 __attribute__((ext_vector_type(MV)));
        const NV4 t = __builtin_nontemporal_load(
            reinterpret_cast<const NV4*>(slice + (int64_t)y * 2 * sx + comp * sx + k0 + kv * MV));
        v[u] = __builtin_bit_cast(V, t);
      }
    }
#pragma unroll
    for (int u = 0; u < MAXU; ++u) {
      const int e = lane + 64 * u;
      if (e < total) {
        const int kv = e % NV, comp = (e / NV) & 1, y = y0 + e / (2 * NV);
        T* dst = comp ? sim : sre;
#pragma unroll
        for (int m = 0; m < MV; ++m) dst[lidx(kv * MV + m, y, ldy, R)] = vget<T>(v[u], m);
      }
    }
  } else {
    const int total = (y1 - y0) * 2 * NB;
    for (int e = lane; e < total; e += 64) {
      const int k = e % NB, comp = (e / NB) & 1, y = y0 + e / (2 * NB);
      (comp ? sim : sre)[lidx(k, y, ldy, R)] = slice[(int64_t)y * 2 * sx + comp * sx + k0 + k];
    }
  }
}

// Block k0 .. k0 + nk - 1 of a slice from wave 0's copy of its solution
// (value i of line q of lane p at (q R + i) 64 + p) to global memory: one
// thread per row y = p R + i writes that row's nk modes (real, then imaginary
// parts), 16-byte vectors when VEC and the block is full.
template <typename T, int NB, int R, bool VEC>
__device__ __forceinline__ void wsol_store(T* slice, const Cx<T>* wsol, int k0, int nk, int sx, int sy, int P,
                                           int tid, int nthr, float* __restrict__ rm) {
  for (int e = tid; e < P * R; e += nthr) {
    const int p = e % P, i = e / P, y = p * R + i;
    if (y >= sy) continue;
    T re[NB], im[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const Cx<T> v = wsol[(q * R + i) * 64 + p];
      re[q] = v.x;
      im[q] = v.y;
    }
    if (rm) {   // running maximum of the row's solved modes (the same thread owns row y at every call)
      float m = rm[y];
#pragma unroll
      for (int q = 0; q < NB; ++q)
        if (q < nk) m = fmaxf(m, fmaxf(fabsf((float)re[q]), fabsf((float)im[q])));
      rm[y] = m;
    }
    T* row = slice + (int64_t)y * 2 * sx + k0;
    if (VEC && nk == NB && sizeof(T) == 4 && NB % 4 == 0) {
      typedef T V4T __attribute__((ext_vector_type(4)));
#pragma unroll
      for (int h = 0; h < NB / 4; ++h) {
        *reinterpret_cast<V4T*>(row + 4 * h) = V4T{re[4 * h], re[4 * h + 1], re[4 * h + 2], re[4 * h + 3]};
        *reinterpret_cast<V4T*>(row + sx + 4 * h) = V4T{im[4 * h], im[4 * h + 1], im[4 * h + 2], im[4 * h + 3]};
      }
    } else {
#pragma unroll
      for (int q = 0; q < NB; ++q)
        if (q < nk) {
          row[q] = re[q];
          row[sx + q] = im[q];
        }
    }
  }
}

// Pipelined back-sweep: one workgroup of 1 + NCW waves per (right-hand side,
// frequency) slice; blocks of NB modes from the last to the first.  Step b:
//   * all waves write block b+1 (solved in the previous step) from LDS to
//     global memory; barrier;
//   * wave 0 takes block b's tile (already carrying its coupling to every
//     mode beyond block b+1), subtracts the coupling to block b+1 from the
//     solution of b+1 it still holds in registers, and solves the NB lines in
//     order (DPP scans, right-looking updates inside the block); the near
//     coupling of a line is independent of the scans before it, so the
//     compiler interleaves the two;
//   * meanwhile waves 1..NCW stage block b-1's tile and subtract lambda2 times
//     its coupling to all modes beyond block b (MFMA products on fragments
//     read from global memory, one 16-mode step prefetched), and stage the
//     coefficients block b-1 needs: lambda2 T inside it and towards block b.
//     Every other step the pass over the modes beyond block b also produces
//     block b-2's coupling to them, which the next step completes with block
//     b's modes alone: the solved lines are streamed once per two blocks;
//   * barrier.
// Tiles and coefficient blocks are double-buffered in LDS.  One wave per SIMD
// per workgroup; with NB = 8 two workgroups share a CU.
constexpr int NCW = 3;
constexpr int SWT = 64 * (NCW + 1);

template <typename T, int R, int P, int NB, int RB, bool VEC, int MINB, int W0B, bool WIN>
__global__ __launch_bounds__(SWT, MINB) void k_schur_sweep(T* __restrict__ spec, const double2* __restrict__ lam,
                                                     const T* __restrict__ tup, const T* __restrict__ lu,
                                                     double lo, double up, int F, int sx, int sy, int ldy,
                                                     int klo, int khi, float* __restrict__ rmax, int b0) {
  static_assert((2 * NB) % 16 == 0, "MFMA column blocks");
  using MF = SweepMfma<T>;
  constexpr int NCB = 2 * NB / 16;
  extern __shared__ __align__(16) unsigned char smraw[];
  T* tiles = reinterpret_cast<T*>(smraw);       // [2 buffers][re, im][NB][ldy]
  const int TS = 2 * NB * ldy;
  T* tbs = tiles + (WIN ? 1 : 2) * TS;          // [2][NB][NB] complex: lambda2 T_{q' q} inside the block, q' < q
  T* tns = tbs + 4 * NB * NB;                   // [2][NB][NB] complex: lambda2 T_{q j} towards the block after
  // wave 0's copy of the block it solved last: value i of line q of lane l at
  // (q R + i) 64 + l (conflict-free), read back by the next step's near coupling
  Cx<T>* wsol = reinterpret_cast<Cx<T>*>(tns + 4 * NB * NB);
  // inverse pivots of the block being solved: row y = p R + i of line q at
  // (q R + i) P + p, so that wave 0's lanes read consecutive entries
  Cx<T>* pivs = wsol + NB * R * 64;
  // The coupling waves load the next block's pivots from global memory at the
  // start of a step (their latency hidden behind the step) and store them here
  // at the start of the following one, after wave 0 has finished with the
  // previous block's: the solves never wait on HBM for them.  Lines of up to
  // 256 rows (beyond, the registers are taken: wave 0 loads them itself, one
  // line ahead).
  constexpr bool PIVL = R * P <= 256;
  using PV = typename PivUnit<T, VEC>::t;
  constexpr int PVW = PivUnit<T, VEC>::n;                        // T per unit
  constexpr int PU = PIVL ? (2 * NB * R * P / PVW + SWT - 64 - 1) / (SWT - 64) : 1;   // units per coupling thread
  PV pv[PU];
  auto piv_store = [&](int ct, int nunits) {   // pv (units ct + u (SWT - 64)) -> pivs
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int e = ct + u * (SWT - 64);
      if (e < nunits)
#pragma unroll
        for (int h = 0; h < PVW / 2; ++h) {
          const int c = e * (PVW / 2) + h;   // complex index q sy + y in the block
          const int q = c / sy, y = c - q * sy;
          pivs[(q * R + y % R) * P + y / R] = Cx<T>{pv[u][2 * h], pv[u][2 * h + 1]};
        }
    }
  };

  const int n = blockIdx.x, b = blockIdx.y + b0;   // right-hand sides b0 .. b0 + gridDim.y - 1
  T* slice = spec + ((int64_t)b * F + n) * sy * 2 * sx;
  // a window's running row maxima of the solved modes (rows of this slice), or null
  float* rm = rmax ? rmax + ((int64_t)b * F + n) * sy : nullptr;
  const T* tre = tup;
  const T* tim = tup + (int64_t)sx * sx;
  const double2 l2 = lam[F + n];
  const T l2r = (T)l2.x, l2i = (T)l2.y;
  const int wave = threadIdx.x >> 6;
  // the window of modes [klo, khi) (klo a multiple of NB; khi one too, or sx):
  // blocks blo .. bhi-1; modes from khi on are already folded into the tiles
  const int blo = klo / NB, bhi = (khi + NB - 1) / NB;
  const int nblk = bhi - blo;
  // Far couplings come in pairs of blocks: in a step with far set, the rows a
  // wave prepares get their coupling to every mode beyond block kb for blocks
  // kb-1 and kb-2 in one pass over those modes (each W fragment read once,
  // multiplied twice); block kb-2's part waits in carry until the next step,
  // which adds only its coupling to block kb.  Neighbouring slices take
  // opposite parities, so half the workgroups stream the solved lines at any
  // time.
  constexpr int RBC = RB > W0B ? RB : W0B;
  typename MF::acc_t carry[RBC][NCB];
#pragma unroll
  for (int i = 0; i < RBC; ++i)
#pragma unroll
    for (int j = 0; j < NCB; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) carry[i][j][v] = 0;
  const int phase = (int)(blockIdx.x & 1);

  // lambda2 T[k0a + qa][k0b + qb] for qa, qb < NB (zero outside the valid
  // range: qb >= nkb, or qa >= qb when the two blocks coincide)
  auto stage_coef = [&](T* dst, int k0a, int k0b, int nkb, bool upper, int t, int nthr) {
    for (int e = t; e < NB * NB; e += nthr) {
      const int qa = e / NB, qb = e - qa * NB;
      T tr = 0, ti = 0;
      if (qb < nkb && (!upper || qa < qb)) {
        tr = tre[(int64_t)(k0a + qa) * sx + k0b + qb];
        ti = tim[(int64_t)(k0a + qa) * sx + k0b + qb];
      }
      dst[2 * e] = l2r * tr - l2i * ti;
      dst[2 * e + 1] = l2r * ti + l2i * tr;
    }
  };

  const T* lun = lu + (int64_t)n * sx * sy * 2;
  {  // prologue: the last block of the window (the only one that may be partial)
    const int k0 = (bhi - 1) * NB, nk = khi - k0;
    tile_load_by(slice, tiles, tiles + NB * ldy, k0, nk, NB, sx, sy, ldy, R, (int)threadIdx.x, SWT);
    stage_coef(tbs, k0, k0, nk, true, (int)threadIdx.x, SWT);
    if constexpr (PIVL)
      for (int c = threadIdx.x; c < nk * sy; c += SWT) {
        const int q = c / sy, y = c - q * sy;
        const T* src = lun + ((int64_t)k0 * sy + c) * 2;
        pivs[(q * R + y % R) * P + y / R] = Cx<T>{src[0], src[1]};
      }
  }
  __syncthreads();

  for (int st = 0; st < nblk; ++st) {
    // Thread indices re-derived each step from an opaque copy: otherwise the
    // compiler hoists every per-thread address of the tile copies out of the
    // loop and keeps them all live, which spills the solve's registers.
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, lr = lane & 15, lk = lane >> 4;
    const int cur = st & 1, nxt = cur ^ 1;
    // tiles: double-buffered, or in a window one buffer (wave 0 takes block kb
    // into registers before the coupling waves stage block kb-1 over it)
    const int tcur = WIN ? 0 : cur, tnxt = WIN ? 0 : nxt;
    const int kb = bhi - 1 - st, k0 = kb * NB, nk = min(NB, khi - k0), kend = k0 + nk;
    T* cre = tiles + tcur * TS;
    T* cim = cre + NB * ldy;
    T* nre = tiles + tnxt * TS;
    T* nim = nre + NB * ldy;
    if (st > 0) {   // block kb+1, solved in the previous step, to global memory
      const int k0p = k0 + NB, nkp = min(NB, khi - k0p);
      if constexpr (WIN) wsol_store<T, NB, R, VEC>(slice, wsol, k0p, nkp, sx, sy, P, tid, SWT, rm);
      else if (VEC && nkp == NB) tile_store_vec<T, NB, R * P>(slice, nre, nim, k0p, sx, sy, ldy, R, tid, SWT);
      else tile_store_by(slice, nre, nim, k0p, nkp, NB, sx, sy, ldy, R, tid, SWT);
      // block kb's pivots, loaded by the coupling waves in the previous step
      if (PIVL && tid >= 64) piv_store(tid - 64, 2 * NB * sy / PVW);
    }
    __syncthreads();   // block kb+1 in global memory; its LDS buffer is free; block kb's pivots staged
    // wave 0: block kb (carrying its coupling to every mode beyond block kb+1)
    // into registers; in a window before the coupling waves overwrite the one
    // tile buffer, else inside wave 0's branch (loaded here, the lines would
    // stay live across the coupling waves' code and spill it)
    Cx<T> d[NB][R];
    auto load_block = [&]() {
      const int p = lane % P;
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int idx = q * ldy + p * (R + 1) + i;
          d[q][i] = (lane < P && q < nk) ? Cx<T>{cre[idx], cim[idx]} : cz<T>();
        }
    };
    if constexpr (WIN) {
      if (wave == 0) load_block();
      __syncthreads();   // the single tile buffer is free for block kb-1
    }
    const int k0n = k0 - NB;   // next block (always full) when kb > blo
    // windowed: no pairing, every step couples block kb-1 to the rest of the window
    const bool far = WIN || ((st + phase) & 1) == 0;
    // Rows [y0, y1) of block kb-1: staged into the LDS buffer, coupled to every
    // mode beyond block kb (read from global memory), and lambda2 times the
    // coupling subtracted.  One wave; it touches only its own rows.
    auto prep_rows = [&](auto rbx, int y0, int y1, int lane, int lr, int lk) {
      constexpr int RBX = decltype(rbx)::value;
      tile_rows_load<T, NB, RBX * 16, VEC>(slice, nre, nim, k0n, sx, y0, y1, ldy, R, lane);
      typename MF::acc_t acc[RBX][NCB];
      if constexpr (WIN) {   // block kb-1 against the window's modes beyond block kb
        typename MF::acc_t a1[1][RBX][NCB];
#pragma unroll
        for (int i = 0; i < RBX; ++i)
#pragma unroll
          for (int j = 0; j < NCB; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) a1[0][i][j][v] = 0;
        const int k0t[1] = {k0n};
        const bool tok[1] = {true};
        coupling_far<T, NB, RBX, 1, VEC>(slice, tre, tim, sx, sy, k0t, tok, kend, khi, y0, lr, lk, a1);
#pragma unroll
        for (int i = 0; i < RBX; ++i)
#pragma unroll
          for (int j = 0; j < NCB; ++j) acc[i][j] = a1[0][i][j];
      } else if (far) {   // blocks kb-1 and kb-2 against every mode beyond block kb
        typename MF::acc_t a2[2][RBX][NCB];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int i = 0; i < RBX; ++i)
#pragma unroll
            for (int j = 0; j < NCB; ++j)
#pragma unroll
              for (int v = 0; v < 4; ++v) a2[h][i][j][v] = 0;
        const int k0t[2] = {k0n, k0n - NB};
        const bool tok[2] = {true, k0n - NB >= klo};
        coupling_far<T, NB, RBX, 2, VEC>(slice, tre, tim, sx, sy, k0t, tok, kend, khi, y0, lr, lk, a2);
#pragma unroll
        for (int i = 0; i < RBX; ++i)
#pragma unroll
          for (int j = 0; j < NCB; ++j) {
            acc[i][j] = a2[0][i][j];
            carry[i][j] = a2[1][i][j];
          }
      } else {     // block kb-1: the carried part plus its coupling to block kb+1
        typename MF::acc_t a1[1][RBX][NCB];
#pragma unroll
        for (int i = 0; i < RBX; ++i)
#pragma unroll
          for (int j = 0; j < NCB; ++j) a1[0][i][j] = carry[i][j];
        const int k0t[1] = {k0n};
        const bool tok[1] = {true};
        coupling_far<T, NB, RBX, 1, VEC>(slice, tre, tim, sx, sy, k0t, tok, kend, min(kend + NB, khi), y0,
                                         lr, lk, a1);
#pragma unroll
        for (int i = 0; i < RBX; ++i)
#pragma unroll
          for (int j = 0; j < NCB; ++j) acc[i][j] = a1[0][i][j];
      }
      // tile -= lambda2 C: all LDS reads first, then all writes (one
      // read-modify-write at a time would expose the LDS latency per value)
      const bool col_ok = NCB == 2 || lr < 8;
      T tr_[RBX][4], ti_[RBX][4];
#pragma unroll
      for (int i = 0; i < RBX; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int y = y0 + i * 16 + MF::row(lk, v);
          const int idx = lidx(lr, y, ldy, R);
          tr_[i][v] = (y < y1 && col_ok) ? nre[idx] : (T)0;   // y1 <= sy: this call's rows only
          ti_[i][v] = (y < y1 && col_ok) ? nim[idx] : (T)0;
        }
#pragma unroll
      for (int i = 0; i < RBX; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int y = y0 + i * 16 + MF::row(lk, v);
          T cr, ci;
          if constexpr (NCB == 2) {
            cr = acc[i][0][v];
            ci = acc[i][1][v];
          } else {
            cr = acc[i][0][v];
            ci = dpp_mov<0x108>(acc[i][0][v]);   // imaginary part from lane lr + 8 (row_shl:8)
          }
          if (y < y1 && col_ok) {
            const int idx = lidx(lr, y, ldy, R);
            nre[idx] = tr_[i][v] - (l2r * cr - l2i * ci);
            nim[idx] = ti_[i][v] - (l2r * ci + l2i * cr);
          }
        }
    };
    if (wave == 0) {
      // ---- block kb: near coupling, then its lines in order ------------
      const bool active = lane < P;
      const int p = lane % P;
      const Cx<T> ca = active ? Cx<T>{(T)(l2.x * lo), (T)(l2.y * lo)} : cz<T>();
      const Cx<T> cc = active ? Cx<T>{(T)(l2.x * up), (T)(l2.y * up)} : cz<T>();
      const Cx<T>* tbc = reinterpret_cast<const Cx<T>*>(tbs + cur * 2 * NB * NB);
      const Cx<T>* tnc = reinterpret_cast<const Cx<T>*>(tns + cur * 2 * NB * NB);
      // inverse pivots of line q (one beyond the line's rows): from LDS, or
      // read once from global memory, non-temporally (they should not push
      // the solved lines, which the coupling product re-reads, out of the
      // last-level cache)
      auto load_inv = [&](int q, Cx<T> (&iv)[R]) {
        if constexpr (PIVL) {
#pragma unroll
          for (int i = 0; i < R; ++i)
            iv[i] = (active && p * R + i < sy) ? pivs[(q * R + i) * P + p] : c1<T>();
          return;
        }
        const T* src = lun + ((int64_t)(k0 + q) * sy + p * R) * 2;
        if constexpr (sizeof(T) == 4 && R % 2 == 0) {
          typedef float f4v __attribute__((ext_vector_type(4)));
          const bool full = active && p * R + R <= sy;
#pragma unroll
          for (int h = 0; h < R / 2; ++h) {
            f4v v = {1.f, 0.f, 1.f, 0.f};
            if (full) v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(src) + h);
            iv[2 * h] = Cx<T>{v.x, v.y};
            iv[2 * h + 1] = Cx<T>{v.z, v.w};
          }
          if (!full)
#pragma unroll
            for (int i = 0; i < R; ++i)
              iv[i] = (active && p * R + i < sy) ? Cx<T>{src[2 * i], src[2 * i + 1]} : c1<T>();
        } else {
#pragma unroll
          for (int i = 0; i < R; ++i)
            iv[i] = (active && p * R + i < sy) ? Cx<T>{src[2 * i], src[2 * i + 1]} : c1<T>();
        }
      };
      if constexpr (!WIN) load_block();
      Cx<T> ivn[R];
      load_inv(nk - 1, ivn);
      // coupling of the whole block to block kb+1 (solved in the previous
      // step; nothing in the first): it does not depend on this block's own
      // lines, so it runs as one batch before them, one solved line of block
      // kb+1 at a time, instead of on the chain of solves
      if (st > 0) {
#pragma unroll
        for (int jq = 0; jq < NB; ++jq) {
          Cx<T> x[R];
#pragma unroll
          for (int i = 0; i < R; ++i) x[i] = wsol[(jq * R + i) * 64 + lane];
#pragma unroll
          for (int q = 0; q < NB; ++q) {
            const Cx<T> t = tnc[q * NB + jq];
#pragma unroll
            for (int i = 0; i < R; ++i) {
              d[q][i].x = fma(-t.x, x[i].x, fma(t.y, x[i].y, d[q][i].x));
              d[q][i].y = fma(-t.x, x[i].y, fma(-t.y, x[i].x, d[q][i].y));
            }
          }
        }
      }
#pragma unroll
      for (int q = NB - 1; q >= 0; --q) {
        if (q < nk) {
          Cx<T> iv[R];
#pragma unroll
          for (int i = 0; i < R; ++i) iv[i] = ivn[i];
          if (q > 0) load_inv(q - 1, ivn);
          lu_scan_dpp<T, R, P>(d[q], iv, ca, cc, sy, lane);
          // d_qa -= t w_q inside the block, four fused multiply-adds per value
#pragma unroll
          for (int qa = 0; qa < q; ++qa) {
            const Cx<T> t = tbc[qa * NB + q];
#pragma unroll
            for (int i = 0; i < R; ++i) {
              const Cx<T> x = d[q][i];
              d[qa][i].x = fma(-t.x, x.x, fma(t.y, x.y, d[qa][i].x));
              d[qa][i].y = fma(-t.x, x.y, fma(-t.y, x.x, d[qa][i].y));
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int i = 0; i < R; ++i) {
          wsol[(q * R + i) * 64 + lane] = (q < nk) ? d[q][i] : cz<T>();
          const int idx = q * ldy + p * (R + 1) + i;
          if (!WIN && active && q < nk) {
            cre[idx] = d[q][i].x;
            cim[idx] = d[q][i].y;
          }
        }
      // the first W0B row blocks of block kb-1's preparation: wave 0 finishes
      // its lines before the coupling waves finish theirs, so it takes a share
      if constexpr (W0B > 0)
        if (kb > blo) prep_rows(std::integral_constant<int, W0B>{}, 0, min(sy, W0B * 16), lane, lr, lk);
    } else if (kb > blo) {
      // ---- block kb-1: tile, coupling to the modes beyond block kb -----
      // Wave cw stages exactly the rows its accumulators cover, so its
      // subtraction depends only on its own LDS writes (in program order).
      const int ct = tid - 64, cw = wave - 1;
      const int y0 = (W0B + cw * RB) * 16, y1 = min(sy, y0 + RB * 16);
      // coefficients of block kb-1 (inside it; towards block kb): loads
      // issued now, their latency hidden behind the tile and the products
      static_assert(NB * NB <= SWT - 64, "one coefficient per thread");
      if constexpr (PIVL) {  // block kb-1's pivots: contiguous in global memory (one unit per PVW values)
        const PV* src = reinterpret_cast<const PV*>(lun + (int64_t)k0n * sy * 2);
        const int nunits = 2 * NB * sy / PVW;
#pragma unroll
        for (int u = 0; u < PU; ++u) {
          const int e = ct + u * (SWT - 64);
          if (e < nunits) pv[u] = __builtin_nontemporal_load(src + e);
        }
      }
      T cbr = 0, cbi = 0, cnr = 0, cni = 0;
      if (ct < NB * NB) {
        const int qa = ct / NB, qb = ct - qa * NB;
        const int64_t row = (int64_t)(k0n + qa) * sx;
        if (qa < qb) {
          cbr = tre[row + k0n + qb];
          cbi = tim[row + k0n + qb];
        }
        if (qb < nk) {
          cnr = tre[row + k0 + qb];
          cni = tim[row + k0 + qb];
        }
      }
      if constexpr (WIN) {   // passes of 32 rows: registers for two workgroups per CU
        for (int yy = y0; yy < y1; yy += 32)
          prep_rows(std::integral_constant<int, 2>{}, yy, min(y1, yy + 32), lane, lr, lk);
      } else {
        prep_rows(std::integral_constant<int, RB>{}, y0, y1, lane, lr, lk);
      }
      if (ct < NB * NB) {
        T* bt = tbs + nxt * 2 * NB * NB;
        T* bn = tns + nxt * 2 * NB * NB;
        bt[2 * ct] = l2r * cbr - l2i * cbi;
        bt[2 * ct + 1] = l2r * cbi + l2i * cbr;
        bn[2 * ct] = l2r * cnr - l2i * cni;
        bn[2 * ct + 1] = l2r * cni + l2i * cnr;
      }
    }
    __syncthreads();   // block kb solved (LDS buffer cur); block kb-1 staged
  }
  {  // the first block of the window, solved in the last step
    const int nkp = min(NB, khi - klo);
    if constexpr (WIN) {
      wsol_store<T, NB, R, VEC>(slice, wsol, klo, nkp, sx, sy, P, (int)threadIdx.x, SWT, rm);
    } else {
      T* pre = tiles + ((nblk - 1) & 1) * TS;
      tile_store_by(slice, pre, pre + NB * ldy, klo, nkp, NB, sx, sy, ldy, R, (int)threadIdx.x, SWT);
    }
  }
}

template <typename T, int R, int P, int NB, int BK, int RB, bool VEC>
__global__ __launch_bounds__(NT, (sizeof(T) == 8 && R >= 8) ? 1 : 2) void k_schur_sweep_wide(T* __restrict__ spec, const double2* __restrict__ lam,
                                                    const double2* __restrict__ tk,
                                                    const T* __restrict__ tup,
                                                    const T* __restrict__ lu, double lo, double di,
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
  T* As = sim + NB * ldy;                // [NYP][LDA]; after the K loop: C[NYP][LDA] (staged path)
  T* Bs = As + (VEC ? 0 : NYP * LDA);    // [2 NB][LDA] (staged path)
  T* Tb = Bs + (VEC ? 0 : 2 * NB * LDA); // block of T: [2][NB][NB] (re, im)
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
    if (VEC && J > 0) {
      typename MF::acc_t acc[RB][NCB];
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < NCB; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;
      coupling_direct<T, NB, RB>(slice, tre, tim, sx, sy, k0, nk, kend, wave, lr, lk, acc);
      __syncthreads();   // the tile is complete before the subtraction
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int y = wave * RB * 16 + i * 16 + MF::row(lk, v);
          T cr, ci;
          int q;
          if constexpr (NCB == 2) {
            cr = acc[i][0][v];
            ci = acc[i][1][v];
            q = lr;
          } else {
            cr = acc[i][0][v];
            ci = __shfl_down(acc[i][0][v], 8, 16);   // imaginary part from lane lr + 8
            q = lr;
          }
          if (y < sy && q < nk && (NCB == 2 || lr < 8)) {
            int idx = lidx(q, y, ldy, R);
            sre[idx] -= l2r * cr - l2i * ci;
            sim[idx] -= l2r * ci + l2i * cr;
          }
        }
    } else if (!VEC && J > 0) {
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
      // Lines of the block in order, each with its precomputed LU (inverse
      // pivots of line (n, k) at lu[((n sx + k) sy + y)], complex) and the
      // coupling to the block's already solved lines gathered left-looking
      // from LDS: r_q -= lambda2 sum_{q' > q} T[k0+q][k0+q'] w_q'.
      const bool active = (seg == 0);
      const Cx<T> ca = active ? Cx<T>{(T)(l2.x * lo), (T)(l2.y * lo)} : cz<T>();
      const Cx<T> cc = active ? Cx<T>{(T)(l2.x * up), (T)(l2.y * up)} : cz<T>();
      const T* lun = lu + (int64_t)n * sx * sy * 2;
      Cx<T> ivn[R];
      auto load_inv = [&](int q, Cx<T> (&iv)[R]) {
        const T* src = lun + ((int64_t)(k0 + q) * sy + p * R) * 2;
#pragma unroll
        for (int i = 0; i < R; ++i)
          iv[i] = (active && p * R + i < sy) ? Cx<T>{src[2 * i], src[2 * i + 1]} : c1<T>();
      };
      if (nk > 0) load_inv(nk - 1, ivn);
      for (int q = nk - 1; q >= 0; --q) {
        Cx<T> iv[R];
#pragma unroll
        for (int i = 0; i < R; ++i) iv[i] = ivn[i];
        if (q > 0) load_inv(q - 1, ivn);     // next line's pivots in flight
        Cx<T> d[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
          int idx = q * ldy + p * (R + 1) + i;
          d[i] = active ? Cx<T>{sre[idx], sim[idx]} : cz<T>();
        }
        for (int qq = q + 1; qq < nk; ++qq) {
          T tr = Tb[q * NB + qq], ti = Tb[NB * NB + q * NB + qq];
          T cr = l2r * tr - l2i * ti, ci = l2r * ti + l2i * tr;
#pragma unroll
          for (int i = 0; i < R; ++i) {
            int idx = qq * ldy + p * (R + 1) + i;
            T wr = sre[idx], wi = sim[idx];
            d[i].x -= cr * wr - ci * wi;
            d[i].y -= cr * wi + ci * wr;
          }
        }
        lu_scan_wave<T, R, P>(d, iv, ca, cc, sy, p);
        if (active) {
#pragma unroll
          for (int i = 0; i < R; ++i) {
            int idx = q * ldy + p * (R + 1) + i;
            sre[idx] = d[i].x;
            sim[idx] = d[i].y;
          }
        }
      }
    }
    __syncthreads();
    tile_store(slice, sre, sim, k0, nk, NB, sx, sy, ldy, R);
    __threadfence_block();
  }
}


// Inverse pivots of the non-pivoted LU factorisation of every line matrix
// [(lambda1_n + lambda2_n T_kk) I + lambda2_n K_y] (float64 recurrence,
// stored in the working precision): one thread per (frequency, mode).
template <typename T>
__global__ __launch_bounds__(NT) void k_line_lu(T* __restrict__ lu, const double2* __restrict__ lam,
                                                const double2* __restrict__ tk, double lo, double di,
                                                double up, int F, int sx, int sy) {
  const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (t >= (int64_t)F * sx) return;
  const int n = (int)(t / sx), k = (int)(t - (int64_t)n * sx);
  const double2 l1 = lam[n], l2 = lam[F + n], tt = tk[k];
  const double shr = tt.x + di, shi = tt.y;
  const double br = l1.x + l2.x * shr - l2.y * shi, bi = l1.y + l2.x * shi + l2.y * shr;
  // a c = lambda2^2 lo up
  const double acr = (l2.x * l2.x - l2.y * l2.y) * lo * up, aci = 2.0 * l2.x * l2.y * lo * up;
  T* out = lu + t * sy * 2;
  double ir = 0, ii = 0;
  for (int y = 0; y < sy; ++y) {
    double mr = br, mi = bi;
    if (y > 0) {  // m = b - a c / m_prev = b - (a c) inv_prev
      mr -= acr * ir - aci * ii;
      mi -= acr * ii + aci * ir;
    }
    const double den = 1.0 / (mr * mr + mi * mi);
    ir = mr * den;
    ii = -mi * den;
    out[2 * y] = (T)ir;
    out[2 * y + 1] = (T)ii;
  }
}

// Far coupling of one window of the back-sweep, over every slice at once.
// For the window of modes [klo, klo + NW) and every row (slice, y) of the
// spectral buffer:
//
//   R[row][klo + q] -= lambda2_n sum_{j >= khi} W[row][j] T[klo + q][j],  q < NW,
//
// with W the solved modes (already final in the buffer) and khi = klo + NW.
// In the real block form, row [Wr | Wi] (the buffer's row-planar layout) times
// B[k][n'] with n' < NW the real and n' >= NW the imaginary part of mode
// klo + n' mod NW:  B^T = [[Tr, -Ti], [Ti, Tr]] restricted to those rows and to
// the columns j >= khi of both halves (tfar holds the whole 2nx x 2nx B^T).
// Operands split on MFMA with float32 accumulation, in one of two forms:
//  * F16 (the default): each W row scaled by the power of two that brings the
//    largest of its solved modes (rmax, kept by the window kernels) into
//    [2^13, 2^14), B^T by the power of two tscale (its largest entry into the
//    same range), both split into fp16 hi + lo (22 significant bits), and the
//    three products hi hi + hi lo + lo hi; the dropped lo lo term is 2^-22 of
//    |W| |T|, below the rounding of a float32 dot product of the same length;
//  * bf16: three parts each, the six products down to relative size 2^-16.
// Tiles of 128 rows x 2 NW = 128 columns x 32, 2 x 2 waves of 64 x 64; the
// accumulators go through LDS so that each thread can combine a mode's real
// and imaginary parts and apply the complex lambda2 of its row's frequency.
// Needs nx % 32 == 0 (k chunks do not straddle the two halves; 16-byte loads).
constexpr int FAR_NW = 64;   // modes per column tile; a window takes SWEEP_WINDOW / 64 of them

// Power of two bringing m into [2^13, 2^14) (1 for m = 0).
__device__ __forceinline__ float far_rowscale(float m) {
  int e = 0;
  (void)frexpf(m, &e);   // m = f 2^e, f in [0.5, 1)
  return m > 0.f ? ldexpf(1.f, 14 - e) : 1.f;
}

template <bool F16>
__global__ __launch_bounds__(NT, 2) void k_sweep_far(float* __restrict__ spec, const unsigned short* __restrict__ Bt,
                                                  const double2* __restrict__ lam, int64_t rows, int F, int sx,
                                                  int sy, int klo, int khi, const float* __restrict__ rmax,
                                                  float tinv, int64_t r0) {
  constexpr int BM = 128, BN = 2 * FAR_NW, BK = 32, NA = F16 ? 2 : 3;
  static_assert(BN == 128, "tile");
  auto off = [](int r, int ch) { return r * BK + 8 * (ch ^ ((r >> 1) & 3)); };
  constexpr int STAGE = 2 * NA * BM * BK;      // unsigned shorts of the A and B staging
  constexpr int LDC = BN + 1;                  // float stride of the accumulator half-tile
  constexpr int WORDS = (STAGE / 2 > 64 * LDC) ? STAGE / 2 : 64 * LDC;
  __shared__ __align__(16) float smem[WORDS];
  unsigned short* As = reinterpret_cast<unsigned short*>(smem);
  unsigned short* Bs = As + NA * BM * BK;
  float* Cs = smem;

  const int64_t m0 = r0 + (int64_t)blockIdx.x * BM;   // rows r0 .. rows - 1
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * 64, wn0 = (wave & 1) * 64;
  const int lr = lane & 15, lk = lane >> 4;
  klo += FAR_NW * (int)blockIdx.y;             // this tile's 64 modes of the window
  const int L = sx - khi;                      // solved modes beyond the window
  const int K2 = 2 * L;
  const int64_t ld = 2 * (int64_t)sx;          // row length of the buffer and of B^T
  const int64_t part = ld * ld;                // elements per bf16 part of B^T

  // the W rows come from HBM once per tile: DA k chunks of them in flight,
  // the B^T chunk (shared by every tile, from L2) one.  Rows beyond the
  // buffer load a valid row and are zeroed afterwards, so the loads carry no
  // branches and the waits can count them.
  constexpr int DA = 2;   // A chunks in flight (a third spills)
  float4 ra[DA][4];
  u32x4 rb[NA][2];   // a native vector type: with HIP's uint4 struct this array went to scratch memory
  int64_t arow[4];
  bool aok[4];
  float rsc[4];   // F16: the staged rows' scales
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t gm = m0 + (tid >> 3) + 32 * i;
    aok[i] = gm < rows;
    const int64_t gc = aok[i] ? gm : rows - 1;
    arow[i] = gc * ld + 4 * (tid & 7);
    rsc[i] = F16 ? far_rowscale(rmax[gc]) : 1.f;
  }
  int64_t brow[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int nl = (tid >> 2) + 64 * i;      // local column: real parts of the window, then imaginary
    const int np = nl < FAR_NW ? klo + nl : sx + klo + (nl - FAR_NW);
    brow[i] = (int64_t)np * ld + 8 * (tid & 3);
  }
  auto gk = [&](int kk) { return kk < L ? khi + kk : sx + khi + (kk - L); };
  auto aload = [&](auto bufc, int kk) {
    constexpr int bb = decltype(bufc)::value;
    const int k = gk(kk);
#pragma unroll
    for (int i = 0; i < 4; ++i) ra[bb][i] = *reinterpret_cast<const float4*>(spec + arow[i] + k);
  };
  auto bload = [&](int kk) {
    const int k = gk(kk);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int a = 0; a < NA; ++a) rb[a][i] = *reinterpret_cast<const u32x4*>(Bt + a * part + brow[i] + k);
  };
  auto sstore = [&](auto bufc) {
    constexpr int bb = decltype(bufc)::value;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = (tid >> 3) + 32 * i, c = 4 * (tid & 7);
      float v[4] = {ra[bb][i].x, ra[bb][i].y, ra[bb][i].z, ra[bb][i].w};
      if (!aok[i]) v[0] = v[1] = v[2] = v[3] = 0.f;
      us4 prt[NA];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if constexpr (F16) {   // exact power-of-two scale, then hi and the exact residual
          const float x = v[q] * rsc[i];
          const _Float16 h = (_Float16)x;
          prt[0][q] = __builtin_bit_cast(unsigned short, h);
          prt[1][q] = __builtin_bit_cast(unsigned short, (_Float16)(x - (float)h));
        } else {
          float rest = v[q];
#pragma unroll
          for (int a = 0; a < NA; ++a) {
            prt[a][q] = bf16_bits(rest);
            if (a + 1 < NA) rest -= bf16_val(prt[a][q]);
          }
        }
      }
#pragma unroll
      for (int a = 0; a < NA; ++a) *reinterpret_cast<us4*>(&As[a * BM * BK + off(r, c >> 3) + (c & 7)]) = prt[a];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = (tid >> 2) + 64 * i, c = 8 * (tid & 3);
#pragma unroll
      for (int a = 0; a < NA; ++a) *reinterpret_cast<u32x4*>(&Bs[a * BN * BK + off(r, c >> 3)]) = rb[a][i];
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
      for (int j = 0; j < 4; ++j) b[x][j] = *reinterpret_cast<const bf8*>(&Bs[x * BN * BK + off(wn0 + 16 * j + lr, lk)]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      bf8 a[NA];
#pragma unroll
      for (int x = 0; x < NA; ++x) a[x] = *reinterpret_cast<const bf8*>(&As[x * BM * BK + off(wm0 + 16 * i + lr, lk)]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if constexpr (F16) {   // small terms first
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a[1]), __builtin_bit_cast(h8, b[0][j]),
                                                             acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a[0]), __builtin_bit_cast(h8, b[1][j]),
                                                             acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a[0]), __builtin_bit_cast(h8, b[0][j]),
                                                             acc[i][j], 0, 0, 0);
        } else {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[NA - 1], b[0][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[NA - 1][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0][j], acc[i][j], 0, 0, 0);
        }
      }
    }
  };
  // one k chunk: stage chunk k (A from buffer dc), issue the loads DA chunks
  // ahead into the freed buffer and B one chunk ahead, multiply
  auto step = [&](auto dc, int k) {
    __syncthreads();
    sstore(dc);
    __syncthreads();
    if (k + DA * BK < K2) aload(dc, k + DA * BK);
    if (k + BK < K2) bload(k + BK);
    compute();
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  aload(I0{}, 0);
  bload(0);
  if (BK < K2) aload(I1{}, BK);
  for (int kk = 0; kk < K2; kk += DA * BK) {
    step(I0{}, kk);
    if (kk + BK >= K2) break;
    step(I1{}, kk + BK);
  }
  // the accumulators through LDS (reusing the staging buffers), 64 rows at a
  // time: the two waves of row half h write, then every thread takes
  // R -= lambda2 C for consecutive modes of one row
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    __syncthreads();
    if ((wave >> 1) == h)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) Cs[(16 * i + 4 * lk + v) * LDC + wn0 + 16 * j + lr] = acc[i][j][v];
    __syncthreads();
    // every global load of the update first (one round trip), then the stores
    static_assert(FAR_NW == 64, "thread -> (row, mode) map");
    constexpr int PER = 64 * FAR_NW / NT;
    const int q = tid & 63;
    float yr[PER], yi[PER], rm[PER];
    double2 l2v[PER];
    // branch-free: rows beyond the buffer read the last row (their results
    // are not stored), so all the loads issue before the first wait; the
    // row's frequency in 32-bit arithmetic (the buffer has far fewer than
    // 2^32 rows)
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int r = (tid >> 6) + 4 * t;
      const int64_t gm = m0 + 64 * h + r;
      const int64_t gc = gm < rows ? gm : rows - 1;
      const float* src = spec + gc * ld + klo + q;
      yr[t] = src[0];
      yi[t] = src[sx];
      l2v[t] = lam[F + (int)(((unsigned)gc / (unsigned)sy) % (unsigned)F)];
      rm[t] = F16 ? rmax[gc] : 0.f;
    }
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int r = (tid >> 6) + 4 * t;
      const int64_t gm = m0 + 64 * h + r;
      if (gm < rows) {
        const float l2r = (float)l2v[t].x, l2i = (float)l2v[t].y;
        const float us = F16 ? tinv / far_rowscale(rm[t]) : 1.f;   // undo the operand scales (powers of two)
        const float cr = us * Cs[r * LDC + q], ci = us * Cs[r * LDC + FAR_NW + q];
        float* dst = spec + gm * ld + klo + q;
        dst[0] = yr[t] - (l2r * cr - l2i * ci);
        dst[sx] = yi[t] - (l2r * ci + l2i * cr);
      }
    }
  }
}

struct SweepShape { int R, P, RB, ldy; size_t lds; bool vec; };

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
  const bool vec = (g.sx % 4) == 0;
  size_t stage = vec ? 0 : (size_t)64 * RB * (BK + 1) + (size_t)2 * NB * (BK + 1);
  size_t lds = sizeof(T) * ((size_t)2 * NB * ldy + stage + (size_t)2 * NB * NB + (size_t)2 * NB);
  return SweepShape{R, P, RB, ldy, lds, vec};
}

template <typename T, int R, int P, int NB, int BK, int RB>
void launch_one(const Plan& pl, const SpaceOp& op, T* spec, hipStream_t s) {
  const Geom& g = pl.g;
  SweepShape sh = sweep_shape<T, NB, BK>(pl);
  auto kfn = sh.vec ? k_schur_sweep_wide<T, R, P, NB, BK, RB, true> : k_schur_sweep_wide<T, R, P, NB, BK, RB, false>;
  lds_limit((const void*)kfn, sh.lds);
  kfn<<<dim3(g.F, g.B), NT, sh.lds, s>>>(spec, pl.d_lam, op.tk, (const T*)op.tup, (const T*)op.lu,
                                         op.lo, op.di, op.up, g.F, g.sx, g.sy, sh.ldy);
}

// Pipelined kernel: LDS bytes of two tiles and two coupling blocks.
template <typename T, int NB>
size_t piped_lds(const SweepShape& sh, bool win) {
  // two tiles, two pairs of coefficient blocks, wave 0's solution copy
  // + the pivots of one block (lines of up to 256 rows, or in a window)
  // (a window keeps one tile; its pivots come from LDS only for short lines)
  return sizeof(T) * ((size_t)(win ? 2 : 4) * NB * sh.ldy + (size_t)8 * NB * NB + (size_t)2 * NB * sh.R * 64 +
                      (sh.R * sh.P <= 256 ? (size_t)2 * NB * sh.R * sh.P : 0));
}

template <typename T, int R, int P, int NB, int RB, int W0B>
void launch_piped(const Plan& pl, const SpaceOp& op, T* spec, hipStream_t s, int klo, int khi, int b0, int nb) {
  const Geom& g = pl.g;
  SweepShape sh = sweep_shape<T, NB, 16>(pl);
  const bool win = khi - klo < g.sx;
  const size_t lds = piped_lds<T, NB>(sh, win);
  // two workgroups per CU where the registers allow (lines of up to 256 rows):
  // an odd number of slices, or more slices than CUs, then leaves no CU idle
  // while a last slice runs alone
  constexpr int MINB = (R == 4) ? 2 : 1;
  // a window's kernel (one tile buffer, no far pairs) fits two workgroups per
  // CU at every line length
  auto kfn = sh.vec ? (win ? k_schur_sweep<T, R, P, NB, RB, true, 2, W0B, true>
                           : k_schur_sweep<T, R, P, NB, RB, true, MINB, W0B, false>)
                    : (win ? k_schur_sweep<T, R, P, NB, RB, false, 2, W0B, true>
                           : k_schur_sweep<T, R, P, NB, RB, false, MINB, W0B, false>);
  lds_limit((const void*)kfn, lds);
  kfn<<<dim3(g.F, nb), SWT, lds, s>>>(spec, pl.d_lam, (const T*)op.tup, (const T*)op.lu, op.lo, op.up,
                                      g.F, g.sx, g.sy, sh.ldy, klo, khi, win ? pl.d_rmax : nullptr, b0);
}

// (NB, BK) of the wide kernel per precision and row count.
template <typename T> struct SweepCfg;
template <> struct SweepCfg<float> { static constexpr int NB = 16, BK = 32, NB8 = 8, BK8 = 16; };
template <> struct SweepCfg<double> { static constexpr int NB = 8, BK = 16, NB8 = 8, BK8 = 16; };

// Modes per block of the pipelined kernel: the block's lines live in wave 0's
// registers (NB x R complex values per lane); 8 keeps the kernel within two
// workgroups per CU (42 KiB of LDS at 256 rows).
template <typename T> struct PipedCfg;
template <> struct PipedCfg<float> { static constexpr int NB4 = 8, NB8 = 8; };
template <> struct PipedCfg<double> { static constexpr int NB4 = 0, NB8 = 0; };

// float64 keeps the one-phase kernel: its coupling product (half the float32
// MFMA rate) is the long pole, and there all four waves run it.

template <typename T>
void launch(const Plan& pl, const SpaceOp& op, T* spec, hipStream_t s, int klo = 0, int khi = -1, int b0 = 0,
            int nb = -1) {
  using C = SweepCfg<T>;
  using PC = PipedCfg<T>;
  SweepShape sh = sweep_shape<T, C::NB, C::BK>(pl);
  if (khi < 0) khi = pl.g.sx;
  if (nb < 0) nb = pl.g.B;
  if constexpr (PC::NB8 > 0) {   // float32: pipelined kernel
    // row blocks of 16 rows: W0 for wave 0 (after its lines), RB per coupling
    // wave, W0 + 3 RB >= rows / 16: <= 64 rows: 0 + 3 x 2, <= 128: 0 + 3 x 3,
    // <= 256: 1 + 3 x 5, <= 512: 2 + 3 x 10
#define PD_PIPED(RR, PP, BB, W0, NBV)                                                     \
  if (sh.R == RR && sh.P == PP) {                                                         \
    launch_piped<T, RR, PP, NBV, BB, W0>(pl, op, spec, s, klo, khi, b0, nb);              \
    return;                                                                               \
  }
    PD_PIPED(4, 1, 2, 0, PC::NB4) PD_PIPED(4, 2, 2, 0, PC::NB4) PD_PIPED(4, 4, 2, 0, PC::NB4)
    PD_PIPED(4, 8, 2, 0, PC::NB4) PD_PIPED(4, 16, 2, 0, PC::NB4) PD_PIPED(4, 32, 3, 0, PC::NB4)
    PD_PIPED(4, 64, 5, 1, PC::NB4)
    PD_PIPED(8, 64, 10, 2, PC::NB8)
#undef PD_PIPED
    return;
  }
  // float64: the one-phase kernel (block in LDS, coupling on all four waves)
  if constexpr (PC::NB8 == 0) {
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
}

}  // namespace

size_t schur_sweep_lds(const Plan& pl) {
  if (pl.prec == Prec::F64) {
    SweepShape a = sweep_shape<double, 8, 16>(pl);
    return a.RB == 8 ? sweep_shape<double, SweepCfg<double>::NB8, SweepCfg<double>::BK8>(pl).lds : a.lds;
  }
  SweepShape a = sweep_shape<float, 16, 32>(pl);
  const bool win = sweep_windowed(pl);
  return a.R == 4 ? piped_lds<float, PipedCfg<float>::NB4>(a, win) : piped_lds<float, PipedCfg<float>::NB8>(a, win);
}

void schur_line_lu(const Plan& pl, const SpaceOp& op, hipStream_t s) {
  const Geom& g = pl.g;
  const int64_t lines = (int64_t)g.F * g.sx;
  dim3 grid((unsigned)((lines + NT - 1) / NT));
  if (pl.prec == Prec::F64)
    k_line_lu<double><<<grid, NT, 0, s>>>((double*)op.lu, pl.d_lam, op.tk, op.lo, op.di, op.up, g.F, g.sx, g.sy);
  else
    k_line_lu<float><<<grid, NT, 0, s>>>((float*)op.lu, pl.d_lam, op.tk, op.lo, op.di, op.up, g.F, g.sx, g.sy);
}

bool sweep_windowed(const Plan& pl) {
  const Geom& g = pl.g;
  return pl.schur && pl.p.dim == 2 && (pl.prec == Prec::BF16 || pl.prec == Prec::F16) && g.sx % SWEEP_WINDOW == 0 &&
         g.sx >= 2 * SWEEP_WINDOW && g.sx % 32 == 0;
}

static __global__ __launch_bounds__(NT) void k_zero_f32(float* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

static void fill_zero_f32(float* p, int64_t n, hipStream_t s) {
  k_zero_f32<<<(unsigned)((n + NT - 1) / NT), NT, 0, s>>>(p, n);
}

void schur_sweep(const Plan& pl, const SpaceOp& op, void* spec, hipStream_t s) {
  if (pl.prec == Prec::F64) {
    launch<double>(pl, op, (double*)spec, s);
    return;
  }
  if (!sweep_windowed(pl) || !op.tfar) {
    launch<float>(pl, op, (float*)spec, s);
    return;
  }
  // windows from the last modes to the first: fold the coupling to every
  // later window into the tiles with one product over all slices, then sweep
  // the window's modes
  const Geom& g = pl.g;
  const int64_t rows = (int64_t)g.B * g.F * g.sy;
  // the rows' running maxima start from zero (a fill kernel: no memset node
  // for callers that capture the sequence)
  fill_zero_f32(pl.d_rmax, rows, s);
  // The sweep is independent per slice.  With a batch of two or more, the
  // second half of the right-hand sides runs on the plan's second stream, so
  // that one half's far products (HBM-bound) and the last round of its window
  // launches overlap the other half's window launches (bound by the serial
  // line solves).
  const bool two = pl.sweep_side != nullptr && g.B >= 2;
  const int bh = two ? g.B / 2 : g.B;
  const int64_t rh = (int64_t)bh * g.F * g.sy;   // first row of the second half
  hipStream_t s2 = two ? pl.sweep_side : s;
  if (two) {
    hipEventRecord(pl.sweep_fork, s);
    hipStreamWaitEvent(s2, pl.sweep_fork, 0);
  }
  auto far = [&](hipStream_t st, int64_t ra, int64_t rb, int klo, int khi) {
    const unsigned tiles = (unsigned)((rb - ra + 127) / 128);
    k_sweep_far<true><<<dim3(tiles, SWEEP_WINDOW / FAR_NW), NT, 0, st>>>(
        (float*)spec, (const unsigned short*)op.tfar, pl.d_lam, rb, g.F, g.sx, g.sy, klo, khi, pl.d_rmax,
        op.tfar_inv, ra);
  };
  for (int khi = g.sx; khi > 0; khi -= SWEEP_WINDOW) {
    const int klo = khi - SWEEP_WINDOW;
    if (khi < g.sx) far(s, 0, rh, klo, khi);
    launch<float>(pl, op, (float*)spec, s, klo, khi, 0, bh);
    if (two) {
      if (khi < g.sx) far(s2, rh, rows, klo, khi);
      launch<float>(pl, op, (float*)spec, s2, klo, khi, bh, g.B - bh);
    }
  }
  if (two) {
    hipEventRecord(pl.sweep_join, s2);
    hipStreamWaitEvent(s, pl.sweep_join, 0);
  }
}

}  // namespace pd
