// Step-(b) of the ParaDiag-II preconditioner (eq1.3, eq2.12): for every
// frequency n the complex shifted spatial system (lambda1_n I + lambda2_n K) S2_n = S1_n.
//
// After the x-direction transform (see kernels_gemm.hip) the 2D system
// decouples -- exactly when K_x is symmetric (sine basis, T diagonal) and by
// back-substitution over x-modes when K_x is non-normal (Schur basis, T upper
// triangular) -- into complex tridiagonal systems along y, one per
// (right-hand side, frequency, x-mode):
//
//   [(lambda1_n + lambda2_n T_kk) I + lambda2_n K_y] w_k = r_k - lambda2_n sum_{j>k} T_kj w_j.
//
// In 1D the whole of Step-(b) is one tridiagonal system per frequency.
//
// Line solver (one wave64 segment of P lanes per line, R rows per lane, P*R >=
// line length): every lane eliminates its chunk of R rows so that each row is
// expressed through the chunk's first and last unknowns (a Thomas-like sweep
// forward and backward), the chunk boundary unknowns form a tridiagonal
// system of size P in the last-row unknowns, solved by parallel cyclic
// reduction across lanes with shuffles, and the lanes finish their rows.
// No pivoting, as in the sequential Thomas algorithm.
//
// Memory: a workgroup stages a tile of TK consecutive x-modes by all rows in
// LDS (coalesced rows in HBM, one read and one write per element), padded so
// the chunk-strided lane accesses are bank-conflict free.

#include "internal.h"

namespace pd {
namespace {

template <typename T> struct Cx { T x, y; };

template <typename T> __device__ __forceinline__ Cx<T> cz() { return Cx<T>{(T)0, (T)0}; }
template <typename T> __device__ __forceinline__ Cx<T> c1() { return Cx<T>{(T)1, (T)0}; }
template <typename T> __device__ __forceinline__ Cx<T> mul(Cx<T> a, Cx<T> b) {
  return Cx<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ Cx<T> sub(Cx<T> a, Cx<T> b) {
  return Cx<T>{a.x - b.x, a.y - b.y};
}
template <typename T> __device__ __forceinline__ Cx<T> neg(Cx<T> a) { return Cx<T>{-a.x, -a.y}; }
template <typename T> __device__ __forceinline__ Cx<T> rcp(Cx<T> a) {
  T d = (T)1 / (a.x * a.x + a.y * a.y);
  return Cx<T>{a.x * d, -a.y * d};
}
template <typename T> __device__ __forceinline__ Cx<T> shup(Cx<T> v, int d, int w) {
  return Cx<T>{__shfl_up(v.x, d, w), __shfl_up(v.y, d, w)};
}
template <typename T> __device__ __forceinline__ Cx<T> shdn(Cx<T> v, int d, int w) {
  return Cx<T>{__shfl_down(v.x, d, w), __shfl_down(v.y, d, w)};
}
template <typename T> __device__ __forceinline__ Cx<T> fromd(double2 v) {
  return Cx<T>{(T)v.x, (T)v.y};
}

// Solve a x_{i-1} + b x_i + c x_{i+1} = d_i, i < N (rows >= N are identity),
// for the line owned by the P-lane segment containing this lane.  d holds the
// lane's rows p*R .. p*R+R-1 on entry and the solution on exit.  Every lane
// of the wave must call this (shuffles).
template <typename T, int R, int P>
__device__ void tri_wave(Cx<T> (&d)[R], Cx<T> a, Cx<T> b, Cx<T> c, int N, int p) {
  static_assert(R >= 3, "chunk must hold at least 3 rows");
  const int row0 = p * R;
  Cx<T> aa[R], cc[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const bool real_row = (row0 + i) < N;
    Cx<T> ai = real_row ? a : cz<T>();
    Cx<T> bi = real_row ? b : c1<T>();
    Cx<T> ci = real_row ? c : cz<T>();
    if (!real_row) d[i] = cz<T>();
    if (i < 2) {
      Cx<T> inv = rcp(bi);
      aa[i] = mul(ai, inv);
      cc[i] = mul(ci, inv);
      d[i] = mul(d[i], inv);
    } else {
      Cx<T> inv = rcp(sub(bi, mul(ai, cc[i - 1])));
      aa[i] = neg(mul(mul(ai, aa[i - 1]), inv));
      cc[i] = mul(ci, inv);
      d[i] = mul(sub(d[i], mul(ai, d[i - 1])), inv);
    }
  }
  // rows 1..R-2 in terms of the chunk's first (x_s) and last (x_e) unknowns
#pragma unroll
  for (int i = R - 3; i >= 1; --i) {
    d[i] = sub(d[i], mul(cc[i], d[i + 1]));
    aa[i] = sub(aa[i], mul(cc[i], aa[i + 1]));
    cc[i] = neg(mul(cc[i], cc[i + 1]));
  }
  // first row: x_s + aB x_{s-1} + gB x_e = dB
  Cx<T> inv = rcp(sub(c1<T>(), mul(cc[0], aa[1])));
  Cx<T> aB = mul(aa[0], inv);
  Cx<T> gB = neg(mul(mul(cc[0], cc[1]), inv));
  Cx<T> dB = mul(sub(d[0], mul(cc[0], d[1])), inv);
  // last row: x_e + aA x_s + gA x_{e+1} = dA
  Cx<T> aA = aa[R - 1], gA = cc[R - 1], dA = d[R - 1];
  Cx<T> aBn = shdn(aB, 1, P), gBn = shdn(gB, 1, P), dBn = shdn(dB, 1, P);
  if (p == P - 1) { aBn = cz<T>(); gBn = cz<T>(); dBn = cz<T>(); }
  // eliminate the first-row unknowns: tridiagonal system in x_e across lanes
  Cx<T> A = (p == 0) ? cz<T>() : neg(mul(aA, aB));
  Cx<T> Bc = sub(sub(c1<T>(), mul(aA, gB)), mul(gA, aBn));
  Cx<T> Cc = neg(mul(gA, gBn));
  Cx<T> D = sub(sub(dA, mul(aA, dB)), mul(gA, dBn));
#pragma unroll
  for (int s = 1; s < P; s <<= 1) {
    Cx<T> Am = shup(A, s, P), Bm = shup(Bc, s, P), Cm = shup(Cc, s, P), Dm = shup(D, s, P);
    Cx<T> Ap = shdn(A, s, P), Bp = shdn(Bc, s, P), Cp = shdn(Cc, s, P), Dp = shdn(D, s, P);
    if (p < s) { Am = cz<T>(); Bm = c1<T>(); Cm = cz<T>(); Dm = cz<T>(); }
    if (p + s >= P) { Ap = cz<T>(); Bp = c1<T>(); Cp = cz<T>(); Dp = cz<T>(); }
    Cx<T> k1 = mul(A, rcp(Bm)), k2 = mul(Cc, rcp(Bp));
    A = neg(mul(k1, Am));
    Cc = neg(mul(k2, Cp));
    Bc = sub(sub(Bc, mul(k1, Cm)), mul(k2, Ap));
    D = sub(sub(D, mul(k1, Dm)), mul(k2, Dp));
  }
  Cx<T> xe = mul(D, rcp(Bc));
  Cx<T> xem = shup(xe, 1, P);
  if (p == 0) xem = cz<T>();
  Cx<T> xs = sub(sub(dB, mul(aB, xem)), mul(gB, xe));
#pragma unroll
  for (int i = 1; i < R - 1; ++i) d[i] = sub(sub(d[i], mul(aa[i], xs)), mul(cc[i], xe));
  d[0] = xs;
  d[R - 1] = xe;
}

constexpr int NT = 256;

// Padded LDS index of row y of mode column k.
__device__ __forceinline__ int lidx(int k, int y, int ldy, int R) { return k * ldy + y + y / R; }

template <typename T>
__device__ void tile_load(const T* slice, T* sre, T* sim, int k0, int nk, int TK, int sx, int sy,
                          int ldy, int R) {
  for (int e = threadIdx.x; e < sy * 2 * TK; e += NT) {
    int k = e % TK, comp = (e / TK) & 1, y = e / (2 * TK);
    T v = 0;
    if (k < nk) v = slice[(int64_t)y * 2 * sx + comp * sx + k0 + k];
    (comp ? sim : sre)[lidx(k, y, ldy, R)] = v;
  }
}

template <typename T>
__device__ void tile_store(T* slice, const T* sre, const T* sim, int k0, int nk, int TK, int sx,
                           int sy, int ldy, int R) {
  for (int e = threadIdx.x; e < sy * 2 * TK; e += NT) {
    int k = e % TK, comp = (e / TK) & 1, y = e / (2 * TK);
    if (k < nk) slice[(int64_t)y * 2 * sx + comp * sx + k0 + k] = (comp ? sim : sre)[lidx(k, y, ldy, R)];
  }
}

// Solve the line of tile column k with this wave's segment (all lanes call).
template <typename T, int R, int P>
__device__ void solve_tile_line(T* sre, T* sim, int k, bool active, Cx<T> a, Cx<T> b, Cx<T> c,
                                int sy, int ldy, int p) {
  Cx<T> d[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    int idx = k * ldy + p * (R + 1) + i;
    d[i] = active ? Cx<T>{sre[idx], sim[idx]} : cz<T>();
  }
  if (!active) { a = cz<T>(); b = c1<T>(); c = cz<T>(); }
  tri_wave<T, R, P>(d, a, b, c, sy, p);
  if (active) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      int idx = k * ldy + p * (R + 1) + i;
      sre[idx] = d[i].x;
      sim[idx] = d[i].y;
    }
  }
}

// Independent lines (1D, or 2D with a diagonal x-mode matrix T).
template <typename T, int R, int P>
__global__ __launch_bounds__(NT) void k_line_solve(T* __restrict__ spec, const double2* __restrict__ lam,
                                                   const double2* __restrict__ tk, double lo, double di,
                                                   double up, int F, int sx, int sy, int TK, int ldy) {
  extern __shared__ __align__(16) unsigned char smraw[];
  T* sre = reinterpret_cast<T*>(smraw);
  T* sim = sre + TK * ldy;
  const int k0 = blockIdx.x * TK, n = blockIdx.y, b = blockIdx.z;
  const int nk = min(TK, sx - k0);
  T* slice = spec + ((int64_t)b * F + n) * sy * 2 * sx;
  tile_load(slice, sre, sim, k0, nk, TK, sx, sy, ldy, R);
  __syncthreads();
  constexpr int LW = 64 / P;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = lane % P, seg = lane / P;
  const double2 l1 = lam[n], l2 = lam[F + n];
  for (int g = wave; g * LW < nk; g += NT / 64) {
    int k = g * LW + seg;
    bool active = k < nk;
    double2 t = (active && tk) ? tk[k0 + k] : double2{0.0, 0.0};
    // a = l2*lo, b = l1 + l2*(t + di), c = l2*up (float64, then rounded)
    double2 sh{t.x + di, t.y};
    Cx<T> ca{(T)(l2.x * lo), (T)(l2.y * lo)};
    Cx<T> cb{(T)(l1.x + l2.x * sh.x - l2.y * sh.y), (T)(l1.y + l2.x * sh.y + l2.y * sh.x)};
    Cx<T> cc{(T)(l2.x * up), (T)(l2.y * up)};
    solve_tile_line<T, R, P>(sre, sim, k, active, ca, cb, cc, sy, ldy, p);
  }
  __syncthreads();
  tile_store(slice, sre, sim, k0, nk, TK, sx, sy, ldy, R);
}

// Non-normal x factor: back-substitution over x-modes k = sx-1 .. 0 in blocks of
// TK modes, one workgroup per (right-hand side, frequency) slice.  Before a
// block is solved, the coupling to the already solved modes j >= end of block
// is subtracted (left-looking update with the strictly upper part of T);
// inside the block the modes are solved one after the other with rank-1
// updates of the remaining block columns in LDS.
template <typename T, typename Tc, int R, int P>
__global__ __launch_bounds__(NT) void k_schur_sweep(T* __restrict__ spec, const double2* __restrict__ lam,
                                                    const double2* __restrict__ tk,
                                                    const Tc* __restrict__ tup, double lo, double di,
                                                    double up, int F, int sx, int sy, int TK, int ldy) {
  extern __shared__ __align__(16) unsigned char smraw[];
  T* sre = reinterpret_cast<T*>(smraw);
  T* sim = sre + TK * ldy;
  const int n = blockIdx.x, b = blockIdx.y;
  T* slice = spec + ((int64_t)b * F + n) * sy * 2 * sx;
  const Tc* tre = tup;
  const Tc* tim = tup + (int64_t)sx * sx;
  const double2 l1 = lam[n], l2 = lam[F + n];
  const T l2r = (T)l2.x, l2i = (T)l2.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = lane % P;
  const int nblk = (sx + TK - 1) / TK;
  for (int kb = nblk - 1; kb >= 0; --kb) {
    const int k0 = kb * TK, nk = min(TK, sx - k0), kend = k0 + nk;
    tile_load(slice, sre, sim, k0, nk, TK, sx, sy, ldy, R);
    __syncthreads();
    // left-looking update from the solved modes j >= kend
    if (kend < sx) {
      for (int y = threadIdx.x; y < sy; y += NT) {
        T accr[16], acci[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) { accr[q] = 0; acci[q] = 0; }
        const T* wr = slice + (int64_t)y * 2 * sx;
        const T* wi = wr + sx;
        for (int j = kend; j < sx; ++j) {
          T xr = wr[j], xi = wi[j];
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            if (q < nk) {
              T tr = (T)tre[(int64_t)(k0 + q) * sx + j], ti = (T)tim[(int64_t)(k0 + q) * sx + j];
              accr[q] += tr * xr - ti * xi;
              acci[q] += tr * xi + ti * xr;
            }
          }
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          if (q < nk) {
            int idx = lidx(q, y, ldy, R);
            // r -= l2 * acc
            sre[idx] -= l2r * accr[q] - l2i * acci[q];
            sim[idx] -= l2r * acci[q] + l2i * accr[q];
          }
        }
      }
      __syncthreads();
    }
    for (int q = nk - 1; q >= 0; --q) {
      if (wave == 0) {
        const int seg = lane / P;
        bool active = (seg == 0);
        double2 t = tk[k0 + q];
        double2 sh{t.x + di, t.y};
        Cx<T> ca{(T)(l2.x * lo), (T)(l2.y * lo)};
        Cx<T> cb{(T)(l1.x + l2.x * sh.x - l2.y * sh.y), (T)(l1.y + l2.x * sh.y + l2.y * sh.x)};
        Cx<T> cc{(T)(l2.x * up), (T)(l2.y * up)};
        solve_tile_line<T, R, P>(sre, sim, q, active, ca, cb, cc, sy, ldy, p);
      }
      __syncthreads();
      if (q > 0) {
        // columns q' < q of the block: r_q' -= l2 * T[k0+q'][k0+q] * w_q
        for (int e = threadIdx.x; e < q * sy; e += NT) {
          int qq = e / sy, y = e - qq * sy;
          T tr = (T)tre[(int64_t)(k0 + qq) * sx + k0 + q], ti = (T)tim[(int64_t)(k0 + qq) * sx + k0 + q];
          T cr = l2r * tr - l2i * ti, ci = l2r * ti + l2i * tr;
          int src = lidx(q, y, ldy, R), dst = lidx(qq, y, ldy, R);
          T xr = sre[src], xi = sim[src];
          sre[dst] -= cr * xr - ci * xi;
          sim[dst] -= cr * xi + ci * xr;
        }
        __syncthreads();
      }
    }
    tile_store(slice, sre, sim, k0, nk, TK, sx, sy, ldy, R);
    __threadfence_block();
    __syncthreads();
  }
}

struct LineShape { int R, P, TK, ldy; size_t lds; };

LineShape line_shape(const Plan& pl, bool sweep) {
  const Geom& g = pl.g;
  int R = 4;
  while (R * 64 < g.sy) R <<= 1;
  int P = 1;
  while (P * R < g.sy) P <<= 1;
  int ldy = P * (R + 1);
  if ((ldy & 1) == 0) ldy += 1;
  size_t esz = (pl.prec == Prec::F64) ? 8 : 4;
  int TK = sweep ? 16 : 16;
  while (TK > 1 && (size_t)2 * TK * ldy * esz > 80 * 1024) TK >>= 1;
  while (TK > 1 && TK / 2 >= g.sx) TK >>= 1;
  return LineShape{R, P, TK, ldy, (size_t)2 * TK * ldy * esz};
}

template <typename T>
void launch_lines(const Plan& pl, const SpaceOp& op, T* spec, hipStream_t s) {
  const Geom& g = pl.g;
  LineShape sh = line_shape(pl, false);
  dim3 grid((g.sx + sh.TK - 1) / sh.TK, g.F, g.B);
#define PD_LINE(RR, PP)                                                                           \
  if (sh.R == RR && sh.P == PP) {                                                                 \
    hipFuncSetAttribute((const void*)k_line_solve<T, RR, PP>,                                     \
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds);                 \
    k_line_solve<T, RR, PP><<<grid, NT, sh.lds, s>>>(spec, pl.d_lam, op.tk, op.lo, op.di, op.up,  \
                                                     g.F, g.sx, g.sy, sh.TK, sh.ldy);             \
    return;                                                                                       \
  }
  PD_LINE(4, 1) PD_LINE(4, 2) PD_LINE(4, 4) PD_LINE(4, 8) PD_LINE(4, 16) PD_LINE(4, 32)
  PD_LINE(4, 64) PD_LINE(8, 64) PD_LINE(16, 64) PD_LINE(32, 64)
#undef PD_LINE
}

template <typename T, typename Tc>
void launch_sweep(const Plan& pl, const SpaceOp& op, T* spec, hipStream_t s) {
  const Geom& g = pl.g;
  LineShape sh = line_shape(pl, true);
  dim3 grid(g.F, g.B);
#define PD_SWEEP(RR, PP)                                                                          \
  if (sh.R == RR && sh.P == PP) {                                                                 \
    hipFuncSetAttribute((const void*)k_schur_sweep<T, Tc, RR, PP>,                                \
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds);                 \
    k_schur_sweep<T, Tc, RR, PP><<<grid, NT, sh.lds, s>>>(spec, pl.d_lam, op.tk,                 \
                                                          (const Tc*)op.tup, op.lo, op.di, op.up, \
                                                          g.F, g.sx, g.sy, sh.TK, sh.ldy);        \
    return;                                                                                       \
  }
  PD_SWEEP(4, 1) PD_SWEEP(4, 2) PD_SWEEP(4, 4) PD_SWEEP(4, 8) PD_SWEEP(4, 16) PD_SWEEP(4, 32)
  PD_SWEEP(4, 64) PD_SWEEP(8, 64) PD_SWEEP(16, 64) PD_SWEEP(32, 64)
#undef PD_SWEEP
}

}  // namespace

void line_solve(const Plan& pl, const SpaceOp& op, void* spec, hipStream_t s) {
  if (pl.prec == Prec::F64) launch_lines<double>(pl, op, (double*)spec, s);
  else launch_lines<float>(pl, op, (float*)spec, s);
}

void schur_sweep(const Plan& pl, const SpaceOp& op, void* spec, hipStream_t s) {
  // the T table is stored in the working precision of the line solves
  if (pl.prec == Prec::F64) launch_sweep<double, double>(pl, op, (double*)spec, s);
  else launch_sweep<float, float>(pl, op, (float*)spec, s);
}

}  // namespace pd
