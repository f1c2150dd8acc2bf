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

#include "tri_device.h"

namespace pd {
namespace {

using namespace tri;

// Independent lines (1D, or 2D with a diagonal x-mode matrix T).  TKV > 0:
// tiles of TKV modes copied with 16-byte vectors (sx % 4 == 0), the last
// partial tile element-wise; TKV = 0: element-wise copies of TK modes.
template <typename T, int R, int P, int TKV>
__global__ __launch_bounds__(NT) void k_line_solve(T* __restrict__ spec, const double2* __restrict__ lam,
                                                   const double2* __restrict__ tk, double lo, double di,
                                                   double up, int F, int sx, int sy, int TK, int ldy) {
  extern __shared__ __align__(16) unsigned char smraw[];
  T* sre = reinterpret_cast<T*>(smraw);
  T* sim = sre + TK * ldy;
  const BlockPos bp = xcd_block();
  const int k0 = bp.x * TK, n = bp.y, b = bp.z;
  const int nk = min(TK, sx - k0);
  T* slice = spec + ((int64_t)b * F + n) * sy * 2 * sx;
  bool vec = false;
  if constexpr (TKV > 0) vec = nk == TKV;
  if constexpr (TKV > 0) {
    if (vec) tile_load_vec<T, TKV, R * P, NT>(slice, sre, sim, k0, sx, sy, ldy, R, (int)threadIdx.x, NT);
    else tile_load(slice, sre, sim, k0, nk, TK, sx, sy, ldy, R);
  } else {
    tile_load(slice, sre, sim, k0, nk, TK, sx, sy, ldy, R);
  }
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
  if constexpr (TKV > 0) {
    if (vec) tile_store_vec<T, TKV, R * P>(slice, sre, sim, k0, sx, sy, ldy, R, (int)threadIdx.x, NT);
    else tile_store(slice, sre, sim, k0, nk, TK, sx, sy, ldy, R);
  } else {
    tile_store(slice, sre, sim, k0, nk, TK, sx, sy, ldy, R);
  }
}

struct LineShape { int R, P, TK, ldy; size_t lds; };

LineShape line_shape(const Plan& pl) {
  const Geom& g = pl.g;
  // R rows per lane: at least 8 from 256 rows on (fewer lanes per line, fewer
  // cyclic-reduction levels: measured 0.42 -> 0.30 ms per launch at 256 rows)
  int R = 4;
  while (R * 64 < g.sy) R <<= 1;
  if (g.sy >= 256 && R < 8) R = 8;
  int P = 1;
  while (P * R < g.sy) P <<= 1;
  int ldy = P * (R + 1);
  if ((ldy & 1) == 0) ldy += 1;
  size_t esz = (pl.prec == Prec::F64) ? 8 : 4;
  // Waves per SIMD that the kernel's registers allow (compiler-reported VGPRs
  // of the instantiations: float 70 / 117 / 214 at R = 4 / 8 / 16, double
  // 98 (P = 1) / 168 / 248 at R = 4 / 4 / 8).  A workgroup is one wave per
  // SIMD, so the tile is sized for that many workgroups per CU: the loads of
  // some overlap the solves of the others.
  int occ;
  if (pl.prec == Prec::F64) occ = (R == 4) ? (P == 1 ? 4 : 3) : (R == 8 ? 2 : 1);
  else occ = (R == 4) ? 7 : (R == 8 ? 4 : (R == 16 ? 2 : 1));
  const size_t lim = std::min<size_t>(80 * 1024, (size_t)158 * 1024 / occ);
  int TK = 16;
  while (TK > 4 && (size_t)2 * TK * ldy * esz > lim) TK >>= 1;
  while (TK > 1 && (size_t)2 * TK * ldy * esz > 158 * 1024) TK >>= 1;
  while (TK > 1 && TK / 2 >= g.sx) TK >>= 1;
  return LineShape{R, P, TK, ldy, (size_t)2 * TK * ldy * esz};
}

template <typename T>
void launch_lines(const Plan& pl, const SpaceOp& op, T* spec, hipStream_t s) {
  const Geom& g = pl.g;
  LineShape sh = line_shape(pl);
  dim3 grid((g.sx + sh.TK - 1) / sh.TK, g.F, g.B);
  const bool vec = (g.sx % 4) == 0;
#define PD_LINE_K(RR, PP, TKV)                                                                    \
  {                                                                                               \
    lds_limit((const void*)k_line_solve<T, RR, PP, TKV>, sh.lds);                                 \
    k_line_solve<T, RR, PP, TKV><<<grid, NT, sh.lds, s>>>(spec, pl.d_lam, op.tk, op.lo, op.di,    \
                                                          op.up, g.F, g.sx, g.sy, sh.TK, sh.ldy); \
    return;                                                                                       \
  }
#define PD_LINE(RR, PP)                                                                           \
  if (sh.R == RR && sh.P == PP) {                                                                 \
    if (vec && sh.TK == 16) PD_LINE_K(RR, PP, 16)                                                 \
    if (vec && sh.TK == 8) PD_LINE_K(RR, PP, 8)                                                   \
    PD_LINE_K(RR, PP, 0)                                                                          \
  }
  PD_LINE(4, 1) PD_LINE(4, 2) PD_LINE(4, 4) PD_LINE(4, 8) PD_LINE(4, 16) PD_LINE(4, 32)
  PD_LINE(4, 64) PD_LINE(8, 64) PD_LINE(16, 64) PD_LINE(32, 64) PD_LINE(8, 32)
#undef PD_LINE
#undef PD_LINE_K
}

}  // namespace

void line_solve(const Plan& pl, const SpaceOp& op, void* spec, hipStream_t s) {
  if (pl.prec == Prec::F64) launch_lines<double>(pl, op, (double*)spec, s);
  else launch_lines<float>(pl, op, (float*)spec, s);
}


}  // namespace pd
