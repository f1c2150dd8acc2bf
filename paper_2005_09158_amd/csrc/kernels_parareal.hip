// Fine propagation of the ParaDiag-II parareal variant (Section 2.2.2), one
// space dimension.
//
// Each parareal iteration first propagates every coarse interval with the
// fine integrator from the previous iterate: Ut_{n+1} = F(U_n), U_0 = U0, F =
// J backward Euler steps of dt = dT / J, i.e. J solves with the constant
// tridiagonal matrix (I + dt K).  The Nt * batch propagations are independent:
// one wave per line, R rows per lane, the J solves done in registers with the
// one-wave tridiagonal solver (chunk elimination per lane, then cyclic
// reduction across the 64 lanes).  The kernel then writes the right-hand side
// of the alpha-periodic coarse-grid correction directly,
//
//   b_n = (I/dT + K) Ut_n - (n == 1 ? alpha U_Nt : U_{n-1}) / dT,
//
// where K Ut_n comes from the last fine step itself: (I + dt K) Ut = U_{J-1}
// gives K Ut = (U_{J-1} - Ut) / dt, so no stencil pass is needed.

#include "tri_device.h"

namespace pd {
namespace {

constexpr int NT = 256;   // 4 waves, one line each

template <int R>
__global__ __launch_bounds__(NT) void k_parareal_fine(const double* __restrict__ U0,
                                                      const double* __restrict__ uprev,
                                                      double* __restrict__ b, int Nt, int nx, int lines,
                                                      int J, double dt, double dT, double alpha,
                                                      double lo, double di, double up) {
  using C = tri::Cx<double>;
  const int lane = threadIdx.x & 63;
  const int line = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  if (line >= lines) return;   // whole waves leave together (tri_wave shuffles within a wave)
  const int bi = line / Nt, n = line - bi * Nt;
  const int64_t N1 = (int64_t)Nt * nx;
  const double* start = (n == 0) ? U0 + (int64_t)bi * nx : uprev + bi * N1 + (int64_t)(n - 1) * nx;
  const int row0 = lane * R;
  C d[R], prev[R];
  double st[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int r = row0 + i;
    st[i] = r < nx ? start[r] : 0.0;
    d[i] = C{st[i], 0.0};
  }
  const C a{dt * lo, 0.0}, bb{1.0 + dt * di, 0.0}, c{dt * up, 0.0};
  for (int j = 0; j < J; ++j) {
#pragma unroll
    for (int i = 0; i < R; ++i) prev[i] = d[i];
    tri::tri_wave<double, R, 64>(d, a, bb, c, nx, lane);
  }
  // the shift of row n: alpha U_Nt for the first interval, else the start value
  const double* shift = (n == 0) ? uprev + bi * N1 + (int64_t)(Nt - 1) * nx : nullptr;
  double* out = b + bi * N1 + (int64_t)n * nx;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int r = row0 + i;
    if (r >= nx) continue;
    const double ut = d[i].x, kut = (prev[i].x - ut) / dt;
    const double sh = (n == 0) ? alpha * shift[r] : st[i];
    out[r] = ut / dT + kut - sh / dT;
  }
}

}  // namespace

void parareal_fine(const Plan& pl, const double* U0, const double* uprev, double* b, int J, double alpha,
                   hipStream_t s) {
  const Geom& g = pl.g;
  const int lines = g.B * g.nt;
  const double dT = pl.p.T / g.nt, dt = dT / J;
  const SpaceOp& op = pl.op[0];
  const dim3 grid((unsigned)((lines + NT / 64 - 1) / (NT / 64)));
  const int nx = g.nx;
#define PD_PF(RR) k_parareal_fine<RR><<<grid, NT, 0, s>>>(U0, uprev, b, g.nt, nx, lines, J, dt, dT, alpha, \
                                                          op.lo, op.di, op.up)
  if (nx <= 64 * 4) PD_PF(4);
  else if (nx <= 64 * 8) PD_PF(8);
  else if (nx <= 64 * 16) PD_PF(16);
  else PD_PF(32);
#undef PD_PF
}

}  // namespace pd
