// float64 kernels around the preconditioner: the all-at-once matvec (eq1.1),
// the right-hand side (eq2.5, eq3.2) and its transpose, and the Krylov
// vector operations of flexible GMRES.
//
// Matvec: y_n = sum_k c1_k u_{n-k} + K (sum_k c2_k u_{n-k}), u_{m<1} = 0,
// with the 5-point stencil of K evaluated on the fly.  A workgroup owns 256
// spatial points of one right-hand side and a chunk of consecutive time
// steps; each thread marches through the chunk keeping the last L values of
// u and K u of its point in registers, so u is read once (plus the L-1 steps
// before the chunk) and y written once.  The transposed operator marches
// backwards in time with the transposed stencil.
//
// Krylov reductions are deterministic: per-workgroup partial sums in a fixed
// order, then a fixed-order reduction over workgroups.  No atomics.

#include "internal.h"

namespace pd {
namespace {

constexpr int NT = 256;
constexpr int MAXV = 33;  // vectors per multi-dot (restart <= 32)

// Sum over the workgroup, valid in thread 0: wave reduction, then across the
// 4 waves in a fixed order.  Every thread of the workgroup must call it.
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0) t = red[0] + red[1] + red[2] + red[3];
  return t;
}

struct Stencil {
  double xl, xu, yl, yu, d;  // K u = xl u[x-1] + xu u[x+1] + yl u[y-1] + yu u[y+1] + d u
};

template <typename Tin>
__device__ __forceinline__ double ld(const Tin* p) { return (double)*p; }

// V consecutive values from p (16-byte aligned when V > 1) as doubles.
template <typename Tin, int V>
__device__ __forceinline__ void ldv(const Tin* p, double (&o)[V]) {
  if constexpr (V == 1) {
    o[0] = (double)*p;
  } else if constexpr (sizeof(Tin) == 4) {
#pragma unroll
    for (int h = 0; h < V; h += 4) {
      const float4 q = *reinterpret_cast<const float4*>(p + h);
      o[h] = q.x; o[h + 1] = q.y; o[h + 2] = q.z; o[h + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int h = 0; h < V; h += 2) {
      const double2 q = *reinterpret_cast<const double2*>(p + h);
      o[h] = q.x; o[h + 1] = q.y;
    }
  }
}

// u and K u at the V points x .. x+V-1 of row y (x % V == 0, nx % V == 0).
// Each point's stencil terms are added in the order centre, x-1, x+1, y-1, y+1.
template <typename Tin, int V>
__device__ __forceinline__ void points_and_k(const Tin* un, int x, int y, int nx, int ny,
                                             const Stencil& st, double (&u)[V], double (&ku)[V]) {
  // Every load is issued unconditionally (a missing neighbour reads the
  // point itself and is then left out), so that they are all in flight
  // together instead of one after another behind divergent branches.
  const Tin* c = un + (int64_t)y * nx + x;
  const int dup = y > 0 ? nx : 0, ddn = y < ny - 1 ? nx : 0;
  const int dl = x > 0 ? 1 : 0, dr = x + V < nx ? V : V - 1;
  double up[V], dn[V];
  ldv<Tin, V>(c, u);
  ldv<Tin, V>(c - dup, up);
  ldv<Tin, V>(c + ddn, dn);
  const double lft = ld(c - dl), rgt = ld(c + dr);
#pragma unroll
  for (int v = 0; v < V; ++v) {
    double k = st.d * u[v];
    if (x + v > 0) k += st.xl * (v ? u[v - 1] : lft);
    if (x + v < nx - 1) k += st.xu * (v + 1 < V ? u[v + 1] : rgt);
    if (y > 0) k += st.yl * up[v];
    if (y < ny - 1) k += st.yu * dn[v];
    ku[v] = k;
  }
}

template <typename Tin>
__device__ __forceinline__ void point_and_k(const Tin* un, int x, int y, int nx, int ny,
                                            const Stencil& st, double& u, double& ku) {
  double uu[1], kk[1];
  points_and_k<Tin, 1>(un, x, y, nx, ny, st, uu, kk);
  u = uu[0];
  ku = kk[0];
}

// One step of the march: r = c1_0 u_0 + c2_0 K u_0 + c1_1 u_1 + ... at V
// points, y = b - r (or r), then shift the history.
template <int V>
__device__ __forceinline__ void march_step(const double (&u0)[V], const double (&k0)[V],
                                           const double (&bv)[V], bool hasb, int L, double c10,
                                           double c11, double c12, double c20, double c21,
                                           double c22, double (&u1)[V], double (&k1)[V],
                                           double (&u2)[V], double (&k2)[V], double* dst,
                                           double (&r)[V]) {
#pragma unroll
  for (int v = 0; v < V; ++v) {
    r[v] = c10 * u0[v] + c20 * k0[v] + c11 * u1[v] + c21 * k1[v];
    if (L > 2) r[v] += c12 * u2[v] + c22 * k2[v];
    if (hasb) r[v] = bv[v] - r[v];
    u2[v] = u1[v]; k2[v] = k1[v]; u1[v] = u0[v]; k1[v] = k0[v];
  }
  if (dst == nullptr) return;   // only the values (for their norm) are wanted
  if constexpr (V == 1) {
    dst[0] = r[0];
  } else {
#pragma unroll
    for (int h = 0; h < V; h += 2) *reinterpret_cast<double2*>(dst + h) = double2{r[h], r[h + 1]};
  }
}

// dir = +1: y = A u ;  dir = -1: y = A^T u (stencil already transposed by the
// caller).  V = 4: four consecutive points per thread with 16-byte row loads
// (nx % 4 == 0), which keeps four times the bytes in flight per load.
// NV != 0: also the dots of the result with the Krylov vectors V_i (i < nv;
// NV > 0 fixed, NV < 0 any nv <= MAXV), one partial sum per workgroup in
// partial[b][chunk][i], chunk = the workgroup's (x, time chunk) index --
// the first Gram-Schmidt pass without a second read of the result.
template <typename Tin, int V, int NV>
__global__ __launch_bounds__(NT) void k_matvec(const Tin* __restrict__ u, const double* __restrict__ b,
                                               double* __restrict__ yv, int Nt, int nx, int ny, int L,
                                               double c10, double c11, double c12, double c20,
                                               double c21, double c22, Stencil st, int chunk, int dir,
                                               const double* __restrict__ Vk, int64_t vstride, int nv,
                                               int sq, double* __restrict__ partial,
                                               const double* __restrict__ V0, int v0sq) {
  constexpr int NR = NV > 0 ? NV : (NV < 0 ? MAXV : 1);
  __shared__ double red[4];
  const int S = nx * ny;
  const BlockPos bp = xcd_block();   // neighbouring rows of the stencil on one L2
  const int s = (bp.x * NT + threadIdx.x) * V;
  double acc[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) acc[i] = 0.0;
  double asq = 0.0;   // y . y when sq
  double abb = 0.0;   // V_0 . V_0 when v0sq
  if (s < S) {
  const int x = s % nx, y = s / nx;
  const int64_t boff = (int64_t)bp.z * Nt * S;
  const Tin* ub = u + boff;
  double* yb = yv ? yv + boff : nullptr;   // null: y is not stored (sq only)
  const double* bb = b ? b + boff : nullptr;
  const int nbeg = bp.y * chunk;
  const int nend = min(Nt, nbeg + chunk);
  double u1[V], k1[V], u2[V], k2[V];  // history: step -1 and -2 along the march
#pragma unroll
  for (int v = 0; v < V; ++v) u1[v] = k1[v] = u2[v] = k2[v] = 0.0;
  // prologue: the L-1 steps preceding the chunk in marching order
  for (int h = L - 1; h >= 1; --h) {
    const int m = (dir > 0) ? (nbeg - h) : (nend - 1 + h);
    double uu[V], kk[V];
#pragma unroll
    for (int v = 0; v < V; ++v) uu[v] = kk[v] = 0.0;
    if (m >= 0 && m < Nt) points_and_k<Tin, V>(ub + (int64_t)m * S, x, y, nx, ny, st, uu, kk);
#pragma unroll
    for (int v = 0; v < V; ++v) { u2[v] = u1[v]; k2[v] = k1[v]; u1[v] = uu[v]; k1[v] = kk[v]; }
  }
  // dots of the values r just written (at element offset off) with V_q, and
  // with themselves when sq
  auto dots_of = [&](const double (&r)[V], int64_t off) {
    if (sq)
#pragma unroll
      for (int v = 0; v < V; ++v) asq += r[v] * r[v];
    if constexpr (NV != 0) {
      const double* Vb = Vk + boff;
#pragma unroll
      for (int q = 0; q < NR; ++q)
        if (NV > 0 || q < nv) {
          double vq[V];
          ldv<double, V>(((q == 0 && V0 != nullptr) ? V0 + boff : Vb + q * vstride) + off, vq);
#pragma unroll
          for (int v = 0; v < V; ++v) acc[q] += vq[v] * r[v];
          if (q == 0 && v0sq)
#pragma unroll
            for (int v = 0; v < V; ++v) abb += vq[v] * vq[v];
        }
    }
  };
  // two time steps per iteration, all of both steps' loads issued first (the
  // second step of an odd tail re-reads the first and is not stored)
  const int cnt = nend - nbeg;
  for (int i = 0; i < cnt; i += 2) {
    const int nA = (dir > 0) ? (nbeg + i) : (nend - 1 - i);
    const int iB = min(i + 1, cnt - 1);
    const int nB = (dir > 0) ? (nbeg + iB) : (nend - 1 - iB);
    double uA[V], kA[V], uB[V], kB[V], bA[V], bB[V];
    points_and_k<Tin, V>(ub + (int64_t)nA * S, x, y, nx, ny, st, uA, kA);
    points_and_k<Tin, V>(ub + (int64_t)nB * S, x, y, nx, ny, st, uB, kB);
    const int64_t offA = (int64_t)nA * S + s, offB = (int64_t)nB * S + s;
    if (bb) {
      ldv<double, V>(bb + offA, bA);
      ldv<double, V>(bb + offB, bB);
    }
    double rA[V], rB[V];
    march_step<V>(uA, kA, bA, bb != nullptr, L, c10, c11, c12, c20, c21, c22, u1, k1, u2, k2, yb ? yb + offA : nullptr, rA);
    dots_of(rA, offA);
    if (i + 1 < cnt) {
      march_step<V>(uB, kB, bB, bb != nullptr, L, c10, c11, c12, c20, c21, c22, u1, k1, u2, k2, yb ? yb + offB : nullptr, rB);
      dots_of(rB, offB);
    }
  }
  }  // s < S
  if (partial != nullptr) {   // nv and sq are uniform: every thread reaches the barriers
    const int chunks = gridDim.x * gridDim.y;
    double* out = partial + ((int64_t)bp.z * chunks + bp.x + (int64_t)gridDim.x * bp.y) * MAXV;
    const int ndots = NV > 0 ? NV : (NV < 0 ? nv : 0);
    if constexpr (NV != 0)
#pragma unroll
      for (int q = 0; q < NR; ++q)
        if (q < ndots) {
          const double t = block_sum(acc[q], red);
          if (threadIdx.x == 0) out[q] = t;
        }
    if (sq) {
      const double t = block_sum(asq, red);
      if (threadIdx.x == 0) out[ndots] = t;
    }
    if (v0sq) {
      const double t = block_sum(abb, red);
      if (threadIdx.x == 0) out[ndots + (sq ? 1 : 0)] = t;
    }
  }
}

// Matvec of the hybrid discretisation (Section 2.1.2): y_n = sum_{|k|<=2}
// band[n][k+2] u_{n+k} + K u_n, the time matrix B (neq2.9c) or B^2 (neq2.15)
// given by its banded rows (or those of its transpose), K by its 5-point
// stencil.  Same grid and partial-sum layout as k_matvec with no Krylov dots:
// y = b - A u when b is given, y not stored when null, and the partial sums
// of y . y in slot 0 when sq.
template <typename Tin, int V>
__global__ __launch_bounds__(NT) void k_matvec_band(const Tin* __restrict__ u, const double* __restrict__ b,
                                                    double* __restrict__ yv, int Nt, int nx, int ny,
                                                    const double* __restrict__ band, Stencil st, int chunk,
                                                    int sq, double* __restrict__ partial) {
  __shared__ double red[4];
  const int S = nx * ny;
  const BlockPos bp = xcd_block();
  const int s = (bp.x * NT + threadIdx.x) * V;
  double asq = 0.0;
  if (s < S) {
    const int x = s % nx, y = s / nx;
    const int64_t boff = (int64_t)bp.z * Nt * S;
    const Tin* ub = u + boff;
    const int nbeg = bp.y * chunk, nend = min(Nt, nbeg + chunk);
    for (int n = nbeg; n < nend; ++n) {
      double uu[V], ku[V], r[V];
      points_and_k<Tin, V>(ub + (int64_t)n * S, x, y, nx, ny, st, uu, ku);
      const double* bn = band + (int64_t)n * 5;
#pragma unroll
      for (int v = 0; v < V; ++v) r[v] = ku[v] + bn[2] * uu[v];
#pragma unroll
      for (int k = -2; k <= 2; ++k) {
        if (k == 0 || n + k < 0 || n + k >= Nt || bn[k + 2] == 0.0) continue;
        double w[V];
        ldv<Tin, V>(ub + (int64_t)(n + k) * S + s, w);
#pragma unroll
        for (int v = 0; v < V; ++v) r[v] += bn[k + 2] * w[v];
      }
      const int64_t off = boff + (int64_t)n * S + s;
      if (b) {
        double bv[V];
        ldv<double, V>(b + off, bv);
#pragma unroll
        for (int v = 0; v < V; ++v) r[v] = bv[v] - r[v];
      }
      if (yv) {
#pragma unroll
        for (int v = 0; v < V; ++v) yv[off + v] = r[v];
      }
      if (sq)
#pragma unroll
        for (int v = 0; v < V; ++v) asq += r[v] * r[v];
    }
  }
  if (partial != nullptr && sq) {
    const int chunks = gridDim.x * gridDim.y;
    double* out = partial + ((int64_t)bp.z * chunks + bp.x + (int64_t)gridDim.x * bp.y) * MAXV;
    const double t = block_sum(asq, red);
    if (threadIdx.x == 0) out[0] = t;
  }
}

// b from U0, u1, f (see paradiag_build_rhs); one thread per (n, point).
__global__ __launch_bounds__(NT) void k_rhs(const double* __restrict__ U0, const double* __restrict__ V1,
                                            const double* __restrict__ f, double* __restrict__ b,
                                            int Nt, int nx, int ny, int scheme, double dt,
                                            double theta, Stencil st) {
  const int S = nx * ny;
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int bi = blockIdx.y;
  if (e >= (int64_t)Nt * S) return;
  const int n = (int)(e / S), s = (int)(e - (int64_t)n * S);
  const int x = s % nx, y = s / nx;
  const double* u0b = U0 + (int64_t)bi * S;
  const double* fb = f ? f + (int64_t)bi * (Nt + 1) * S : nullptr;
  double r = 0.0;
  double uu, ku;
  if (scheme == PD_HYBRID || scheme == PD_HYBRID_WAVE) {
    // rows n = 1 .. Nt carry f(t_n); the first-order form adds U0/(2 dt) to
    // row 1, the second-order form u1/(2 dt) to row 1 and -U0/(4 dt^2) to row 2
    if (fb) r = fb[(int64_t)(n + 1) * S + s];
    if (scheme == PD_HYBRID) {
      if (n == 0) r += u0b[s] / (2.0 * dt);
    } else {
      if (n == 0 && V1) r += V1[(int64_t)bi * S + s] / (2.0 * dt);
      if (n == 1) r -= u0b[s] / (4.0 * dt * dt);
    }
  } else if (scheme != PD_LEAPFROG) {
    if (n == 0) {
      point_and_k(u0b, x, y, nx, ny, st, uu, ku);
      r = uu / dt - (1.0 - theta) * ku;
    }
    if (fb) r += theta * fb[(int64_t)(n + 1) * S + s] + (1.0 - theta) * fb[(int64_t)n * S + s];
  } else {
    if (n == 0) {
      point_and_k(u0b, x, y, nx, ny, st, uu, ku);
      r = uu / (dt * dt);
      if (V1) {
        double vv, kv;
        point_and_k(V1 + (int64_t)bi * S, x, y, nx, ny, st, vv, kv);
        r += vv / dt + 0.5 * dt * kv;
      }
      if (fb) r += 0.5 * fb[s];
    } else if (n == 1) {
      point_and_k(u0b, x, y, nx, ny, st, uu, ku);
      r = -uu / (dt * dt) - 0.5 * ku;
      if (fb) r += fb[(int64_t)S + s];
    } else {
      if (fb) r = fb[(int64_t)n * S + s];
    }
  }
  b[(int64_t)bi * Nt * S + e] = r;
}

// Transpose of the right-hand side map; st is the transposed stencil.
// One thread per (level n in 0..Nt, point): writes gf[n] and, at n == 0, gU0 / gu1.
__global__ __launch_bounds__(NT) void k_rhs_t(const double* __restrict__ lam, double* __restrict__ gU0,
                                              double* __restrict__ gu1, double* __restrict__ gf,
                                              int Nt, int nx, int ny, int scheme, double dt,
                                              double theta, Stencil st) {
  const int S = nx * ny;
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int bi = blockIdx.y;
  if (e >= (int64_t)(Nt + 1) * S) return;
  const int n = (int)(e / S), s = (int)(e - (int64_t)n * S);
  const int x = s % nx, y = s / nx;
  const double* lb = lam + (int64_t)bi * Nt * S;   // lam_1 .. lam_Nt at rows 0..Nt-1
  auto L = [&](int m) { return (m >= 1 && m <= Nt) ? lb[(int64_t)(m - 1) * S + s] : 0.0; };
  if (scheme != PD_LEAPFROG) {
    if (gf) gf[(int64_t)bi * (Nt + 1) * S + e] = theta * L(n) + (1.0 - theta) * L(n + 1);
    if (n == 0) {
      double l1, kl1;
      point_and_k(lb, x, y, nx, ny, st, l1, kl1);
      gU0[(int64_t)bi * S + s] = l1 / dt - (1.0 - theta) * kl1;
      if (gu1) gu1[(int64_t)bi * S + s] = 0.0;
    }
  } else {
    if (gf) {
      double v = (n == 0) ? 0.5 * L(1) : (n < Nt ? L(n + 1) : 0.0);
      gf[(int64_t)bi * (Nt + 1) * S + e] = v;
    }
    if (n == 0) {
      double l1, kl1, l2 = 0, kl2 = 0;
      point_and_k(lb, x, y, nx, ny, st, l1, kl1);
      if (Nt > 1) point_and_k(lb + S, x, y, nx, ny, st, l2, kl2);
      gU0[(int64_t)bi * S + s] = l1 / (dt * dt) - l2 / (dt * dt) - 0.5 * kl2;
      if (gu1) gu1[(int64_t)bi * S + s] = l1 / dt + 0.5 * dt * kl1;
    }
  }
}


// partial[b][chunk][0] = sum over the chunk of (u - v)^2, [1] = sum of u^2
// (the relative change of a fixed-point iterate, e.g. parareal's)
__global__ __launch_bounds__(NT) void k_diff_sq(const double* __restrict__ u, const double* __restrict__ v,
                                                double* __restrict__ partial, int64_t N1, int chunks) {
  __shared__ double red[4];
  const int b = blockIdx.y, c = blockIdx.x;
  const int64_t len = (N1 + chunks - 1) / chunks, beg = (int64_t)c * len, end = min(N1, beg + len);
  const double* ub = u + (int64_t)b * N1;
  const double* vb = v + (int64_t)b * N1;
  double dd = 0.0, uu = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += NT) {
    const double x = ub[i], y = x - vb[i];
    dd += y * y;
    uu += x * x;
  }
  double* out = partial + ((int64_t)b * chunks + c) * MAXV;
  const double t0 = block_sum(dd, red);
  if (threadIdx.x == 0) out[0] = t0;
  const double t1 = block_sum(uu, red);
  if (threadIdx.x == 0) out[1] = t1;
}

// Nonlinear problems U' + K U + g(U) = 0, g(u) = k1 u + k2 u^2 + k3 u^3
// (eq1.4): the nonlinear part of the residual, r_n -= c2_0 g(U_n) + c2_1
// g(U_{n-1}) (n >= 1; row 1's U_0 term sits in b), with partial sums of r^2
// (slot 0) and of g'(U) (slot 1, for the averaged Jacobian) per chunk.
struct CubicG {
  double k1, k2, k3;
  __device__ __forceinline__ double g(double u) const { return u * (k1 + u * (k2 + u * k3)); }
  __device__ __forceinline__ double dg(double u) const { return k1 + u * (2.0 * k2 + 3.0 * k3 * u); }
};

__global__ __launch_bounds__(NT) void k_nl_residual(const double* __restrict__ u, double* __restrict__ r,
                                                    int64_t N1, int S, double c20, double c21, CubicG gc,
                                                    double* __restrict__ partial, int chunks) {
  __shared__ double red[4];
  const int b = blockIdx.y, c = blockIdx.x;
  const int64_t len = (N1 + chunks - 1) / chunks, beg = (int64_t)c * len, end = min(N1, beg + len);
  const double* ub = u + (int64_t)b * N1;
  double* rb = r + (int64_t)b * N1;
  double rr = 0.0, gs = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += NT) {
    const double x = ub[i];
    double v = rb[i] - c20 * gc.g(x);
    if (c21 != 0.0 && i >= S) v -= c21 * gc.g(ub[i - S]);
    rb[i] = v;
    rr += v * v;
    gs += gc.dg(x);
  }
  double* out = partial + ((int64_t)b * chunks + c) * MAXV;
  const double t0 = block_sum(rr, red);
  if (threadIdx.x == 0) out[0] = t0;
  const double t1 = block_sum(gs, red);
  if (threadIdx.x == 0) out[1] = t1;
}

// b_1 -= w g(U0) (the known initial state's share of row 1; w = 1 - theta)
__global__ __launch_bounds__(NT) void k_nl_rhs_fix(const double* __restrict__ U0, double* __restrict__ b,
                                                   int S, int64_t N1, double w, CubicG gc) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= S) return;
  b[(int64_t)blockIdx.y * N1 + e] -= w * gc.g(U0[(int64_t)blockIdx.y * S + e]);
}

// u_n = U0 for every n (the starting iterate), and the gather of the last
// time step of a block of rows: dst[b] = src[b][nt-1]
__global__ __launch_bounds__(NT) void k_bcast_rows(const double* __restrict__ U0, double* __restrict__ u,
                                                   int S, int nt) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= (int64_t)nt * S) return;
  u[(int64_t)blockIdx.y * nt * S + e] = U0[(int64_t)blockIdx.y * S + e % S];
}
__global__ __launch_bounds__(NT) void k_last_rows(const double* __restrict__ src, double* __restrict__ dst,
                                                  int S, int nt) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= S) return;
  dst[(int64_t)blockIdx.y * S + e] = src[((int64_t)blockIdx.y * nt + nt - 1) * S + e];
}

// Multi-dot and update kernels, templated on the number of Krylov vectors
// (NV <= 8; larger counts use the generic predicated form).  Each thread
// handles pairs of consecutive doubles (16-byte loads); a workgroup owns one
// contiguous chunk of one right-hand side.

// partial[b][chunk][i] = sum over the chunk of V_i[b] . w[b]  (i < nv)
template <int NV>
__global__ __launch_bounds__(NT) void k_mdot_t(const double* __restrict__ V, int64_t vstride, int nv,
                                               const double* __restrict__ w, double* __restrict__ partial,
                                               int64_t N1, int chunks, int slot0) {
  __shared__ double red[4];
  constexpr int NR = NV > 0 ? NV : MAXV;
  const int b = blockIdx.y, c = blockIdx.x;
  const int64_t per = ((N1 + chunks - 1) / chunks + 1) & ~(int64_t)1;
  const int64_t beg = c * per, end = min(N1, beg + per);
  const double* wb = w + (int64_t)b * N1;
  const double* Vb = V + (int64_t)b * N1;
  double acc[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) acc[i] = 0;
  for (int64_t e = beg + 2 * threadIdx.x; e < end; e += 2 * NT) {
    double2 wv = *reinterpret_cast<const double2*>(wb + e);
#pragma unroll
    for (int i = 0; i < NR; ++i)
      if (NV > 0 || i < nv) {
        double2 v = *reinterpret_cast<const double2*>(Vb + i * vstride + e);
        acc[i] += v.x * wv.x + v.y * wv.y;
      }
  }
  double* out = partial + ((int64_t)b * chunks + c) * MAXV + slot0;
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    if (NV > 0 || i < nv) {  // nv is uniform: the barrier inside is reached by all threads
      double t = block_sum(acc[i], red);
      if (threadIdx.x == 0) out[i] = t;
    }
  }
}

// t = sum_c partial[b][c][i]; with the Krylov scale s = sigma[b][i] (1 for
// i >= nscaled or sigma == null): h[b][i] = t s and coef[b][i] = t s^2.
__global__ __launch_bounds__(NT) void k_reduce(const double* __restrict__ partial, int nv, int chunks,
                                               const double* __restrict__ sigma, int nscaled,
                                               double* __restrict__ h, double* __restrict__ coef,
                                               int ldh, double* __restrict__ hhost) {
  __shared__ double red[4];
  const int b = blockIdx.y, i = blockIdx.x;
  double v = 0;
  for (int c = threadIdx.x; c < chunks; c += NT) v += partial[((int64_t)b * chunks + c) * MAXV + i];
  double t = block_sum(v, red);
  if (threadIdx.x == 0) {
    double sg = (sigma && i < nscaled) ? sigma[b * ldh + i] : 1.0;
    h[b * ldh + i] = t * sg;
    if (coef) coef[b * ldh + i] = t * sg * sg;
    if (hhost) hhost[b * ldh + i] = t * sg;   // pinned host copy, read after the stream sync
  }
}

// The completion word of a solver round trip, stored once every kernel
// queued before this one has finished.  The store is a release at system
// scope (one vector store from one lane): the earlier kernels' writes to the
// coherent pinned buffer are visible to the host before the word is, and the
// host reads the word with acquire ordering.
__global__ void k_signal(int* __restrict__ word, int v) {
  if (threadIdx.x == 0) __hip_atomic_store(word, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// dst[i] = src[i] for i < n: the solver's per-step scalars, staged by the
// host in pinned memory, fetched by one small kernel instead of a copy.
__global__ __launch_bounds__(NT) void k_fetch(const double* __restrict__ src, double* __restrict__ dst,
                                              int n) {
  for (int i = threadIdx.x; i < n; i += NT) dst[i] = src[i];
}

// w[b] -= sum_i coef[b][i] V_i[b]; optionally partial dots of the new w with
// V_i (slots 0..nv-1) and with itself (slot nv).  Nothing happens when skip
// is given and set (see k_arnoldi_skip).
template <int NV, bool DOTS>
__global__ __launch_bounds__(NT) void k_update_t(const double* __restrict__ V, int64_t vstride, int nv,
                                                 const double* __restrict__ coef, int ldc,
                                                 double* __restrict__ w, double* __restrict__ partial,
                                                 int64_t N1, int chunks, const int* __restrict__ skip,
                                                 const double* __restrict__ V0) {
  if (skip != nullptr && *skip != 0) return;
  __shared__ double red[4];
  constexpr int NR = NV > 0 ? NV : MAXV;
  const int b = blockIdx.y, c = blockIdx.x;
  const int64_t per = ((N1 + chunks - 1) / chunks + 1) & ~(int64_t)1;
  const int64_t beg = c * per, end = min(N1, beg + per);
  double* wb = w + (int64_t)b * N1;
  const double* Vb = V + (int64_t)b * N1;
  double cf[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) cf[i] = (NV > 0 || i < nv) ? coef[b * ldc + i] : 0.0;
  double acc[NR + 1];
#pragma unroll
  for (int i = 0; i <= NR; ++i) acc[i] = 0;
  for (int64_t e = beg + 2 * threadIdx.x; e < end; e += 2 * NT) {
    double2 vv[NR];
    double2 wv = *reinterpret_cast<const double2*>(wb + e);
#pragma unroll
    for (int i = 0; i < NR; ++i)
      if (NV > 0 || i < nv) {
        vv[i] = *reinterpret_cast<const double2*>(((i == 0 && V0 != nullptr) ? V0 + (int64_t)b * N1 : Vb + i * vstride) + e);
        wv.x -= cf[i] * vv[i].x;
        wv.y -= cf[i] * vv[i].y;
      }
    *reinterpret_cast<double2*>(wb + e) = wv;
    if (DOTS) {
#pragma unroll
      for (int i = 0; i < NR; ++i)
        if (NV > 0 || i < nv) acc[i] += vv[i].x * wv.x + vv[i].y * wv.y;
      acc[NR] += wv.x * wv.x + wv.y * wv.y;
    }
  }
  if (!DOTS) return;
  double* out = partial + ((int64_t)b * chunks + c) * MAXV;
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    if (NV > 0 || i < nv) {
      double t = block_sum(acc[i], red);
      if (threadIdx.x == 0) out[i] = t;
    }
  }
  double t = block_sum(acc[NR], red);
  if (threadIdx.x == 0) out[nv] = t;
}

// x[b] += sum_i y[b][i] Z_i[b]  (x[b] = ... when overwrite: x is not read)
template <typename Tz>
__global__ __launch_bounds__(NT) void k_xupd(const Tz* __restrict__ Z, int64_t zstride, int nz,
                                             const double* __restrict__ yc, int ldy,
                                             double* __restrict__ x, int64_t N1, int overwrite) {
  const int b = blockIdx.y;
  double cf[MAXV];
#pragma unroll
  for (int i = 0; i < MAXV; ++i) cf[i] = (i < nz) ? yc[b * ldy + i] : 0.0;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < N1; e += (int64_t)gridDim.x * NT) {
    double v = overwrite ? 0.0 : x[(int64_t)b * N1 + e];
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
      if (i < nz) v += cf[i] * (double)Z[i * zstride + (int64_t)b * N1 + e];
    x[(int64_t)b * N1 + e] = v;
  }
}

// The same update, four consecutive elements per thread with every Z load of
// an iteration issued before the first use (NZ known at compile time; N1 a
// multiple of 4 and Z rows 16-byte aligned).
template <typename Tz> struct Quad;
template <> struct Quad<float> {
  static __device__ __forceinline__ void load(const float* p, double (&v)[4]) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
};
template <> struct Quad<double> {
  static __device__ __forceinline__ void load(const double* p, double (&v)[4]) {
    const double2 a = reinterpret_cast<const double2*>(p)[0], c = reinterpret_cast<const double2*>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = c.x; v[3] = c.y;
  }
};

template <typename Tz, int NZ>
__global__ __launch_bounds__(NT) void k_xupd4(const Tz* __restrict__ Z, int64_t zstride,
                                              const double* __restrict__ yc, int ldy,
                                              double* __restrict__ x, int64_t N1, int overwrite) {
  const int b = blockIdx.y;
  double cf[NZ];
#pragma unroll
  for (int i = 0; i < NZ; ++i) cf[i] = yc[b * ldy + i];
  const int64_t n4 = N1 / 4;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n4; e += (int64_t)gridDim.x * NT) {
    const int64_t off = (int64_t)b * N1 + 4 * e;
    double z[NZ][4];
#pragma unroll
    for (int i = 0; i < NZ; ++i) Quad<Tz>::load(Z + i * zstride + off, z[i]);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (!overwrite) Quad<double>::load(x + off, v);
#pragma unroll
    for (int i = 0; i < NZ; ++i)
#pragma unroll
      for (int c = 0; c < 4; ++c) v[c] = fma(cf[i], z[i][c], v[c]);
    double2* xo = reinterpret_cast<double2*>(x + off);
    xo[0] = double2{v[0], v[1]};
    xo[1] = double2{v[2], v[3]};
  }
}

// Whether the Arnoldi step j can end its cycle without orthogonalising w.
// h[b][q] (q <= j) are the first Gram-Schmidt pass's coefficients v_q . w and
// h[b][j+1] = w . w, so the new subdiagonal entry is
// sqrt(w . w - sum_q h_q^2) (Pythagoras, V orthonormal).  giv[b] holds
// [threshold (negative: right-hand side no longer live), g_j, c_0..c_{j-1},
// s_0..s_{j-1}]: the residual estimate so far and the cycle's Givens
// rotations.  Rotating the new column and forming the next rotation gives the
// least-squares residual estimate |s_j g_j| after this step.  The step skips
// the update (flag = 1) when that subtraction is well conditioned for every
// live right-hand side (w . w - sum h^2 above 1e-12 w . w) and either every
// estimate is within its threshold or the host forces the end of the cycle
// (restart length or iteration limit reached): the next basis vector is then
// never used.  With `first` (step 0 of a cycle run on the unnormalised
// V_0 = b, whose h[b][2] holds b . b) the kernel also derives beta = ||b||:
// it stores the V_0 scale 1/beta in sigma, scales the first-pass coefficient
// in c1 by 1/beta^2 before the update reads it, and tests against rtol beta
// with g_0 = beta.  A zero b is then not live.  One thread: a few
// multiply-adds per right-hand side.
__global__ void k_arnoldi_skip(const double* __restrict__ h, const double* __restrict__ giv, int gs,
                               int j, int B, int force, int* __restrict__ flag,
                               int* __restrict__ flag_host, int first, double* __restrict__ c1,
                               double* __restrict__ sigma, double rtol) {
  if (threadIdx.x != 0) return;
  bool all_done = true, well = true;
  for (int b = 0; b < B; ++b) {
    const double* G = giv + (int64_t)b * gs;
    const double* hc = h + (int64_t)b * MAXV;
    double thr = G[0], g = G[1], sc = 1.0;
    if (first) {
      // step 0 of a cycle started from the unnormalised V_0 = b: h[2] = b . b
      // gives beta = ||b||, the scale of V_0 (for this step's update and the
      // later reductions), the threshold rtol beta and g_0 = beta; the step's
      // dots and w . w carry a factor beta^2
      const double beta = sqrt(hc[2]);
      const double s0 = beta > 0.0 ? 1.0 / beta : 0.0;
      sigma[(int64_t)b * MAXV] = s0;
      c1[(int64_t)b * MAXV] *= s0 * s0;
      if (!(beta > 0.0)) continue;   // b = 0: not live (NaN: the host stops)
      sc = s0 * s0;
      thr = rtol * beta;
      g = beta;
    }
    if (thr < 0.0) continue;
    const double w2 = hc[j + 1] * sc;
    double nn = w2, cur = hc[0] * sc;
    for (int q = 0; q <= j; ++q) nn -= (hc[q] * sc) * (hc[q] * sc);
    for (int q = 0; q < j; ++q) {   // the previous rotations applied to the new column
      const double c = G[2 + q], sn = G[2 + j + q], nx = hc[q + 1] * sc;
      cur = -sn * cur + c * nx;
    }
    if (!(nn > 1e-12 * w2)) { well = false; continue; }
    const double hn = sqrt(nn);
    const double est = fabs(hn / hypot(cur, hn) * g);
    if (!(est <= thr)) all_done = false;
  }
  const int f = (well && (force || all_done)) ? 1 : 0;
  *flag = f;
  if (flag_host) *flag_host = f;
}

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) b[e] = a[e];
}
__global__ void k_zero(double* __restrict__ b, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) b[e] = 0.0;
}

Stencil stencil_of(const SpaceOp& op) { return Stencil{op.sxl, op.sxu, op.syl, op.syu, op.sd}; }

int grid_for(int64_t n) {
  int64_t g = (n + NT - 1) / NT;
  if (g > 65536) g = 65536;
  return (int)std::max<int64_t>(g, 1);
}

}  // namespace

static dim3 matvec_grid(const Plan& pl, int& V, int& chunk) {
  const Geom& g = pl.g;
  chunk = 16;
  V = (g.nx % 4) == 0 ? 4 : 1;
  return dim3((unsigned)((g.S / V + NT - 1) / NT), (g.nt + chunk - 1) / chunk, g.B);
}

int matvec_chunks(const Plan& pl) {
  if (pl.oc) return dot_chunks(pl);   // its dots come from multi_dot
  int V, chunk;
  const dim3 gr = matvec_grid(pl, V, chunk);
  return (int)(gr.x * gr.y);
}

void matvec_plain(const Plan& pl, const SpaceOp& op, const void* u, bool u_is_f32, const double* b,
                  double* y, int transpose, hipStream_t s) {
  int V, chunk;
  const dim3 grid = matvec_grid(pl, V, chunk);
  Stencil st = stencil_of(op);
  const int dir = transpose ? -1 : 1;
  const Geom& g = pl.g;
#define PD_MVP(TIN, VV)                                                                            \
  k_matvec<TIN, VV, 0><<<grid, NT, 0, s>>>((const TIN*)u, b, y, g.nt, g.nx, g.ny, pl.L, pl.c1[0],  \
                                           pl.c1[1], pl.c1[2], pl.c2[0], pl.c2[1], pl.c2[2], st,  \
                                           chunk, dir, nullptr, 0, 0, 0, nullptr, nullptr, 0)
  if (u_is_f32) { if (V == 4) PD_MVP(float, 4); else PD_MVP(float, 1); }
  else { if (V == 4) PD_MVP(double, 4); else PD_MVP(double, 1); }
#undef PD_MVP
}

void matvec(const Plan& pl, const SpaceOp& op, const void* u, bool u_is_f32, const double* b,
            double* y, int transpose, hipStream_t s, const double* Vk, int64_t vstride, int nv,
            double* partial, int sq, const double* V0, int v0sq) {
  int V, chunk;
  const dim3 grid = matvec_grid(pl, V, chunk);
  Stencil st = stencil_of(op);
  int dir = transpose ? -1 : 1;
  const Geom& g = pl.g;
  if (pl.oc) {
    oc_matvec(pl, u, u_is_f32, b, y, s, Vk, vstride, nv, partial, sq, V0, v0sq);
    return;
  }
  if (pl.hybrid) {   // banded time matrix; Krylov dots are not fused here
    const double* band = transpose ? pl.d_band_t : pl.d_band;
#define PD_MVB(TIN, VV) \
    k_matvec_band<TIN, VV><<<grid, NT, 0, s>>>((const TIN*)u, b, y, g.nt, g.nx, g.ny, band, st, chunk, sq, partial)
    if (u_is_f32) { if (V == 4) PD_MVB(float, 4); else PD_MVB(float, 1); }
    else { if (V == 4) PD_MVB(double, 4); else PD_MVB(double, 1); }
#undef PD_MVB
    return;
  }
#define PD_MV(TIN, VV, K)                                                                         \
  k_matvec<TIN, VV, K><<<grid, NT, 0, s>>>((const TIN*)u, b, y, g.nt, g.nx, g.ny, pl.L, pl.c1[0], \
                                           pl.c1[1], pl.c1[2], pl.c2[0], pl.c2[1], pl.c2[2], st,  \
                                           chunk, dir, Vk, vstride, nv, sq, partial, V0, v0sq)
#define PD_MV_NV(TIN, VV)                                                                         \
  switch (nv) {                                                                                   \
    case 0: PD_MV(TIN, VV, 0); break;                                                             \
    case 1: PD_MV(TIN, VV, 1); break;                                                             \
    case 2: PD_MV(TIN, VV, 2); break;                                                             \
    case 3: PD_MV(TIN, VV, 3); break;                                                             \
    case 4: PD_MV(TIN, VV, 4); break;                                                             \
    default: PD_MV(TIN, VV, -1); break;                                                           \
  }
  if (u_is_f32) {
    if (V == 4) { PD_MV_NV(float, 4) }
    else { PD_MV_NV(float, 1) }
  } else {
    if (V == 4) { PD_MV_NV(double, 4) }
    else { PD_MV_NV(double, 1) }
  }
#undef PD_MV_NV
#undef PD_MV
}

void build_rhs(const Plan& pl, const double* U0, const double* u1, const double* f, double* b,
               hipStream_t s) {
  const Geom& g = pl.g;
  dim3 grid((unsigned)(((int64_t)g.nt * g.S + NT - 1) / NT), g.B);
  k_rhs<<<grid, NT, 0, s>>>(U0, u1, f, b, g.nt, g.nx, g.ny, pl.p.scheme, pl.p.T / g.nt, pl.theta,
                            stencil_of(pl.op[0]));
}

void rhs_transpose(const Plan& pl, const double* lam, double* gU0, double* gu1, double* gf,
                   hipStream_t s) {
  const Geom& g = pl.g;
  dim3 grid((unsigned)(((int64_t)(g.nt + 1) * g.S + NT - 1) / NT), g.B);
  k_rhs_t<<<grid, NT, 0, s>>>(lam, gU0, gu1, gf, g.nt, g.nx, g.ny, pl.p.scheme, pl.p.T / g.nt,
                              pl.theta, stencil_of(pl.op[1]));
}

int dot_chunks(const Plan& pl) {
  // about 16 pairs per thread per chunk, at most 2048 chunks per right-hand side
  int64_t c = pl.g.N1 / (NT * 32);
  if (c < 1) c = 1;
  if (c > 2048) c = 2048;
  return (int)c;
}

void multi_dot(const Plan& pl, const double* V, int64_t vstride, int nv, const double* w,
               double* partial, hipStream_t s, int slot0) {
  int chunks = dot_chunks(pl);
  dim3 grid(chunks, pl.g.B);
  switch (nv) {
#define PD_MD(K) case K: k_mdot_t<K><<<grid, NT, 0, s>>>(V, vstride, nv, w, partial, pl.g.N1, chunks, slot0); return;
    PD_MD(1) PD_MD(2) PD_MD(3) PD_MD(4) PD_MD(5) PD_MD(6) PD_MD(7) PD_MD(8)
#undef PD_MD
    default: k_mdot_t<0><<<grid, NT, 0, s>>>(V, vstride, nv, w, partial, pl.g.N1, chunks, slot0);
  }
}

void reduce_partials(const Plan& pl, const double* partial, int nv, const double* sigma,
                     int nscaled, double* h, double* coef, hipStream_t s, int chunks,
                     double* hhost) {
  if (chunks <= 0) chunks = dot_chunks(pl);
  k_reduce<<<dim3(nv, pl.g.B), NT, 0, s>>>(partial, nv, chunks, sigma, nscaled, h, coef, MAXV, hhost);
}

void fetch_host(const double* src, double* dst, int n, hipStream_t s) {
  k_fetch<<<1, NT, 0, s>>>(src, dst, n);
}

void signal_host(int* word, int v, hipStream_t s) { k_signal<<<1, 64, 0, s>>>(word, v); }

void update_dot(const Plan& pl, const double* V, int64_t vstride, int nv, const double* coef,
                double* w, double* partial, int want_dots, hipStream_t s, const int* skip,
                const double* V0) {
  int chunks = dot_chunks(pl);
  dim3 grid(chunks, pl.g.B);
#define PD_UP(K)                                                                                  \
  case K:                                                                                         \
    if (want_dots) k_update_t<K, true><<<grid, NT, 0, s>>>(V, vstride, nv, coef, MAXV, w, partial, pl.g.N1, chunks, skip, V0); \
    else k_update_t<K, false><<<grid, NT, 0, s>>>(V, vstride, nv, coef, MAXV, w, partial, pl.g.N1, chunks, skip, V0); \
    return;
  switch (nv) {
    PD_UP(1) PD_UP(2) PD_UP(3) PD_UP(4) PD_UP(5) PD_UP(6) PD_UP(7) PD_UP(8)
    default:
      if (want_dots) k_update_t<0, true><<<grid, NT, 0, s>>>(V, vstride, nv, coef, MAXV, w, partial, pl.g.N1, chunks, skip, V0);
      else k_update_t<0, false><<<grid, NT, 0, s>>>(V, vstride, nv, coef, MAXV, w, partial, pl.g.N1, chunks, skip, V0);
  }
#undef PD_UP
}

void arnoldi_skip(const Plan& pl, const double* h, const double* giv, int gs, int j, bool force,
                  int* flag, hipStream_t s, int* flag_host, bool first, double* c1, double* sigma,
                  double rtol) {
  k_arnoldi_skip<<<1, 64, 0, s>>>(h, giv, gs, j, pl.g.B, force ? 1 : 0, flag, flag_host,
                                  first ? 1 : 0, c1, sigma, rtol);
}

void x_update(const Plan& pl, const void* Z, bool z_is_f32, int64_t zstride, int nz,
              const double* y, double* x, bool overwrite, hipStream_t s) {
  if (pl.g.N1 % 4 == 0 && zstride % 4 == 0 && nz >= 1 && nz <= 8 && (uintptr_t)x % 16 == 0 &&
      (uintptr_t)Z % 16 == 0) {
    dim3 grid(grid_for(pl.g.N1 / 4), pl.g.B);
#define PD_XUPD(K)                                                                                  \
  case K:                                                                                           \
    if (z_is_f32)                                                                                   \
      k_xupd4<float, K><<<grid, NT, 0, s>>>((const float*)Z, zstride, y, MAXV, x, pl.g.N1, overwrite); \
    else                                                                                            \
      k_xupd4<double, K><<<grid, NT, 0, s>>>((const double*)Z, zstride, y, MAXV, x, pl.g.N1, overwrite); \
    return;
    switch (nz) { PD_XUPD(1) PD_XUPD(2) PD_XUPD(3) PD_XUPD(4) PD_XUPD(5) PD_XUPD(6) PD_XUPD(7) PD_XUPD(8) }
#undef PD_XUPD
  }
  dim3 grid(grid_for(pl.g.N1), pl.g.B);
  if (z_is_f32)
    k_xupd<float><<<grid, NT, 0, s>>>((const float*)Z, zstride, nz, y, MAXV, x, pl.g.N1, overwrite);
  else
    k_xupd<double><<<grid, NT, 0, s>>>((const double*)Z, zstride, nz, y, MAXV, x, pl.g.N1, overwrite);
}

void diff_norms(const Plan& pl, const double* u, const double* v, double* partial, int chunks,
                hipStream_t s) {
  k_diff_sq<<<dim3(chunks, pl.g.B), NT, 0, s>>>(u, v, partial, pl.g.N1, chunks);
}

void nl_residual(const Plan& pl, const double* u, double* r, const double* gk, double* partial, int chunks,
                 hipStream_t s) {
  k_nl_residual<<<dim3(chunks, pl.g.B), NT, 0, s>>>(u, r, pl.g.N1, (int)pl.g.S, pl.c2[0], pl.c2[1],
                                                    CubicG{gk[0], gk[1], gk[2]}, partial, chunks);
}
void nl_rhs_fix(const Plan& pl, const double* U0, double* b, const double* gk, hipStream_t s) {
  const dim3 grid((unsigned)((pl.g.S + NT - 1) / NT), pl.g.B);
  k_nl_rhs_fix<<<grid, NT, 0, s>>>(U0, b, (int)pl.g.S, pl.g.N1, 1.0 - pl.theta, CubicG{gk[0], gk[1], gk[2]});
}
void bcast_rows(const Plan& pl, const double* U0, double* u, hipStream_t s) {
  const dim3 grid((unsigned)((pl.g.N1 + NT - 1) / NT), pl.g.B);
  k_bcast_rows<<<grid, NT, 0, s>>>(U0, u, (int)pl.g.S, pl.g.nt);
}
void last_rows(const Plan& pl, const double* src, double* dst, hipStream_t s) {
  const dim3 grid((unsigned)((pl.g.S + NT - 1) / NT), pl.g.B);
  k_last_rows<<<grid, NT, 0, s>>>(src, dst, (int)pl.g.S, pl.g.nt);
}

void copy_vec(const double* src, double* dst, int64_t n, hipStream_t s) {
  k_copy<<<grid_for(n), NT, 0, s>>>(src, dst, n);
}

void fill_zero(double* dst, int64_t n, hipStream_t s) { k_zero<<<grid_for(n), NT, 0, s>>>(dst, n); }

}  // namespace pd
