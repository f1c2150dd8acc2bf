// Device helpers shared by the line-solve kernels: complex arithmetic, the
// one-wave tridiagonal solver and the padded LDS tile of line data.
#pragma once

#include "internal.h"

namespace pd {
namespace tri {

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
// 1 / (a.x + i a.y) = conj(a) / |a|^2.  float: the hardware reciprocal (1 ulp),
// well inside the float32 preconditioner's tolerance; double: IEEE division.
__device__ __forceinline__ float recip(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double recip(double v) { return 1.0 / v; }
template <typename T> __device__ __forceinline__ Cx<T> rcp(Cx<T> a) {
  T d = recip(a.x * a.x + a.y * a.y);
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

// Global -> LDS copy of a tile of TK mode columns by sy rows.  Loads are
// issued in batches of 8 per thread before their LDS stores, so each thread
// has several loads in flight instead of one load-wait-store chain.
template <typename T>
__device__ void tile_load(const T* slice, T* sre, T* sim, int k0, int nk, int TK, int sx, int sy,
                          int ldy, int R) {
  const int total = sy * 2 * TK;
  for (int base = 0; base < total; base += 8 * NT) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * NT + threadIdx.x;
      int k = e % TK, comp = (e / TK) & 1, y = e / (2 * TK);
      v[u] = (e < total && k < nk) ? slice[(int64_t)y * 2 * sx + comp * sx + k0 + k] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * NT + threadIdx.x;
      int k = e % TK, comp = (e / TK) & 1, y = e / (2 * TK);
      if (e < total) (comp ? sim : sre)[lidx(k, y, ldy, R)] = v[u];
    }
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


// Solve a x_{i-1} + b_i x_i + c x_{i+1} = d_i (i < N) given the inverse pivots
// inv_i = 1/m_i of its non-pivoted LU factorisation (m_0 = b_0, m_i = b_i -
// a c / m_{i-1}): the forward and backward substitutions are first-order
// linear recurrences, evaluated as affine scans across the P lanes of the
// segment (R rows per lane; rows >= N are identity).  Every lane of the wave
// must call this (shuffles).
template <typename T, int R, int P>
__device__ void lu_scan_wave(Cx<T> (&d)[R], const Cx<T> (&inv)[R], Cx<T> a, Cx<T> c, int N, int p) {
  const int row0 = p * R;
  // forward: d'_y = (d_y - a_y d'_{y-1}) inv_y  ->  d'_i = al_i + be_i * (entering d')
  Cx<T> al[R], be[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int y = row0 + i;
    const Cx<T> ay = (y > 0 && y < N) ? a : cz<T>();
    const Cx<T> iv = (y < N) ? inv[i] : c1<T>();
    const Cx<T> dy = (y < N) ? d[i] : cz<T>();
    if (i == 0) {
      al[0] = mul(dy, iv);
      be[0] = neg(mul(ay, iv));
    } else {
      al[i] = mul(sub(dy, mul(ay, al[i - 1])), iv);
      be[i] = neg(mul(mul(ay, be[i - 1]), iv));
    }
  }
  Cx<T> A = al[R - 1], B = be[R - 1];
#pragma unroll
  for (int o = 1; o < P; o <<= 1) {
    Cx<T> Ap = shup(A, o, P), Bp = shup(B, o, P);
    if (p >= o) {
      A = Cx<T>{A.x + B.x * Ap.x - B.y * Ap.y, A.y + B.x * Ap.y + B.y * Ap.x};
      B = mul(B, Bp);
    }
  }
  Cx<T> din = shup(A, 1, P);
  if (p == 0) din = cz<T>();
#pragma unroll
  for (int i = 0; i < R; ++i) {
    Cx<T> t = mul(be[i], din);
    d[i] = Cx<T>{al[i].x + t.x, al[i].y + t.y};
  }
  // backward: x_y = d'_y - c'_y x_{y+1}, c'_y = c inv_y (0 on the last row)
  Cx<T> ga[R], de[R];
#pragma unroll
  for (int i = R - 1; i >= 0; --i) {
    const int y = row0 + i;
    const Cx<T> cy = (y < N - 1) ? mul(c, inv[i]) : cz<T>();
    if (i == R - 1) {
      ga[i] = d[i];
      de[i] = neg(cy);
    } else {
      ga[i] = sub(d[i], mul(cy, ga[i + 1]));
      de[i] = neg(mul(cy, de[i + 1]));
    }
  }
  Cx<T> G = ga[0], D = de[0];
#pragma unroll
  for (int o = 1; o < P; o <<= 1) {
    Cx<T> Gn = shdn(G, o, P), Dn = shdn(D, o, P);
    if (p + o < P) {
      G = Cx<T>{G.x + D.x * Gn.x - D.y * Gn.y, G.y + D.x * Gn.y + D.y * Gn.x};
      D = mul(D, Dn);
    }
  }
  Cx<T> xn = shdn(G, 1, P);
  if (p == P - 1) xn = cz<T>();
#pragma unroll
  for (int i = 0; i < R; ++i) {
    Cx<T> t = mul(de[i], xn);
    d[i] = Cx<T>{ga[i].x + t.x, ga[i].y + t.y};
  }
}

}  // namespace tri
}  // namespace pd
