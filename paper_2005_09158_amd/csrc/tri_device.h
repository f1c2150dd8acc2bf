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
  // eliminate the first-row unknowns: tridiagonal system in x_e across lanes,
  // each equation scaled to a unit diagonal, so that cyclic reduction moves
  // three coefficients per neighbour and takes one reciprocal per level
  Cx<T> A = (p == 0) ? cz<T>() : neg(mul(aA, aB));
  Cx<T> Bc = sub(sub(c1<T>(), mul(aA, gB)), mul(gA, aBn));
  Cx<T> Cc = neg(mul(gA, gBn));
  Cx<T> D = sub(sub(dA, mul(aA, dB)), mul(gA, dBn));
  {
    const Cx<T> ib = rcp(Bc);
    A = mul(A, ib);
    Cc = mul(Cc, ib);
    D = mul(D, ib);
  }
#pragma unroll
  for (int s = 1; s < P; s <<= 1) {
    Cx<T> Am = shup(A, s, P), Cm = shup(Cc, s, P), Dm = shup(D, s, P);
    Cx<T> Ap = shdn(A, s, P), Cp = shdn(Cc, s, P), Dp = shdn(D, s, P);
    if (p < s) { Am = cz<T>(); Cm = cz<T>(); Dm = cz<T>(); }       // x = 0 outside the line
    if (p + s >= P) { Ap = cz<T>(); Cp = cz<T>(); Dp = cz<T>(); }
    // row - A row_{p-s} - C row_{p+s}, then rescaled to a unit diagonal
    const Cx<T> ib = rcp(sub(sub(c1<T>(), mul(A, Cm)), mul(Cc, Ap)));
    const Cx<T> nA = neg(mul(A, Am)), nC = neg(mul(Cc, Cp));
    const Cx<T> nD = sub(sub(D, mul(A, Dm)), mul(Cc, Dp));
    A = mul(nA, ib);
    Cc = mul(nC, ib);
    D = mul(nD, ib);
  }
  Cx<T> xe = D;
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

// Global -> LDS copy of a tile of TK mode columns by sy rows, by threads
// t = 0..nthr-1.  Loads are issued in batches of 8 per thread before their LDS
// stores, so each thread has several loads in flight instead of one
// load-wait-store chain.
template <typename T>
__device__ void tile_load_by(const T* slice, T* sre, T* sim, int k0, int nk, int TK, int sx, int sy,
                             int ldy, int R, int t, int nthr) {
  const int total = sy * 2 * TK;
  for (int base = 0; base < total; base += 8 * nthr) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * nthr + t;
      int k = e % TK, comp = (e / TK) & 1, y = e / (2 * TK);
      v[u] = (e < total && k < nk) ? slice[(int64_t)y * 2 * sx + comp * sx + k0 + k] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * nthr + t;
      int k = e % TK, comp = (e / TK) & 1, y = e / (2 * TK);
      if (e < total) (comp ? sim : sre)[lidx(k, y, ldy, R)] = v[u];
    }
  }
}

template <typename T>
__device__ void tile_store_by(T* slice, const T* sre, const T* sim, int k0, int nk, int TK, int sx,
                              int sy, int ldy, int R, int t, int nthr) {
  for (int e = t; e < sy * 2 * TK; e += nthr) {
    int k = e % TK, comp = (e / TK) & 1, y = e / (2 * TK);
    if (k < nk) slice[(int64_t)y * 2 * sx + comp * sx + k0 + k] = (comp ? sim : sre)[lidx(k, y, ldy, R)];
  }
}

template <typename T>
__device__ void tile_load(const T* slice, T* sre, T* sim, int k0, int nk, int TK, int sx, int sy,
                          int ldy, int R) {
  tile_load_by(slice, sre, sim, k0, nk, TK, sx, sy, ldy, R, (int)threadIdx.x, NT);
}

template <typename T>
__device__ void tile_store(T* slice, const T* sre, const T* sim, int k0, int nk, int TK, int sx,
                           int sy, int ldy, int R) {
  tile_store_by(slice, sre, sim, k0, nk, TK, sx, sy, ldy, R, (int)threadIdx.x, NT);
}

// 16-byte copies of a full tile (NB modes, sx % 4 == 0, k0 % 4 == 0): each
// vector holds MV consecutive modes of one row part; every thread issues all
// its loads before its LDS stores.  MAXROWS bounds sy, MINTHR bounds nthr
// from below.
template <typename T> struct Vec16;
template <> struct Vec16<float> { using t = float4; static constexpr int n = 4; };
template <> struct Vec16<double> { using t = double2; static constexpr int n = 2; };

template <typename T> __device__ __forceinline__ T vget(const float4& v, int m) {
  return m == 0 ? v.x : m == 1 ? v.y : m == 2 ? v.z : v.w;
}
template <typename T> __device__ __forceinline__ T vget(const double2& v, int m) {
  return m == 0 ? v.x : v.y;
}

template <typename T, int NB, int MAXROWS, int MINTHR>
__device__ __forceinline__ void tile_load_vec(const T* slice, T* sre, T* sim, int k0, int sx, int sy,
                                              int ldy, int R, int t, int nthr) {
  using V = typename Vec16<T>::t;
  constexpr int MV = Vec16<T>::n, NV = NB / MV;
  constexpr int MAXE = MAXROWS * 2 * NV;
  constexpr int MAXU = (MAXE + MINTHR - 1) / MINTHR;   // nthr >= MINTHR
  const int total = sy * 2 * NV;
  V v[MAXU];
#pragma unroll
  for (int u = 0; u < MAXU; ++u) {
    const int e = t + u * nthr;
    if (e < total) {
      const int kv = e % NV, comp = (e / NV) & 1, y = e / (2 * NV);
      v[u] = *reinterpret_cast<const V*>(slice + (int64_t)y * 2 * sx + comp * sx + k0 + kv * MV);
    }
  }
#pragma unroll
  for (int u = 0; u < MAXU; ++u) {
    const int e = t + u * nthr;
    if (e < total) {
      const int kv = e % NV, comp = (e / NV) & 1, y = e / (2 * NV);
      T* dst = comp ? sim : sre;
#pragma unroll
      for (int m = 0; m < MV; ++m) dst[lidx(kv * MV + m, y, ldy, R)] = vget<T>(v[u], m);
    }
  }
}

template <typename T, int NB, int MAXROWS>
__device__ __forceinline__ void tile_store_vec(T* slice, const T* sre, const T* sim, int k0, int sx,
                                               int sy, int ldy, int R, int t, int nthr) {
  using V = typename Vec16<T>::t;
  constexpr int MV = Vec16<T>::n, NV = NB / MV;
  const int total = sy * 2 * NV;
  for (int e = t; e < total; e += nthr) {
    const int kv = e % NV, comp = (e / NV) & 1, y = e / (2 * NV);
    const T* src = comp ? sim : sre;
    V v;
    T* vv = reinterpret_cast<T*>(&v);
#pragma unroll
    for (int m = 0; m < MV; ++m) vv[m] = src[lidx(kv * MV + m, y, ldy, R)];
    *reinterpret_cast<V*>(slice + (int64_t)y * 2 * sx + comp * sx + k0 + kv * MV) = v;
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


// ---------------------------------------------------------------------------
// The same substitutions with the cross-lane steps on DPP row shifts (a VALU
// operand modifier, no LDS round trip) and readlane for the carries between
// rows of 16 lanes.  Segment of P lanes (P <= 16: several segments per row;
// P = 32, 64: two or four rows); only the lanes of a segment exchange data.

template <int CTRL> __device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL> __device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL, typename T> __device__ __forceinline__ Cx<T> dpp_c(Cx<T> v) {
  return Cx<T>{dpp_mov<CTRL>(v.x), dpp_mov<CTRL>(v.y)};
}
__device__ __forceinline__ float lane_read(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_read(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <typename T> __device__ __forceinline__ Cx<T> lane_read(Cx<T> v, int l) {
  return Cx<T>{lane_read(v.x, l), lane_read(v.y, l)};
}
template <typename T> __device__ __forceinline__ Cx<T> fma_c(Cx<T> a, Cx<T> b, Cx<T> c) {
  // a + b c
  return Cx<T>{a.x + b.x * c.x - b.y * c.y, a.y + b.x * c.y + b.y * c.x};
}

// DPP move whose lanes without a source in their row keep `old`.
template <int CTRL> __device__ __forceinline__ float dpp_keep(float old, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double dpp_keep(double old, double v) {
  const long long b = __double_as_longlong(v), o = __double_as_longlong(old);
  const int lo = __builtin_amdgcn_update_dpp((int)(o & 0xffffffffll), (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// Complex DPP move that brings in the identity map (A = 0, B = 1) where the
// source lane lies outside the row: composing with it changes nothing, so
// rows of 16 lanes scan without branches.
template <int CTRL, typename T> __device__ __forceinline__ void dpp_affine(Cx<T>& A, Cx<T>& B, Cx<T>& Ap, Cx<T>& Bp) {
  Ap = Cx<T>{dpp_keep<CTRL>((T)0, A.x), dpp_keep<CTRL>((T)0, A.y)};
  Bp = Cx<T>{dpp_keep<CTRL>((T)1, B.x), dpp_keep<CTRL>((T)0, B.y)};
}

// One level of the inclusive affine scan toward higher lanes: lanes at
// position >= O in their row segment compose with the lane O below.  Whole
// rows (P >= 16) rely on the identity fill; segments inside a row select.
template <int O, int W, typename T>
__device__ __forceinline__ void scan_up_level(Cx<T>& A, Cx<T>& B, int pw) {
  if constexpr (O < W) {
    Cx<T> Ap, Bp;
    dpp_affine<0x110 + O>(A, B, Ap, Bp);
    const Cx<T> An = fma_c(A, B, Ap), Bn = mul(B, Bp);
    if constexpr (W == 16) {
      A = An;
      B = Bn;
    } else {
      const bool take = pw >= O;
      A = Cx<T>{take ? An.x : A.x, take ? An.y : A.y};
      B = Cx<T>{take ? Bn.x : B.x, take ? Bn.y : B.y};
    }
  }
}
// ... and toward lower lanes (suffix): lanes with position + O < W.
template <int O, int W, typename T>
__device__ __forceinline__ void scan_down_level(Cx<T>& G, Cx<T>& D, int pw) {
  if constexpr (O < W) {
    Cx<T> Gn, Dn;
    dpp_affine<0x100 + O>(G, D, Gn, Dn);
    const Cx<T> Gc = fma_c(G, D, Gn), Dc = mul(D, Dn);
    if constexpr (W == 16) {
      G = Gc;
      D = Dc;
    } else {
      const bool take = pw + O < W;
      G = Cx<T>{take ? Gc.x : G.x, take ? Gc.y : G.y};
      D = Cx<T>{take ? Dc.x : D.x, take ? Dc.y : D.y};
    }
  }
}

// lu_scan_wave with DPP exchanges.  d, inv: rows p*R .. p*R+R-1 of the line
// of this lane's segment (p = lane % P); all 64 lanes call it.
template <typename T, int R, int P>
__device__ __forceinline__ void lu_scan_dpp(Cx<T> (&d)[R], const Cx<T> (&inv)[R], Cx<T> a, Cx<T> c,
                                            int N, int lane) {
  constexpr int W = P < 16 ? P : 16;   // lanes of a segment inside one row
  constexpr int NR = P < 16 ? 1 : P / 16;
  const int p = lane % P;
  const int pw = P < 16 ? p : (lane & 15);
  const int rs = P < 16 ? 0 : (p >> 4);   // row of the lane inside its segment
  const int row0 = p * R;
  // forward: d'_y = inv_y d_y + e_y d'_{y-1} with e_y = -a inv_y, as
  // d'_i = al_i + be_i (entering d'); e and be do not depend on the data and
  // run beside the al chain
  Cx<T> al[R], be[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int y = row0 + i;
    const Cx<T> iv = (y < N) ? inv[i] : c1<T>();
    const Cx<T> dy = (y < N) ? d[i] : cz<T>();
    const Cx<T> na = (y > 0 && y < N) ? neg(a) : cz<T>();
    const Cx<T> e = mul(na, iv);
    const Cx<T> f = mul(dy, iv);
    if (i == 0) {
      al[0] = f;
      be[0] = e;
    } else {
      al[i] = fma_c(f, e, al[i - 1]);
      be[i] = mul(e, be[i - 1]);
    }
  }
  Cx<T> A = al[R - 1], B = be[R - 1];
  scan_up_level<1, W>(A, B, pw);
  scan_up_level<2, W>(A, B, pw);
  scan_up_level<4, W>(A, B, pw);
  scan_up_level<8, W>(A, B, pw);
  Cx<T> carry_in = cz<T>();   // d' entering the first lane of this lane's row
  if constexpr (NR > 1) {
    Cx<T> run = cz<T>();
#pragma unroll
    for (int r = 0; r < NR - 1; ++r) {
      const Cx<T> At = lane_read(A, 16 * r + 15), Bt = lane_read(B, 16 * r + 15);
      run = fma_c(At, Bt, run);
      if (rs == r + 1) carry_in = run;
    }
    A = fma_c(A, B, carry_in);
  }
  // d' entering this lane: the lane below in the row, else the row carry
  // (zero at the start of a segment)
  Cx<T> din = Cx<T>{dpp_keep<0x111>(carry_in.x, A.x), dpp_keep<0x111>(carry_in.y, A.y)};
  if constexpr (P < 16) {
    if (p == 0) din = cz<T>();
  }
#pragma unroll
  for (int i = 0; i < R; ++i) d[i] = fma_c(al[i], be[i], din);
  // backward: x_y = d'_y + g_y x_{y+1}, g_y = -c inv_y (no coupling beyond
  // row N-1)
  Cx<T> ga[R], de[R];
  const Cx<T> nc = neg(c);
#pragma unroll
  for (int i = R - 1; i >= 0; --i) {
    const int y = row0 + i;
    const Cx<T> g = (y < N - 1) ? mul(nc, inv[i]) : cz<T>();
    if (i == R - 1) {
      ga[i] = d[i];
      de[i] = g;
    } else {
      ga[i] = fma_c(d[i], g, ga[i + 1]);
      de[i] = mul(g, de[i + 1]);
    }
  }
  Cx<T> G = ga[0], D = de[0];
  scan_down_level<1, W>(G, D, pw);
  scan_down_level<2, W>(G, D, pw);
  scan_down_level<4, W>(G, D, pw);
  scan_down_level<8, W>(G, D, pw);
  Cx<T> carry_dn = cz<T>();   // x at the first row of the next row of lanes
  if constexpr (NR > 1) {
    Cx<T> run = cz<T>();
#pragma unroll
    for (int r = NR - 2; r >= 0; --r) {
      const Cx<T> Gt = lane_read(G, 16 * (r + 1)), Dt = lane_read(D, 16 * (r + 1));
      run = fma_c(Gt, Dt, run);
      if (rs == r) carry_dn = run;
    }
    G = fma_c(G, D, carry_dn);
  }
  Cx<T> xn = Cx<T>{dpp_keep<0x101>(carry_dn.x, G.x), dpp_keep<0x101>(carry_dn.y, G.y)};
  if constexpr (P < 16) {
    if (p == P - 1) xn = cz<T>();
  }
#pragma unroll
  for (int i = 0; i < R; ++i) d[i] = fma_c(ga[i], de[i], xn);
}

}  // namespace tri
}  // namespace pd
