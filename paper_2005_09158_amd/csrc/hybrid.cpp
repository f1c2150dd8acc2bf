// Eigendecomposition of the time matrix of the hybrid discretisation
// (explicit midpoint for Nt - 1 steps, backward Euler for the last; Section
// 2.1.2, neq2.9c), in closed form after Thm thmCondU: B = V D V^{-1} with
//
//   D = diag(i x_n / dt),  v_{n,l} = i^l U_l(x_n),  l = 0 .. Nt-1,
//
// where x_n are the Nt roots of U_{Nt-1}(x) - i T_Nt(x) (T, U the Chebyshev
// polynomials of the first and second kind).  The second-order form uses
// B^2 = V D^2 V^{-1} (neq2.15).
//
// Roots.  With x = cos(theta), U_{N-1}(x) = sin(N theta)/sin(theta) and
// T_N(x) = cos(N theta), so the roots solve
//   g(theta) = sin(N theta) - i sin(theta) cos(N theta) = 0,
// i.e. tan(N theta) = i sin(theta), or N theta = k pi + i atanh(sin theta).
// For k = 1 .. N/2-1 the map theta -> (k pi + i atanh(sin theta)) / N
// contracts (its derivative is 1 / (N cos theta), at most about 1/pi here),
// so a few dozen fixed-point steps from k pi / N land next to the root and
// Newton's iteration on g finishes it.  The last root of the half plane
// Re theta < pi/2 lies near theta N / pi = N/2 - 0.4 + 0.27 i ln N (the two
// central roots push apart); Newton from there finds it.  B is real, so the
// other half are the mirror images x -> -conj(x) (eigenvalue -> its
// conjugate), and only the half Re x > 0 is kept.
//
// Inverse.  D_s^{-1} B D_s is complex symmetric for the diagonal scaling
// d_l = i^l (l < Nt-1), d_{Nt-1} = i sqrt(2) d_{Nt-2}, so its eigenvectors
// are orthogonal under the plain (unconjugated) product and
// V^{-1}[n][l] = (-i)^l U_l(x_n) w_l / sum_j w_j U_j(x_n)^2 with w_l = 1,
// except w_{Nt-1} = 1/2.  This orthogonality holds for exact roots only, and
// the Chebyshev values reach |U_l| ~ Nt / 3, so in double precision the
// products V^{-1} V miss the identity by ~1e-10 at Nt = 512 (close roots
// amplify root and recurrence rounding).  Roots, recurrences and sums are
// therefore carried in long double (64-bit significand) and rounded to
// double at the end.  The setup checks |V^{-1} V - I| and B V = V D.

#include <cmath>

#include "internal.h"

namespace pd {

namespace {

using ld = long double;
using cl = std::complex<long double>;

void g_dg(cl th, int N, cl& g, cl& dg) {
  const cl I(0.0L, 1.0L);
  const cl s = std::sin((ld)N * th), c = std::cos((ld)N * th);
  g = s - I * std::sin(th) * c;
  dg = (ld)N * c - I * std::cos(th) * c + I * (ld)N * std::sin(th) * s;
}

cl newton(cl th, int N) {
  for (int it = 0; it < 60; ++it) {
    cl g, dg;
    g_dg(th, N, g, dg);
    const cl step = g / dg;
    th -= step;
    if (std::abs(step) < 1e-18L * std::max(1.0L, std::abs(th))) break;
  }
  return th;
}

}  // namespace

bool hybrid_eigen(int nt, double dt, int order, HybridTables& out, std::string& err) {
  const ld PI = 3.141592653589793238462643383279502884L;
  const int N = nt, h = nt / 2;
  if (nt < 4 || (nt & 1)) { err = "the hybrid scheme needs an even nt >= 4"; return false; }
  const cl I(0.0L, 1.0L);
  std::vector<cl> x(h);
  for (int k = 1; k < h; ++k) {
    cl th = k * PI / N;
    for (int it = 0; it < 80; ++it) th = (k * PI + I * std::atanh(std::sin(th))) / (ld)N;
    x[k - 1] = std::cos(newton(th, N));
  }
  x[h - 1] = std::cos(newton(cl(h - 0.4L, 0.27L * std::log((ld)N)) * (PI / N), N));
  // the half set must hold h distinct roots strictly inside Re x > 0
  for (int a = 0; a < h; ++a) {
    if (!(x[a].real() > 0.0L) || !std::isfinite((double)x[a].real()) || !std::isfinite((double)x[a].imag())) {
      err = "hybrid eigenvalue search left the half plane";
      return false;
    }
    for (int b = 0; b < a; ++b)
      if (std::abs(x[a] - x[b]) < 1e-3L / ((ld)N * N)) { err = "hybrid eigenvalue search found a double root"; return false; }
  }
  // U_l(x_n) for the half set, l = 0 .. N-1
  std::vector<cl> U((size_t)N * h);
  for (int n = 0; n < h; ++n) {
    cl um = 1.0L, u = 2.0L * x[n];
    U[n] = 1.0L;
    U[(size_t)h + n] = u;
    for (int l = 2; l < N; ++l) {
      cl un = 2.0L * x[n] * u - um;
      um = u;
      u = un;
      U[(size_t)l * h + n] = u;
    }
  }
  auto ipow = [&](int l) { static const cl p[4] = {cl(1, 0), cl(0, 1), cl(-1, 0), cl(0, -1)}; return p[l & 3]; };
  out.d.resize(h);
  out.wf.assign((size_t)2 * h * N, 0.0);
  out.wi.assign((size_t)N * 2 * h, 0.0);
  ld res = 0.0L, vnorm = 0.0L;
  for (int n = 0; n < h; ++n) {
    const cl lam = I * x[n] / (ld)dt;
    const cl dn = order == 1 ? lam : lam * lam;
    out.d[n] = cd((double)dn.real(), (double)dn.imag());
    cl nn = 0.0L;
    for (int l = 0; l < N; ++l) {
      const cl u = U[(size_t)l * h + n];
      nn += (l == N - 1 ? 0.5L : 1.0L) * u * u;
    }
    for (int l = 0; l < N; ++l) {
      const cl u = U[(size_t)l * h + n];
      const cl vi = std::conj(ipow(l)) * u * (l == N - 1 ? 0.5L : 1.0L) / nn;   // V^{-1}[n][l]
      const cl v = ipow(l) * u;                                                 // V[l][n]
      out.wf[(size_t)(2 * n) * N + l] = (double)vi.real();
      out.wf[(size_t)(2 * n + 1) * N + l] = (double)vi.imag();
      out.wi[(size_t)l * 2 * h + 2 * n] = (double)(2.0L * v.real());
      out.wi[(size_t)l * 2 * h + 2 * n + 1] = (double)(-2.0L * v.imag());
      vnorm = std::max(vnorm, std::abs(v));
    }
    // B v = lam v, row by row (B of neq2.9c times dt)
    for (int l = 0; l < N; ++l) {
      cl bv;
      if (l == N - 1) bv = -ipow(l - 1) * U[(size_t)(l - 1) * h + n] + ipow(l) * U[(size_t)l * h + n];
      else {
        bv = 0.5L * ipow(l + 1) * U[(size_t)(l + 1) * h + n];
        if (l > 0) bv -= 0.5L * ipow(l - 1) * U[(size_t)(l - 1) * h + n];
      }
      res = std::max(res, std::abs(bv - I * x[n] * ipow(l) * U[(size_t)l * h + n]));
    }
  }
  if (!(res <= 1e-12L * vnorm)) { err = "hybrid eigenvectors fail B V = V D"; return false; }
  // V^{-1} V = I: rows n of V^{-1} (a strided sample of at most 32) against
  // every column m of V and its mirror
  double worst = 0.0;
  const int rstep = std::max(1, h / 32);
  for (int n = 0; n < h; n += rstep)
    for (int m = 0; m < h; ++m) {
      cd dot = 0.0, dotc = 0.0;
      for (int l = 0; l < N; ++l) {
        const cd vi(out.wf[(size_t)(2 * n) * N + l], out.wf[(size_t)(2 * n + 1) * N + l]);
        const cd v(0.5 * out.wi[(size_t)l * 2 * h + 2 * m], -0.5 * out.wi[(size_t)l * 2 * h + 2 * m + 1]);
        dot += vi * v;
        dotc += vi * std::conj(v);
      }
      worst = std::max(worst, std::abs(dot - (n == m ? 1.0 : 0.0)));
      worst = std::max(worst, std::abs(dotc));
    }
  out.inverse_error = worst;
  if (!(worst <= 1e-9)) { err = "hybrid left eigenvectors are not the inverse"; return false; }
  // banded rows of the time matrix (B or B^2) for the matvec: coefficients of
  // u_{n-2} .. u_{n+2}
  auto Bent = [&](int r, int c) {   // entry (r, c) of B (neq2.9c)
    if (r == N - 1) return c == N - 2 ? -1.0 / dt : (c == N - 1 ? 1.0 / dt : 0.0);
    return c == r + 1 ? 0.5 / dt : (c == r - 1 ? -0.5 / dt : 0.0);
  };
  out.band.assign((size_t)N * 5, 0.0);
  for (int r = 0; r < N; ++r)
    for (int k = -2; k <= 2; ++k) {
      const int c = r + k;
      if (c < 0 || c >= N) continue;
      double v = 0.0;
      if (order == 1) v = Bent(r, c);
      else
        for (int j = std::max(0, r - 1); j <= std::min(N - 1, r + 1); ++j) v += Bent(r, j) * Bent(j, c);
      out.band[(size_t)r * 5 + k + 2] = v;
    }
  return true;
}

}  // namespace pd
