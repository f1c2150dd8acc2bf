// Complex Schur decomposition of a real upper-Hessenberg matrix on the host.
//
// The x-direction factor K_x of a Dirichlet advection-diffusion operator is a
// non-normal Toeplitz tridiagonal matrix.  Its eigenvector matrix has a
// condition number growing like ((1+Pe)/(1-Pe))^{(n-1)/2} (Pe the cell Peclet
// number), far beyond 1/eps at the grid sizes of interest, so a
// diagonalisation is useless in floating point.  A unitary Schur basis
// K_x = Q T Q^H (T upper triangular) is perfectly conditioned and turns the
// 2D shifted solve of Step-(b) into a back-substitution over x-modes of
// y-direction tridiagonal solves (the Bartels-Stewart scheme).
//
// Algorithm: Francis implicit single-shift QR iteration in complex
// arithmetic on the Hessenberg matrix (a tridiagonal matrix already is one),
// Wilkinson shifts with periodic exceptional shifts, deflation on negligible
// subdiagonals, rotations accumulated into Q.  O(n^3); n <= 4096.

#include <cmath>
#include <complex>
#include <vector>

#include "internal.h"

namespace pd {

using cd = std::complex<double>;

namespace {

// Rotation G = [[c, s], [-conj(s), c]] with G [a; b] = [r; 0], c real.
inline void make_rotation(cd a, cd b, double& c, cd& s) {
  double aa = std::abs(a), ab = std::abs(b);
  if (ab == 0.0) { c = 1.0; s = 0.0; return; }
  if (aa == 0.0) { c = 0.0; s = std::conj(b) / ab; return; }
  double r = std::hypot(aa, ab);
  c = aa / r;
  s = (a / aa) * std::conj(b) / r;
}

}  // namespace

// h: n x n row-major complex, upper Hessenberg on entry, upper triangular on
// exit.  q: n x n row-major, receives the accumulated unitary factor so that
// H_in = Q H_out Q^H.  Returns false if the iteration fails to converge.
bool complex_schur(int n, std::vector<cd>& h, std::vector<cd>& q) {
  q.assign(static_cast<size_t>(n) * n, cd(0.0));
  for (int i = 0; i < n; ++i) q[static_cast<size_t>(i) * n + i] = 1.0;
  auto H = [&](int i, int j) -> cd& { return h[static_cast<size_t>(i) * n + j]; };
  auto Q = [&](int i, int j) -> cd& { return q[static_cast<size_t>(i) * n + j]; };
  const double eps = 2.220446049250313e-16;
  double hnorm = 0.0;
  for (auto& v : h) hnorm = std::max(hnorm, std::abs(v));
  if (hnorm == 0.0) return true;

  int ihi = n - 1;
  int its = 0, total = 0;
  const int max_total = 60 * n + 100;
  while (ihi > 0) {
    // locate the start of the unreduced block ending at ihi
    int l = ihi;
    for (; l > 0; --l) {
      double s = std::abs(H(l, l)) + std::abs(H(l - 1, l - 1));
      if (s == 0.0) s = hnorm;
      if (std::abs(H(l, l - 1)) <= eps * s) {
        H(l, l - 1) = 0.0;
        break;
      }
    }
    if (l == ihi) {  // 1x1 block converged
      --ihi;
      its = 0;
      continue;
    }
    if (++total > max_total) return false;
    ++its;
    cd mu;
    if (its % 11 == 0) {
      // exceptional shift breaks rare cycles of the Wilkinson shift
      mu = H(ihi, ihi) + 0.75 * std::abs(H(ihi, ihi - 1)) * cd(1.0, 0.5);
    } else {
      cd a = H(ihi - 1, ihi - 1), b = H(ihi - 1, ihi), c = H(ihi, ihi - 1), d = H(ihi, ihi);
      cd tr2 = 0.5 * (a + d);
      cd disc = std::sqrt(0.25 * (a - d) * (a - d) + b * c);
      cd m1 = tr2 + disc, m2 = tr2 - disc;
      mu = (std::abs(m1 - d) < std::abs(m2 - d)) ? m1 : m2;
    }
    // implicit single-shift sweep over the block l..ihi
    cd x = H(l, l) - mu, y = H(l + 1, l);
    for (int k = l; k < ihi; ++k) {
      if (k > l) { x = H(k, k - 1); y = H(k + 1, k - 1); }
      double c; cd s;
      make_rotation(x, y, c, s);
      // rows k, k+1 (all columns from k-1 to the right: keeps the full Schur form)
      int j0 = (k > l) ? k - 1 : l;
      for (int j = j0; j < n; ++j) {
        cd h1 = H(k, j), h2 = H(k + 1, j);
        H(k, j) = c * h1 + s * h2;
        H(k + 1, j) = -std::conj(s) * h1 + c * h2;
      }
      if (k > l) H(k + 1, k - 1) = 0.0;
      // columns k, k+1 (rows 0 .. min(k+2, ihi))
      int i1 = std::min(k + 2, ihi);
      for (int i = 0; i <= i1; ++i) {
        cd h1 = H(i, k), h2 = H(i, k + 1);
        H(i, k) = h1 * c + h2 * std::conj(s);
        H(i, k + 1) = -h1 * s + h2 * c;
      }
      for (int i = 0; i < n; ++i) {
        cd q1 = Q(i, k), q2 = Q(i, k + 1);
        Q(i, k) = q1 * c + q2 * std::conj(s);
        Q(i, k + 1) = -q1 * s + q2 * c;
      }
    }
  }
  // clean the strictly lower part
  for (int i = 1; i < n; ++i)
    for (int j = 0; j < i; ++j) H(i, j) = 0.0;
  return true;
}

}  // namespace pd
