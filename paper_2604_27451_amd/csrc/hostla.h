// hostla.h -- small dense host algebra of the folded eigensolver: a complex
// Hermitian eigensolver (cyclic Jacobi) for the projected matrices (order
// <= 64) and the Chebyshev coefficients of the resolvent 1/(x - t).
#pragma once
#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
#include <vector>

namespace adc2 {
namespace hostla {

using cplx = std::complex<double>;

// Eigen-decomposition of a Hermitian n x n matrix A (row-major).  On return
// w[0..n) holds the eigenvalues in ascending order and Z (row-major, n x n)
// the orthonormal eigenvectors as columns: A Z[:, i] = w[i] Z[:, i].
// Cyclic Jacobi: each plane rotation R = [[c, s e], [-s conj(e), c]] with
// e = a_pq / |a_pq| and t = s / c the smaller root of
// t^2 + 2 theta t - 1 = 0, theta = (a_qq - a_pp) / (2 |a_pq|), zeroes a_pq.
inline void herm_eig(int n, const cplx* A, double* w, cplx* Z) {
  std::vector<cplx> a(A, A + (size_t)n * n);
  std::vector<cplx> z((size_t)n * n, cplx(0.0, 0.0));
  for (int i = 0; i < n; ++i) z[(size_t)i * n + i] = 1.0;
  double diag2 = 0.0;
  for (int i = 0; i < n; ++i) diag2 += std::norm(a[(size_t)i * n + i]);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += std::norm(a[(size_t)p * n + q]);
    if (off <= 1e-32 * std::max(diag2, 1e-300) || off == 0.0) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const cplx apq = a[(size_t)p * n + q];
        const double g = std::abs(apq);
        if (g == 0.0) continue;
        const double app = a[(size_t)p * n + p].real(), aqq = a[(size_t)q * n + q].real();
        if (g < 1e-300 + 1e-18 * (std::fabs(app) + std::fabs(aqq)) && sweep > 2) {
          a[(size_t)p * n + q] = a[(size_t)q * n + p] = 0.0;
          continue;
        }
        const cplx e = apq / g;
        const double th = (aqq - app) / (2.0 * g);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        const cplx se = s * e, sce = s * std::conj(e);
        // A <- A R   (columns p, q)
        for (int i = 0; i < n; ++i) {
          const cplx aip = a[(size_t)i * n + p], aiq = a[(size_t)i * n + q];
          a[(size_t)i * n + p] = c * aip - sce * aiq;
          a[(size_t)i * n + q] = se * aip + c * aiq;
        }
        // A <- R^H A (rows p, q)
        for (int j = 0; j < n; ++j) {
          const cplx apj = a[(size_t)p * n + j], aqj = a[(size_t)q * n + j];
          a[(size_t)p * n + j] = c * apj - se * aqj;
          a[(size_t)q * n + j] = sce * apj + c * aqj;
        }
        a[(size_t)p * n + q] = a[(size_t)q * n + p] = 0.0;
        a[(size_t)p * n + p] = a[(size_t)p * n + p].real();
        a[(size_t)q * n + q] = a[(size_t)q * n + q].real();
        // Z <- Z R
        for (int i = 0; i < n; ++i) {
          const cplx zip = z[(size_t)i * n + p], ziq = z[(size_t)i * n + q];
          z[(size_t)i * n + p] = c * zip - sce * ziq;
          z[(size_t)i * n + q] = se * zip + c * ziq;
        }
      }
    }
  }
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int x, int y) { return a[(size_t)x * n + x].real() < a[(size_t)y * n + y].real(); });
  for (int i = 0; i < n; ++i) {
    w[i] = a[(size_t)ord[i] * n + ord[i]].real();
    for (int r = 0; r < n; ++r) Z[(size_t)r * n + i] = z[(size_t)r * n + ord[i]];
  }
}

// Same, warm-started from an orthonormal basis Zp (columns, row-major n x n)
// close to the eigenvectors: A is rotated into that basis, where it is nearly
// diagonal, so the Jacobi sweeps converge in one or two passes.
inline void herm_eig_warm(int n, const cplx* A, const cplx* Zp, double* w, cplx* Z) {
  std::vector<cplx> T((size_t)n * n, cplx(0.0, 0.0)), B((size_t)n * n, cplx(0.0, 0.0)), Y((size_t)n * n);
  for (int i = 0; i < n; ++i)          // T = A Zp
    for (int l = 0; l < n; ++l) {
      const cplx a = A[(size_t)i * n + l];
      if (a == cplx(0.0, 0.0)) continue;
      const cplx* zr = &Zp[(size_t)l * n];
      cplx* tr = &T[(size_t)i * n];
      for (int c = 0; c < n; ++c) tr[c] += a * zr[c];
    }
  for (int i = 0; i < n; ++i)          // B = Zp^H T
    for (int r = 0; r < n; ++r) {
      const cplx z = std::conj(Zp[(size_t)i * n + r]);
      const cplx* tr = &T[(size_t)i * n];
      cplx* br = &B[(size_t)r * n];
      for (int c = 0; c < n; ++c) br[c] += z * tr[c];
    }
  for (int r = 0; r < n; ++r) {
    B[(size_t)r * n + r] = B[(size_t)r * n + r].real();
    for (int c = r + 1; c < n; ++c) {
      const cplx a = 0.5 * (B[(size_t)r * n + c] + std::conj(B[(size_t)c * n + r]));
      B[(size_t)r * n + c] = a;
      B[(size_t)c * n + r] = std::conj(a);
    }
  }
  herm_eig(n, B.data(), w, Y.data());
  for (int i = 0; i < n; ++i) {        // Z = Zp Y
    cplx* zr = &Z[(size_t)i * n];
    for (int c = 0; c < n; ++c) zr[c] = 0.0;
    for (int l = 0; l < n; ++l) {
      const cplx zp = Zp[(size_t)i * n + l];
      const cplx* yr = &Y[(size_t)l * n];
      for (int c = 0; c < n; ++c) zr[c] += zp * yr[c];
    }
  }
}

// Chebyshev expansions of the resolvent for real |x| > 1 and t in [-1, 1]:
//   1/(x - t)   = sum_m b[m] T_m(t),   1/(x - t)^2 = sum_m e[m] T_m(t).
// With u = |x|, s = sqrt(u^2 - 1), r = u - s < 1 and sg = sign(x), the
// generating function of the T_m gives b[m] = sg (m ? 2 : 1) (sg r)^m / s;
// e = -db/dx.  Returns the number of terms after which r^m < 1e-17, or -1
// if that exceeds mmax.
inline int cheb_resolvent(double x, int mmax, double* b, double* e) {
  const double sg = x > 0.0 ? 1.0 : -1.0;
  const double u = std::fabs(x);
  if (!(u > 1.0)) return -1;
  const double s = std::sqrt(u * u - 1.0), r = u - s;
  int need = (int)std::ceil(std::log(1e-17) / std::log(r)) + 1;
  if (need < 2) need = 2;
  if (need > mmax) return -1;
  double rm = 1.0, sgm = 1.0;
  for (int m = 0; m < need; ++m) {
    const double pref = m == 0 ? 1.0 : 2.0;
    b[m] = sg * pref * sgm * rm / s;
    const double db = sg * pref * sgm * (rm * (-x / (s * s * s)) + m * rm * (-sg / s) / s);
    e[m] = -db;
    rm *= r;
    sgm *= sg;
  }
  return need;
}

}  // namespace hostla
}  // namespace adc2
