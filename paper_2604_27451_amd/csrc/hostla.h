// hostla.h -- small dense host algebra of the folded eigensolver: a complex
// Hermitian eigensolver (Householder tridiagonalisation and implicit QL) for
// the projected matrices (order <= 64) and the Chebyshev coefficients of the
// resolvent 1/(x - t).
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
// Householder reduction to a real symmetric tridiagonal T = Q^H A Q, then the
// implicit QL iteration with Wilkinson shifts on T (Bowdler, Martin, Reinsch
// and Wilkinson 1968; eigenvectors accumulated in a real matrix), then the
// back-transformation Z = Q Y.
//   Reflector of step i (column i, rows i+1..n-1): H = I - tau v v^H with
//   v[0] = 1, chosen so that H^H (alpha, x) = (beta, 0) with beta real,
//   beta = -sign(Re alpha) |(alpha, x)|, tau = (beta - alpha) / beta,
//   v[1:] = x / (alpha - beta); the trailing block is updated as
//   A <- A - v w^H - w v^H with p = tau A v, w = p - (tau/2)(p^H v) v.
// Returns the number of eigenvalues whose QL iteration did not converge
// within max_iter sweeps (0 on success); callers treat a nonzero count as a
// failed eigensolve.
inline int herm_eig(int n, const cplx* A, double* w, cplx* Z, int max_iter = 60) {
  if (n <= 0) return 0;
  std::vector<cplx> a(A, A + (size_t)n * n);
  for (int i = 0; i < n; ++i) {          // Hermitian part, real diagonal
    a[(size_t)i * n + i] = a[(size_t)i * n + i].real();
    for (int j = i + 1; j < n; ++j) {
      const cplx h = 0.5 * (a[(size_t)i * n + j] + std::conj(a[(size_t)j * n + i]));
      a[(size_t)i * n + j] = h;
      a[(size_t)j * n + i] = std::conj(h);
    }
  }
  std::vector<double> d(n), e(n, 0.0);
  std::vector<cplx> tau(n, cplx(0.0, 0.0)), V((size_t)n * n, cplx(0.0, 0.0));   // V column i = v_i
  std::vector<cplx> p(n), wv(n), vc(n);
  for (int i = 0; i + 1 < n; ++i) {
    const int m = n - i - 1;               // length of the column below the diagonal
    const cplx alpha = a[(size_t)(i + 1) * n + i];
    double xn2 = 0.0;
    for (int r = i + 2; r < n; ++r) xn2 += std::norm(a[(size_t)r * n + i]);
    cplx t = 0.0;
    double beta = alpha.real();
    if (xn2 > 0.0 || alpha.imag() != 0.0) {
      const double nrm = std::sqrt(std::norm(alpha) + xn2);
      beta = alpha.real() >= 0.0 ? -nrm : nrm;
      t = (beta - alpha) / beta;
      const cplx sc = 1.0 / (alpha - beta);
      V[(size_t)(i + 1) * n + i] = 1.0;
      for (int r = i + 2; r < n; ++r) V[(size_t)r * n + i] = a[(size_t)r * n + i] * sc;
      // p = tau A22 v  (A22 = rows/cols i+1..n-1); the O(n^3) loops below
      // spell out the complex arithmetic on the (re, im) pairs
      for (int c = i + 1; c < n; ++c) vc[c] = V[(size_t)c * n + i];
      for (int r = i + 1; r < n; ++r) {
        const double* ar = reinterpret_cast<const double*>(&a[(size_t)r * n]);
        const double* vv = reinterpret_cast<const double*>(vc.data());
        double sr = 0.0, si = 0.0;
        for (int c = i + 1; c < n; ++c) {
          const double xr = ar[2 * c], xi = ar[2 * c + 1], yr = vv[2 * c], yi = vv[2 * c + 1];
          sr += xr * yr - xi * yi;
          si += xr * yi + xi * yr;
        }
        p[r] = t * cplx(sr, si);
      }
      cplx pv = 0.0;                       // p^H v
      for (int r = i + 1; r < n; ++r) pv += std::conj(p[r]) * V[(size_t)r * n + i];
      const cplx half = -0.5 * t * pv;
      for (int r = i + 1; r < n; ++r) wv[r] = p[r] + half * V[(size_t)r * n + i];
      for (int r = i + 1; r < n; ++r) {
        double* ar = reinterpret_cast<double*>(&a[(size_t)r * n]);
        const double* ww = reinterpret_cast<const double*>(wv.data());
        const double* vv = reinterpret_cast<const double*>(vc.data());
        const double vr = vv[2 * r], vi = vv[2 * r + 1], wr = ww[2 * r], wi = ww[2 * r + 1];
        for (int c = i + 1; c < n; ++c) {
          // v_r conj(w_c) + w_r conj(v_c)
          const double wcr = ww[2 * c], wci = ww[2 * c + 1], vcr = vv[2 * c], vci = vv[2 * c + 1];
          ar[2 * c] -= vr * wcr + vi * wci + wr * vcr + wi * vci;
          ar[2 * c + 1] -= vi * wcr - vr * wci + wi * vcr - wr * vci;
        }
      }
    }
    (void)m;
    tau[i] = t;
    d[i] = a[(size_t)i * n + i].real();
    e[i] = beta;                           // T[i+1][i] = T[i][i+1]
  }
  d[n - 1] = a[(size_t)(n - 1) * n + (n - 1)].real();

  // implicit QL on (d, e), e[i] coupling i and i+1; Y accumulates the rotations
  std::vector<double> Y((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Y[(size_t)i * n + i] = 1.0;
  int unconverged = 0;
  for (int l = 0; l < n; ++l) {
    for (int iter = 0;; ++iter) {
      int m = l;
      for (; m + 1 < n; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 1e-16 * dd) break;
      }
      if (m == l) break;
      if (iter >= max_iter) {
        ++unconverged;
        break;
      }
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, pp = 0.0;
      int i = m - 1;
      for (; i >= l; --i) {
        double f = s * e[i];
        const double b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= pp;
          e[m] = 0.0;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - pp;
        r = (d[i] - g) * s + 2.0 * c * b;
        pp = s * r;
        d[i + 1] = g + pp;
        g = c * r - b;
        for (int k = 0; k < n; ++k) {       // rotate columns i and i+1 of Y
          f = Y[(size_t)k * n + i + 1];
          Y[(size_t)k * n + i + 1] = s * Y[(size_t)k * n + i] + c * f;
          Y[(size_t)k * n + i] = c * Y[(size_t)k * n + i] - s * f;
        }
      }
      if (r == 0.0 && i >= l) continue;
      d[l] -= pp;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  // Z = Q Y, Q = H_0 H_1 ... H_{n-2}: apply the reflectors last to first
  std::vector<cplx> X((size_t)n * n);
  for (size_t q = 0; q < X.size(); ++q) X[q] = Y[q];
  std::vector<double> acc(2 * n);
  for (int i = n - 2; i >= 0; --i) {
    if (tau[i] == cplx(0.0, 0.0)) continue;
    // acc[c] = tau v^H X[:, c], then X -= v acc^T (row by row, contiguous)
    std::fill(acc.begin(), acc.end(), 0.0);
    for (int r = i + 1; r < n; ++r) {
      const cplx v = V[(size_t)r * n + i];
      const double vr = v.real(), vi = -v.imag();   // conj(v_r)
      const double* xr = reinterpret_cast<const double*>(&X[(size_t)r * n]);
      for (int c = 0; c < n; ++c) {
        acc[2 * c] += vr * xr[2 * c] - vi * xr[2 * c + 1];
        acc[2 * c + 1] += vr * xr[2 * c + 1] + vi * xr[2 * c];
      }
    }
    const double tr = tau[i].real(), ti = tau[i].imag();
    for (int c = 0; c < n; ++c) {
      const double ar = acc[2 * c], ai = acc[2 * c + 1];
      acc[2 * c] = tr * ar - ti * ai;
      acc[2 * c + 1] = tr * ai + ti * ar;
    }
    for (int r = i + 1; r < n; ++r) {
      const cplx v = V[(size_t)r * n + i];
      const double vr = v.real(), vi = v.imag();
      double* xr = reinterpret_cast<double*>(&X[(size_t)r * n]);
      for (int c = 0; c < n; ++c) {
        xr[2 * c] -= vr * acc[2 * c] - vi * acc[2 * c + 1];
        xr[2 * c + 1] -= vr * acc[2 * c + 1] + vi * acc[2 * c];
      }
    }
  }
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int i = 0; i < n; ++i) {
    w[i] = d[ord[i]];
    for (int r = 0; r < n; ++r) Z[(size_t)r * n + i] = X[(size_t)r * n + ord[i]];
  }
  return unconverged;
}

// Same contract, for a matrix close to diagonal in the basis Zp: the direct
// solver above costs the same either way, so Zp is not needed.
inline int herm_eig_warm(int n, const cplx* A, const cplx* Zp, double* w, cplx* Z) {
  (void)Zp;
  return herm_eig(n, A, w, Z);
}

// Chebyshev expansions of the resolvent for real |x| > 1 and t in [-1, 1]:
//   1/(x - t)   = sum_m b[m] T_m(t),   1/(x - t)^2 = sum_m e[m] T_m(t).
// With u = |x|, s = sqrt(u^2 - 1), r = u - s < 1 and sg = sign(x), the
// generating function of the T_m gives b[m] = sg (m ? 2 : 1) (sg r)^m / s;
// e = -db/dx.  Returns the number of terms after which r^m < tol, or -1 if
// that exceeds mmax.
inline int cheb_resolvent(double x, int mmax, double* b, double* e, double tol = 1e-17) {
  const double sg = x > 0.0 ? 1.0 : -1.0;
  const double u = std::fabs(x);
  if (!(u > 1.0)) return -1;
  const double s = std::sqrt(u * u - 1.0), r = u - s;
  int need = (int)std::ceil(std::log(tol) / std::log(r)) + 1;
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

// Chebyshev variable of the doubles energies D in [Dmin, Dmax] and the
// expansion coefficients of the resolvent in it, for omega < Dmin:
//   (omega - D)^-1 = sum_m g[m] T_m(tau(D)),  (omega - D)^-2 = sum_m h[m] T_m(tau(D)).
// Linear: tau = (D - c) / hw, c and hw the centre and half-width of the
// interval, and (omega - D)^-1 = (1/hw) / (x - tau), x = (omega - c) / hw.
// Shifted inverse, w0 < Dmin: v = 1/(D - w0) maps the interval onto
// [1/(Dmax - w0), 1/(Dmin - w0)] (centre c, half-width hw), and with
// v* = 1/(omega - w0) the resolvent is v* - v*^2 / (v* - v), whose pole x =
// (v* - c) / hw lies far outside [-1, 1] when w0 is well below omega, so the
// series converges much faster.
struct ResolventMap {
  bool inv = false;
  double c = 0.0, ih = 1.0, w0 = 0.0;   // tau = (v - c) * ih
  double tol = 1e-17;                   // truncation: terms until r^m < tol (scaled for the shifted map)

  static ResolventMap linear(double Dmin, double Dmax) {
    ResolventMap r;
    r.c = 0.5 * (Dmin + Dmax);
    r.ih = 1.0 / std::max(0.5 * (Dmax - Dmin), 1e-6 * std::max(1.0, std::fabs(r.c)));
    return r;
  }
  static ResolventMap shifted_inverse(double Dmin, double Dmax, double w0) {
    ResolventMap r;
    r.inv = true;
    r.w0 = w0;
    const double lo = 1.0 / (Dmax - w0), hi = 1.0 / (Dmin - w0);
    r.c = 0.5 * (lo + hi);
    r.ih = 1.0 / std::max(0.5 * (hi - lo), 1e-12 * hi);
    return r;
  }
  double tau(double D) const { return ((inv ? 1.0 / (D - w0) : D) - c) * ih; }
  // largest omega whose pole has |x| >= xmin
  double reach(double xmin) const { return inv ? w0 + 1.0 / (c + xmin / ih) : c - xmin / ih; }
  // g, h as above (b, e: work arrays); returns the number of terms, or -1 if
  // more than mmax are needed or omega is not below the interval
  int coeffs(double omega, int mmax, double* b, double* e, double* g, double* h) const {
    if (!inv) {
      const int M = cheb_resolvent((omega - c) * ih, mmax, b, e, tol);
      for (int m = 0; m < M; ++m) {
        g[m] = b[m] * ih;
        h[m] = e[m] * ih * ih;
      }
      return M;
    }
    if (!(omega > w0)) return -1;
    const double vs = 1.0 / (omega - w0);
    // the truncated tail is scaled by v*^2 / hw relative to the linear case
    const int M = cheb_resolvent((vs - c) * ih, mmax, b, e, tol * std::min(1.0, c / vs));
    // (omega - D)^-1 = v* - (v*^2/hw) sum b T;  (omega - D)^-2 = v*^2 - 2 (v*^3/hw) sum b T + (v*^4/hw^2) sum e T
    const double g1 = vs * vs * ih, h1 = 2.0 * vs * vs * vs * ih, h2 = vs * vs * vs * vs * ih * ih;
    for (int m = 0; m < M; ++m) {
      g[m] = -g1 * b[m];
      h[m] = -h1 * b[m] + h2 * e[m];
    }
    if (M > 0) {
      g[0] += vs;
      h[0] += vs * vs;
    }
    return M;
  }
};

}  // namespace hostla
}  // namespace adc2
