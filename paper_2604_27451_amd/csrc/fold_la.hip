// fold_la.hip -- the subspace linear algebra of the folded (doubles-free)
// Davidson solver, FP64 on the GPU.
//
// The folded solver works in the singles space: the search space V (s <= 64
// orthonormal singles vectors), S1 = the singles part of sigma(v, 0), the
// projected singles block H11 = V^H S1 and the Chebyshev moments
// K_m = U^H T_m(tau(D)) U of the doubles parts U = M21 V.  The effective
// matrix of the folded eigenproblem (the ADC(2) matrix with M22 = diag(D),
// Eq. 11 with the doubles eliminated) projected on V is
//   G(omega) = H11 + sum_m g_m(omega) K_m,
// and a root is a fixed point lambda_b(G(omega)) = omega of branch b.  Every
// step that touches these arrays runs here: the Newton iteration on omega with
// its eigensolves (one workgroup per projected root, jacobi.h), Ritz vectors
// and singles residuals, the preconditioned new directions, Gram-Schmidt,
// restarts (rotation of V, S1, H11 and every K_m), the root-following
// overlaps and the Hermitian bookkeeping of H11 and K.  The host only reads
// per-root status words and residual norms to steer the iteration.
#include <algorithm>
#include <cmath>

#include "fold_la.h"
#include "internal.h"
#include "jacobi.h"
#include "tile.h"

namespace adc2 {

// ---------------------------------------------------------------------------
// Chebyshev expansion of the resolvent (device side of the host map in
// hostla.h, same formulas):
//   1/(x - t) = sum_m b[m] T_m(t),  1/(x - t)^2 = sum_m e[m] T_m(t),  |x| > 1,
// b[m] = sg (m ? 2 : 1) (sg r)^m / s with u = |x|, s = sqrt(u^2 - 1),
// r = u - s, sg = sign(x); e = -db/dx.  Linear map: t = (D - c) ih; shifted
// inverse: t = (1/(D - w0) - c) ih and (omega - D)^-1 = v* - v*^2 / (v* - v),
// v* = 1/(omega - w0).  Returns the number of terms, -1 if omega is outside
// the map's range or more than mmax terms are needed.
// ---------------------------------------------------------------------------
__device__ int fold_cheb_resolvent(double x, int mmax, double* b, double* e, double tol) {
  const double sg = x > 0.0 ? 1.0 : -1.0;
  const double u = fabs(x);
  if (!(u > 1.0)) return -1;
  const double s = sqrt(u * u - 1.0), r = u - s;
  int need = (int)ceil(log(tol) / log(r)) + 1;
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

__device__ int fold_coeffs(const FoldMap& r, double omega, int mmax, double* b, double* e, double* g, double* h) {
  if (!r.inv) {
    const int M = fold_cheb_resolvent((omega - r.c) * r.ih, mmax, b, e, r.tol);
    for (int m = 0; m < M; ++m) {
      g[m] = b[m] * r.ih;
      h[m] = e[m] * r.ih * r.ih;
    }
    return M;
  }
  if (!(omega > r.w0)) return -1;
  const double vs = 1.0 / (omega - r.w0);
  const int M = fold_cheb_resolvent((vs - r.c) * r.ih, mmax, b, e, r.tol * fmin(1.0, r.c / vs));
  const double g1 = vs * vs * r.ih, h1 = 2.0 * vs * vs * vs * r.ih, h2 = vs * vs * vs * vs * r.ih * r.ih;
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

// ---------------------------------------------------------------------------
// Projected nonlinear problem, one workgroup per projected root (entry).
// Entry b solves lambda_j(G(omega)) = omega for its branch j by the Newton
// step omega' = omega + (lambda_j - omega) / (1 + |x2|^2) safeguarded by
// bisection, |x2|^2 = y^H (sum_m h_m K_m) y (the norm of the folded doubles
// of the Ritz vector), each step an eigensolve of G(omega).  The eigensolve
// of the step after the first starts from the previous step's eigenvectors
// (Zp^H G Zp, nearly diagonal); so does the first step when the entry's slot
// holds eigenvectors of the previous iteration (padded with the identity for
// the new basis vectors).  Writes the status, omega, the Rayleigh quotient
// (lambda_j + omega |x2|^2) / (1 + |x2|^2), |x2|^2, the eigenvector y of the
// branch and all eigenvectors Z of G (its slot).
// Status: 0 converged step, 1 not below the reach of the expansion, 2 no
// expansion at omega, 3 more moments needed (need), 4 below the shifted
// map's range, 5 eigensolve did not converge, 6 branch beyond the space.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fold_solve(const double2* __restrict__ H, const double2* __restrict__ K,
                                                     int s, int Mmax, FoldMap map, double Dmin, double hi0,
                                                     double tol, const double* __restrict__ hw,
                                                     const FoldEntry* __restrict__ ent,
                                                     FoldResult* __restrict__ res, double2* __restrict__ Ybr,
                                                     double2* __restrict__ Zbr, FoldBounds* __restrict__ bnd) {
  __shared__ JacobiSmem S;
  __shared__ double cb[FOLD_MM], ce[FOLD_MM], cg[FOLD_MM], chh[FOLD_MM];
  __shared__ double2 ys[JMAX];
  __shared__ double wsh[JMAX];
  __shared__ double red2[256];
  __shared__ int sM, sflag, sdone;
  __shared__ double swv, slo, shi, swlo, slo0;
  const int tid = threadIdx.x;
  const FoldEntry E = ent[blockIdx.x];
  FoldResult R;
  R.omega = E.omega;
  R.rq = R.n2 = R.w = 0.0;
  R.status = R.need = R.ysize = R.zsize = 0;
  const int j = E.branch;
  double2* Zg = Zbr + (long)E.slot * JMAX * JMAX;
  if (tid == 0) {
    double T0 = 0.0;
    for (int i = 0; i < s; ++i) T0 += K[(long)i * JMAX + i].x;
    const double lam_min = hw[0];
    const double zb = 0.5 * (-(lam_min - Dmin) + sqrt((lam_min - Dmin) * (lam_min - Dmin) + 4.0 * fmax(T0, 0.0))) + 1.0;
    const double lo0 = Dmin - zb;
    const double wlo = map.inv ? fmax(lo0, map.w0 + 0.1 * (Dmin - map.w0)) : lo0;
    double wv = E.has_prev ? E.omega : wlo;
    if (!(wv > wlo && wv < hi0)) wv = E.has_prev ? fmin(fmax(wv, wlo), hi0 - 1e-9 * fabs(hi0)) : wlo;
    swv = wv;
    slo = wlo;
    shi = hi0;
    swlo = wlo;
    slo0 = lo0;
    if (blockIdx.x == 0) *bnd = FoldBounds{lam_min, lo0, wlo, hi0};
  }
  __syncthreads();
  if (j >= s) {   // fewer basis vectors than this branch index
    if (tid == 0) {
      R.status = 6;
      res[blockIdx.x] = R;
    }
    return;
  }
  int warm = (E.zwarm > 0 && E.zwarm <= s) ? E.zwarm : 0;
  int status = 0;
  bool wrote = false;
  for (int nit = 0; nit < 80; ++nit) {
    if (tid == 0) {
      const int M = fold_coeffs(map, swv, FOLD_MM, cb, ce, cg, chh);
      sM = M;
      sflag = M < 0 ? 2 : (M > Mmax ? 3 : 0);
    }
    __syncthreads();
    if (sflag != 0) {
      status = sflag;
      if (tid == 0) {
        R.status = sflag;
        R.need = sM;
      }
      break;
    }
    const int M = sM;
    // G = H11 + sum_m g_m K_m into S.ar / S.ai
    for (int e = tid; e < s * s; e += 256) {
      const int i = e / s, l = e % s;
      double2 a = H[(long)i * JMAX + l];
      for (int m = 0; m < M; ++m) {
        const double2 k = K[((long)m * JMAX + i) * JMAX + l];
        a.x += cg[m] * k.x;
        a.y += cg[m] * k.y;
      }
      S.ar[i][l] = a.x;
      S.ai[i][l] = a.y;
    }
    __syncthreads();
    // Hermitian part
    for (int e = tid; e < s * s; e += 256) {
      const int i = e / s, l = e % s;
      if (i < l) {
        const double xr = 0.5 * (S.ar[i][l] + S.ar[l][i]), xi = 0.5 * (S.ai[i][l] - S.ai[l][i]);
        S.ar[i][l] = xr;
        S.ai[i][l] = xi;
        S.ar[l][i] = xr;
        S.ai[l][i] = -xi;
      } else if (i == l) {
        S.ai[i][i] = 0.0;
      }
    }
    __syncthreads();
    if (warm > 0) {
      // G <- Zp^H G Zp, Zp = the stored eigenvectors padded with the identity
      for (int e = tid; e < s * s; e += 256) {
        const int i = e / s, c = e % s;
        double2 a = make_double2(0.0, 0.0);
        for (int l = 0; l < s; ++l) {
          const double2 z = (l < warm && c < warm) ? Zg[(long)l * JMAX + c] : make_double2(l == c ? 1.0 : 0.0, 0.0);
          a = cadd(a, cmul(make_double2(S.ar[i][l], S.ai[i][l]), z));
        }
        S.zs[i][c] = a;
      }
      __syncthreads();
      for (int e = tid; e < s * s; e += 256) {
        const int r = e / s, c = e % s;
        double2 a = make_double2(0.0, 0.0);
        for (int i = 0; i < s; ++i) {
          const double2 z = (i < warm && r < warm) ? Zg[(long)i * JMAX + r] : make_double2(i == r ? 1.0 : 0.0, 0.0);
          a = cadd(a, cmul(cconj(z), S.zs[i][c]));
        }
        S.ar[r][c] = a.x;
        S.ai[r][c] = a.y;
      }
      __syncthreads();
      for (int e = tid; e < s * s; e += 256) {
        const int i = e / s, l = e % s;
        if (i < l) {
          const double xr = 0.5 * (S.ar[i][l] + S.ar[l][i]), xi = 0.5 * (S.ai[i][l] - S.ai[l][i]);
          S.ar[i][l] = xr;
          S.ai[i][l] = xi;
          S.ar[l][i] = xr;
          S.ai[l][i] = -xi;
        } else if (i == l) {
          S.ai[i][i] = 0.0;
        }
      }
      __syncthreads();
    }
    jacobi_lds(S, s);
    if (!S.done) {
      status = 5;
      if (tid == 0) R.status = 5;
      break;
    }
    for (int i = tid; i < s; i += 256) wsh[i] = S.ar[S.perm[i]][S.perm[i]];
    __syncthreads();
    // eigenvectors of G in ascending order: Z = Zp Z' (into S.ar / S.ai), then to the slot
    for (int e = tid; e < s * s; e += 256) {
      const int r = e / s, c = e % s;
      double2 a;
      if (warm > 0) {
        a = make_double2(0.0, 0.0);
        for (int i = 0; i < s; ++i) {
          const double2 z = (r < warm && i < warm) ? Zg[(long)r * JMAX + i] : make_double2(r == i ? 1.0 : 0.0, 0.0);
          a = cadd(a, cmul(z, S.zs[i][S.perm[c]]));
        }
      } else {
        a = S.zs[r][S.perm[c]];
      }
      S.ar[r][c] = a.x;
      S.ai[r][c] = a.y;
    }
    __syncthreads();
    for (int e = tid; e < s * s; e += 256) {
      const int r = e / s, c = e % s;
      Zg[(long)r * JMAX + c] = make_double2(S.ar[r][c], S.ai[r][c]);
    }
    for (int i = tid; i < s; i += 256) ys[i] = make_double2(S.ar[i][j], S.ai[i][j]);
    warm = s;
    __syncthreads();
    // |x2|^2 = y^H (sum_m h_m K_m) y
    double acc = 0.0;
    for (int e = tid; e < s * s; e += 256) {
      const int i = e / s, l = e % s;
      double2 kk = make_double2(0.0, 0.0);
      for (int m = 0; m < M; ++m) {
        const double2 k = K[((long)m * JMAX + i) * JMAX + l];
        kk.x += chh[m] * k.x;
        kk.y += chh[m] * k.y;
      }
      acc += cmul(cconj(ys[i]), cmul(kk, ys[l])).x;
    }
    red2[tid] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) red2[tid] += red2[tid + st];
      __syncthreads();
    }
    if (tid == 0) {
      const double n2 = red2[0];
      const double wv = swv;
      const double f = wsh[j] - wv;
      if (f > 0.0) slo = fmax(slo, wv);
      else shi = fmin(shi, wv);
      double wn = wv + f / (1.0 + fmax(n2, 0.0));
      if (!(wn > slo && wn < shi)) wn = 0.5 * (slo + shi);
      // (wv, y) is an exact eigenpair of G(wv); its distance to the root is ~|wn - wv|, which only has
      // to stay well below the residual tolerance of the outer iteration
      const double wtol = fmin(1e-10, 1e-3 * tol) * fmax(1.0, fabs(wv));
      sdone = (fabs(wn - wv) <= wtol || (shi - slo) <= 1e-15 * fmax(1.0, fabs(wv))) ? 1 : 0;
      R.omega = wv;
      R.w = wsh[j];
      R.rq = (wsh[j] + wv * fmax(n2, 0.0)) / (1.0 + fmax(n2, 0.0));
      R.n2 = n2;
      R.status = 0;
      R.ysize = s;
      if (!sdone) swv = wn;
    }
    wrote = true;
    for (int i = tid; i < s; i += 256) Ybr[(long)E.slot * JMAX + i] = ys[i];
    __syncthreads();
    if (sdone) break;
  }
  if (tid == 0) {
    if (status == 0 && wrote) {
      if (!(R.omega < hi0 - 1e-12 * fabs(hi0))) R.status = 1;
      // the root lies below the lowest point the shifted map may evaluate
      if (map.inv && swlo > slo0 && R.omega <= swlo + 1e-9 * fmax(1.0, fabs(swlo))) R.status = 4;
    }
    R.zsize = wrote ? s : 0;
    res[blockIdx.x] = R;
  }
}

// ---------------------------------------------------------------------------
// Small kernels on the singles space (ns = nc nv elements per vector)
// ---------------------------------------------------------------------------

// Y[i][c] = scale_c Ybr[slot_c][i]  (s x q, ld q)
__global__ void k_fold_gather_y(const double2* __restrict__ Ybr, const int* __restrict__ slot,
                                const double* __restrict__ scale, int s, int q, double2* __restrict__ Y) {
  for (int e = threadIdx.x; e < s * q; e += blockDim.x) {
    const int i = e / q, c = e % q;
    Y[e] = cscale(Ybr[(long)slot[c] * JMAX + i], scale ? scale[c] : 1.0);
  }
}

// For the c-th of q roots (grid (blocks over e, q)): x1 = V y_c, r1 = S1 y_c + Sx[c] - om_c x1 (Sx: the
// M12 x2 part, singles of rows with stride ldx), written to row row[c] of X1 and R1 (row c without a
// row list); npart[c][blk] = the block's share of |r1|^2.
__global__ __launch_bounds__(256) void k_fold_resid(const double2* __restrict__ V, const double2* __restrict__ S1,
                                                     int s, long ns, const double2* __restrict__ Y, int q,
                                                     const double* __restrict__ om, const double2* __restrict__ Sx,
                                                     long ldx, const int* __restrict__ row,
                                                     double2* __restrict__ X1, double2* __restrict__ R1,
                                                     double* __restrict__ npart) {
  __shared__ double2 yc[JMAX];
  __shared__ double red[256];
  const int j = blockIdx.y;
  const long orow = row ? row[j] : j;
  for (int i = threadIdx.x; i < s; i += 256) yc[i] = Y[(long)i * q + j];
  __syncthreads();
  double acc = 0.0;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < ns; e += (long)gridDim.x * 256) {
    double2 x = make_double2(0.0, 0.0), r = Sx[(long)j * ldx + e];
    for (int i = 0; i < s; ++i) {
      x = cadd(x, cmul(V[(long)i * ns + e], yc[i]));
      r = cadd(r, cmul(S1[(long)i * ns + e], yc[i]));
    }
    r.x -= om[j] * x.x;
    r.y -= om[j] * x.y;
    X1[orow * ns + e] = x;
    R1[orow * ns + e] = r;
    acc += r.x * r.x + r.y * r.y;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) npart[(long)j * gridDim.x + blockIdx.x] = red[0];
}

// T[c][e] = r1[root_c][e] / (om_c - d11_e - nu_e / (om_c - Dbar_e)), the approximate diagonal of the
// folded operator minus omega, kept away from zero
__global__ void k_fold_newdir(const double2* __restrict__ R1, long ns, const int* __restrict__ root,
                              const double* __restrict__ om, int q, const double* __restrict__ d11,
                              const double* __restrict__ pnu, const double* __restrict__ pdb,
                              double2* __restrict__ T) {
  const long total = (long)q * ns;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int c = (int)(t / ns);
    const long e = t - (long)c * ns;
    const double w = om[c];
    double den = w - d11[e];
    const double gap = w - pdb[e];
    if (pnu[e] > 0.0 && fabs(gap) > 1e-12) den -= pnu[e] / gap;
    if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
    const double2 r = R1[(long)root[c] * ns + e];
    T[t] = make_double2(r.x / den, r.y / den);
  }
}

// rows r < q of T (ld ns): unit vectors at idx[r]
__global__ void k_fold_unit(double2* __restrict__ T, int q, long ns, const int* __restrict__ idx) {
  const long total = (long)q * ns;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int r = (int)(t / ns);
    const long e = t - (long)r * ns;
    T[t] = make_double2(e == idx[r] ? 1.0 : 0.0, 0.0);
  }
}

// H (ld JMAX): the rows i < snew of the new columns [s, snew) are computed; mirror them into the new rows
// (upper triangle of the new block wins) and make the diagonal real
__global__ void k_fold_herm_fill(double2* __restrict__ H, int s, int snew) {
  const int q = snew - s;
  for (int e = threadIdx.x; e < snew * q; e += blockDim.x) {
    const int i = e / q, jn = s + e % q;
    if (i < jn) H[(long)jn * JMAX + i] = cconj(H[(long)i * JMAX + jn]);
    else if (i == jn) H[(long)i * JMAX + i].y = 0.0;
  }
}

// Moments of the columns [c0, c0 + qc) from the reduced tile Kt[m][i][j] (i < srows, j < qc):
// K[m][i][c0 + j] = Kt, and for the old rows i < c0 the mirror K[m][c0 + j][i] = conj(Kt)
__global__ void k_fold_cheb_scatter(const double2* __restrict__ Kt, int mm, int srows, int c0, int qc,
                                    double2* __restrict__ K) {
  const long total = (long)mm * srows * qc;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int j = (int)(t % qc);
    const long r = t / qc;
    const int i = (int)(r % srows), m = (int)(r / srows);
    const double2 v = Kt[t];
    K[((long)m * JMAX + i) * JMAX + c0 + j] = v;
    if (i < c0) K[((long)m * JMAX + c0 + j) * JMAX + i] = cconj(v);
  }
}

// ov[c][b] = |sum_i conj(PG[i][c]) y_b[i]|^2 / ((1 + n2_b) gn_c): overlap of the Ritz singles of entry b
// (normalised with |x|^2 = 1 + |x2|^2) with guess c.  PG = V^H g (s x k, ld k).
__global__ void k_fold_overlap(const double2* __restrict__ PG, int s, int k, const double2* __restrict__ Ybr,
                               const FoldEntry* __restrict__ ent, const FoldResult* __restrict__ res, int nbr,
                               const double* __restrict__ gn, double* __restrict__ ov) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < k * nbr; t += gridDim.x * blockDim.x) {
    const int c = t / nbr, b = t % nbr;
    const double2* y = Ybr + (long)ent[b].slot * JMAX;
    double2 a = make_double2(0.0, 0.0);
    for (int i = 0; i < s; ++i) a = cadd(a, cmul(cconj(PG[(long)i * k + c]), y[i]));
    ov[t] = (a.x * a.x + a.y * a.y) / ((1.0 + fmax(res[b].n2, 0.0)) * fmax(gn[c], 1e-300));
  }
}

// Restart basis: columns c < k are the Ritz vectors y of the roots (slots rs[c]), columns k <= c < nk the
// next eigenvectors of G of the highest root (Zbr of slot zslot); two passes of modified Gram-Schmidt,
// columns whose norm falls below 1e-8 dropped.  C (s x kc, ld kc) and kc = *count.
__global__ __launch_bounds__(256) void k_fold_restart_basis(const double2* __restrict__ Ybr,
                                                             const double2* __restrict__ Zbr,
                                                             const int* __restrict__ rs, int k, int zslot, int s,
                                                             int nk, double2* __restrict__ C,
                                                             int* __restrict__ count) {
  __shared__ double2 cm[JMAX][JMAX + 1];
  __shared__ double2 red[256];
  __shared__ int kc;
  const int tid = threadIdx.x;
  for (int e = tid; e < s * nk; e += 256) {
    const int i = e / nk, c = e % nk;
    cm[i][c] = c < k ? Ybr[(long)rs[c] * JMAX + i] : Zbr[((long)zslot * JMAX + i) * JMAX + c];
  }
  if (tid == 0) kc = 0;
  __syncthreads();
  for (int c = 0; c < nk; ++c) {
    for (int pass = 0; pass < 2; ++pass)
      for (int p = 0; p < kc; ++p) {
        double2 a = make_double2(0.0, 0.0);
        for (int i = tid; i < s; i += 256) a = cadd(a, cmul(cconj(cm[i][p]), cm[i][c]));
        red[tid] = a;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
          if (tid < st) red[tid] = cadd(red[tid], red[tid + st]);
          __syncthreads();
        }
        const double2 d = red[0];
        __syncthreads();
        for (int i = tid; i < s; i += 256) {
          const double2 v = cmul(d, cm[i][p]);
          cm[i][c].x -= v.x;
          cm[i][c].y -= v.y;
        }
        __syncthreads();
      }
    double a = 0.0;
    for (int i = tid; i < s; i += 256) a += cm[i][c].x * cm[i][c].x + cm[i][c].y * cm[i][c].y;
    red[tid] = make_double2(a, 0.0);
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) red[tid].x += red[tid + st].x;
      __syncthreads();
    }
    const double nn = sqrt(red[0].x);
    __syncthreads();
    if (nn >= 1e-8) {
      for (int i = tid; i < s; i += 256) cm[i][kc] = cscale(cm[i][c], 1.0 / nn);
      __syncthreads();
      if (tid == 0) ++kc;
    }
    __syncthreads();
  }
  for (int e = tid; e < s * kc; e += 256) {
    const int i = e / kc, c = e % kc;
    C[e] = cm[i][c];
  }
  if (tid == 0) *count = kc;
}

// A_b <- C^H A_b C for the matrices A_b = base + b * stride (s x s, ld JMAX); C is s x kc (ld kc).
// One workgroup per matrix; A is read from global memory before it is overwritten.
__global__ __launch_bounds__(256) void k_fold_rot_small(double2* __restrict__ base, long stride, int s,
                                                         const double2* __restrict__ C, int kc) {
  __shared__ double2 cs[JMAX][JMAX + 1];
  __shared__ double2 t1[JMAX][JMAX + 1];
  double2* A = base + (long)blockIdx.x * stride;
  const int tid = threadIdx.x;
  for (int e = tid; e < s * kc; e += 256) cs[e / kc][e % kc] = C[e];
  __syncthreads();
  for (int e = tid; e < s * kc; e += 256) {
    const int i = e / kc, c = e % kc;
    double2 a = make_double2(0.0, 0.0);
    for (int l = 0; l < s; ++l) a = cadd(a, cmul(A[(long)i * JMAX + l], cs[l][c]));
    t1[i][c] = a;
  }
  __syncthreads();
  for (int e = tid; e < kc * kc; e += 256) {
    const int r = e / kc, c = e % kc;
    double2 a = make_double2(0.0, 0.0);
    for (int i = 0; i < s; ++i) a = cadd(a, cmul(cconj(cs[i][r]), t1[i][c]));
    A[(long)r * JMAX + c] = a;
  }
}

// Squared norms of the rows of T (q x ns): one workgroup per row
__global__ __launch_bounds__(256) void k_fold_rownorm(const double2* __restrict__ T, long ns,
                                                       double* __restrict__ n2) {
  __shared__ double red[256];
  const double2* t = T + (long)blockIdx.x * ns;
  double a = 0.0;
  for (long e = threadIdx.x; e < ns; e += 256) a += t[e].x * t[e].x + t[e].y * t[e].y;
  red[threadIdx.x] = a;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) n2[blockIdx.x] = red[0];
}

// Modified Gram-Schmidt of the rows of T (q x ns) among themselves, two
// passes per row, in row order: row r is kept (normalised, moved to position
// kept) unless its norm after the projections is at most 1e-10 of its norm
// n0[r] = sqrt(n2[r]) before any projection, or n0[r] is zero or not finite.
// One workgroup of 1024 threads; *count = the number kept.
__global__ __launch_bounds__(1024) void k_fold_mgs(double2* __restrict__ T, int q, long ns,
                                                    const double* __restrict__ n2, int* __restrict__ count) {
  __shared__ double2 red[1024];
  __shared__ int kept;
  const int tid = threadIdx.x;
  if (tid == 0) kept = 0;
  __syncthreads();
  for (int r = 0; r < q; ++r) {
    const double n0 = sqrt(n2[r]);
    if (!(n0 > 0.0) || !isfinite(n0)) continue;   // uniform: n2 is the same for every thread
    double2* t = T + (long)r * ns;
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < kept; ++i) {
        const double2* v = T + (long)i * ns;
        double2 a = make_double2(0.0, 0.0);
        for (long e = tid; e < ns; e += 1024) a = cadd(a, cmul(cconj(v[e]), t[e]));
        red[tid] = a;
        __syncthreads();
        for (int st = 512; st > 0; st >>= 1) {
          if (tid < st) red[tid] = cadd(red[tid], red[tid + st]);
          __syncthreads();
        }
        const double2 d = red[0];
        __syncthreads();
        for (long e = tid; e < ns; e += 1024) {
          const double2 w = cmul(d, v[e]);
          t[e].x -= w.x;
          t[e].y -= w.y;
        }
        __syncthreads();
      }
    double a = 0.0;
    for (long e = tid; e < ns; e += 1024) a += t[e].x * t[e].x + t[e].y * t[e].y;
    red[tid] = make_double2(a, 0.0);
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
      if (tid < st) red[tid].x += red[tid + st].x;
      __syncthreads();
    }
    const double n1 = sqrt(red[0].x);
    const int kk = kept;
    __syncthreads();
    if (n1 <= 1e-10 * n0) continue;
    double2* dst = T + (long)kk * ns;
    for (long e = tid; e < ns; e += 1024) dst[e] = cscale(t[e], 1.0 / n1);
    __syncthreads();
    if (tid == 0) kept = kk + 1;
    __syncthreads();
  }
  if (tid == 0) *count = kept;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
adc2_status fold_solve_launch(const double2* H, const double2* K, int s, int Mmax, const FoldMap& map, double Dmin,
                              double hi0, double tol, const double* hw, const FoldEntry* ent, int n,
                              FoldResult* res, double2* Ybr, double2* Zbr, FoldBounds* bnd, hipStream_t st) {
  if (s <= 0 || s > JMAX || n <= 0) {
    set_error("adc2_davidson (folded): projected problem size out of range");
    return ADC2_ERR_ARG;
  }
  k_fold_solve<<<n, 256, 0, st>>>(H, K, s, Mmax, map, Dmin, hi0, tol, hw, ent, res, Ybr, Zbr, bnd);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

adc2_status fold_gather_y(const double2* Ybr, const int* slot, const double* scale, int s, int q, double2* Y,
                          hipStream_t st) {
  k_fold_gather_y<<<1, 256, 0, st>>>(Ybr, slot, scale, s, q, Y);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

int fold_resid_blocks(long ns) { return (int)std::max<long>(1, std::min<long>(256, (ns + 1023) / 1024)); }

adc2_status fold_resid(const double2* V, const double2* S1, int s, long ns, const double2* Y, int q, const double* om,
                       const double2* Sx, long ldx, const int* row, double2* X1, double2* R1, double* npart,
                       hipStream_t st) {
  if (q <= 0) return ADC2_OK;
  dim3 g(fold_resid_blocks(ns), q);
  k_fold_resid<<<g, 256, 0, st>>>(V, S1, s, ns, Y, q, om, Sx, ldx, row, X1, R1, npart);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

adc2_status fold_newdir(const double2* R1, long ns, const int* root, const double* om, int q, const double* d11,
                        const double* pnu, const double* pdb, double2* T, hipStream_t st) {
  const long total = (long)q * ns;
  k_fold_newdir<<<(unsigned)std::min<long>(4096, (total + 255) / 256), 256, 0, st>>>(R1, ns, root, om, q, d11, pnu,
                                                                                       pdb, T);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

adc2_status fold_unit(double2* T, int q, long ns, const int* idx, hipStream_t st) {
  const long total = (long)q * ns;
  k_fold_unit<<<(unsigned)std::min<long>(4096, (total + 255) / 256), 256, 0, st>>>(T, q, ns, idx);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

adc2_status fold_herm_fill(double2* H, int s, int snew, hipStream_t st) {
  k_fold_herm_fill<<<1, 256, 0, st>>>(H, s, snew);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

adc2_status fold_cheb_scatter(const double2* Kt, int mm, int srows, int c0, int qc, double2* K, hipStream_t st) {
  const long total = (long)mm * srows * qc;
  k_fold_cheb_scatter<<<(unsigned)std::min<long>(4096, (total + 255) / 256), 256, 0, st>>>(Kt, mm, srows, c0, qc, K);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

adc2_status fold_overlap(const double2* PG, int s, int k, const double2* Ybr, const FoldEntry* ent,
                         const FoldResult* res, int nbr, const double* gn, double* ov, hipStream_t st) {
  k_fold_overlap<<<(unsigned)std::max(1, (k * nbr + 255) / 256), 256, 0, st>>>(PG, s, k, Ybr, ent, res, nbr, gn, ov);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

adc2_status fold_restart_basis(const double2* Ybr, const double2* Zbr, const int* rs, int k, int zslot, int s, int nk,
                               double2* C, int* count, hipStream_t st) {
  if (s > JMAX || nk > JMAX) {
    set_error("adc2_davidson (folded): restart basis out of range");
    return ADC2_ERR_ARG;
  }
  k_fold_restart_basis<<<1, 256, 0, st>>>(Ybr, Zbr, rs, k, zslot, s, nk, C, count);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

adc2_status fold_rot_small(double2* base, long stride, int nmat, int s, const double2* C, int kc, hipStream_t st) {
  if (nmat <= 0) return ADC2_OK;
  k_fold_rot_small<<<nmat, 256, 0, st>>>(base, stride, s, C, kc);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

adc2_status fold_rownorm(const double2* T, int q, long ns, double* n2, hipStream_t st) {
  if (q <= 0) return ADC2_OK;
  k_fold_rownorm<<<q, 256, 0, st>>>(T, ns, n2);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

adc2_status fold_mgs(double2* T, int q, long ns, const double* n2, int* count, hipStream_t st) {
  k_fold_mgs<<<1, 1024, 0, st>>>(T, q, ns, n2, count);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

}  // namespace adc2
