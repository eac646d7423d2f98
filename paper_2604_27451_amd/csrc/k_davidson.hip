// k_davidson.hip -- FP64 kernels of the block Davidson solver for the
// Hermitian eigenproblem M X = X Omega, X^H X = 1 (paper Eq. 11).
//
// All of these stream ADC vectors (complex128, length dim) from HBM once per
// call and are bandwidth-bound: block Gram products V^H W, linear
// combinations V C, the Ritz residual M x - theta x with its norms, and the
// diagonal preconditioner (theta - diag M)^-1.  The subspace matrix is
// diagonalised by a one-workgroup parallel cyclic Jacobi method (complex
// Hermitian rotations), so no step of the solver leaves the GPU except the
// handful of residual norms the host reads to decide convergence.
#include <algorithm>
#include <cmath>

#include "internal.h"
#include "tile.h"

namespace adc2 {

constexpr int GB = 16;     // Gram tile (rows of V x rows of W)
constexpr int GCH = 64;    // elements per LDS chunk

int dav_nblk(long dim) { return (int)std::max<long>(1, std::min<long>(1024, (dim + 4095) / 4096)); }

// partial[blk][ii][jj] = sum_{e in this block's chunks} conj(V[i0+ii][e]) W[j0+jj][e]
__global__ __launch_bounds__(256) void k_gram_part(const double2* __restrict__ V, int s,
                                                    const double2* __restrict__ W, int m, long dim, int nchunkblk,
                                                    double2* __restrict__ part) {
  __shared__ double2 vs[GB][GCH + 1];
  __shared__ double2 ws[GB][GCH + 1];
  const int nbj = (m + GB - 1) / GB;
  const int tileid = blockIdx.y;
  const int i0 = (tileid / nbj) * GB, j0 = (tileid % nbj) * GB;
  const int tid = threadIdx.x;
  const int ii = tid / GB, jj = tid % GB;
  double2 acc = make_double2(0, 0);
  const long nch = (dim + GCH - 1) / GCH;
  for (long ch = blockIdx.x; ch < nch; ch += nchunkblk) {
    const long e0 = ch * GCH;
    __syncthreads();
    for (int q = 0; q < (2 * GB * GCH) / 256; ++q) {
      const int idx = q * 256 + tid;
      const int row = idx / GCH, e = idx % GCH;
      const long ge = e0 + e;
      if (row < GB) {
        const int i = i0 + row;
        vs[row][e] = (i < s && ge < dim) ? V[(long)i * dim + ge] : make_double2(0, 0);
      } else {
        const int j = j0 + row - GB;
        ws[row - GB][e] = (j < m && ge < dim) ? W[(long)j * dim + ge] : make_double2(0, 0);
      }
    }
    __syncthreads();
#pragma unroll 8
    for (int e = 0; e < GCH; ++e) acc = cadd(acc, cdotc(vs[ii][e], ws[jj][e]));
  }
  part[((long)tileid * nchunkblk + blockIdx.x) * 256 + tid] = acc;
}

__global__ void k_gram_reduce(const double2* __restrict__ part, int s, int m, int nchunkblk, double2* __restrict__ G,
                              int ldg) {
  const int nbj = (m + GB - 1) / GB;
  const int i = blockIdx.x;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    const int tileid = (i / GB) * nbj + j / GB;
    const int t = (i % GB) * GB + (j % GB);
    double2 acc = make_double2(0, 0);
    for (int b = 0; b < nchunkblk; ++b) acc = cadd(acc, part[((long)tileid * nchunkblk + b) * 256 + t]);
    G[(long)i * ldg + j] = acc;
  }
}

adc2_status dav_gram(const double2* V, int s, const double2* W, int m, long dim, double2* G, int ldg,
                     double2* scratch, hipStream_t st) {
  if (s <= 0 || m <= 0) return ADC2_OK;
  const int ntile = ((s + GB - 1) / GB) * ((m + GB - 1) / GB);
  const int nb = dav_nblk(dim);
  dim3 g(nb, ntile);
  k_gram_part<<<g, 256, 0, st>>>(V, s, W, m, dim, nb, scratch);
  ADC2_CHECK_LAUNCH();
  k_gram_reduce<<<s, 64, 0, st>>>(scratch, s, m, nb, G, ldg);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

// out[j][e] (+)= alpha * sum_i V[i][e] C[i*ldc + j]   for j < m (<= 32), i < s (<= 64)
__global__ __launch_bounds__(256) void k_combine(const double2* __restrict__ V, int s,
                                                  const double2* __restrict__ C, int ldc, int m, long dim,
                                                  double2* __restrict__ out, double alpha, int accumulate) {
  __shared__ double2 cs[64 * 32];
  for (int t = threadIdx.x; t < s * m; t += blockDim.x) {
    const int i = t / m, j = t % m;
    cs[i * 32 + j] = C[(long)i * ldc + j];
  }
  __syncthreads();
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < dim; e += (long)gridDim.x * blockDim.x) {
    for (int jb = 0; jb < m; jb += 8) {
      double2 acc[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = make_double2(0, 0);
      for (int i = 0; i < s; ++i) {
        const double2 v = V[(long)i * dim + e];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (jb + q < m) acc[q] = cadd(acc[q], cmul(v, cs[i * 32 + jb + q]));
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (jb + q < m) {
          double2* p = out + (long)(jb + q) * dim + e;
          const double2 r = cscale(acc[q], alpha);
          *p = accumulate ? cadd(*p, r) : r;
        }
      }
    }
  }
}

adc2_status dav_combine(const double2* V, int s, const double2* C, int ldc, int m, long dim, double2* out,
                        double alpha, bool accumulate, hipStream_t st) {
  if (m <= 0) return ADC2_OK;
  if (s > 64 || m > 32) {
    set_error("dav_combine: subspace block too large");
    return ADC2_ERR_ARG;
  }
  const int g = (int)std::min<long>(8192, (dim + 255) / 256);
  k_combine<<<g, 256, 0, st>>>(V, s, C, ldc, m, dim, out, alpha, accumulate);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

// X[k][e] = sum_i V[i][e] Y[i][k];  R[k][e] = sum_i S[i][e] Y[i][k] - theta_k X[k][e]
// norms2_partial[blk][k] = sum over this block's elements |R[k][e]|^2
// Roots are processed in groups of 8 so every accumulator index is static.
__global__ __launch_bounds__(256) void k_residual(const double2* __restrict__ V, const double2* __restrict__ Sg, int s,
                                                   const double2* __restrict__ Yc, int ldy,
                                                   const double* __restrict__ theta, int k, long dim,
                                                   double2* __restrict__ Xout, double2* __restrict__ R,
                                                   double* __restrict__ npart) {
  __shared__ double2 ys[64 * 32];
  __shared__ double th[32];
  __shared__ double red[8][256];
  for (int t = threadIdx.x; t < s * k; t += blockDim.x) {
    const int i = t / k, j = t % k;
    ys[i * 32 + j] = Yc[(long)i * ldy + j];
  }
  if (threadIdx.x < k) th[threadIdx.x] = theta[threadIdx.x];
  __syncthreads();
  for (int jb = 0; jb < k; jb += 8) {
    double nrm[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) nrm[q] = 0.0;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < dim; e += (long)gridDim.x * blockDim.x) {
      double2 ax[8], ar[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) ax[q] = ar[q] = make_double2(0, 0);
      for (int i = 0; i < s; ++i) {
        const double2 v = V[(long)i * dim + e];
        const double2 sv = Sg[(long)i * dim + e];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (jb + q < k) {
            const double2 y = ys[i * 32 + jb + q];
            ax[q] = cadd(ax[q], cmul(v, y));
            ar[q] = cadd(ar[q], cmul(sv, y));
          }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (jb + q < k) {
          const int j = jb + q;
          const double2 r = csub(ar[q], cscale(ax[q], th[j]));
          if (Xout) Xout[(long)j * dim + e] = ax[q];
          R[(long)j * dim + e] = r;
          nrm[q] += r.x * r.x + r.y * r.y;
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) red[q][threadIdx.x] = nrm[q];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st) {
#pragma unroll
        for (int q = 0; q < 8; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + st];
      }
      __syncthreads();
    }
    if (threadIdx.x < 8 && jb + threadIdx.x < k) npart[(long)blockIdx.x * 32 + jb + threadIdx.x] = red[threadIdx.x][0];
    __syncthreads();
  }
}

adc2_status dav_residual(const double2* V, const double2* Sg, int s, const double2* Yc, int ldy,
                         const double* theta, int k, long dim, double2* Xout, double2* R, double* npart, int nblk,
                         hipStream_t st) {
  if (s > 64 || k > 32) {
    set_error("dav_residual: block too large");
    return ADC2_ERR_ARG;
  }
  k_residual<<<nblk, 256, 0, st>>>(V, Sg, s, Yc, ldy, theta, k, dim, Xout, R, npart);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

__global__ void k_norms(const double2* __restrict__ T, int k, long dim, double* __restrict__ npart) {
  __shared__ double red[256];
  for (int j = 0; j < k; ++j) {
    double a = 0.0;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < dim; e += (long)gridDim.x * blockDim.x) {
      const double2 v = T[(long)j * dim + e];
      a += v.x * v.x + v.y * v.y;
    }
    red[threadIdx.x] = a;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) npart[(long)blockIdx.x * 32 + j] = red[0];
    __syncthreads();
  }
}

adc2_status dav_norms(const double2* T, int k, long dim, double* npart, int nblk, hipStream_t st) {
  k_norms<<<nblk, 256, 0, st>>>(T, k, dim, npart);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

// T[k][e] /= (theta_k - diag[e]), with |denominator| floored at 1e-6
__global__ void k_precond(double2* __restrict__ T, const double* __restrict__ theta, const double* __restrict__ diag,
                          int k, long dim) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < dim; e += (long)gridDim.x * blockDim.x) {
    const double d = diag[e];
    for (int j = 0; j < k; ++j) {
      double den = theta[j] - d;
      if (fabs(den) < 1e-6) den = den < 0 ? -1e-6 : 1e-6;
      double2* p = T + (long)j * dim + e;
      *p = cscale(*p, 1.0 / den);
    }
  }
}

adc2_status dav_precondition(double2* T, const double* theta, const double* diag, int k, long dim, hipStream_t st) {
  const int g = (int)std::min<long>(8192, (dim + 255) / 256);
  k_precond<<<g, 256, 0, st>>>(T, theta, diag, k, dim);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

__global__ void k_scale_cols(double2* __restrict__ T, int k, long dim, const double* __restrict__ s) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < dim * k; e += (long)gridDim.x * blockDim.x) {
    const int j = (int)(e / dim);
    T[e] = cscale(T[e], s[j]);
  }
}

adc2_status dav_scale_columns(double2* T, int k, long dim, const double* s, hipStream_t st) {
  const int g = (int)std::min<long>(8192, (dim * k + 255) / 256);
  k_scale_cols<<<g, 256, 0, st>>>(T, k, dim, s);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

__global__ void k_unit_guess(double2* __restrict__ V, int g, long dim, const int* __restrict__ idx) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < dim * g; e += (long)gridDim.x * blockDim.x) {
    const int j = (int)(e / dim);
    const long r = e % dim;
    V[e] = make_double2(r == idx[j] ? 1.0 : 0.0, 0.0);
  }
}

adc2_status dav_unit_guess(double2* V, int g, long dim, const int* idx, hipStream_t st) {
  const int gr = (int)std::min<long>(8192, (dim * g + 255) / 256);
  k_unit_guess<<<gr, 256, 0, st>>>(V, g, dim, idx);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

// ---------------------------------------------------------------------------
// Parallel cyclic Jacobi for a complex Hermitian n x n matrix (n <= 64).
// Reads the upper triangle of G (row-major, ldg), writes ascending
// eigenvalues w[n] and eigenvectors as columns of Z (row-major, ldz).
// Pair (p,q) rotation J = [[c, s e], [-s conj(e), c]], e = a_pq/|a_pq|,
// t = sign(tau)/(|tau| + sqrt(1+tau^2)), tau = (a_qq - a_pp)/(2|a_pq|),
// zeroes a_pq of J^H A J; all n/2 disjoint pairs of a round-robin round are
// applied together.
// ---------------------------------------------------------------------------
constexpr int JMAX = 64;

__global__ __launch_bounds__(256) void k_heevj(const double2* __restrict__ G, int n, int ldg,
                                                double* __restrict__ w, double2* __restrict__ Z, int ldz) {
  __shared__ double ar[JMAX][JMAX];
  __shared__ double ai[JMAX][JMAX];
  __shared__ double2 zs[JMAX][JMAX];
  __shared__ double rc[JMAX / 2], rs[JMAX / 2];
  __shared__ double2 re[JMAX / 2];
  __shared__ int rp[JMAX / 2], rq[JMAX / 2];
  __shared__ double red[256];
  __shared__ int done;
  const int tid = threadIdx.x;
  const int N = (n + 1) & ~1;   // even number of players (player n is a dummy if n is odd)
  for (int e = tid; e < JMAX * JMAX; e += 256) {
    const int i = e / JMAX, j = e % JMAX;
    double x = 0, y = 0;
    if (i < n && j < n) {
      if (i <= j) {
        const double2 g = G[(long)i * ldg + j];
        x = g.x;
        y = (i == j) ? 0.0 : g.y;
      } else {
        const double2 g = G[(long)j * ldg + i];
        x = g.x;
        y = -g.y;
      }
    }
    ar[i][j] = x;
    ai[i][j] = y;
    zs[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int npair = N / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    // convergence test: off-diagonal Frobenius norm vs full norm
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n * n; e += 256) {
      const int i = e / n, j = e % n;
      const double v = ar[i][j] * ar[i][j] + ai[i][j] * ai[i][j];
      tot += v;
      if (i != j) off += v;
    }
    red[tid] = off;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) red[tid] += red[tid + st];
      __syncthreads();
    }
    const double offs = red[0];
    __syncthreads();
    red[tid] = tot;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) red[tid] += red[tid + st];
      __syncthreads();
    }
    if (tid == 0) done = (offs <= 1e-30 * red[0] || offs == 0.0) ? 1 : 0;
    __syncthreads();
    if (done) break;
    for (int round = 0; round < N - 1; ++round) {
      if (tid < npair) {
        // round-robin: player 0 fixed, players 1..N-1 rotate
        int a, b;
        if (tid == 0) {
          a = 0;
          b = 1 + (round % (N - 1));
        } else {
          a = 1 + ((round + tid) % (N - 1));
          b = 1 + ((round + N - 1 - tid) % (N - 1));
        }
        const int p = min(a, b), q = max(a, b);
        double c = 1.0, s = 0.0;
        double2 ee = make_double2(1.0, 0.0);
        if (q < n) {
          const double br = ar[p][q], bi = ai[p][q];
          const double mag = sqrt(br * br + bi * bi);
          const double app = ar[p][p], aqq = ar[q][q];
          if (mag > 1e-300 && mag > 1e-18 * (fabs(app) + fabs(aqq))) {
            const double tau = (aqq - app) / (2.0 * mag);
            const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            ee = make_double2(br / mag, bi / mag);
          }
        }
        rp[tid] = p;
        rq[tid] = q;
        rc[tid] = c;
        rs[tid] = s;
        re[tid] = ee;
      }
      __syncthreads();
      // column update A <- A J and Z <- Z J
      for (int it = tid; it < npair * n; it += 256) {
        const int pr = it / n, r = it % n;
        const int p = rp[pr], q = rq[pr];
        if (q >= n || rs[pr] == 0.0) continue;
        const double c = rc[pr], s = rs[pr];
        const double2 e = re[pr];
        const double2 x = make_double2(ar[r][p], ai[r][p]);
        const double2 y = make_double2(ar[r][q], ai[r][q]);
        // new_p = c x - s conj(e) y ; new_q = s e x + c y
        const double2 ny = cmul(cconj(e), y);
        const double2 nx = cmul(e, x);
        ar[r][p] = c * x.x - s * ny.x;
        ai[r][p] = c * x.y - s * ny.y;
        ar[r][q] = s * nx.x + c * y.x;
        ai[r][q] = s * nx.y + c * y.y;
        const double2 zx = zs[r][p], zy = zs[r][q];
        const double2 zny = cmul(cconj(e), zy);
        const double2 znx = cmul(e, zx);
        zs[r][p] = make_double2(c * zx.x - s * zny.x, c * zx.y - s * zny.y);
        zs[r][q] = make_double2(s * znx.x + c * zy.x, s * znx.y + c * zy.y);
      }
      __syncthreads();
      // row update A <- J^H A : new_p = c x - s e y ; new_q = s conj(e) x + c y
      for (int it = tid; it < npair * n; it += 256) {
        const int pr = it / n, r = it % n;
        const int p = rp[pr], q = rq[pr];
        if (q >= n || rs[pr] == 0.0) continue;
        const double c = rc[pr], s = rs[pr];
        const double2 e = re[pr];
        const double2 x = make_double2(ar[p][r], ai[p][r]);
        const double2 y = make_double2(ar[q][r], ai[q][r]);
        const double2 ey = cmul(e, y);
        const double2 cx = cmul(cconj(e), x);
        ar[p][r] = c * x.x - s * ey.x;
        ai[p][r] = c * x.y - s * ey.y;
        ar[q][r] = s * cx.x + c * y.x;
        ai[q][r] = s * cx.y + c * y.y;
      }
      __syncthreads();
      if (tid < npair) {
        const int p = rp[tid], q = rq[tid];
        if (q < n && rs[tid] != 0.0) {
          ar[p][q] = ai[p][q] = ar[q][p] = ai[q][p] = 0.0;
          ai[p][p] = ai[q][q] = 0.0;
        }
      }
      __syncthreads();
    }
  }
  // sort ascending (selection by one thread; n <= 64)
  __shared__ int perm[JMAX];
  if (tid == 0) {
    for (int i = 0; i < n; ++i) perm[i] = i;
    for (int i = 0; i < n; ++i) {
      int best = i;
      for (int j = i + 1; j < n; ++j)
        if (ar[perm[j]][perm[j]] < ar[perm[best]][perm[best]]) best = j;
      const int t = perm[i];
      perm[i] = perm[best];
      perm[best] = t;
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += 256) w[i] = ar[perm[i]][perm[i]];
  for (int e = tid; e < n * n; e += 256) {
    const int r = e / n, c = e % n;
    Z[(long)r * ldz + c] = zs[r][perm[c]];
  }
}

adc2_status dav_heevj(const double2* G, int n, int ldg, double* w, double2* Z, int ldz, hipStream_t st) {
  if (n > JMAX || n <= 0) {
    set_error("dav_heevj: subspace dimension out of range");
    return ADC2_ERR_ARG;
  }
  k_heevj<<<1, 256, 0, st>>>(G, n, ldg, w, Z, ldz);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

}  // namespace adc2
