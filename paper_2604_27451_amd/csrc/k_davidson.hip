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
#include "jacobi.h"
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
// Subspace eigensolve: the upper triangle of G (row-major, ldg) into LDS and
// the parallel cyclic Jacobi of jacobi.h; ascending eigenvalues w[n] and
// eigenvectors as columns of Z (row-major, ldz).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_heevj(const double2* __restrict__ G, int n, int ldg,
                                                double* __restrict__ w, double2* __restrict__ Z, int ldz) {
  __shared__ JacobiSmem S;
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += 256) {
    const int i = e / n, j = e % n;
    double x, y;
    if (i <= j) {
      const double2 g = G[(long)i * ldg + j];
      x = g.x;
      y = (i == j) ? 0.0 : g.y;
    } else {
      const double2 g = G[(long)j * ldg + i];
      x = g.x;
      y = -g.y;
    }
    S.ar[i][j] = x;
    S.ai[i][j] = y;
  }
  __syncthreads();
  jacobi_lds(S, n);
  for (int i = tid; i < n; i += 256) w[i] = S.ar[S.perm[i]][S.perm[i]];
  for (int e = tid; e < n * n; e += 256) {
    const int r = e / n, c = e % n;
    Z[(long)r * ldz + c] = S.zs[r][S.perm[c]];
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
