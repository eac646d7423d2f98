// k_sigma.hip -- sigma = M x for the CVS-ADC(2) matrix (paper Eq. 11-12,
// CVS section), FP64 complex on the FP64 MFMA.
//
// With r = [r1 (I,a) | r2 (I,j,a<b)] and the doubles state a+_a a+_b a_j a_I:
//   M21[(Ijab),(Kc)] = d_IK <ab||cj> - d_ac <Kb||Ij> + d_bc <Ka||Ij>
//   M22 = diag(e_a + e_b - e_I - e_j),  M12 = M21^H.
// The three-virtual integral <ab||cj> = (ac|bj) - (aj|bc) is never formed:
//   X^P_{Ia} = sum_c L^P_{ac} r_{Ic}                               (X-build)
//   s2_{Ijab} = sum_P (X^P_{Ia} L^P_{bj} - L^P_{aj} X^P_{Ib})
//             + sum_K (<Ka||Ij> r_{Kb} - r_{Ka} <Kb||Ij>) + D r2      (sigma2)
//   Y^P_{Ic}  = sum_{jd} conj(L^P_{dj}) r_{Ijcd}                       (Y-build)
//   s1_{Ia}   = sum_{Jb} M11 r1 + sum_{Pc} L^P_{ac} Y^P_{Ic}
//             - sum_{I',jb} conj(<Ib||I'j>) r_{I'jab}                 (sigma1)
// The sigma2 contraction is an antisymmetric rank-2K product evaluated on
// the upper tile pairs (a-blk <= b-blk) only, with the light core terms
// appended as nc extra K entries and D r2 fused into the epilogue.
#include <algorithm>
#include <vector>

#include "internal.h"
#include "tile.h"

namespace adc2 {

__host__ __device__ static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// generic  C[i][j] = alpha * sum_k A[i][k] B^T[j][k]  (both k-contiguous)
// ---------------------------------------------------------------------------
template <bool CA, bool CB>
__global__ __launch_bounds__(256) void k_gemm_rr(int M, int N, int K, const double2* __restrict__ A, long lda,
                                                  const double2* __restrict__ B, long ldb,
                                                  double2* __restrict__ C, long ldc, double alpha, int accumulate) {
  __shared__ TileSmem s;
  const int nbj = cdiv(N, TN);
  const int i0 = (blockIdx.x / nbj) * TM, j0 = (blockIdx.x % nbj) * TN;
  SrcR<CA> sa{A + (long)i0 * lda, lda, K, M - i0, 1.0};
  SrcR<CB> sb{B + (long)j0 * ldb, ldb, K, N - j0, 1.0};
  Acc acc;
  acc.zero();
  mainloop(s, sa, sb, 0, cdiv(K, TK), acc);
  for_each_acc(acc, [&](int r, int c, double2 v) {
    const int i = i0 + r, j = j0 + c;
    if (i < M && j < N) {
      double2* p = C + (long)i * ldc + j;
      v = cscale(v, alpha);
      *p = accumulate ? cadd(*p, v) : v;
    }
  });
}

adc2_status gemm_rr(int M, int N, int K, const double2* A, long lda, bool conjA, const double2* B, long ldb,
                    bool conjB, double2* C, long ldc, double alpha, bool accumulate, hipStream_t st) {
  if (M <= 0 || N <= 0) return ADC2_OK;
  const int nblk = cdiv(M, TM) * cdiv(N, TN);
  if (!conjA && !conjB)
    k_gemm_rr<false, false><<<nblk, 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc, alpha, accumulate);
  else if (conjA && !conjB)
    k_gemm_rr<true, false><<<nblk, 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc, alpha, accumulate);
  else if (!conjA && conjB)
    k_gemm_rr<false, true><<<nblk, 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc, alpha, accumulate);
  else
    k_gemm_rr<true, true><<<nblk, 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc, alpha, accumulate);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

// ---------------------------------------------------------------------------
// X-build:  X[mI][(P,a)] = sum_c r1[m][I][c] Lvv[P][a][c]
// ---------------------------------------------------------------------------
struct SrcR1Rows {   // element (k=c, i=mI) = r1 of vector m, core I
  static constexpr int MAP = RMAJOR;
  const double2* x;
  long dim;
  int nc, nv, nrows, i0;
  __device__ __forceinline__ double2 get(int k, int i) const {
    const int mi = i0 + i;
    if (k >= nv || mi >= nrows) return czero();
    const int m = mi / nc, I = mi - m * nc;
    return x[(long)m * dim + (long)I * nv + k];
  }
};

__global__ __launch_bounds__(256) void k_xbuild(const double2* __restrict__ x, long dim, int nc, int nv, int naux,
                                                 int nrows, const double2* __restrict__ Lvv,
                                                 double2* __restrict__ X) {
  __shared__ TileSmem s;
  const long ncol = (long)naux * nv;
  const int nbj = cdiv(ncol, TN);
  const long nblocks = (long)cdiv(nrows, TM) * nbj;
  const long lid = xcd_remap(blockIdx.x, nblocks);
  const int i0 = (int)(lid / nbj) * TM;
  const long j0 = (lid % nbj) * TN;
  SrcR1Rows sa{x, dim, nc, nv, nrows, i0};
  SrcR<false> sb{Lvv + j0 * nv, nv, nv, (int)min((long)TN, ncol - j0), 1.0};
  Acc acc;
  acc.zero();
  mainloop(s, sa, sb, 0, cdiv(nv, TK), acc);
  for_each_acc(acc, [&](int r, int c, double2 v) {
    const int mi = i0 + r;
    const long j = j0 + c;
    if (mi < nrows && j < ncol) X[(long)mi * ncol + j] = v;
  });
}

// ---------------------------------------------------------------------------
// sigma2 (antisymmetric rank-2K product + light core terms + D r2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void upper_pair(int t, int nb, int& ab, int& bb) {
  int r = 0;
  while (t >= nb - r) {
    t -= nb - r;
    ++r;
  }
  ab = r;
  bb = r + t;
}

__device__ __forceinline__ long pair_offset(int a, int b, int nv) {
  return (long)a * nv - (long)a * (a + 1) / 2 + (b - a - 1);
}

__global__ __launch_bounds__(256) void k_sigma2(const double2* __restrict__ xin, double2* __restrict__ sout,
                                                 long dim, const double2* __restrict__ X,
                                                 const double2* __restrict__ Lvo, const double2* __restrict__ Vt,
                                                 const double* __restrict__ eps, int m, int nc, int no, int nv,
                                                 int naux) {
  __shared__ TileSmem s;
  __shared__ double ea[TM], eb[TN];
  const int nb = (nv + TM - 1) / TM;
  const int ntp = nb * (nb + 1) / 2;
  const long nblocks = (long)m * nc * no * ntp;
  const long lid = xcd_remap(blockIdx.x, nblocks);
  const int t = (int)(lid % ntp);
  const int j = (int)((lid / ntp) % no);
  const int mI = (int)(lid / ((long)ntp * no));
  const int mv = mI / nc, I = mI - mv * nc;
  int abk, bbk;
  upper_pair(t, nb, abk, bbk);
  const int a0 = abk * TM, b0 = bbk * TN;
  const int o = nc + no;
  const long lds = (long)naux * nv;
  const double2* Xm = X + (long)mI * lds;
  const double2* Lj = Lvo + (long)(nc + j) * lds;
  const double2* Vij = Vt + ((long)(I * no + j) * nc) * nv;
  const double2* r1 = xin + (long)mv * dim;
  const int tid = threadIdx.x;
  if (tid < TM) ea[tid] = (a0 + tid < nv) ? eps[o + a0 + tid] : 0.0;
  else if (tid < TM + TN) eb[tid - TM] = (b0 + tid - TM < nv) ? eps[o + b0 + tid - TM] : 0.0;

  Acc acc;
  acc.zero();
  const int nkc = cdiv(naux + nc, TK);
  {
    SrcK2 A{Xm + a0, nv, naux, Vij + a0, nv, nc, nv - a0, 1.0};
    SrcK2 B{Lj + b0, nv, naux, r1 + b0, nv, nc, nv - b0, 1.0};
    mainloop(s, A, B, 0, nkc, acc);
  }
  {
    SrcK2 A{Lj + a0, nv, naux, r1 + a0, nv, nc, nv - a0, 1.0};
    SrcK2 B{Xm + b0, nv, naux, Vij + b0, nv, nc, nv - b0, -1.0};
    mainloop(s, A, B, 0, nkc, acc);
  }
  const long ns = (long)nc * nv;
  const long npair = (long)nv * (nv - 1) / 2;
  const long off = (long)mv * dim + ns + ((long)I * no + j) * npair;
  const double2* r2 = xin + off;
  double2* s2 = sout + off;
  const double eIj = eps[I] + eps[nc + j];
  for_each_acc(acc, [&](int r, int c, double2 v) {
    const int a = a0 + r, b = b0 + c;
    if (a < b && b < nv) {
      const long q = pair_offset(a, b, nv);
      const double D = ea[r] + eb[c] - eIj;
      const double2 x2 = r2[q];
      s2[q] = make_double2(v.x + D * x2.x, v.y + D * x2.y);
    }
  });
}

// ---------------------------------------------------------------------------
// Y-build:  Y[mI][P][c] = sum_{j,d} conj(L^P_{dj}) R_{Ij}[c][d]   (P < naux)
//           Y[mI][naux+K][c] = sum_{j,d} conj(<Kd||Ij>) R_{Ij}[c][d]
// with R_{Ij}[c][d] the antisymmetric doubles block of vector m.
// K index = (j, d) with d padded to a multiple of TK per j.
// ---------------------------------------------------------------------------
struct SrcLconj {    // element (k=(j,d), i=P) ; rows P >= naux read <Kd||Ij>
  static constexpr int MAP = RMAJOR;
  const double2* Lvo;   // + nc*naux*nv already (valence rows)
  const double2* VI;    // Vt + I*no*nc*nv
  int naux, nv, nc, cpe, p0;
  long lds;
  __device__ __forceinline__ double2 get(int k, int i) const {
    const int chunk = k / TK;
    const int j = chunk / cpe;
    const int d = (chunk - j * cpe) * TK + (k % TK);
    const int P = p0 + i;
    if (d >= nv) return czero();
    double2 v;
    if (P < naux) v = Lvo[(long)j * lds + (long)P * nv + d];
    else if (P < naux + nc) v = VI[((long)j * nc + (P - naux)) * nv + d];
    else return czero();
    return make_double2(v.x, -v.y);
  }
};

struct SrcR2 {       // element (k=(j,d), i=c) = R_{Ij}[c][d] from packed a<b storage
  static constexpr int MAP = KMAJOR;
  const double2* r2;    // doubles of (m, I, j=0)
  long npair;
  int nv, cpe, c0;
  __device__ __forceinline__ double2 get(int k, int i) const {
    const int chunk = k / TK;
    const int j = chunk / cpe;
    const int d = (chunk - j * cpe) * TK + (k % TK);
    const int c = c0 + i;
    if (d >= nv || c >= nv || c == d) return czero();
    const double2* blk = r2 + (long)j * npair;
    if (c < d) return blk[pair_offset(c, d, nv)];
    const double2 v = blk[pair_offset(d, c, nv)];
    return make_double2(-v.x, -v.y);
  }
};

__global__ __launch_bounds__(256) void k_ybuild(const double2* __restrict__ xin, long dim,
                                                 const double2* __restrict__ Lvo, const double2* __restrict__ Vt,
                                                 int m, int nc, int no, int nv, int naux,
                                                 double2* __restrict__ Y) {
  __shared__ TileSmem s;
  const int nrow = naux + nc;
  const int nbp = cdiv(nrow, TM), nbc = cdiv(nv, TN);
  const long nblocks = (long)m * nc * nbp * nbc;
  const long lid = xcd_remap(blockIdx.x, nblocks);
  const int cb = (int)(lid % nbc);
  const int pb = (int)((lid / nbc) % nbp);
  const int mI = (int)(lid / ((long)nbc * nbp));
  const int mv = mI / nc, I = mI - mv * nc;
  const int p0 = pb * TM, c0 = cb * TN;
  const int cpe = cdiv(nv, TK);
  const long lds = (long)naux * nv;
  const long ns = (long)nc * nv;
  const long npair = (long)nv * (nv - 1) / 2;
  SrcLconj A{Lvo + (long)nc * lds, Vt + (long)I * no * nc * nv, naux, nv, nc, cpe, p0, lds};
  SrcR2 B{xin + (long)mv * dim + ns + (long)I * no * npair, npair, nv, cpe, c0};
  Acc acc;
  acc.zero();
  mainloop(s, A, B, 0, no * cpe, acc);
  double2* Ym = Y + (long)mI * nrow * nv;
  for_each_acc(acc, [&](int r, int c, double2 v) {
    const int P = p0 + r, cc = c0 + c;
    if (P < nrow && cc < nv) Ym[(long)P * nv + cc] = v;
  });
}

// ---------------------------------------------------------------------------
// back-contraction:  part[split][mI][a] = sum_{P in split} sum_c Y[mI][P][c] Lvv[P][a][c]
// ---------------------------------------------------------------------------
struct SrcYrows {    // element (k=(P,c), i=mI)
  static constexpr int MAP = RMAJOR;
  const double2* Y;
  int nrow_y, nv, cpe, nrows, i0;
  __device__ __forceinline__ double2 get(int k, int i) const {
    const int chunk = k / TK;
    const int P = chunk / cpe;
    const int c = (chunk - P * cpe) * TK + (k % TK);
    const int mi = i0 + i;
    if (c >= nv || mi >= nrows) return czero();
    return Y[((long)mi * nrow_y + P) * nv + c];
  }
};

struct SrcLvvT {     // element (k=(P,c), i=a) = Lvv[P][a][c]
  static constexpr int MAP = RMAJOR;
  const double2* Lvv;
  int nv, cpe, a0;
  __device__ __forceinline__ double2 get(int k, int i) const {
    const int chunk = k / TK;
    const int P = chunk / cpe;
    const int c = (chunk - P * cpe) * TK + (k % TK);
    const int a = a0 + i;
    if (c >= nv || a >= nv) return czero();
    return Lvv[((long)P * nv + a) * nv + c];
  }
};

__global__ __launch_bounds__(256) void k_backc(const double2* __restrict__ Y, const double2* __restrict__ Lvv,
                                                int nrows, int nv, int naux, int nc, int nsplit,
                                                double2* __restrict__ part) {
  __shared__ TileSmem s;
  const int nbi = cdiv(nrows, TM), nba = cdiv(nv, TN);
  const long nblocks = (long)nbi * nba * nsplit;
  const long lid = xcd_remap(blockIdx.x, nblocks);
  const int split = (int)(lid / ((long)nbi * nba));
  const int tile = (int)(lid % ((long)nbi * nba));
  const int i0 = (tile / nba) * TM, a0 = (tile % nba) * TN;
  const int cpe = cdiv(nv, TK);
  const int nchunks = naux * cpe;
  const int per = cdiv(nchunks, nsplit);
  const int kc0 = split * per, kc1 = min(nchunks, kc0 + per);
  SrcYrows A{Y, naux + nc, nv, cpe, nrows, i0};
  SrcLvvT B{Lvv, nv, cpe, a0};
  Acc acc;
  acc.zero();
  mainloop(s, A, B, kc0, kc1, acc);
  double2* out = part + (long)split * nrows * nv;
  for_each_acc(acc, [&](int r, int c, double2 v) {
    const int mi = i0 + r, a = a0 + c;
    if (mi < nrows && a < nv) out[(long)mi * nv + a] = v;
  });
}

// s1[m][K][a] += sum_split part[split][mK][a] - sum_I Y[m*nc+I][naux+K][a]
__global__ void k_sigma1_finish(const double2* __restrict__ part, int nsplit, const double2* __restrict__ Y,
                                int m, int nc, int nv, int naux, long dim, double2* __restrict__ sout) {
  const long total = (long)m * nc * nv;
  const int nrow = naux + nc;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int a = (int)(e % nv);
    const int mK = (int)(e / nv);
    const int mv = mK / nc, K = mK - mv * nc;
    double2 acc = make_double2(0, 0);
    for (int sp = 0; sp < nsplit; ++sp) acc = cadd(acc, part[((long)sp * m * nc + mK) * nv + a]);
    for (int I = 0; I < nc; ++I) acc = csub(acc, Y[((long)(mv * nc + I) * nrow + naux + K) * nv + a]);
    double2* p = sout + (long)mv * dim + (long)K * nv + a;
    *p = cadd(*p, acc);
  }
}

// ---------------------------------------------------------------------------
static adc2_status ensure_ws(adc2_handle h, int m) {
  if (h->ws_m >= m) return ADC2_OK;
  const Dims& d = h->d;
  hipFree(h->X);
  hipFree(h->Y);
  hipFree(h->part);
  h->X = h->Y = h->part = nullptr;
  h->ws_m = 0;
  const long rows = (long)m * d.nc;
  ADC2_HIP(hipMalloc(&h->X, sizeof(double2) * rows * d.naux * d.nv));
  ADC2_HIP(hipMalloc(&h->Y, sizeof(double2) * rows * (d.naux + d.nc) * d.nv));
  const int nbi = cdiv(rows, TM), nba = cdiv(d.nv, TN);
  int nsplit = std::max(1, std::min(256, 2048 / std::max(1, nbi * nba)));
  nsplit = std::min(nsplit, d.naux);
  h->nsplit = nsplit;
  ADC2_HIP(hipMalloc(&h->part, sizeof(double2) * nsplit * rows * d.nv));
  h->ws_m = m;
  return ADC2_OK;
}

adc2_status sigma_fp64(adc2_handle h, int m, const double2* xin, double2* sout, hipStream_t st) {
  adc2_status rc = ensure_ws(h, m);
  if (rc != ADC2_OK) return rc;
  const Dims& d = h->d;
  const int nc = d.nc, no = d.no, nv = d.nv, naux = d.naux;
  const int rows = m * nc;
  // X-build
  {
    const long nblk = (long)cdiv(rows, TM) * cdiv((long)naux * nv, TN);
    k_xbuild<<<(unsigned)nblk, 256, 0, st>>>(xin, d.dim, nc, nv, naux, rows, h->Lvv, h->X);
    ADC2_CHECK_LAUNCH();
  }
  // sigma2
  {
    const int nb = cdiv(nv, TM);
    const long nblk = (long)m * nc * no * (nb * (nb + 1) / 2);
    k_sigma2<<<(unsigned)nblk, 256, 0, st>>>(xin, sout, d.dim, h->X, h->Lvo, h->Vt, h->eps, m, nc, no, nv, naux);
    ADC2_CHECK_LAUNCH();
  }
  // Y-build
  {
    const long nblk = (long)m * nc * cdiv(naux + nc, TM) * cdiv(nv, TN);
    k_ybuild<<<(unsigned)nblk, 256, 0, st>>>(xin, d.dim, h->Lvo, h->Vt, m, nc, no, nv, naux, h->Y);
    ADC2_CHECK_LAUNCH();
  }
  // sigma1 = M11 r1 (writes the singles of S), then back-contraction
  {
    adc2_status r2 = gemm_rr(m, (int)d.ns, (int)d.ns, xin, d.dim, false, h->M11, d.ns, false, sout, d.dim, 1.0,
                             false, st);
    if (r2 != ADC2_OK) return r2;
    const long nblk = (long)cdiv(rows, TM) * cdiv(nv, TN) * h->nsplit;
    k_backc<<<(unsigned)nblk, 256, 0, st>>>(h->Y, h->Lvv, rows, nv, naux, nc, h->nsplit, h->part);
    ADC2_CHECK_LAUNCH();
    const long tot = (long)rows * nv;
    const int g = (int)std::min<long>(4096, (tot + 255) / 256);
    k_sigma1_finish<<<g, 256, 0, st>>>(h->part, h->nsplit, h->Y, m, nc, nv, naux, d.dim, sout);
    ADC2_CHECK_LAUNCH();
  }
  return ADC2_OK;
}

}  // namespace adc2
