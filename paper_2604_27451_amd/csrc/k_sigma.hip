// k_sigma.hip -- sigma = M x for the CVS-ADC(2) matrix (paper Eq. 11-12,
// CVS section), FP64 complex on the FP64 MFMA.
//
// With r = [r1 (I,a) | r2 (I,j,a<b)] and the doubles state a+_a a+_b a_j a_I:
//   M21[(Ijab),(Kc)] = d_IK <ab||cj> - d_ac <Kb||Ij> + d_bc <Ka||Ij>
//   M22 = diag(e_a + e_b - e_I - e_j),  M12 = M21^H.
// The three-virtual integral <ab||cj> = (ac|bj) - (aj|bc) is never formed:
//   X^P_{Ia}  = sum_c L^P_{ac} r_{Ic}                                  (X-build)
//   Z_{Ij}[a][b] = sum_P X^P_{Ia} L^P_{bj}                             (sigma2 GEMM)
//   s2_{Ijab} = Z_ab - Z_ba + sum_K (<Ka||Ij> r_Kb - r_Ka <Kb||Ij>) + D r2 (pack)
//   Y^P_{Ic}  = sum_{jd} conj(L^P_{dj}) r_{Ijcd}                          (Y GEMM)
//   s1_{Ia}   = sum_{Jb} M11 r1 + sum_{Pc} L^P_{ac} Y^P_{Ic}
//             - sum_{I',jb} conj(<Ib||I'j>) r_{I'jab}                    (sigma1)
// The two heavy contractions (8 nc no nv^2 naux flops per vector each) are
// plain complex GEMMs on 128x128 tiles (zgemm.h) with no redundant work; the
// antisymmetrisation, the denominators and the light core terms run in
// bandwidth-bound kernels around them.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include <mutex>

#include "internal.h"
#include "tile.h"
#include "zgemm.h"
#include "zgemm32.h"
#include "zgemmb.h"

namespace adc2 {

__host__ __device__ static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }
static inline unsigned grid_for(long n, long per = 256, long cap = 16384) {
  long g = (n + per - 1) / per;
  return (unsigned)std::max<long>(1, std::min<long>(g, cap));
}

// storage conversions of the precision form (complex64 operands, FP64 arithmetic around them)
__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2((double)v.x, (double)v.y); }
template <class T> __device__ __forceinline__ T from_d2(double2 v);
template <> __device__ __forceinline__ double2 from_d2<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 from_d2<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }

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

template <class TO>
__global__ __launch_bounds__(256) void k_xbuild(const double2* __restrict__ x, long dim, int nc, int nv, int naux,
                                                 int nrows, const double2* __restrict__ Lvv,
                                                 TO* __restrict__ X) {
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
    if (mi < nrows && j < ncol) X[(long)mi * ncol + j] = from_d2<TO>(v);
  });
}

// Y-build A: element (k = (j, d), i = P) = conj(L^P_{d j}) = conj(Lvo[nc+j][P][d]);
// k runs over j-blocks of cpe chunks (d padded to a multiple of BK).
template <int NS>
struct SrcLconjRows {
  static constexpr int MAP = RMAJOR;
  const double2* base;   // Lvo + nc*naux*nv
  long jstride;          // naux*nv
  int nv, cpe, nrows;
  long off[NS];
  unsigned okmask;
  int kk;
  __device__ __forceinline__ void begin(int tid, int i0) {
    kk = tid & 15;
    okmask = 0;
#pragma unroll
    for (int e = 0; e < NS; ++e) {
      const int P = i0 + (tid >> 4) + 16 * e;
      off[e] = (long)P * nv;
      if (P < nrows) okmask |= 1u << e;
    }
  }
  __device__ __forceinline__ void load(int kc, RegsN<NS>& r) const {
    const int j = kc / cpe;
    const int d = (kc - j * cpe) * BK + kk;
    const long jo = (long)j * jstride + d;
    const bool dok = d < nv;
#pragma unroll
    for (int e = 0; e < NS; ++e) {
      if (((okmask >> e) & 1u) && dok) {
        const double2 v = base[off[e] + jo];
        r.v[e] = make_double2(v.x, -v.y);
      } else {
        r.v[e] = czero();
      }
    }
  }
};

// Y-build B: element (k = (j, d), col = (mI, c)) = R_{mI j}[c][d] from the
// unpacked antisymmetric doubles Rf[mI][j][c][d].
template <int NS>
struct SrcRfull {
  static constexpr int MAP = RMAJOR;
  const double2* R;
  int nv, no, cpe, ncols;
  long off[NS];
  unsigned okmask;
  int kk;
  __device__ __forceinline__ void begin(int tid, int i0) {
    kk = tid & 15;
    okmask = 0;
#pragma unroll
    for (int e = 0; e < NS; ++e) {
      const int col = i0 + (tid >> 4) + 16 * e;
      const int g = col / nv, c = col - g * nv;
      off[e] = ((long)g * no * nv + c) * nv;
      if (col < ncols) okmask |= 1u << e;
    }
  }
  __device__ __forceinline__ void load(int kc, RegsN<NS>& r) const {
    const int j = kc / cpe;
    const int d = (kc - j * cpe) * BK + kk;
    const long jo = (long)j * nv * nv + d;
    const bool dok = d < nv;
#pragma unroll
    for (int e = 0; e < NS; ++e) r.v[e] = (((okmask >> e) & 1u) && dok) ? R[off[e] + jo] : czero();
  }
};

// sigma2 core:  Z[mI][j][a][b] = sum_P X[mI][P][a] Lvo[nc+j][P][b]
// G3: three-multiplication 128x64 tiles; otherwise four-multiplication 128x128.
template <bool G3>
__global__ __launch_bounds__(256) void k_zsig2(const double2* __restrict__ X, const double2* __restrict__ Lvo,
                                                int rows, int nc, int no, int nv, int naux,
                                                double2* __restrict__ Z) {
  constexpr int TNC = G3 ? BT3N : BT;
  constexpr int NSB = G3 ? 4 : 8;
  const int ncols = no * nv;
  const int nbm = (rows + BT - 1) / BT, nbn = (ncols + TNC - 1) / TNC;
  const long lid = xcd_remap(blockIdx.x, (long)nbm * nbn);
  int bm, bn;
  big_tile_coords(lid, nbm, nbn, bm, bn);
  const int i0 = bm * BT, j0 = bn * TNC;
  const long lds = (long)naux * nv;
  SrcGroupedK<8> A{X, lds, nv, nv, rows, naux};
  SrcGroupedK<NSB> B{Lvo + (long)nc * lds, lds, nv, nv, ncols, naux};
  A.begin(threadIdx.x, i0);
  B.begin(threadIdx.x, j0);
  auto store = [&](int r, int c, double2 v) {
    const int i = i0 + r, jc = j0 + c;
    if (i < rows && jc < ncols) {
      const int mI = i / nv, a = i - mI * nv;
      const int j = jc / nv, b = jc - j * nv;
      Z[(((long)mI * no + j) * nv + a) * nv + b] = v;
    }
  };
  const int nkc = (naux + BK - 1) / BK;
  if constexpr (G3) {
    __shared__ BigSmem3 s;
    BigAcc3 acc;
    acc.zero();
    big_mainloop3(s, A, B, 0, nkc, acc);
    big_for_each3(acc, store);
  } else {
    __shared__ BigSmem s[2];
    BigAcc acc;
    acc.zero();
    big_mainloop(s, A, B, 0, nkc, acc);
    big_for_each(acc, store);
  }
}

// Y-build:  Y[mI][P][c] = sum_{(j,d)} LvT[(j,d)][P] Rt[(j,d)][(mI,c)]
//                      = sum_{j,d} conj(L^P_{dj}) R_{mIj}[c][d]
// Both operands are k-major rows (contiguous in P and in (mI,c)).
template <bool G3>
__global__ __launch_bounds__(256) void k_ygemm(const double2* __restrict__ LvT, const double2* __restrict__ Rt,
                                                int rows, int nc, int no, int nv, int naux,
                                                double2* __restrict__ Y) {
  constexpr int TNC = G3 ? BT3N : BT;
  constexpr int NSB = G3 ? 4 : 8;
  const int ncols = rows * nv;
  const int nbm = (naux + BT - 1) / BT, nbn = (ncols + TNC - 1) / TNC;
  const long lid = xcd_remap(blockIdx.x, (long)nbm * nbn);
  int bm, bn;
  big_tile_coords(lid, nbm, nbn, bm, bn);
  const int i0 = bm * BT, j0 = bn * TNC;
  const int K = no * nv;
  SrcGroupedK<8> A{LvT, 0, naux, naux, naux, K};
  SrcGroupedK<NSB> B{Rt, 0, ncols, ncols, ncols, K};
  A.begin(threadIdx.x, i0);
  B.begin(threadIdx.x, j0);
  // split over K: blockIdx.y of gridDim.y writes its own partial of Y
  const int nchunks = (K + BK - 1) / BK;
  const int per = (nchunks + gridDim.y - 1) / gridDim.y;
  const int kc0 = blockIdx.y * per, kc1 = min(nchunks, kc0 + per);
  double2* Ys = Y + (long)blockIdx.y * ((long)rows * naux * nv);
  auto store = [&](int r, int c, double2 v) {
    const int P = i0 + r, col = j0 + c;
    if (P < naux && col < ncols) {
      const int mI = col / nv, cc = col - mI * nv;
      Ys[((long)mI * naux + P) * nv + cc] = v;
    }
  };
  if constexpr (G3) {
    __shared__ BigSmem3 s;
    BigAcc3 acc;
    acc.zero();
    big_mainloop3(s, A, B, kc0, kc1, acc);
    big_for_each3(acc, store);
  } else {
    __shared__ BigSmem s[2];
    BigAcc acc;
    acc.zero();
    big_mainloop(s, A, B, kc0, kc1, acc);
    big_for_each(acc, store);
  }
}

// The same two contractions on the two-per-CU engine (128 x 64 tiles, chunks
// of 8 k).  The Y-build's K-splits are cut at the 16-k boundaries of the
// 128 x 128 kernel, so both kernels sum every partial in the same order.
__global__ __launch_bounds__(256, 2) void k_zsig2_mid(const double2* __restrict__ X,
                                                       const double2* __restrict__ Lvo, int rows, int nc, int no,
                                                       int nv, int naux, double2* __restrict__ Z) {
  __shared__ MidSmem s[2];
  const int ncols = no * nv;
  const int nbm = (rows + BT - 1) / BT, nbn = (ncols + MTN - 1) / MTN;
  const long lid = xcd_remap(blockIdx.x, (long)nbm * nbn);
  int bm, bn;
  big_tile_coords(lid, nbm, nbn, bm, bn);
  const int i0 = bm * BT, j0 = bn * MTN;
  const long lds = (long)naux * nv;
  SrcGroupedK8<4> A{X, lds, nv, nv, rows, naux};
  SrcGroupedK8<2> B{Lvo + (long)nc * lds, lds, nv, nv, ncols, naux};
  A.begin(threadIdx.x, i0);
  B.begin(threadIdx.x, j0);
  MidAcc acc;
  acc.zero();
  mid_mainloop(s, A, B, 0, (naux + MBK - 1) / MBK, acc);
  mid_for_each(acc, [&](int r, int c, double2 v) {
    const int i = i0 + r, jc = j0 + c;
    if (i < rows && jc < ncols) {
      const int mI = i / nv, a = i - mI * nv;
      const int j = jc / nv, b = jc - j * nv;
      Z[(((long)mI * no + j) * nv + a) * nv + b] = v;
    }
  });
}

__global__ __launch_bounds__(256, 2) void k_ygemm_mid(const double2* __restrict__ LvT,
                                                       const double2* __restrict__ Rt, int rows, int no, int nv,
                                                       int naux, double2* __restrict__ Y) {
  __shared__ MidSmem s[2];
  const int ncols = rows * nv;
  const int nbm = (naux + BT - 1) / BT, nbn = (ncols + MTN - 1) / MTN;
  const long lid = xcd_remap(blockIdx.x, (long)nbm * nbn);
  int bm, bn;
  big_tile_coords(lid, nbm, nbn, bm, bn);
  const int i0 = bm * BT, j0 = bn * MTN;
  const int K = no * nv;
  SrcGroupedK8<4> A{LvT, 0, naux, naux, naux, K};
  SrcGroupedK8<2> B{Rt, 0, ncols, ncols, ncols, K};
  A.begin(threadIdx.x, i0);
  B.begin(threadIdx.x, j0);
  const int n16 = (K + BK - 1) / BK;
  const int per = (n16 + gridDim.y - 1) / gridDim.y;   // in 16-k chunks
  const int kc0 = 2 * blockIdx.y * per, kc1 = min((K + MBK - 1) / MBK, kc0 + 2 * per);
  double2* Ys = Y + (long)blockIdx.y * ((long)rows * naux * nv);
  MidAcc acc;
  acc.zero();
  mid_mainloop(s, A, B, kc0, kc1, acc);
  mid_for_each(acc, [&](int r, int c, double2 v) {
    const int P = i0 + r, col = j0 + c;
    if (P < naux && col < ncols) {
      const int mI = col / nv, cc = col - mI * nv;
      Ys[((long)mI * naux + P) * nv + cc] = v;
    }
  });
}

// The same two contractions on the eight-wave engine (128 x 128 tiles, 16-k
// chunks, two waves per SIMD).
__global__ __launch_bounds__(512) void k_zsig2_wide(const double2* __restrict__ X, const double2* __restrict__ Lvo,
                                                     int rows, int nc, int no, int nv, int naux,
                                                     double2* __restrict__ Z) {
  __shared__ BigSmem s[2];
  const int ncols = no * nv;
  const int nbm = (rows + BT - 1) / BT, nbn = (ncols + BT - 1) / BT;
  const long lid = xcd_remap(blockIdx.x, (long)nbm * nbn);
  int bm, bn;
  big_tile_coords(lid, nbm, nbn, bm, bn);
  const int i0 = bm * BT, j0 = bn * BT;
  const long lds = (long)naux * nv;
  SrcGroupedK8<4, BK> A{X, lds, nv, nv, rows, naux};
  SrcGroupedK8<4, BK> B{Lvo + (long)nc * lds, lds, nv, nv, ncols, naux};
  A.begin(threadIdx.x, i0);
  B.begin(threadIdx.x, j0);
  MidAcc acc;
  acc.zero();
  wide_mainloop(s, A, B, 0, (naux + BK - 1) / BK, acc);
  wide_for_each(acc, [&](int r, int c, double2 v) {
    const int i = i0 + r, jc = j0 + c;
    if (i < rows && jc < ncols) {
      const int mI = i / nv, a = i - mI * nv;
      const int j = jc / nv, b = jc - j * nv;
      Z[(((long)mI * no + j) * nv + a) * nv + b] = v;
    }
  });
}

__global__ __launch_bounds__(512) void k_ygemm_wide(const double2* __restrict__ LvT, const double2* __restrict__ Rt,
                                                     int rows, int no, int nv, int naux, double2* __restrict__ Y) {
  __shared__ BigSmem s[2];
  const int ncols = rows * nv;
  const int nbm = (naux + BT - 1) / BT, nbn = (ncols + BT - 1) / BT;
  const long lid = xcd_remap(blockIdx.x, (long)nbm * nbn);
  int bm, bn;
  big_tile_coords(lid, nbm, nbn, bm, bn);
  const int i0 = bm * BT, j0 = bn * BT;
  const int K = no * nv;
  SrcGroupedK8<4, BK> A{LvT, 0, naux, naux, naux, K};
  SrcGroupedK8<4, BK> B{Rt, 0, ncols, ncols, ncols, K};
  A.begin(threadIdx.x, i0);
  B.begin(threadIdx.x, j0);
  const int nchunks = (K + BK - 1) / BK;
  const int per = (nchunks + gridDim.y - 1) / gridDim.y;
  const int kc0 = blockIdx.y * per, kc1 = min(nchunks, kc0 + per);
  double2* Ys = Y + (long)blockIdx.y * ((long)rows * naux * nv);
  MidAcc acc;
  acc.zero();
  wide_mainloop(s, A, B, kc0, kc1, acc);
  wide_for_each(acc, [&](int r, int c, double2 v) {
    const int P = i0 + r, col = j0 + c;
    if (P < naux && col < ncols) {
      const int mI = col / nv, cc = col - mI * nv;
      Ys[((long)mI * naux + P) * nv + cc] = v;
    }
  });
}

// Precision form: the two heavy contractions on complex64 operands with the
// FP32 MFMA and FP32 accumulation.  Each kernel body is an "item" (one output
// tile and one K-split) so that the plain launches below and the grouped
// launches of several systems (GemmJobs) share it.
//   sigma2: Z[mI][j][a][b] = sum_P X^P_{(mI)a} L^P_{bj}      (rows = m*nc*nv)
//   Y-build: Y[s][mI][P][c] = sum_{(j,d) in split s} conj(L^P_dj) Rt[(j,d)][(mI,c)]
__device__ __forceinline__ void zsig2_c64_item(BigSmemF (&s)[2], const float2* __restrict__ X32,
                                               const float2* __restrict__ Lv32, int rows, int no, int nv, int naux,
                                               float2* __restrict__ Z, long lid) {
  const int ncols = no * nv;
  const int nbm = (rows + BT - 1) / BT, nbn = (ncols + BT - 1) / BT;
  int bm, bn;
  big_tile_coords(lid, nbm, nbn, bm, bn);
  const int i0 = bm * BT, j0 = bn * BT;
  const long lds = (long)naux * nv;
  SrcGroupedKF A{X32, lds, nv, nv, rows, naux};
  SrcGroupedKF B{Lv32, lds, nv, nv, ncols, naux};
  A.begin(threadIdx.x, i0);
  B.begin(threadIdx.x, j0);
  BigAccF acc;
  acc.zero();
  big_mainloopF(s, A, B, 0, (naux + BK - 1) / BK, acc);
  big_for_eachF(acc, [&](int r, int c, float2 v) {
    const int i = i0 + r, jc = j0 + c;
    if (i < rows && jc < ncols) {
      const int mI = i / nv, a = i - mI * nv;
      const int j = jc / nv, b = jc - j * nv;
      Z[(((long)mI * no + j) * nv + a) * nv + b] = v;
    }
  });
}

__device__ __forceinline__ void ygemm_c64_item(BigSmemF (&s)[2], const float2* __restrict__ LvT32,
                                               const float2* __restrict__ Rt32, int rows, int no, int nv, int naux,
                                               double2* __restrict__ Y, long lid, int split, int nsplit) {
  const int ncols = rows * nv;
  const int nbm = (naux + BT - 1) / BT, nbn = (ncols + BT - 1) / BT;
  int bm, bn;
  big_tile_coords(lid, nbm, nbn, bm, bn);
  const int i0 = bm * BT, j0 = bn * BT;
  const int K = no * nv;
  SrcGroupedKF A{LvT32, 0, naux, naux, naux, K};
  SrcGroupedKF B{Rt32, 0, ncols, ncols, ncols, K};
  A.begin(threadIdx.x, i0);
  B.begin(threadIdx.x, j0);
  const int nchunks = (K + BK - 1) / BK;
  const int per = (nchunks + nsplit - 1) / nsplit;
  const int kc0 = split * per, kc1 = min(nchunks, kc0 + per);
  double2* Ys = Y + (long)split * ((long)rows * naux * nv);
  BigAccF acc;
  acc.zero();
  big_mainloopF(s, A, B, kc0, kc1, acc);
  big_for_eachF(acc, [&](int r, int c, float2 v) {
    const int P = i0 + r, col = j0 + c;
    if (P < naux && col < ncols) {
      const int mI = col / nv, cc = col - mI * nv;
      Ys[((long)mI * naux + P) * nv + cc] = make_double2((double)v.x, (double)v.y);
    }
  });
}

// Precision form, split-BF16 variant: the same two contractions on the BF16
// matrix cores with hi/lo operands in the blocked split layout (zgemmb.h),
// FP32 accumulation, 512-thread workgroups (consumer waves 0-3 write the
// tile).  XB, LvB: sigma2 operands (rows (mI,a) and (j,b), K = naux); LvTB, RB:
// Y-build operands (rows P and (mI,c), K = (j,d)).
__device__ __forceinline__ void zsig2_b3_item(BigSmemB (&s)[2], const __bf16* __restrict__ XB,
                                              const __bf16* __restrict__ LvB, int rows, int no, int nv, int naux,
                                              float2* __restrict__ Z, long lid) {
  const int ncols = no * nv;
  const int nbm = (rows + BT - 1) / BT, nbn = (ncols + BT - 1) / BT;
  int bm, bn;
  big_tile_coords(lid, nbm, nbn, bm, bn);
  const int i0 = bm * BT, j0 = bn * BT;
  const int nkc = (naux + BKB - 1) / BKB;
  SrcBL A{(const char*)XB, nkc};
  SrcBL B{(const char*)LvB, nkc};
  A.begin(threadIdx.x & 255, i0);
  B.begin(threadIdx.x & 255, j0);
  BigAccF acc;
  acc.zero();
  big_mainloopB(s, A, B, 0, nkc, acc);
  if (wave_id() >= 4) return;
  big_for_eachF(acc, [&](int r, int c, float2 v) {
    const int i = i0 + r, jc = j0 + c;
    if (i < rows && jc < ncols) {
      const int mI = i / nv, a = i - mI * nv;
      const int j = jc / nv, b = jc - j * nv;
      Z[(((long)mI * no + j) * nv + a) * nv + b] = v;
    }
  });
}

__device__ __forceinline__ void ygemm_b3_item(BigSmemB (&s)[2], const __bf16* __restrict__ LvTB,
                                              const __bf16* __restrict__ RB, int rows, int no, int nv, int naux,
                                              double2* __restrict__ Y, long lid, int split, int nsplit) {
  const int ncols = rows * nv;
  const int nbm = (naux + BT - 1) / BT, nbn = (ncols + BT - 1) / BT;
  int bm, bn;
  big_tile_coords(lid, nbm, nbn, bm, bn);
  const int i0 = bm * BT, j0 = bn * BT;
  const int nchunks = (no * nv + BKB - 1) / BKB;
  SrcBL A{(const char*)LvTB, nchunks};
  SrcBL B{(const char*)RB, nchunks};
  A.begin(threadIdx.x & 255, i0);
  B.begin(threadIdx.x & 255, j0);
  const int per = (nchunks + nsplit - 1) / nsplit;
  const int kc0 = split * per, kc1 = min(nchunks, kc0 + per);
  double2* Ys = Y + (long)split * ((long)rows * naux * nv);
  BigAccF acc;
  acc.zero();
  big_mainloopB(s, A, B, kc0, kc1, acc);
  if (wave_id() >= 4) return;
  big_for_eachF(acc, [&](int r, int c, float2 v) {
    const int P = i0 + r, col = j0 + c;
    if (P < naux && col < ncols) {
      const int mI = col / nv, cc = col - mI * nv;
      Ys[((long)mI * naux + P) * nv + cc] = make_double2((double)v.x, (double)v.y);
    }
  });
}

// Split a K-major complex operand (element (k, row) at src[g*gstride +
// x*xstride + k*ld], row = g*inner + x < R, k < K; complex64, or complex128
// rounded to complex64 first) into the blocked split layout of zgemmb.h (rows
// padded to 128, k to 32, padding zero).  Thread t of a block's 512 owns row
// r = (t / 4) % 128 and the k-group stored in 16-byte slot t % 4 of that row,
// so every plane store of a wave covers 16 whole 64-byte rows (1 KB
// contiguous); with xstride 1 the source reads of a wave are 4 runs of 16 rows.
template <class TS>
__global__ void k_split_pack(const TS* __restrict__ src, long gstride, long xstride, long ld, int inner, int R,
                             int K, int nrt, int nkc, __bf16* __restrict__ dst) {
  const long total = (long)nrt * nkc * 512;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int slot = (int)(t & 3), r = (int)((t >> 2) & 127);
    const long blk = t >> 9;
    const int kc = (int)(blk % nkc), rt = (int)(blk / nkc);
    const int row = rt * BT + r;
    const int k0 = kc * BKB + 8 * (slot ^ ((r >> 1) & 3));
    float re[8], im[8];
    if (row < R) {
      const int g = row / inner;
      const TS* p = src + (long)g * gstride + (long)(row - g * inner) * xstride;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        float2 v = make_float2(0.f, 0.f);
        if (k0 + e < K) {
          const TS w = p[(long)(k0 + e) * ld];
          v = make_float2((float)w.x, (float)w.y);
        }
        re[e] = v.x;
        im[e] = v.y;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) re[e] = im[e] = 0.f;
    }
    bf8 rh, rl, ih, il;
    split8(re, rh, rl);
    split8(im, ih, il);
    const long o0 = split_block_offset(row, k0, 0, nkc);   // = plane-0 base of the block + r*32 + 8*slot
    const long ps = (long)BT * BLDB;                      // plane stride
    *(bf8*)(dst + o0) = rh;
    *(bf8*)(dst + o0 + ps) = rl;
    *(bf8*)(dst + o0 + 2 * ps) = ih;
    *(bf8*)(dst + o0 + 3 * ps) = il;
  }
}

long split_bytes(long R, long K) { return (long)cdiv(R, BT) * cdiv(K, BKB) * BLOCK_BYTES; }

template <class TS>
static adc2_status split_pack(const TS* src, long gstride, long ld, int inner, long R, long K, __bf16* dst,
                              hipStream_t st, long xstride = 1) {
  const int nrt = cdiv(R, BT), nkc = cdiv(K, BKB);
  const long total = (long)nrt * nkc * 512;
  k_split_pack<TS><<<grid_for(total, 256, 1L << 20), 256, 0, st>>>(src, gstride, xstride, ld, inner, (int)R, (int)K,
                                                                    nrt, nkc, dst);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

__global__ __launch_bounds__(256) void k_zsig2_c64(const float2* __restrict__ X32, const float2* __restrict__ Lv32,
                                                    int rows, int no, int nv, int naux, float2* __restrict__ Z) {
  __shared__ BigSmemF s[2];
  const long nt = (long)((rows + BT - 1) / BT) * ((no * nv + BT - 1) / BT);
  zsig2_c64_item(s, X32, Lv32, rows, no, nv, naux, Z, xcd_remap(blockIdx.x, nt));
}

// Two workgroups per CU: the accumulators then live in the unified register
// file (no AGPR split) within 256 registers per lane.
__global__ __launch_bounds__(256, 2) void k_ygemm_c64(const float2* __restrict__ LvT32, const float2* __restrict__ Rt32,
                                                    int rows, int no, int nv, int naux, double2* __restrict__ Y) {
  __shared__ BigSmemF s[2];
  const long nt = (long)((naux + BT - 1) / BT) * ((rows * nv + BT - 1) / BT);
  ygemm_c64_item(s, LvT32, Rt32, rows, no, nv, naux, Y, xcd_remap(blockIdx.x, nt), blockIdx.y, gridDim.y);
}

__global__ __launch_bounds__(512) void k_zsig2_b3(const __bf16* __restrict__ XB, const __bf16* __restrict__ LvB,
                                                   int rows, int no, int nv, int naux, float2* __restrict__ Z) {
  __shared__ BigSmemB s[2];
  const long nt = (long)((rows + BT - 1) / BT) * ((no * nv + BT - 1) / BT);
  zsig2_b3_item(s, XB, LvB, rows, no, nv, naux, Z, xcd_remap(blockIdx.x, nt));
}

__global__ __launch_bounds__(512) void k_ygemm_b3(const __bf16* __restrict__ LvTB, const __bf16* __restrict__ RB,
                                                   int rows, int no, int nv, int naux, double2* __restrict__ Y) {
  __shared__ BigSmemB s[2];
  const long nt = (long)((naux + BT - 1) / BT) * ((rows * nv + BT - 1) / BT);
  ygemm_b3_item(s, LvTB, RB, rows, no, nv, naux, Y, xcd_remap(blockIdx.x, nt), blockIdx.y, gridDim.y);
}

// ---------------------------------------------------------------------------
// Grouped launches of the heavy GEMMs over several systems (batching form).
// One job per system; its work items are (K-split, tile) pairs.  Job q owns
// the slots [w0, w0 + npad) of the launch, npad = its item count rounded up
// to a multiple of 8 and w0 a multiple of 8, so that slot w runs on XCD
// w mod 8 and every job is spread evenly over the eight XCDs (the items of
// different systems differ in K, hence in cost, by an order of magnitude:
// an equal item count per XCD would leave some XCDs idle).  Within a job,
// xcd_remap gives each XCD a contiguous run of items, which share operand
// panels in its L2.  Jobs are ordered by decreasing cost per item, so the
// tail of the launch is made of the cheapest items.  Workgroup b takes slots
// b, b + gridDim.x, ... (gridDim.x a multiple of 8).
constexpr int GMAX = 16;   // systems per grouped launch
struct GemmJob {
  const void* A;     // Y-build: LvT32 (complex64) or LvTB (split);  sigma2: X32 or XB
  const void* B;     // Y-build: Rt32 or RB;  sigma2: Lv32 or LvB
  void* C;           // Y (double2, nsplit partials) or Z (float2)
  int rows, no, nv, naux, nsplit;
  long ntile;        // output tiles of one K-split
  long w0;           // first slot (a multiple of 8)
};
struct GemmJobs {
  int n;
  long total;
  GemmJob j[GMAX];
};

__device__ __forceinline__ int job_of(const GemmJobs& J, long item) {
  int q = 0;
  for (int t = 1; t < J.n; ++t)
    if (item >= J.j[t].w0) q = t;
  return q;
}

// Item of slot w of job g, or -1 for a padding slot.
__device__ __forceinline__ long job_item(const GemmJob& g, long w) {
  const long nit = g.ntile * g.nsplit;
  const long item = xcd_remap(w - g.w0, (nit + 7) & ~7L);
  return item < nit ? item : -1;
}

template <bool YBUILD>
__global__ __launch_bounds__(256, 2) void k_gemm_c64_grouped(const GemmJobs J) {
  __shared__ BigSmemF s[2];
  for (long w = blockIdx.x; w < J.total; w += gridDim.x) {
    const GemmJob& g = J.j[job_of(J, w)];
    const long loc = job_item(g, w);
    if (loc < 0) continue;
    const int split = (int)(loc / g.ntile);
    const long lid = loc - (long)split * g.ntile;
    if (YBUILD)
      ygemm_c64_item(s, (const float2*)g.A, (const float2*)g.B, g.rows, g.no, g.nv, g.naux, (double2*)g.C, lid,
                     split, g.nsplit);
    else
      zsig2_c64_item(s, (const float2*)g.A, (const float2*)g.B, g.rows, g.no, g.nv, g.naux, (float2*)g.C, lid);
  }
}

template <bool YBUILD>
__global__ __launch_bounds__(512) void k_gemm_b3_grouped(const GemmJobs J) {
  __shared__ BigSmemB s[2];
  for (long w = blockIdx.x; w < J.total; w += gridDim.x) {
    const GemmJob& g = J.j[job_of(J, w)];
    const long loc = job_item(g, w);
    if (loc < 0) continue;
    const int split = (int)(loc / g.ntile);
    const long lid = loc - (long)split * g.ntile;
    if (YBUILD)
      ygemm_b3_item(s, (const __bf16*)g.A, (const __bf16*)g.B, g.rows, g.no, g.nv, g.naux, (double2*)g.C, lid,
                    split, g.nsplit);
    else
      zsig2_b3_item(s, (const __bf16*)g.A, (const __bf16*)g.B, g.rows, g.no, g.nv, g.naux, (float2*)g.C, lid);
  }
}

__global__ void k_to_c64(const double2* __restrict__ src, long n, float2* __restrict__ dst) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    dst[e] = make_float2((float)src[e].x, (float)src[e].y);
}

// Y = sum of the split partials (in place into split 0)
__global__ void k_ysum(double2* __restrict__ Y, long len, int nsplit) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < len; e += (long)gridDim.x * blockDim.x) {
    double2 a = Y[e];
    for (int s = 1; s < nsplit; ++s) a = cadd(a, Y[(long)s * len + e]);
    Y[e] = a;
  }
}

__device__ __forceinline__ long pair_offset(int a, int b, int nv) {
  return (long)a * nv - (long)a * (a + 1) / 2 + (b - a - 1);
}

// Unpack the doubles of all m vectors into the k-major Y-build operand
//   Rt[(j, d)][(mI, c)] = R_{mI j}[c][d]   (c<d packed, c>d negated, 0 on c=d)
// with row (j,d) = j*nv + d of length m*nc*nv.  One workgroup per
// (mI, j, 32x32 tile pair cb <= db): the packed upper tile is read along d
// (contiguous) and written both straight and, through LDS, transposed; every
// global access is coalesced.
constexpr int UT = 32;
template <class TO, bool WTS>
__global__ __launch_bounds__(256) void k_unpack(const double2* __restrict__ xin, long dim, int m, int nc, int no,
                                                 int nv, TO* __restrict__ Rt, const double* __restrict__ wts) {
  __shared__ double2 t[UT][UT + 1];
  const int nb = (nv + UT - 1) / UT;
  const int ntp = nb * (nb + 1) / 2;
  const long g = blockIdx.x / ntp;           // g = mI*no + j
  int tt = blockIdx.x % ntp, cbk = 0;
  while (tt >= nb - cbk) {
    tt -= nb - cbk;
    ++cbk;
  }
  const int dbk = cbk + tt;
  const int c0 = cbk * UT, d0 = dbk * UT;
  const long ns = (long)nc * nv;
  const long npair = (long)nv * (nv - 1) / 2;
  const int mI = (int)(g / no), j = (int)(g % no);
  const int mv = mI / nc, I = mI - mv * nc;
  const double2* r2 = xin + (long)mv * dim + ns + ((long)I * no + j) * npair;
  const long ld = (long)m * nc * nv;
  TO* R = Rt + (long)j * nv * ld + (long)mI * nv;   // R[d*ld + c] = R_{mIj}[c][d]
  const int tid = threadIdx.x;
  for (int e = tid; e < UT * UT; e += 256) {
    const int rc = e / UT, cd = e % UT;
    const int c = c0 + rc, d = d0 + cd;
    double2 v = czero();
    if (c < nv && d < nv && c < d) v = r2[pair_offset(c, d, nv)];
    if (WTS) v = cscale(v, wts[mv]);
    t[rc][cd] = v;    // t[c][d] = R[c][d] on the upper tile
  }
  __syncthreads();
  // rows d of the d-tile, columns c of the c-tile: R[c][d] = t[c][d] (c<d)
  for (int e = tid; e < UT * UT; e += 256) {
    const int rd = e / UT, cc = e % UT;
    const int d = d0 + rd, c = c0 + cc;
    if (c < nv && d < nv) {
      double2 v;
      if (cbk == dbk) v = (c < d) ? t[cc][rd] : (c > d ? cneg(t[rd][cc]) : czero());
      else v = t[cc][rd];
      R[(long)d * ld + c] = from_d2<TO>(v);
    }
  }
  if (cbk != dbk) {
    // rows c of the c-tile, columns d of the d-tile: R[d][c] = -R[c][d]
    for (int e = tid; e < UT * UT; e += 256) {
      const int rc = e / UT, cd = e % UT;
      const int c = c0 + rc, d = d0 + cd;
      if (c < nv && d < nv) R[(long)c * ld + d] = from_d2<TO>(cneg(t[rc][cd]));
    }
  }
}

// One-time conjugate transpose of the occupied Cholesky block:
//   LoT[(l, d)][P] = conj(L^P_{d l}) = conj(Lvo[l][P][d])   for every occupied l.
// Its valence rows are the Y-build operand; the adjoint also uses the core rows.
__global__ __launch_bounds__(256) void k_lvo_transpose(const double2* __restrict__ Lvo, int nv, int naux,
                                                        double2* __restrict__ LoT) {
  __shared__ double2 t[UT][UT + 1];
  const int nbd = (nv + UT - 1) / UT, nbp = (naux + UT - 1) / UT;
  const int l = blockIdx.x / (nbd * nbp);
  const int rem = blockIdx.x % (nbd * nbp);
  const int p0 = (rem / nbd) * UT, d0 = (rem % nbd) * UT;
  const double2* src = Lvo + (long)l * naux * nv;
  for (int e = threadIdx.x; e < UT * UT; e += 256) {
    const int rp = e / UT, cd = e % UT;
    const int P = p0 + rp, d = d0 + cd;
    t[rp][cd] = (P < naux && d < nv) ? src[(long)P * nv + d] : czero();
  }
  __syncthreads();
  for (int e = threadIdx.x; e < UT * UT; e += 256) {
    const int rd = e / UT, cp = e % UT;
    const int d = d0 + rd, P = p0 + cp;
    if (P < naux && d < nv) LoT[((long)l * nv + d) * naux + P] = cconj(t[cp][rd]);
  }
}

// light sigma1 term, partial over a group of 4 valence j:
//   Tp[mI][jg][K][c] = sum_{j in group} sum_d conj(<Kd||Ij>) R_{mIj}[c][d]
//                    = -sum_j sum_d conj(Vt[I][j][K][d]) Rf[mI][j][d][c]
constexpr int LJG = 4;
//   Tp[mI][jg][K][c] = sum_{j in group} sum_d conj(<Kd||Ij>) R_{mIj}[c][d]
//                    = sum_j sum_d conj(Vt[I][j][K][d]) Rt[(j,d)][(mI,c)]
template <class TI>
__global__ __launch_bounds__(256) void k_light1(const TI* __restrict__ Rt, const double2* __restrict__ Vt,
                                                 int rows, int nc, int no, int nv, double2* __restrict__ Tp) {
  __shared__ double2 vs[8][256];
  const int ncb = (nv + 255) / 256;
  const int njg = (no + LJG - 1) / LJG;
  const int cb = blockIdx.x % ncb;
  const int jg = (blockIdx.x / ncb) % njg;
  const int mI = blockIdx.x / (ncb * njg);
  const int I = mI % nc;
  const int c = cb * 256 + threadIdx.x;
  const bool cok = c < nv;
  const int cs = cok ? c : 0;
  const long ld = (long)rows * nv;
  for (int K0 = 0; K0 < nc; K0 += 8) {
    double2 acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = czero();
    for (int j = jg * LJG; j < min(no, (jg + 1) * LJG); ++j) {
      const TI* R = Rt + (long)j * nv * ld + (long)mI * nv;   // R[d*ld + c]
      const double2* V = Vt + ((long)I * no + j) * nc * nv;
      for (int dd0 = 0; dd0 < nv; dd0 += 256) {
        __syncthreads();
        for (int e = threadIdx.x; e < 8 * 256; e += 256) {
          const int q = e / 256, dd = e % 256;
          const int K = K0 + q, d = dd0 + dd;
          vs[q][dd] = (K < nc && d < nv) ? cconj(V[(long)K * nv + d]) : czero();
        }
        __syncthreads();
        const int dend = min(256, nv - dd0);
        int dd = 0;
        // DU loads in flight per thread (16 for complex64 operands, where more loads
        // in flight paid; 4 for complex128, where the registers would cost occupancy); a lane
        // past the last column reads column 0 and its sums are never stored
        constexpr int DU = sizeof(TI) == 8 ? 16 : 4;
        for (; dd + DU <= dend; dd += DU) {
          TI r[DU];
#pragma unroll
          for (int u = 0; u < DU; ++u) r[u] = R[(long)(dd0 + dd + u) * ld + cs];
#pragma unroll
          for (int u = 0; u < DU; ++u) {
            const double2 x = to_d2(r[u]);
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] = cadd(acc[q], cmul(vs[q][dd + u], x));
          }
        }
        for (; dd < dend; ++dd) {
          const double2 x = to_d2(R[(long)(dd0 + dd) * ld + cs]);
#pragma unroll
          for (int q = 0; q < 8; ++q) acc[q] = cadd(acc[q], cmul(vs[q][dd], x));
        }
      }
    }
    if (cok)
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (K0 + q < nc) Tp[(((long)mI * njg + jg) * nc + K0 + q) * nv + c] = acc[q];
  }
}

// sigma2 = Z_ab - Z_ba + D r2 + sum_K (<Ka||Ij> r1_Kb - r1_Ka <Kb||Ij>), a < b, packed.
// One workgroup per (g = (m,I,j), 32x32 tile pair ab <= bb); the mirror tile
// is staged in LDS so that both reads of Z are coalesced.
constexpr int PT = 32;
constexpr int PK = 8;    // core spinors staged in LDS by the pack kernel (more read from global memory)
template <class TZ>
__global__ __launch_bounds__(256) void k_pack2(const TZ* __restrict__ Z, const double2* __restrict__ xin,
                                                double2* __restrict__ sout, long dim, const double2* __restrict__ Vt,
                                                const double* __restrict__ eps, int m, int nc, int no, int nv,
                                                int with_d) {
  __shared__ double2 zt[PT][PT + 1];
  __shared__ double2 va[PK][PT], vb[PK][PT], ra[PK][PT], rb[PK][PT];
  __shared__ double ea[PT], eb[PT];
  const int nb = (nv + PT - 1) / PT;
  const int ntp = nb * (nb + 1) / 2;
  const long g = blockIdx.x / ntp;
  int t = blockIdx.x % ntp, abk = 0;
  while (t >= nb - abk) {
    t -= nb - abk;
    ++abk;
  }
  const int bbk = abk + t;
  const int a0 = abk * PT, b0 = bbk * PT;
  const int mv = (int)(g / ((long)nc * no));
  const int I = (int)((g / no) % nc), j = (int)(g % no);
  const int o = nc + no;
  const TZ* Zg = Z + g * (long)nv * nv;
  const double2* r1 = xin + (long)mv * dim;
  const double2* V = Vt + ((long)I * no + j) * nc * nv;
  const int tid = threadIdx.x;
  const bool staged = nc <= PK;
  // mirror tile Z[b][a] -> zt[b - b0][a - a0]
  for (int e = tid; e < PT * PT; e += 256) {
    const int rb_ = e / PT, ca = e % PT;
    const int b = b0 + rb_, a = a0 + ca;
    zt[rb_][ca] = (b < nv && a < nv) ? to_d2(Zg[(long)b * nv + a]) : czero();
  }
  if (staged) {
    for (int e = tid; e < nc * PT; e += 256) {
      const int K = e / PT, x = e % PT;
      const int a = a0 + x, b = b0 + x;
      va[K][x] = a < nv ? V[(long)K * nv + a] : czero();
      ra[K][x] = a < nv ? r1[(long)K * nv + a] : czero();
      vb[K][x] = b < nv ? V[(long)K * nv + b] : czero();
      rb[K][x] = b < nv ? r1[(long)K * nv + b] : czero();
    }
  }
  if (tid < PT) ea[tid] = (a0 + tid < nv) ? eps[o + a0 + tid] : 0.0;
  else if (tid < 2 * PT) eb[tid - PT] = (b0 + tid - PT < nv) ? eps[o + b0 + tid - PT] : 0.0;
  __syncthreads();
  const long ns = (long)nc * nv;
  const long npair = (long)nv * (nv - 1) / 2;
  const long off = (long)mv * dim + ns + ((long)I * no + j) * npair;
  const double eIj = eps[I] + eps[nc + j];
  for (int e = tid; e < PT * PT; e += 256) {
    const int ra_ = e / PT, cb = e % PT;
    const int a = a0 + ra_, b = b0 + cb;
    if (a < b && b < nv) {
      double2 v = csub(to_d2(Zg[(long)a * nv + b]), zt[cb][ra_]);
      if (staged) {
        for (int K = 0; K < nc; ++K)
          v = cadd(v, csub(cmul(va[K][ra_], rb[K][cb]), cmul(ra[K][ra_], vb[K][cb])));
      } else {
        for (int K = 0; K < nc; ++K)
          v = cadd(v, csub(cmul(V[(long)K * nv + a], r1[(long)K * nv + b]),
                           cmul(r1[(long)K * nv + a], V[(long)K * nv + b])));
      }
      const long q = pair_offset(a, b, nv);
      const double D = ea[ra_] + eb[cb] - eIj;
      if (with_d) {
        const double2 x2 = xin[off + q];
        v = make_double2(v.x + D * x2.x, v.y + D * x2.y);
      }
      sout[off + q] = v;
    }
  }
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
                                                int nrows, int nv, int naux, int nsplit,
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
  SrcYrows A{Y, naux, nv, cpe, nrows, i0};
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

// s1[m][K][a] += sum_split part[split][mK][a] + sum_{I,jg} Tp[mI][jg][K][a]
__global__ void k_sigma1_finish(const double2* __restrict__ part, int nsplit, const double2* __restrict__ Tp,
                                int m, int nc, int no, int nv, long dim, double2* __restrict__ sout) {
  const long total = (long)m * nc * nv;
  const int njg = (no + LJG - 1) / LJG;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int a = (int)(e % nv);
    const int mK = (int)(e / nv);
    const int mv = mK / nc, K = mK - mv * nc;
    double2 acc = make_double2(0, 0);
    for (int sp = 0; sp < nsplit; ++sp) acc = cadd(acc, part[((long)sp * m * nc + mK) * nv + a]);
    for (int I = 0; I < nc; ++I)
      for (int jg = 0; jg < njg; ++jg)
        acc = csub(acc, Tp[((((long)(mv * nc + I)) * njg + jg) * nc + K) * nv + a]);
    double2* p = sout + (long)mv * dim + (long)K * nv + a;
    *p = cadd(*p, acc);
  }
}

// ---------------------------------------------------------------------------

adc2_status build_lvt(adc2_handle h, hipStream_t st) {
  const Dims& d = h->d;
  if (h->LoT) return ADC2_OK;
  ADC2_HIP(dmalloc(h, &h->LoT, sizeof(double2) * (long)d.o * d.nv * d.naux));
  h->LvT = h->LoT + (long)d.nc * d.nv * d.naux;
  const long nblk = (long)d.o * cdiv(d.nv, UT) * cdiv(d.naux, UT);
  k_lvo_transpose<<<(unsigned)nblk, 256, 0, st>>>(h->Lvo, d.nv, d.naux, h->LoT);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

adc2_status build_c64(adc2_handle h, hipStream_t st) {
  const Dims& d = h->d;
  if (h->Lv32 && h->LvT32) return ADC2_OK;
  const long nlv = (long)d.no * d.naux * d.nv;
  ADC2_HIP(dmalloc(h, &h->Lv32, sizeof(float2) * nlv));
  ADC2_HIP(dmalloc(h, &h->LvT32, sizeof(float2) * nlv));
  k_to_c64<<<grid_for(nlv), 256, 0, st>>>(h->Lvo + (long)d.nc * d.naux * d.nv, nlv, h->Lv32);
  ADC2_CHECK_LAUNCH();
  k_to_c64<<<grid_for(nlv), 256, 0, st>>>(h->LvT, nlv, h->LvT32);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

// Split-BF16 copies of the two static operands (blocked split layout).
adc2_status build_b3(adc2_handle h, hipStream_t st) {
  adc2_status rc = build_c64(h, st);
  if (rc != ADC2_OK) return rc;
  if (h->LvB && h->LvTB) return ADC2_OK;
  const Dims& d = h->d;
  const long K1 = d.naux, R1 = (long)d.no * d.nv;   // sigma2 B: rows (j,b), K = P
  const long K2 = (long)d.no * d.nv, R2 = d.naux;   // Y-build A: rows P, K = (j,d)
  ADC2_HIP(dmalloc(h, &h->LvB, split_bytes(R1, K1)));
  ADC2_HIP(dmalloc(h, &h->LvTB, split_bytes(R2, K2)));
  if ((rc = split_pack(h->Lv32, (long)d.naux * d.nv, d.nv, d.nv, R1, K1, (__bf16*)h->LvB, st)) != ADC2_OK) return rc;
  return split_pack(h->LvT32, 0, d.naux, d.naux, R2, K2, (__bf16*)h->LvTB, st);
}

// Split-BF16 operands and GEMM of the Schur preconditioner's three-virtual
// column.  pack_valence_b3 writes the valence rows of L in the sigma2 B layout
// (rows (j,b), K = P; the same bits as the handle's LvB).  schur_gemm_b3
// packs, for virtuals c in [c0, c0 + nck), A rows (cc,a) with element
// L^P_{a,c0+cc} (from Lvv[P][a][c]) into Ab and forms
//   Z[cc][j][a][b] = sum_P L^P_{a,c0+cc} L^P_{b,j}     (all j, a, b)
// on the sigma2 split-BF16 kernel.
adc2_status pack_valence_b3(adc2_handle h, __bf16* dst, hipStream_t st) {
  const Dims& d = h->d;
  return split_pack(h->Lvo + (long)d.nc * d.naux * d.nv, (long)d.naux * d.nv, d.nv, d.nv, (long)d.no * d.nv, d.naux,
                    dst, st);
}

adc2_status schur_gemm_b3(adc2_handle h, int c0, int nck, const __bf16* LvB, __bf16* Ab, float2* Z,
                          hipStream_t st) {
  const Dims& d = h->d;
  const long R = (long)nck * d.nv;
  // row (cc, a): group cc (stride 1 in Lvv), position a (stride nv), k = P (stride nv^2)
  adc2_status rc = split_pack(h->Lvv + c0, 1, (long)d.nv * d.nv, d.nv, R, d.naux, Ab, st, (long)d.nv);
  if (rc != ADC2_OK) return rc;
  const long nblk = (long)cdiv(R, BT) * cdiv((long)d.no * d.nv, BT);
  k_zsig2_b3<<<(unsigned)nblk, 512, 0, st>>>(Ab, LvB, (int)R, d.no, d.nv, d.naux, Z);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

adc2_status ensure_ws_b3(adc2_handle h, int m) {
  if (h->wsb_m >= m) return ADC2_OK;
  dfree(h, h->XB);
  dfree(h, h->RB);
  h->XB = h->RB = nullptr;
  h->wsb_m = 0;
  const Dims& d = h->d;
  const long rows = (long)m * d.nc * d.nv;
  ADC2_HIP(dmalloc(h, &h->XB, split_bytes(rows, d.naux)));
  ADC2_HIP(dmalloc(h, &h->RB, split_bytes(rows, (long)d.no * d.nv)));
  h->wsb_m = m;
  return ADC2_OK;
}

// Sizes of the FP64 sigma work spaces for a block of m vectors and the two
// split counts that go with them.
struct WsPlan {
  int ysplit, nsplit;
  size_t x, y, zb, tp, part;   // bytes of h->X, h->Y, h->Zb, h->Tp, h->part
};

// ys, ns > 0 impose the split counts instead of choosing them.
// The Y-build's K-split count (1..8) whose tiles fill whole rounds of the
// engine's workgroup slots best (the last round of a launch runs partly
// empty), each further split charged 0.2% for its partial sum.
int ysplit_rule(adc2_handle h, int m) {
  const Dims& d = h->d;
  const long rows = (long)m * d.nc;
  const bool fp64 = h->prec == ADC2_FP64;
  const int tn = fp64 && h->zgemm != ZGEMM_BIG && h->zgemm != ZGEMM_WIDE ? BT3N : BT;
  const long slots = 256L * ((fp64 && h->zgemm != ZGEMM_MID) || h->prec == ADC2_BF16X3 ? 1 : 2);
  const long ytiles = (long)cdiv(d.naux, BT) * cdiv(rows * d.nv, tn);
  int ys = 1;
  double best = 0.0;
  for (int c = 1; c <= 8; ++c) {
    const double rounds = (double)(ytiles * c) / slots;
    const double cost = std::ceil(rounds) / rounds * (1.0 + 0.002 * (c - 1));
    if (c == 1 || cost < best) {
      best = cost;
      ys = c;
    }
  }
  return ys;
}

static WsPlan ws_plan(adc2_handle h, int m, int ys = 0, int ns = 0) {
  const Dims& d = h->d;
  WsPlan p;
  const long rows = (long)m * d.nc;
  if (ys <= 0) {
    ys = ysplit_rule(h, m);
    if (const char* v = getenv("ADC2_YSPLIT")) ys = std::max(1, std::min(16, atoi(v)));
    if (h->ysplit_tuned > 0) ys = h->ysplit_tuned;   // adc2_autotune's choice
  }
  p.ysplit = ys;
  if (ns <= 0) {
    const int nbi = cdiv(rows, TM), nba = cdiv(d.nv, TN);
    ns = std::max(1, std::min(256, 2048 / std::max(1, nbi * nba)));
    ns = std::min(ns, d.naux);
  }
  p.nsplit = ns;
  const int njg = (d.no + LJG - 1) / LJG;
  p.x = sizeof(double2) * rows * d.naux * d.nv;
  p.y = sizeof(double2) * rows * d.naux * d.nv * p.ysplit;
  p.zb = sizeof(double2) * rows * d.no * (long)d.nv * d.nv;
  p.tp = sizeof(double2) * rows * njg * d.nc * d.nv;
  p.part = sizeof(double2) * p.nsplit * rows * d.nv;
  return p;
}

adc2_status ensure_ws(adc2_handle h, int m) {
  if (h->ws_m >= m) return ADC2_OK;
  dfree(h, h->X);
  dfree(h, h->Y);
  dfree(h, h->part);
  dfree(h, h->Zb);
  dfree(h, h->Tp);
  h->X = h->Y = h->part = h->Zb = h->Tp = nullptr;
  h->ws_m = 0;
  const WsPlan p = ws_plan(h, m);
  h->ysplit = p.ysplit;
  h->nsplit = p.nsplit;
  ADC2_HIP(dmalloc(h, &h->X, p.x));
  ADC2_HIP(dmalloc(h, &h->Y, p.y));
  ADC2_HIP(dmalloc(h, &h->Zb, p.zb));
  ADC2_HIP(dmalloc(h, &h->Tp, p.tp));
  ADC2_HIP(dmalloc(h, &h->part, p.part));
  h->ws_m = m;
  return ADC2_OK;
}


// Weighted unpack Rt[(j,d)][(mI,c)] = w_m R_{mIj}[c][d] into h->Zb, and the
// FP64 Y-build on it into h->Y (split partials summed); used by the adjoint.
adc2_status unpack_weighted(adc2_handle h, int m, const double2* xin, const double* wts, hipStream_t st) {
  const Dims& d = h->d;
  const int nb = cdiv(d.nv, UT);
  const long nblk = (long)m * d.nc * d.no * (nb * (nb + 1) / 2);
  k_unpack<double2, true><<<(unsigned)nblk, 256, 0, st>>>(xin, d.dim, m, d.nc, d.no, d.nv, h->Zb, wts);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

adc2_status ybuild_fp64(adc2_handle h, int m, hipStream_t st) {
  const Dims& d = h->d;
  const int rows = m * d.nc;
  const long nblk = (long)cdiv(d.naux, BT) * cdiv((long)rows * d.nv, BT);
  dim3 grid((unsigned)nblk, h->ysplit);
  k_ygemm<false><<<grid, 256, 0, st>>>(h->LvT, h->Zb, rows, d.nc, d.no, d.nv, d.naux, h->Y);
  ADC2_CHECK_LAUNCH();
  if (h->ysplit > 1) {
    const long len = (long)rows * d.naux * d.nv;
    k_ysum<<<grid_for(len), 256, 0, st>>>(h->Y, len, h->ysplit);
    ADC2_CHECK_LAUNCH();
  }
  return ADC2_OK;
}

adc2_status sigma_fp64(adc2_handle h, int m, const double2* xin, double2* sout, hipStream_t st) {
  return sigma_parts(h, m, xin, sout, SIGMA_SINGLES_IN | SIGMA_DOUBLES_IN, st);
}

// zero the singles block of m vectors
__global__ void k_zero_singles(double2* __restrict__ s, long dim, long ns, int m) {
  const long total = ns * m;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x)
    s[(e / ns) * dim + e % ns] = make_double2(0.0, 0.0);
}

// parts = SIGMA_SINGLES_IN: sigma of (r1, 0):  s1 = M11 r1, s2 = M21 r1 (doubles of xin not read)
// parts = SIGMA_DOUBLES_IN: singles of the sigma of (0, r2): s1 = M12 r2 (singles of xin not read,
//                           doubles of sout not written)
// both: the full sigma.
adc2_status sigma_parts(adc2_handle h, int m, const double2* xin, double2* sout, int parts, hipStream_t st) {
  const SigReq r{h, m, xin, sout, parts};
  return sigma_multi(1, &r, st);
}

adc2_status sigma_call(adc2_handle h, int m, const double2* xin, double2* sout, int parts, hipStream_t st) {
  if (h->sigma_hook) return h->sigma_hook(m, xin, sout, parts, st);
  return sigma_parts(h, m, xin, sout, parts, st);
}

// The Y-build GEMM of one request (m vectors) in the handle's precision form,
// h->ysplit K-split partials into h->Y.
adc2_status ybuild_launch(adc2_handle h, int m, hipStream_t st) {
  const Dims& d = h->d;
  const int rows = m * d.nc;
  const int ys = h->ysplit;
  if (h->prec != ADC2_FP64) {
    const long nblk = (long)cdiv(d.naux, BT) * cdiv((long)rows * d.nv, BT);
    dim3 grid((unsigned)nblk, ys);
    if (h->prec == ADC2_BF16X3)
      k_ygemm_b3<<<grid, 512, 0, st>>>((const __bf16*)h->LvTB, (const __bf16*)h->RB, rows, d.no, d.nv, d.naux, h->Y);
    else
      k_ygemm_c64<<<grid, 256, 0, st>>>(h->LvT32, (const float2*)h->Zb, rows, d.no, d.nv, d.naux, h->Y);
  } else {
    const bool wide_tile = h->zgemm == ZGEMM_BIG || h->zgemm == ZGEMM_WIDE;
    const long nblk = (long)cdiv(d.naux, BT) * cdiv((long)rows * d.nv, wide_tile ? BT : BT3N);
    dim3 grid((unsigned)nblk, ys);
    if (h->zgemm == ZGEMM_WIDE)
      k_ygemm_wide<<<grid, 512, 0, st>>>(h->LvT, h->Zb, rows, d.no, d.nv, d.naux, h->Y);
    else if (h->zgemm == ZGEMM_MID)
      k_ygemm_mid<<<grid, 256, 0, st>>>(h->LvT, h->Zb, rows, d.no, d.nv, d.naux, h->Y);
    else if (h->zgemm == ZGEMM_3M)
      k_ygemm<true><<<grid, 256, 0, st>>>(h->LvT, h->Zb, rows, d.nc, d.no, d.nv, d.naux, h->Y);
    else
      k_ygemm<false><<<grid, 256, 0, st>>>(h->LvT, h->Zb, rows, d.nc, d.no, d.nv, d.naux, h->Y);
  }
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

// Sum of the Y-build's K-split partials into the first one.
adc2_status ybuild_sum(adc2_handle h, int m, hipStream_t st) {
  const Dims& d = h->d;
  if (h->ysplit > 1) {
    const long len = (long)m * d.nc * d.naux * d.nv;
    k_ysum<<<grid_for(len), 256, 0, st>>>(h->Y, len, h->ysplit);
    ADC2_CHECK_LAUNCH();
  }
  return ADC2_OK;
}

// Launch the grouped heavy GEMM (Y-build if ybuild, else sigma2) of the
// requests selected by use[] whose handles share the precision form prec
// (complex64 or split-BF16), GMAX systems per launch.
static adc2_status grouped_gemm(int nreq, const SigReq* rq, const std::vector<char>& use, int prec, bool ybuild,
                                hipStream_t st) {
  GemmJobs J;
  J.n = 0;
  J.total = 0;
  auto flush = [&]() -> adc2_status {
    if (J.n == 0) return ADC2_OK;
    const unsigned grid = (unsigned)std::min<long>(J.total, 1L << 20);   // both multiples of 8
    if (prec == ADC2_BF16X3) {
      if (ybuild) k_gemm_b3_grouped<true><<<grid, 512, 0, st>>>(J);
      else k_gemm_b3_grouped<false><<<grid, 512, 0, st>>>(J);
    } else {
      if (ybuild) k_gemm_c64_grouped<true><<<grid, 256, 0, st>>>(J);
      else k_gemm_c64_grouped<false><<<grid, 256, 0, st>>>(J);
    }
    ADC2_CHECK_LAUNCH();
    J.n = 0;
    J.total = 0;
    return ADC2_OK;
  };
  // requests of this form, by decreasing K per item (ties: request order)
  std::vector<std::pair<long, int>> order;
  for (int q = 0; q < nreq; ++q) {
    if (!use[q] || rq[q].h->prec != prec) continue;
    const Dims& d = rq[q].h->d;
    const long kpi = ybuild ? (long)d.no * d.nv / std::max(1, rq[q].h->ysplit) : (long)d.naux;
    order.push_back({-kpi, q});
  }
  std::stable_sort(order.begin(), order.end(),
                   [](const std::pair<long, int>& a, const std::pair<long, int>& b) { return a.first < b.first; });
  for (const auto& oq : order) {
    const int q = oq.second;
    adc2_handle h = rq[q].h;
    const Dims& d = h->d;
    const int rows = rq[q].m * d.nc;
    GemmJob& g = J.j[J.n];
    g.rows = ybuild ? rows : rows * d.nv;
    g.no = d.no;
    g.nv = d.nv;
    g.naux = d.naux;
    const bool split = prec == ADC2_BF16X3;
    if (ybuild) {
      g.A = split ? h->LvTB : (const void*)h->LvT32;
      g.B = split ? h->RB : (const void*)h->Zb;
      g.C = h->Y;
      g.nsplit = h->ysplit;
      g.ntile = (long)cdiv(d.naux, BT) * cdiv((long)rows * d.nv, BT);
    } else {
      g.A = split ? h->XB : (const void*)h->X;
      g.B = split ? h->LvB : (const void*)h->Lv32;
      g.C = h->Zb;
      g.nsplit = 1;
      g.ntile = (long)cdiv((long)rows * d.nv, BT) * cdiv((long)d.no * d.nv, BT);
    }
    g.w0 = J.total;
    J.total += (g.ntile * g.nsplit + 7) & ~7L;
    if (++J.n == GMAX) {
      adc2_status r = flush();
      if (r != ADC2_OK) return r;
    }
  }
  return flush();
}

// Several sigma requests (possibly of different systems) on one stream.  Each
// phase runs for every request before the next phase; with more than one
// request the two heavy GEMMs of the requests in the complex64 and split-BF16
// forms are one grouped launch per form.  Per-kernel profiling (adc2_profile)
// is recorded for single requests only.
adc2_status sigma_multi(int nreq, const SigReq* rq, hipStream_t st) {
  adc2_status rc;
  for (int q = 0; q < nreq; ++q) {
    adc2_handle h = rq[q].h;
    if ((rc = ensure_ws(h, rq[q].m)) != ADC2_OK) return rc;
    const bool b3 = h->prec == ADC2_BF16X3;
    const bool c64 = h->prec == ADC2_C64 || b3;   // complex64 operand copies
    if (c64 && (rc = build_c64(h, st)) != ADC2_OK) return rc;
    if (b3 && ((rc = build_b3(h, st)) != ADC2_OK || (rc = ensure_ws_b3(h, rq[q].m)) != ADC2_OK)) return rc;
  }
  adc2_handle h0 = rq[0].h;
  const bool prof = nreq == 1 && h0->profiling != 0;
  auto mark = [&](int i) -> adc2_status {
    if (prof) ADC2_HIP(hipEventRecord(h0->kev[i], st));
    return ADC2_OK;
  };
  std::vector<char> sgl(nreq), dbl(nreq);
  for (int q = 0; q < nreq; ++q) {
    sgl[q] = (rq[q].parts & SIGMA_SINGLES_IN) != 0;
    dbl[q] = (rq[q].parts & SIGMA_DOUBLES_IN) != 0;
  }
  // precision forms that have a grouped GEMM and more than one request
  auto grouped = [&](const std::vector<char>& use, int prec) {
    if (nreq < 2) return false;
    int n = 0;
    for (int q = 0; q < nreq; ++q) n += use[q] && rq[q].h->prec == prec;
    return n > 0;
  };
  auto is_grouped = [&](int q) { return nreq > 1 && rq[q].h->prec != ADC2_FP64; };

  // kernel order (profiling slots): unpack, ygemm, light1, xbuild, zsig2, pack2, backc, m11mv+finish
  if ((rc = mark(0)) != ADC2_OK) return rc;
  for (int q = 0; q < nreq; ++q) {
    if (!dbl[q]) continue;
    adc2_handle h = rq[q].h;
    const Dims& d = h->d;
    const bool c64 = h->prec != ADC2_FP64;
    const int nb = cdiv(d.nv, UT);
    const long nblk = (long)rq[q].m * d.nc * d.no * (nb * (nb + 1) / 2);
    if (c64)
      k_unpack<float2, false><<<(unsigned)nblk, 256, 0, st>>>(rq[q].xin, d.dim, rq[q].m, d.nc, d.no, d.nv,
                                                               (float2*)h->Zb, nullptr);
    else
      k_unpack<double2, false><<<(unsigned)nblk, 256, 0, st>>>(rq[q].xin, d.dim, rq[q].m, d.nc, d.no, d.nv, h->Zb,
                                                                nullptr);
    ADC2_CHECK_LAUNCH();
  }
  for (int q = 0; q < nreq; ++q) {   // split-BF16: the unpacked doubles into the blocked split layout
    adc2_handle h = rq[q].h;
    if (!dbl[q] || h->prec != ADC2_BF16X3) continue;
    const Dims& d = h->d;
    const long ncols = (long)rq[q].m * d.nc * d.nv;
    if ((rc = split_pack((const float2*)h->Zb, 0, ncols, (int)ncols, ncols, (long)d.no * d.nv, (__bf16*)h->RB, st)) !=
        ADC2_OK)
      return rc;
  }
  if ((rc = mark(1)) != ADC2_OK) return rc;
  for (int prec : {ADC2_C64, ADC2_BF16X3})
    if (grouped(dbl, prec) && (rc = grouped_gemm(nreq, rq, dbl, prec, true, st)) != ADC2_OK) return rc;
  for (int q = 0; q < nreq; ++q) {
    if (!dbl[q]) continue;
    adc2_handle h = rq[q].h;
    if (!is_grouped(q) && (rc = ybuild_launch(h, rq[q].m, st)) != ADC2_OK) return rc;
    if ((rc = ybuild_sum(h, rq[q].m, st)) != ADC2_OK) return rc;
  }
  if ((rc = mark(2)) != ADC2_OK) return rc;
  for (int q = 0; q < nreq; ++q) {
    if (!dbl[q]) continue;
    adc2_handle h = rq[q].h;
    const Dims& d = h->d;
    const int rows = rq[q].m * d.nc;
    const int njg = (d.no + LJG - 1) / LJG;
    const unsigned g = (unsigned)(rows * njg * ((d.nv + 255) / 256));
    if (h->prec != ADC2_FP64)
      k_light1<float2><<<g, 256, 0, st>>>((const float2*)h->Zb, h->Vt, rows, d.nc, d.no, d.nv, h->Tp);
    else
      k_light1<double2><<<g, 256, 0, st>>>(h->Zb, h->Vt, rows, d.nc, d.no, d.nv, h->Tp);
    ADC2_CHECK_LAUNCH();
  }
  if ((rc = mark(3)) != ADC2_OK) return rc;
  for (int q = 0; q < nreq; ++q) {
    if (!sgl[q]) continue;
    adc2_handle h = rq[q].h;
    const Dims& d = h->d;
    const int rows = rq[q].m * d.nc;
    const long nblk = (long)cdiv(rows, TM) * cdiv((long)d.naux * d.nv, TN);
    if (h->prec != ADC2_FP64)
      k_xbuild<float2><<<(unsigned)nblk, 256, 0, st>>>(rq[q].xin, d.dim, d.nc, d.nv, d.naux, rows, h->Lvv,
                                                       (float2*)h->X);
    else
      k_xbuild<double2><<<(unsigned)nblk, 256, 0, st>>>(rq[q].xin, d.dim, d.nc, d.nv, d.naux, rows, h->Lvv, h->X);
    ADC2_CHECK_LAUNCH();
  }
  for (int q = 0; q < nreq; ++q) {   // split-BF16: X into the blocked split layout
    adc2_handle h = rq[q].h;
    if (!sgl[q] || h->prec != ADC2_BF16X3) continue;
    const Dims& d = h->d;
    if ((rc = split_pack((const float2*)h->X, (long)d.naux * d.nv, d.nv, d.nv, (long)rq[q].m * d.nc * d.nv, d.naux,
                         (__bf16*)h->XB, st)) != ADC2_OK)
      return rc;
  }
  if ((rc = mark(4)) != ADC2_OK) return rc;
  for (int prec : {ADC2_C64, ADC2_BF16X3})
    if (grouped(sgl, prec) && (rc = grouped_gemm(nreq, rq, sgl, prec, false, st)) != ADC2_OK) return rc;
  for (int q = 0; q < nreq; ++q) {
    if (!sgl[q] || is_grouped(q)) continue;
    adc2_handle h = rq[q].h;
    const Dims& d = h->d;
    const int rows = rq[q].m * d.nc;
    if (h->prec != ADC2_FP64) {
      const long nblk = (long)cdiv((long)rows * d.nv, BT) * cdiv((long)d.no * d.nv, BT);
      if (h->prec == ADC2_BF16X3)
        k_zsig2_b3<<<(unsigned)nblk, 512, 0, st>>>((const __bf16*)h->XB, (const __bf16*)h->LvB, rows * d.nv, d.no,
                                                     d.nv, d.naux, (float2*)h->Zb);
      else
        k_zsig2_c64<<<(unsigned)nblk, 256, 0, st>>>((const float2*)h->X, h->Lv32, rows * d.nv, d.no, d.nv, d.naux,
                                                      (float2*)h->Zb);
    } else if (h->zgemm == ZGEMM_WIDE) {
      const long nblk = (long)cdiv((long)rows * d.nv, BT) * cdiv((long)d.no * d.nv, BT);
      k_zsig2_wide<<<(unsigned)nblk, 512, 0, st>>>(h->X, h->Lvo, rows * d.nv, d.nc, d.no, d.nv, d.naux, h->Zb);
    } else if (h->zgemm == ZGEMM_MID) {
      const long nblk = (long)cdiv((long)rows * d.nv, BT) * cdiv((long)d.no * d.nv, MTN);
      k_zsig2_mid<<<(unsigned)nblk, 256, 0, st>>>(h->X, h->Lvo, rows * d.nv, d.nc, d.no, d.nv, d.naux, h->Zb);
    } else if (h->zgemm == ZGEMM_3M) {
      const long nblk = (long)cdiv((long)rows * d.nv, BT) * cdiv((long)d.no * d.nv, BT3N);
      k_zsig2<true><<<(unsigned)nblk, 256, 0, st>>>(h->X, h->Lvo, rows * d.nv, d.nc, d.no, d.nv, d.naux, h->Zb);
    } else {
      const long nblk = (long)cdiv((long)rows * d.nv, BT) * cdiv((long)d.no * d.nv, BT);
      k_zsig2<false><<<(unsigned)nblk, 256, 0, st>>>(h->X, h->Lvo, rows * d.nv, d.nc, d.no, d.nv, d.naux, h->Zb);
    }
    ADC2_CHECK_LAUNCH();
  }
  if ((rc = mark(5)) != ADC2_OK) return rc;
  for (int q = 0; q < nreq; ++q) {
    if (!sgl[q]) continue;
    adc2_handle h = rq[q].h;
    const Dims& d = h->d;
    const int m = rq[q].m;
    const int with_d = dbl[q] ? 1 : 0;
    const int nb = cdiv(d.nv, PT);
    const long nblk = (long)m * d.nc * d.no * (nb * (nb + 1) / 2);
    if (h->prec != ADC2_FP64)
      k_pack2<float2><<<(unsigned)nblk, 256, 0, st>>>((const float2*)h->Zb, rq[q].xin, rq[q].sout, d.dim, h->Vt,
                                                      h->eps, m, d.nc, d.no, d.nv, with_d);
    else
      k_pack2<double2><<<(unsigned)nblk, 256, 0, st>>>(h->Zb, rq[q].xin, rq[q].sout, d.dim, h->Vt, h->eps, m, d.nc,
                                                       d.no, d.nv, with_d);
    ADC2_CHECK_LAUNCH();
  }
  if ((rc = mark(6)) != ADC2_OK) return rc;
  for (int q = 0; q < nreq; ++q) {
    if (!dbl[q]) continue;
    adc2_handle h = rq[q].h;
    const Dims& d = h->d;
    const int rows = rq[q].m * d.nc;
    const long nblk = (long)cdiv(rows, TM) * cdiv(d.nv, TN) * h->nsplit;
    k_backc<<<(unsigned)nblk, 256, 0, st>>>(h->Y, h->Lvv, rows, d.nv, d.naux, h->nsplit, h->part);
    ADC2_CHECK_LAUNCH();
  }
  if ((rc = mark(7)) != ADC2_OK) return rc;
  for (int q = 0; q < nreq; ++q) {
    adc2_handle h = rq[q].h;
    const Dims& d = h->d;
    const int m = rq[q].m;
    if (sgl[q]) {
      adc2_status r2 = gemm_rr(m, (int)d.ns, (int)d.ns, rq[q].xin, d.dim, false, h->M11, d.ns, false, rq[q].sout,
                               d.dim, 1.0, false, st);
      if (r2 != ADC2_OK) return r2;
    } else {
      k_zero_singles<<<grid_for(d.ns * m), 256, 0, st>>>(rq[q].sout, d.dim, d.ns, m);
      ADC2_CHECK_LAUNCH();
    }
    if (dbl[q]) {
      const int rows = m * d.nc;
      k_sigma1_finish<<<grid_for((long)rows * d.nv, 256, 4096), 256, 0, st>>>(h->part, h->nsplit, h->Tp, m, d.nc,
                                                                                d.no, d.nv, d.dim, rq[q].sout);
      ADC2_CHECK_LAUNCH();
    }
  }
  if ((rc = mark(8)) != ADC2_OK) return rc;
  // ADC(2)-x: the first-order doubles block (FP64), on whole sigma requests only
  for (int q = 0; q < nreq; ++q) {
    adc2_handle h = rq[q].h;
    if (h->method != ADC2_METHOD_ADC2X) continue;
    if (!sgl[q] || !dbl[q]) {
      set_error("sigma: ADC(2)-x needs whole sigma products (partial products assume a diagonal doubles block)");
      return ADC2_ERR_ARG;
    }
    if ((rc = adc2x_apply(h, rq[q].m, rq[q].xin, rq[q].sout, st)) != ADC2_OK) return rc;
  }
  if (prof) {
    adc2_handle h = h0;
    const Dims& d = h->d;
    ADC2_HIP(hipEventSynchronize(h->kev[8]));
    const double nc_ = d.nc, no_ = d.no, nv_ = d.nv, na_ = d.naux, m_ = rq[0].m;
    const double heavy = 8.0 * m_ * nc_ * no_ * nv_ * nv_ * na_;
    const double fs = sgl[0] ? 1.0 : 0.0, fd = dbl[0] ? 1.0 : 0.0;
    const double fl[adc2_handle_s::NK] = {
        0.0,                                             // unpack (data movement)
        fd * heavy,                                      // Y-build GEMM
        fd * 8.0 * m_ * nc_ * no_ * nv_ * nv_ * nc_,     // light sigma1 core term
        fs * 8.0 * m_ * nc_ * nv_ * nv_ * na_,           // X-build
        fs * heavy,                                      // sigma2 GEMM
        fs * 8.0 * m_ * nc_ * no_ * nv_ * nv_ * nc_,     // pack + light sigma2 core term
        fd * 8.0 * m_ * nc_ * nv_ * nv_ * na_,           // back-contraction
        fs * 8.0 * m_ * (nc_ * nv_) * (nc_ * nv_)};      // M11 r1 + finish
    const bool ran[adc2_handle_s::NK] = {(bool)dbl[0], (bool)dbl[0], (bool)dbl[0], (bool)sgl[0],
                                          (bool)sgl[0], (bool)sgl[0], (bool)dbl[0], true};
    for (int i = 0; i < adc2_handle_s::NK; ++i) {
      if (!ran[i]) continue;
      float ms = 0.f;
      ADC2_HIP(hipEventElapsedTime(&ms, h->kev[i], h->kev[i + 1]));
      h->k_ms[i] += ms;
      h->k_launches[i] += 1;
      h->k_flops[i] += fl[i];
    }
  }
  return ADC2_OK;
}

}  // namespace adc2

// ---------------------------------------------------------------------------
// Sigma without device allocation: the FP64 sigma build of adc2_sigma with its
// work spaces (X, Y, unpacked doubles, light partials, back-contraction
// partials) carved from one static device array instead of the handle's
// buffers.  The array is a fixed part of the code object, so each device the
// library runs on holds one copy until the process ends; the host reaches it
// only through the address hipGetSymbolAddress returns for the current
// device (the array's own name is a host-side stand-in).
// ---------------------------------------------------------------------------
namespace adc2 {
namespace {
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(128) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
}  // namespace
}  // namespace adc2

static __device__ __align__(256) unsigned char scratch[adc2::NOALLOC_SCRATCH_BYTES];

namespace adc2 {

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per device.
static adc2_status scratch_address(void** out) {
  int dev = 0;
  ADC2_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
    set_error("adc2_sigma_noalloc: device index out of range");
    return ADC2_ERR_ARG;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    ADC2_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("adc2_sigma_noalloc: hipGetSymbolAddress returned NULL");
      return ADC2_ERR_HIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ADC2_OK;
}

// The plan of a no-allocation sigma: the split counts adc2_sigma would use
// on this handle now (those of its current work spaces when they already
// hold m vectors), so that both give the same result.
static WsPlan noalloc_plan(adc2_handle h, int m) {
  return h->ws_m >= m ? ws_plan(h, m, h->ysplit, h->nsplit) : ws_plan(h, m);
}

static size_t plan_bytes(const WsPlan& p) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return al(p.x) + al(p.y) + al(p.zb) + al(p.tp) + al(p.part);
}

}  // namespace adc2

extern "C" adc2_status adc2_sigma_noalloc(adc2_handle h, int m, const void* X, void* S, void* stream) {
  using namespace adc2;
  if (!h || !X || !S || m <= 0) {
    set_error("adc2_sigma_noalloc: bad arguments");
    return ADC2_ERR_ARG;
  }
  if (X == S) {
    set_error("adc2_sigma_noalloc: S must not alias X");
    return ADC2_ERR_ARG;
  }
  if (h->prec != ADC2_FP64) {
    set_error("adc2_sigma_noalloc: only the FP64 form (the handle is in a precision form)");
    return ADC2_ERR_ARG;
  }
  if (h->method != ADC2_METHOD_ADC2) {
    set_error("adc2_sigma_noalloc: only the ADC(2) matrix (the handle is set to ADC(2)-x)");
    return ADC2_ERR_ARG;
  }
  const WsPlan p = noalloc_plan(h, m);
  const size_t need = plan_bytes(p);
  if (need > NOALLOC_SCRATCH_BYTES) {
    char buf[256];
    snprintf(buf, sizeof buf,
             "adc2_sigma_noalloc: m=%d needs %zu bytes of scratch, above its maximum of %zu bytes "
             "(use adc2_sigma)",
             m, need, NOALLOC_SCRATCH_BYTES);
    set_error(buf);
    return ADC2_ERR_ARG;
  }
  void* base = nullptr;
  adc2_status rc = scratch_address(&base);
  if (rc != ADC2_OK) return rc;
  // point the handle's work spaces into the scratch for this call only; the
  // kernels take these addresses as arguments at launch
  double2 *sX = h->X, *sY = h->Y, *sZb = h->Zb, *sTp = h->Tp, *spart = h->part;
  const int sws = h->ws_m, sys = h->ysplit, sns = h->nsplit;
  unsigned char* q = static_cast<unsigned char*>(base);
  auto take = [&](size_t b) {
    double2* r = reinterpret_cast<double2*>(q);
    q += (b + 255) & ~size_t(255);
    return r;
  };
  h->X = take(p.x);
  h->Y = take(p.y);
  h->Zb = take(p.zb);
  h->Tp = take(p.tp);
  h->part = take(p.part);
  h->ws_m = m;
  h->ysplit = p.ysplit;
  h->nsplit = p.nsplit;
  rc = sigma_parts(h, m, static_cast<const double2*>(X), static_cast<double2*>(S),
                   SIGMA_SINGLES_IN | SIGMA_DOUBLES_IN, static_cast<hipStream_t>(stream));
  h->X = sX;
  h->Y = sY;
  h->Zb = sZb;
  h->Tp = sTp;
  h->part = spart;
  h->ws_m = sws;
  h->ysplit = sys;
  h->nsplit = sns;
  return rc;
}

