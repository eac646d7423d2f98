// k_adjoint.hip -- adjoint of the CVS-ADC(2) eigenvalues with respect to the
// Cholesky vectors and the spinor energies (Hellmann-Feynman).
//
// For normalised eigenvectors x_k of the Hermitian secular matrix M(L, eps)
// (Eq. 11, truncated at second order, Eq. 12), d omega_k = x_k^H dM x_k.  The
// library differentiates
//     f(L, eps) = sum_k g_k x_k^H M(L, eps) x_k / (x_k^H x_k)
// with the x_k held fixed, which is sum_k g_k omega_k to first order when the
// x_k are eigenvectors.  With r1 (singles) and r2 (doubles, antisymmetric in
// the two virtual indices) of every vector and w_k = g_k / |x_k|^2:
//
//   f = sum gamma . M11  +  2 Re sum_k w_k r2^H M21 r1  +  sum_k w_k r2^H D r2,
//   gamma_{Ia,Jb} = sum_k w_k conj(r1_{k,Ia}) r1_{k,Jb}.
//
// Every integral is (pq|rs) = sum_P L^P_pq L^P_rs, so f is a polynomial in L
// (through <aJ||Ib>, the couplings <ab||cj>, <Ka||Ij> and the quadratic
// second-order terms in W_{ac,kl} = <ac||kl>) and rational in eps (through
// the MP2 denominators).  The gradient g^P_pq = df/dRe L + i df/dIm L of this
// expression is accumulated block by block:
//   hvo[k][P][a]  = g^P_{ak} + conj(g^P_{ka})   (virtual-occupied blocks)
//   gvv[P][a][c]  = g^P_{ac},   goo[P][k][l] = g^P_{kl}
// and the result is its Hermitian projection G^P = (g^P + g^P^H) / 2, the
// unique gradient on Hermitian L:  df = Re sum conj(G) dL for Hermitian dL.
//
// Second-order terms.  Writing f2 = sum gamma . M11^(2) with W_{ac,kl} for
// every ordered occupied pair as independent variables, E = df2/dconj(W) is
//   E_{bc,kl} = Q_{bc,kl} + P_{bc,kl} / D^{bc}_{kl},   P = G(W), Q = G(W / D),
// with the linear map G
//   (i)        1/4 sum_a Gamma_ab X_{ac,kl},        Gamma_ab = sum_I gamma_{Ia,Ib}
//   (ii)+(iii) sum_{Ia} Gc_{(Ia),(Jb)} X_{ac,Ik}    (first occupied index core J)
//   Gc_{(Ia),(Jb)} = -1/2 gamma_{Ia,Jb} + 1/4 delta_ab Gamma'_IJ,  Gamma'_IJ = sum_a gamma_{Ia,Ja}.
// Since W is antisymmetric in (a,c) and in (k,l), only the antisymmetric part
// E^A of E enters, and  dW = dL L + L dL  gives
//   g^P_{ak} += 8 sum_{c,l} E^A_{ac,kl} conj(L^P_{cl}).
// The denominator derivative is df2/dD^{ac}_{kl} = -2 Re(W conj(P)) / D^2.
#include <algorithm>
#include <vector>

#include "internal.h"
#include "tile.h"
#include "zgemm.h"

namespace adc2 {

__host__ __device__ static inline int cdv(long a, long b) { return (int)((a + b - 1) / b); }

static inline unsigned grid1(long n, long per = 256, long cap = 16384) {
  long g = (n + per - 1) / per;
  return (unsigned)std::max<long>(1, std::min<long>(g, cap));
}

// ---------------------------------------------------------------------------
// Generic 64x64-tile complex GEMM over functor sources.
//   C(i, j; b) = sum_k A(k, i; b) B(k, j; b),  i < M, j < N, k < K, batch b,
// A/B provide  MAP  and  double2 get(int k, int i, int b) const  (absolute
// indices, always in range); the epilogue EP(i, j, b, value) consumes C.
// K may be split over workgroups; the partials then go through a reduction
// kernel that applies the same epilogue.
// ---------------------------------------------------------------------------
template <class S>
struct AtTile {
  static constexpr int MAP = S::MAP;
  S s;
  int i0, ni, nk, b;
  __device__ __forceinline__ double2 get(int k, int i) const {
    if (k >= nk || i >= ni) return czero();
    return s.get(k, i0 + i, b);
  }
};

template <class SA, class SB, class EP>
__global__ __launch_bounds__(256) void k_fgemm(int M, int N, int K, int nsplit, SA A, SB B, EP ep,
                                                double2* __restrict__ part) {
  __shared__ TileSmem s;
  const int nbi = cdv(M, TM), nbj = cdv(N, TN);
  const long ntile = (long)nbi * nbj;
  const long lid = xcd_remap(blockIdx.x, ntile * nsplit);
  const int split = (int)(lid / ntile);
  const long tile = lid % ntile;
  const int i0 = (int)(tile / nbj) * TM, j0 = (int)(tile % nbj) * TN;
  const int b = blockIdx.y;
  const int nch = cdv(K, TK);
  const int per = cdv(nch, nsplit);
  const int kc0 = split * per, kc1 = min(nch, kc0 + per);
  AtTile<SA> a{A, i0, M - i0, K, b};
  AtTile<SB> bb{B, j0, N - j0, K, b};
  Acc acc;
  acc.zero();
  mainloop(s, a, bb, kc0, kc1, acc);
  for_each_acc(acc, [&](int r, int c, double2 v) {
    const int i = i0 + r, j = j0 + c;
    if (i < M && j < N) {
      if (nsplit == 1) ep(i, j, b, v);
      else part[(((long)split * gridDim.y + b) * M + i) * N + j] = v;
    }
  });
}

template <class EP>
__global__ void k_fgemm_reduce(int M, int N, int nb, int nsplit, const double2* __restrict__ part, EP ep) {
  const long len = (long)M * N;
  const long total = len * nb;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int b = (int)(e / len);
    const long r = e - (long)b * len;
    double2 acc = czero();
    for (int s = 0; s < nsplit; ++s) acc = cadd(acc, part[((long)s * nb + b) * len + r]);
    ep((int)(r / N), (int)(r % N), b, acc);
  }
}

struct Scratch {
  double2* p;
  long n;
};

template <class SA, class SB, class EP>
static adc2_status fgemm(int M, int N, int K, int nb, const SA& A, const SB& B, const EP& ep, Scratch scr,
                         hipStream_t st) {
  if (M <= 0 || N <= 0 || nb <= 0) return ADC2_OK;
  const long tiles = (long)cdv(M, TM) * cdv(N, TN);
  const int nch = std::max(1, cdv(K, TK));
  int nsplit = 1;
  if (tiles * nb < 512) {
    nsplit = (int)std::min<long>((1024 + tiles * nb - 1) / (tiles * nb), std::max(1, nch / 8));
    const long cap = scr.n / std::max<long>(1, (long)M * N * nb);
    nsplit = (int)std::max<long>(1, std::min<long>(nsplit, cap));
  }
  dim3 grid((unsigned)(tiles * nsplit), (unsigned)nb);
  k_fgemm<SA, SB, EP><<<grid, 256, 0, st>>>(M, N, K, nsplit, A, B, ep, scr.p);
  ADC2_CHECK_LAUNCH();
  if (nsplit > 1) {
    k_fgemm_reduce<EP><<<grid1((long)M * N * nb), 256, 0, st>>>(M, N, nb, nsplit, scr.p, ep);
    ADC2_CHECK_LAUNCH();
  }
  return ADC2_OK;
}

// ---------------------------------------------------------------------------
// Large-tile (128x128, FP64 MFMA) GEMM of two K-major grouped operands into a
// dense C[split][M][N], and the scatter-add of alpha * sum_split C into a
// [g][P][x] block (column j = (g, x), x < inner):  dst[(g0+g)*gs + i*ld + x].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bgemm(SrcGroupedK<8> A, SrcGroupedK<8> B, int M, int N, int K,
                                                double2* __restrict__ C) {
  const int nbm = (M + BT - 1) / BT, nbn = (N + BT - 1) / BT;
  const long lid = xcd_remap(blockIdx.x, (long)nbm * nbn);
  int bm, bn;
  big_tile_coords(lid, nbm, nbn, bm, bn);
  const int i0 = bm * BT, j0 = bn * BT;
  A.begin(threadIdx.x, i0);
  B.begin(threadIdx.x, j0);
  const int nchunks = (K + BK - 1) / BK;
  const int per = (nchunks + gridDim.y - 1) / gridDim.y;
  const int kc0 = blockIdx.y * per, kc1 = min(nchunks, kc0 + per);
  double2* Cs = C + (long)blockIdx.y * M * N;
  __shared__ BigSmem s[2];
  BigAcc acc;
  acc.zero();
  big_mainloop(s, A, B, kc0, kc1, acc);
  big_for_each(acc, [&](int r, int c, double2 v) {
    const int i = i0 + r, j = j0 + c;
    if (i < M && j < N) Cs[(long)i * N + j] = v;
  });
}

// Host launcher of k_bgemm for other translation units: both operands
// K-major grouped rows (SrcGroupedK), output C[split][M][N].
adc2_status bgemm_kmajor(const double2* A, long a_gstride, long a_ld, int a_inner, const double2* B, long b_gstride,
                         long b_ld, int b_inner, int M, int N, int K, int nsplit, double2* C, hipStream_t st) {
  if (M <= 0 || N <= 0) return ADC2_OK;
  SrcGroupedK<8> sa{A, a_gstride, a_ld, a_inner, M, K};
  SrcGroupedK<8> sb{B, b_gstride, b_ld, b_inner, N, K};
  const long tiles = (long)cdv(M, BT) * cdv(N, BT);
  k_bgemm<<<dim3((unsigned)tiles, nsplit), 256, 0, st>>>(sa, sb, M, N, K, C);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

__global__ void k_scatter_add(const double2* __restrict__ C, int nsplit, int M, int N, int inner, long gs, long ld,
                              double alpha, double2* __restrict__ dst) {
  const long len = (long)M * N;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < len; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e % N);
    double2 v = czero();
    for (int s = 0; s < nsplit; ++s) v = cadd(v, C[(long)s * len + e]);
    const int g = j / inner, x = j - g * inner;
    double2* p = dst + (long)g * gs + (long)i * ld + x;
    *p = cadd(*p, cscale(v, alpha));
  }
}

// ---------------------------------------------------------------------------
// Sources and epilogues of the small contractions.
// ---------------------------------------------------------------------------
// gamma:  A(k, i) = w_k conj(x_k[i]),  B(k, j) = x_k[j]   (singles part, i,j < ns)
struct SrcWr1c {
  static constexpr int MAP = KMAJOR;
  const double2* x;
  long dim;
  const double* w;
  __device__ double2 get(int k, int i, int) const { return cscale(cconj(x[(long)k * dim + i]), w[k]); }
};
struct SrcR1 {
  static constexpr int MAP = KMAJOR;
  const double2* x;
  long dim;
  __device__ double2 get(int k, int j, int) const { return x[(long)k * dim + j]; }
};
struct EpStore {
  double2* C;
  long ld;
  __device__ void operator()(int i, int j, int, double2 v) const { C[(long)i * ld + j] = v; }
};

// XT[(mI,a)][P] = conj(X^P_{mI,a}) = conj(sum_c Lvv[P][a][c] r1[m][I][c])
struct SrcR1rows {  // (k = c, i = mI)
  static constexpr int MAP = RMAJOR;
  const double2* x;
  long dim;
  int nc, nv;
  __device__ double2 get(int k, int i, int) const {
    const int m = i / nc, I = i - m * nc;
    return x[(long)m * dim + (long)I * nv + k];
  }
};
struct SrcLvvRows {  // (k = c, j = (P,a)) = Lvv[P][a][c]
  static constexpr int MAP = RMAJOR;
  const double2* Lvv;
  int nv;
  __device__ double2 get(int k, int j, int) const { return Lvv[(long)j * nv + k]; }
};
struct EpXT {
  double2* XT;
  int nv, naux;
  __device__ void operator()(int i, int j, int, double2 v) const {
    const int P = j / nv, a = j - P * nv;
    XT[((long)i * nv + a) * naux + P] = cconj(v);
  }
};

// gvv[P][a][c] += 2 sum_{mI} Y[mI][P][a] conj(r1[m][I][c])
struct SrcYk {  // (k = mI, i = (P,a))
  static constexpr int MAP = KMAJOR;
  const double2* Y;
  long len;
  __device__ double2 get(int k, int i, int) const { return Y[(long)k * len + i]; }
};
struct SrcR1cK {  // (k = mI, j = c) = conj(r1[m][I][c])
  static constexpr int MAP = KMAJOR;
  const double2* x;
  long dim;
  int nc, nv;
  __device__ double2 get(int k, int j, int) const {
    const int m = k / nc, I = k - m * nc;
    return cconj(x[(long)m * dim + (long)I * nv + j]);
  }
};
struct EpAdd {  // C[i*ld + j] += alpha v
  double2* C;
  long ld;
  double alpha;
  __device__ void operator()(int i, int j, int, double2 v) const {
    double2* p = C + (long)i * ld + j;
    *p = cadd(*p, cscale(v, alpha));
  }
};

// T[I][j][K][a] = sum_{k,b} conj(R~_{kIj}[a][b]) r1[k][K][b],  batch b = I*no + j
// with R~_{kIj}[a][b] = Rt[(j*nv + b)*ld + (k*nc + I)*nv + a]
struct SrcRtc {  // (kk = (k, b), i = a)
  static constexpr int MAP = KMAJOR;
  const double2* Rt;
  long ld;
  int nc, nv, no;
  __device__ double2 get(int kk, int i, int bt) const {
    const int k = kk / nv, bv = kk - k * nv;
    const int I = bt / no, j = bt - I * no;
    return cconj(Rt[((long)j * nv + bv) * ld + ((long)k * nc + I) * nv + i]);
  }
};
struct SrcR1kb {  // (kk = (k, b), j = K) = r1[k][K][b]
  static constexpr int MAP = RMAJOR;
  const double2* x;
  long dim;
  int nv;
  __device__ double2 get(int kk, int K, int) const {
    const int k = kk / nv, bv = kk - k * nv;
    return x[(long)k * dim + (long)K * nv + bv];
  }
};
struct EpT {
  double2* T;
  int nc, nv;
  __device__ void operator()(int a, int K, int bt, double2 v) const { T[((long)bt * nc + K) * nv + a] = v; }
};

// Light coupling terms <Ka||Ij> = (KI|aj) - (Kj|aI) against T.
// (9a) hvo[nc+j][P][a] += 2 sum_{K,I} conj(T[I][j][K][a]) conj(Loo[P][K][I])      batch j
struct SrcLooKI {  // (k = (K,I), i = P)
  static constexpr int MAP = RMAJOR;
  const double2* Loo;
  int o, nc;
  __device__ double2 get(int k, int P, int) const {
    const int K = k / nc, I = k - K * nc;
    return cconj(Loo[((long)P * o + K) * o + I]);
  }
};
struct SrcTcKI {  // (k = (K,I), j = a; batch j) = conj(T[I][j][K][a])
  static constexpr int MAP = KMAJOR;
  const double2* T;
  int nc, no, nv;
  __device__ double2 get(int k, int a, int j) const {
    const int K = k / nc, I = k - K * nc;
    return cconj(T[(((long)I * no + j) * nc + K) * nv + a]);
  }
};
struct EpHvo {  // hvo[(g0 + b)][P][a] += alpha v   (i = P, j = a)
  double2* hvo;
  int g0, naux, nv;
  double alpha;
  __device__ void operator()(int P, int a, int b, double2 v) const {
    double2* p = hvo + ((long)(g0 + b) * naux + P) * nv + a;
    *p = cadd(*p, cscale(v, alpha));
  }
};
// (9b) hvo[I][P][a] += -2 sum_{K,j} conj(T[I][j][K][a]) conj(Loo[P][K][nc+j])      batch I
struct SrcLooKj {  // (k = (K,j), i = P)
  static constexpr int MAP = RMAJOR;
  const double2* Loo;
  int o, nc, no;
  __device__ double2 get(int k, int P, int) const {
    const int K = k / no, j = k - K * no;
    return cconj(Loo[((long)P * o + K) * o + nc + j]);
  }
};
struct SrcTcKj {  // (k = (K,j), j = a; batch I)
  static constexpr int MAP = KMAJOR;
  const double2* T;
  int nc, no, nv;
  __device__ double2 get(int k, int a, int I) const {
    const int K = k / no, j = k - K * no;
    return cconj(T[(((long)I * no + j) * nc + K) * nv + a]);
  }
};
// (9c) goo[P][K][I] += 2 sum_{j,a} conj(T[I][j][K][a]) conj(Lvo[nc+j][P][a])
struct SrcLvoc {  // (k = (g, a), i = P) = conj(Lvo[g0 + g][P][a])
  static constexpr int MAP = RMAJOR;
  const double2* Lvo;
  int g0, naux, nv;
  __device__ double2 get(int k, int P, int) const {
    const int g = k / nv, a = k - g * nv;
    return cconj(Lvo[((long)(g0 + g) * naux + P) * nv + a]);
  }
};
struct SrcTc_ja_KI {  // (k = (j,a), col = (K,I))
  static constexpr int MAP = RMAJOR;
  const double2* T;
  int nc, no, nv;
  __device__ double2 get(int k, int col, int) const {
    const int j = k / nv, a = k - j * nv;
    const int K = col / nc, I = col - K * nc;
    return cconj(T[(((long)I * no + j) * nc + K) * nv + a]);
  }
};
struct EpGooKI {  // goo[P][K][I] += alpha v   (col = (K,I))
  double2* goo;
  int o, nc;
  double alpha;
  __device__ void operator()(int P, int col, int, double2 v) const {
    const int K = col / nc, I = col - K * nc;
    double2* p = goo + ((long)P * o + K) * o + I;
    *p = cadd(*p, cscale(v, alpha));
  }
};
// (9d) goo[P][K][nc+j] += -2 sum_{I,a} conj(T[I][j][K][a]) conj(Lvo[I][P][a])
struct SrcTc_Ia_Kj {  // (k = (I,a), col = (K,j))
  static constexpr int MAP = RMAJOR;
  const double2* T;
  int nc, no, nv;
  __device__ double2 get(int k, int col, int) const {
    const int I = k / nv, a = k - I * nv;
    const int K = col / no, j = col - K * no;
    return cconj(T[(((long)I * no + j) * nc + K) * nv + a]);
  }
};
struct EpGooKj {  // goo[P][K][nc+j] += alpha v   (col = (K,j))
  double2* goo;
  int o, nc, no;
  double alpha;
  __device__ void operator()(int P, int col, int, double2 v) const {
    const int K = col / no, j = col - K * no;
    double2* p = goo + ((long)P * o + K) * o + nc + j;
    *p = cadd(*p, cscale(v, alpha));
  }
};

// First-order M11 = (aI|Jb) - (ab|JI).
// (10a) hvo[I][P][a] += 2 sum_{J,b} gamma[(J,b)][(I,a)] Lvo[J][P][b]
struct SrcLvo {  // (k = (J,b), i = P) = Lvo[J][P][b]
  static constexpr int MAP = RMAJOR;
  const double2* Lvo;
  int naux, nv;
  __device__ double2 get(int k, int P, int) const {
    const int J = k / nv, b = k - J * nv;
    return Lvo[((long)J * naux + P) * nv + b];
  }
};
struct SrcMatK {  // (k, j) = Mt[k*ld + j]
  static constexpr int MAP = KMAJOR;
  const double2* Mt;
  long ld;
  __device__ double2 get(int k, int j, int) const { return Mt[(long)k * ld + j]; }
};
struct EpHvoIa {  // hvo[I][P][a] += alpha v   (col = (I,a))
  double2* hvo;
  int naux, nv;
  double alpha;
  __device__ void operator()(int P, int col, int, double2 v) const {
    const int I = col / nv, a = col - I * nv;
    double2* p = hvo + ((long)I * naux + P) * nv + a;
    *p = cadd(*p, cscale(v, alpha));
  }
};
// (10b) gvv[P][a][b] -= sum_{I,J} gamma[(J,b)][(I,a)] Loo[P][I][J]
struct SrcLooIJ {  // (k = (I,J), i = P)
  static constexpr int MAP = RMAJOR;
  const double2* Loo;
  int o, nc;
  __device__ double2 get(int k, int P, int) const {
    const int I = k / nc, J = k - I * nc;
    return Loo[((long)P * o + I) * o + J];
  }
};
struct SrcGamIJ_ab {  // (k = (I,J), col = (a,b)) = gamma[(J,b)][(I,a)]
  static constexpr int MAP = KMAJOR;
  const double2* gam;
  int nc, nv;
  __device__ double2 get(int k, int col, int) const {
    const int I = k / nc, J = k - I * nc;
    const int a = col / nv, b = col - a * nv;
    const long ns = (long)nc * nv;
    return gam[((long)J * nv + b) * ns + (long)I * nv + a];
  }
};
// (10c) goo[P][J][I] -= sum_{b,a} gamma[(J,b)][(I,a)] Lvv[P][b][a]
struct SrcLvvFlat {  // (k = (b,a), i = P) = Lvv[P][b][a]
  static constexpr int MAP = RMAJOR;
  const double2* Lvv;
  long nv2;
  __device__ double2 get(int k, int P, int) const { return Lvv[(long)P * nv2 + k]; }
};
struct SrcGam_ba_JI {  // (k = (b,a), col = (J,I)) = gamma[(J,b)][(I,a)]
  static constexpr int MAP = RMAJOR;
  const double2* gam;
  int nc, nv;
  __device__ double2 get(int k, int col, int) const {
    const int b = k / nv, a = k - b * nv;
    const int J = col / nc, I = col - J * nc;
    const long ns = (long)nc * nv;
    return gam[((long)J * nv + b) * ns + (long)I * nv + a];
  }
};
struct EpGooJI {  // goo[P][J][I] += alpha v   (col = (J,I))
  double2* goo;
  int o, nc;
  double alpha;
  __device__ void operator()(int P, int col, int, double2 v) const {
    const int J = col / nc, I = col - J * nc;
    double2* p = goo + ((long)P * o + J) * o + I;
    *p = cadd(*p, cscale(v, alpha));
  }
};

// Second order.  pair index of k < l in the row-major enumeration of pairs
__device__ __forceinline__ long pair_id(int k, int l, int o) {
  return (long)k * (o - 1) - (long)k * (k - 1) / 2 + (l - k - 1);
}
// (12) PQ[g][b][c] = 1/4 sum_a Gamma[a][b] WT[g][a][c]   (g over W then W/D)
struct SrcGam4 {  // (k = a, i = b)
  static constexpr int MAP = KMAJOR;
  const double2* Gam;
  int nv;
  __device__ double2 get(int k, int i, int) const { return cscale(Gam[(long)k * nv + i], 0.25); }
};
struct SrcWT {  // (k = a, j = (g, c))
  static constexpr int MAP = KMAJOR;
  const double2* WT;
  int nv;
  __device__ double2 get(int k, int j, int) const {
    const int g = j / nv, c = j - g * nv;
    return WT[((long)g * nv + k) * nv + c];
  }
};
struct EpPQ {
  double2* PQ;
  int nv;
  __device__ void operator()(int b, int j, int, double2 v) const {
    const int g = j / nv, c = j - g * nv;
    PQ[((long)g * nv + b) * nv + c] = v;
  }
};
// (13) PQG[h][(J,b)][(k,c)] = sum_{(I,a)} Gc[(I,a)][(J,b)] X^h_{ac,Ik},
//      X^0 = W, X^1 = W / D, taken from the pair store with the sign of (I,k)
struct SrcWcore {  // (k = (I,a), j = (kk,c); batch h)
  static constexpr int MAP = KMAJOR;
  const double2* WT;
  long npairs;
  int nv, o;
  __device__ double2 get(int k, int j, int hh) const {
    const int I = k / nv, a = k - I * nv;
    const int kk = j / nv, c = j - kk * nv;
    if (kk == I) return czero();
    const bool lo = I < kk;
    const long p = lo ? pair_id(I, kk, o) : pair_id(kk, I, o);
    const double2 v = WT[(((long)hh * npairs + p) * nv + a) * nv + c];
    return lo ? v : cneg(v);
  }
};
struct EpPQG {
  double2* PQG;
  long ns, ldo;
  __device__ void operator()(int i, int j, int hh, double2 v) const { PQG[((long)hh * ns + i) * ldo + j] = v; }
};

// ---------------------------------------------------------------------------
// Elementwise kernels
// ---------------------------------------------------------------------------
// Gamma[a][b] = sum_I gamma[(I,a)][(I,b)],  Gamma'[I][J] = sum_a gamma[(I,a)][(J,a)]
__global__ void k_gamma_sums(const double2* __restrict__ gam, int nc, int nv, double2* __restrict__ Gam,
                             double2* __restrict__ Gp) {
  const long ns = (long)nc * nv;
  const long nv2 = (long)nv * nv;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nv2 + nc * nc; e += (long)gridDim.x * blockDim.x) {
    double2 acc = czero();
    if (e < nv2) {
      const int a = (int)(e / nv), b = (int)(e % nv);
      for (int I = 0; I < nc; ++I) acc = cadd(acc, gam[((long)I * nv + a) * ns + (long)I * nv + b]);
      Gam[e] = acc;
    } else {
      const int q = (int)(e - nv2);
      const int I = q / nc, J = q % nc;
      for (int a = 0; a < nv; ++a) acc = cadd(acc, gam[((long)I * nv + a) * ns + (long)J * nv + a]);
      Gp[q] = acc;
    }
  }
}

// Gc[(I,a)][(J,b)] = -1/2 gamma[(I,a)][(J,b)] + 1/4 delta_ab Gamma'[I][J]
__global__ void k_gc(const double2* __restrict__ gam, const double2* __restrict__ Gp, int nc, int nv,
                     double2* __restrict__ Gc) {
  const long ns = (long)nc * nv;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < ns * ns; e += (long)gridDim.x * blockDim.x) {
    const long r = e / ns, c = e % ns;
    const int I = (int)(r / nv), a = (int)(r % nv), J = (int)(c / nv), b = (int)(c % nv);
    double2 v = cscale(gam[e], -0.5);
    if (a == b) v = cadd(v, cscale(Gp[I * nc + J], 0.25));
    Gc[e] = v;
  }
}

__device__ __forceinline__ long pair_off(int a, int b, int nv) {
  return (long)a * nv - (long)a * (a + 1) / 2 + (b - a - 1);
}

// Rn[(mI,a)][(j,b)] = w_m R_{mIj}[a][b] (full antisymmetric form).  One
// workgroup per (g = mI*no + j, 32x32 tile pair ab <= bb).
constexpr int AT = 32;
__global__ __launch_bounds__(256) void k_unpack_rows(const double2* __restrict__ xin, long dim, int nc, int no,
                                                      int nv, const double* __restrict__ wts,
                                                      double2* __restrict__ Rn) {
  __shared__ double2 t[AT][AT + 1];
  const int nb = (nv + AT - 1) / AT;
  const int ntp = nb * (nb + 1) / 2;
  const long g = blockIdx.x / ntp;
  int tt = blockIdx.x % ntp, abk = 0;
  while (tt >= nb - abk) {
    tt -= nb - abk;
    ++abk;
  }
  const int bbk = abk + tt;
  const int a0 = abk * AT, b0 = bbk * AT;
  const int mI = (int)(g / no), j = (int)(g % no);
  const int mv = mI / nc, I = mI - mv * nc;
  const long ns = (long)nc * nv;
  const long npair = (long)nv * (nv - 1) / 2;
  const double2* r2 = xin + (long)mv * dim + ns + ((long)I * no + j) * npair;
  const double w = wts[mv];
  const long ldr = (long)no * nv;
  double2* R = Rn + (long)mI * nv * ldr + (long)j * nv;   // R[a*ldr + b]
  const int tid = threadIdx.x;
  for (int e = tid; e < AT * AT; e += 256) {
    const int ra = e / AT, cb = e % AT;
    const int a = a0 + ra, b = b0 + cb;
    double2 v = czero();
    if (a < nv && b < nv && a < b) v = cscale(r2[pair_off(a, b, nv)], w);
    t[ra][cb] = v;
  }
  __syncthreads();
  for (int e = tid; e < AT * AT; e += 256) {
    const int ra = e / AT, cb = e % AT;
    const int a = a0 + ra, b = b0 + cb;
    if (a < nv && b < nv) {
      double2 v;
      if (abk == bbk) v = (a < b) ? t[ra][cb] : (a > b ? cneg(t[cb][ra]) : czero());
      else v = t[ra][cb];
      R[(long)a * ldr + b] = v;
    }
  }
  if (abk != bbk) {
    for (int e = tid; e < AT * AT; e += 256) {
      const int rb = e / AT, ca = e % AT;
      const int b = b0 + rb, a = a0 + ca;
      if (a < nv && b < nv) R[(long)b * ldr + a] = cneg(t[ca][rb]);
    }
  }
}

// tau = W / D in the second half of WT; blockIdx.y = pair p = (k<l)
__global__ void k_tau(double2* __restrict__ WT, long npairs, const double* __restrict__ eps, int o, int nv) {
  const long nv2 = (long)nv * nv;
  const long p = blockIdx.y;
  int k = 0;
  long base = 0;
  while (base + (o - 1 - k) <= p) {
    base += o - 1 - k;
    ++k;
  }
  const int l = k + 1 + (int)(p - base);
  const double ekl = eps[k] + eps[l];
  const double2* W = WT + p * nv2;
  double2* tau = WT + (npairs + p) * nv2;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nv2; e += (long)gridDim.x * blockDim.x) {
    const int a = (int)(e / nv), c = (int)(e % nv);
    const double D = eps[o + a] + eps[o + c] - ekl;
    tau[e] = (a == c) ? czero() : cscale(W[e], 1.0 / D);
  }
}

// Antisymmetrised E for every occupied pair p = (k<l), written in both
// orders as Ef[k][l][c][a] = E^A_{ac,kl} = -Ef[l][k][c][a], and the per-pair
// denominator-derivative row sums hr[p][a] = sum_{c != a} (h(a,c) + h(c,a)).
// One workgroup per (p, 16-row block of a); 16x16 tiles through LDS so that
// both the (a,c) and the (c,a) reads are coalesced.
constexpr int ET = 16;
struct TilePair {
  double2 ac[ET][ET + 1];
  double2 ca[ET][ET + 1];
};
__device__ __forceinline__ void load_pair(TilePair& t, const double2* base, long rs, int a0, int c0, int nv,
                                          int tid) {
  const int r = tid / ET, q = tid % ET;
  const int a = a0 + r, c = c0 + q;
  t.ac[r][q] = (a < nv && c < nv) ? base[(long)a * rs + c] : czero();
  const int c2 = c0 + r, a2 = a0 + q;
  t.ca[r][q] = (a2 < nv && c2 < nv) ? base[(long)c2 * rs + a2] : czero();
}

__global__ __launch_bounds__(256) void k_efill(const double2* __restrict__ W, const double2* __restrict__ PQ,
                                                const double2* __restrict__ PQG, const double* __restrict__ eps,
                                                int nc, int o, int nv, long npairs, double2* __restrict__ Ef,
                                                double* __restrict__ hr) {
  __shared__ TilePair tw, tpi, tqi, tpk, tqk, tpl, tql;
  __shared__ double hs[ET][ET + 1];
  const int nab = (nv + ET - 1) / ET;
  const long p = blockIdx.x / nab;
  const int a0 = (int)(blockIdx.x % nab) * ET;
  int k = 0;
  long base = 0;
  while (base + (o - 1 - k) <= p) {
    base += o - 1 - k;
    ++k;
  }
  const int l = k + 1 + (int)(p - base);
  const bool kc = k < nc, lc = l < nc;
  const long nv2 = (long)nv * nv;
  const long ns = (long)nc * nv, ldo = (long)o * nv;
  const int tid = threadIdx.x;
  const int tx = tid % ET, ty = tid / ET;   // compute phase: a = a0 + tx, c = c0 + ty
  const int a = a0 + tx;
  const double ekl = eps[k] + eps[l];
  const double ea = a < nv ? eps[o + a] : 0.0;
  double hsum = 0.0;
  double2* Efkl = Ef + ((long)k * o + l) * nv2;
  double2* Eflk = Ef + ((long)l * o + k) * nv2;
  for (int c0 = 0; c0 < nv; c0 += ET) {
    __syncthreads();
    load_pair(tw, W + p * nv2, nv, a0, c0, nv, tid);
    load_pair(tpi, PQ + p * nv2, nv, a0, c0, nv, tid);
    load_pair(tqi, PQ + (npairs + p) * nv2, nv, a0, c0, nv, tid);
    if (kc) {
      load_pair(tpk, PQG + ((long)k * nv) * ldo + (long)l * nv, ldo, a0, c0, nv, tid);
      load_pair(tqk, PQG + (ns + (long)k * nv) * ldo + (long)l * nv, ldo, a0, c0, nv, tid);
    }
    if (lc) {
      load_pair(tpl, PQG + ((long)l * nv) * ldo + (long)k * nv, ldo, a0, c0, nv, tid);
      load_pair(tql, PQG + (ns + (long)l * nv) * ldo + (long)k * nv, ldo, a0, c0, nv, tid);
    }
    __syncthreads();
    const int c = c0 + ty;
    if (a < nv && c < nv) {
      double2 v = czero();
      if (a != c) {
        const double D = ea + eps[o + c] - ekl;
        const double iD = 1.0 / D, iD2 = iD * iD;
        const double2 w = tw.ac[tx][ty];
        // (i): A_ac[Q + P/D]
        const double2 pac = tpi.ac[tx][ty], pca = tpi.ca[ty][tx];
        const double2 Eac = cadd(tqi.ac[tx][ty], cscale(pac, iD));
        const double2 Eca = cadd(tqi.ca[ty][tx], cscale(pca, iD));
        v = cscale(csub(Eac, Eca), 0.5);
        // h(a,c) + h(c,a) with W_ca = -W_ac
        double hh = -4.0 * (w.x * pac.x + w.y * pac.y) + 4.0 * (w.x * pca.x + w.y * pca.y);
        if (kc) {
          const double2 gac = tpk.ac[tx][ty], gca = tpk.ca[ty][tx];
          const double2 Fac = cadd(tqk.ac[tx][ty], cscale(gac, iD));
          const double2 Fca = cadd(tqk.ca[ty][tx], cscale(gca, iD));
          v = cadd(v, cscale(csub(Fac, Fca), 0.25));
          hh += -2.0 * (w.x * gac.x + w.y * gac.y) + 2.0 * (w.x * gca.x + w.y * gca.y);
        }
        if (lc) {
          const double2 gac = tpl.ac[tx][ty], gca = tpl.ca[ty][tx];
          const double2 Fac = cadd(tql.ac[tx][ty], cscale(gac, iD));
          const double2 Fca = cadd(tql.ca[ty][tx], cscale(gca, iD));
          v = csub(v, cscale(csub(Fac, Fca), 0.25));
          hh += 2.0 * (w.x * gac.x + w.y * gac.y) - 2.0 * (w.x * gca.x + w.y * gca.y);
        }
        hsum += hh * iD2;
      }
      Efkl[(long)c * nv + a] = v;
      Eflk[(long)c * nv + a] = cneg(v);
    }
  }
  hs[ty][tx] = hsum;
  __syncthreads();
  if (ty == 0 && a < nv) {
    double s = 0.0;
    for (int r = 0; r < ET; ++r) s += hs[r][tx];
    hr[p * nv + a] = s;
  }
}

// Ef[k][k] = 0
__global__ void k_zero_diag_blocks(double2* __restrict__ Ef, int o, int nv) {
  const long nv2 = (long)nv * nv;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)o * nv2; e += (long)gridDim.x * blockDim.x) {
    const long k = e / nv2;
    Ef[(k * o + k) * nv2 + e % nv2] = czero();
  }
}

// Doubles diagonal: rho_{Ijab} = sum_k w_k |r2_{k,Ijab}|^2 (a<b).  One
// workgroup per (I, j): Sv[(I,j)][a] = sum_b rho over pairs containing a,
// Sv[(I,j)][nv] = sum of rho over the block.
__global__ __launch_bounds__(256) void k_rho(const double2* __restrict__ xin, long dim, int m, int nc, int no,
                                              int nv, const double* __restrict__ wts, double* __restrict__ Sv) {
  extern __shared__ double sm[];
  __shared__ double red4[4];
  double* col = sm;            // [nv]  sums over a of rho(a, b) for column b
  double* row = sm + nv;       // [nv][4] per-wave row sums
  const int g = blockIdx.x;    // I*no + j
  const int I = g / no, j = g % no;
  const long ns = (long)nc * nv;
  const long npair = (long)nv * (nv - 1) / 2;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int b = tid; b < nv; b += 256) col[b] = 0.0;
  for (int e = tid; e < 4 * nv; e += 256) row[e] = 0.0;
  __syncthreads();
  for (int mv = 0; mv < m; ++mv) {
    const double2* r2 = xin + (long)mv * dim + ns + ((long)I * no + j) * npair;
    const double w = wts[mv];
    for (int a = 0; a < nv - 1; ++a) {
      double rs = 0.0;
      for (int b = tid; b < nv; b += 256) {
        if (b > a) {
          const double2 v = r2[pair_off(a, b, nv)];
          const double q = w * (v.x * v.x + v.y * v.y);
          col[b] += q;   // b is owned by this thread
          rs += q;
        }
      }
      for (int off = 32; off > 0; off >>= 1) rs += __shfl_xor(rs, off);
      if (lane == 0) row[a * 4 + wv] += rs;
    }
  }
  __syncthreads();
  double tot = 0.0;
  for (int a = tid; a < nv; a += 256) {
    const double r = row[a * 4] + row[a * 4 + 1] + row[a * 4 + 2] + row[a * 4 + 3];
    Sv[(long)g * (nv + 1) + a] = r + col[a];
    tot += r;
  }
  // block sum of tot
  for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
  __syncthreads();
  if (lane == 0) red4[wv] = tot;
  __syncthreads();
  if (tid == 0) Sv[(long)g * (nv + 1) + nv] = red4[0] + red4[1] + red4[2] + red4[3];
}

// d eps, one thread per spinor.
__global__ void k_eps_final(const double2* __restrict__ gam, const double* __restrict__ Sv,
                            const double* __restrict__ hr, int nc, int no, int nv, double* __restrict__ deps) {
  const int o = nc + no, n = o + nv;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const long ns = (long)nc * nv;
  double v = 0.0;
  if (q >= o) {
    const int a = q - o;
    for (int I = 0; I < nc; ++I) v += gam[((long)I * nv + a) * ns + (long)I * nv + a].x;
    for (int g = 0; g < nc * no; ++g) v += Sv[(long)g * (nv + 1) + a];
    const long npairs = (long)o * (o - 1) / 2;
    for (long p = 0; p < npairs; ++p) v += hr[p * nv + a];
  } else {
    if (q < nc) {
      for (int a = 0; a < nv; ++a) v -= gam[((long)q * nv + a) * ns + (long)q * nv + a].x;
      for (int j = 0; j < no; ++j) v -= Sv[((long)q * no + j) * (nv + 1) + nv];
    } else {
      const int j = q - nc;
      for (int I = 0; I < nc; ++I) v -= Sv[((long)I * no + j) * (nv + 1) + nv];
    }
    double hp = 0.0;
    for (int l = 0; l < o; ++l) {
      if (l == q) continue;
      const long p = q < l ? pair_id(q, l, o) : pair_id(l, q, o);
      for (int a = 0; a < nv; ++a) hp += hr[p * nv + a];
    }
    v -= 0.5 * hp;
  }
  deps[q] = v;
}

// dL[P][p][q] = 1/2 (g[p][q] + conj(g[q][p])) with g assembled from the blocks
//   g = gvv (virtual, virtual), goo (occupied, occupied),
//       hvo[k][P][a] at (o+a, k) and 0 at (k, o+a).
__device__ __forceinline__ double2 graw(const double2* gvv, const double2* goo, const double2* hvo, int P, int p,
                                        int q, int o, int nv, int naux) {
  if (p >= o && q >= o) return gvv[((long)P * nv + (p - o)) * nv + (q - o)];
  if (p < o && q < o) return goo[((long)P * o + p) * o + q];
  if (p >= o) return hvo[((long)q * naux + P) * nv + (p - o)];
  return czero();
}

constexpr int DT = 32;
__global__ __launch_bounds__(256) void k_dl_assemble(const double2* __restrict__ gvv, const double2* __restrict__ goo,
                                                      const double2* __restrict__ hvo, int o, int nv, int naux,
                                                      double2* __restrict__ dL) {
  __shared__ double2 tB[DT][DT + 1];
  const int n = o + nv;
  const int nt = (n + DT - 1) / DT;
  const int tile = blockIdx.x, P = blockIdx.y;
  const int pb = tile / nt, qb = tile % nt;
  const int tid = threadIdx.x;
  // mirror tile: tB[r][c] = g[qb*DT + r][pb*DT + c]
  for (int e = tid; e < DT * DT; e += 256) {
    const int r = e / DT, c = e % DT;
    const int p = qb * DT + r, q = pb * DT + c;
    tB[r][c] = (p < n && q < n) ? graw(gvv, goo, hvo, P, p, q, o, nv, naux) : czero();
  }
  __syncthreads();
  double2* out = dL + (long)P * n * n;
  for (int e = tid; e < DT * DT; e += 256) {
    const int r = e / DT, c = e % DT;
    const int p = pb * DT + r, q = qb * DT + c;
    if (p < n && q < n) {
      const double2 a = graw(gvv, goo, hvo, P, p, q, o, nv, naux);
      const double2 b = tB[c][r];   // g[q][p]
      out[(long)p * n + q] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    }
  }
}

// per-vector norms |x_k|^2 (one workgroup per vector)
__global__ __launch_bounds__(256) void k_vnorm2(const double2* __restrict__ x, long dim, double* __restrict__ out) {
  __shared__ double red[256];
  const double2* v = x + (long)blockIdx.x * dim;
  double s = 0.0;
  for (long e = threadIdx.x; e < dim; e += 256) s += v[e].x * v[e].x + v[e].y * v[e].y;
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// Driver
// ---------------------------------------------------------------------------
adc2_status omega_backward(adc2_handle h, int m, const double2* X, const double* g, double2* dL, double* deps,
                           hipStream_t st) {
  const Dims& d = h->d;
  const int nc = d.nc, no = d.no, nv = d.nv, naux = d.naux, o = d.o;
  const long ns = d.ns, dim = d.dim, nv2 = (long)nv * nv;
  const long npairs = (long)o * (o - 1) / 2;
  if (npairs > 65535 || (long)nc * no > 65535) {
    set_error("adc2_omega_backward: more than 65535 occupied pairs or core-valence pairs");
    return ADC2_ERR_ARG;
  }
  adc2_status rc = ensure_ws(h, m);
  if (rc != ADC2_OK) return rc;

  std::vector<void*> owned;
  auto release = [&]() {
    for (void* p : owned) dfree(h, p);
    owned.clear();
  };
  auto alloc = [&](void** p, size_t bytes) -> adc2_status {
    *p = nullptr;
    hipError_t e = dmalloc(h, p, std::max<size_t>(bytes, 16));
    if (e != hipSuccess) {
      set_error(std::string("adc2_omega_backward: hipMalloc: ") + hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? ADC2_ERR_OOM : ADC2_ERR_HIP;
    }
    owned.push_back(*p);
    return ADC2_OK;
  };
#define BW_TRY(expr)            \
  do {                          \
    adc2_status r_ = (expr);    \
    if (r_ != ADC2_OK) {        \
      hipStreamSynchronize(st); \
      release();                \
      return r_;                \
    }                           \
  } while (0)
#define BW_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      set_error(std::string("adc2_omega_backward: ") + #call + ": " + hipGetErrorString(e_)); \
      hipStreamSynchronize(st);                                                       \
      release();                                                                      \
      return e_ == hipErrorOutOfMemory ? ADC2_ERR_OOM : ADC2_ERR_HIP;                 \
    }                                                                                 \
  } while (0)

  // weights w_k = g_k / |x_k|^2
  double *wts = nullptr, *nrm = nullptr;
  BW_TRY(alloc((void**)&wts, sizeof(double) * m));
  BW_TRY(alloc((void**)&nrm, sizeof(double) * m));
  k_vnorm2<<<m, 256, 0, st>>>(X, dim, nrm);
  BW_HIP(hipGetLastError());
  std::vector<double> hn(m), hw(m);
  BW_HIP(hipMemcpyAsync(hn.data(), nrm, sizeof(double) * m, hipMemcpyDeviceToHost, st));
  BW_HIP(hipStreamSynchronize(st));
  for (int k = 0; k < m; ++k) {
    if (!(hn[k] > 0.0) || !std::isfinite(hn[k])) {
      release();
      set_error("adc2_omega_backward: a vector has zero or non-finite norm");
      return ADC2_ERR_ARG;
    }
    hw[k] = g[k] / hn[k];
  }
  BW_HIP(hipMemcpyAsync(wts, hw.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));

  // accumulators and small matrices
  double2 *hvo, *gvv, *goo, *gam, *Gam, *Gp, *Gc, *T, *scr;
  const long scr_n = std::max<long>(1L << 16, std::min<long>(16L << 20, 64L * naux * std::max<long>(nc * no, nc * nc)));
  BW_TRY(alloc((void**)&hvo, sizeof(double2) * o * naux * nv));
  BW_TRY(alloc((void**)&gvv, sizeof(double2) * naux * nv2));
  BW_TRY(alloc((void**)&goo, sizeof(double2) * naux * o * o));
  BW_TRY(alloc((void**)&gam, sizeof(double2) * ns * ns));
  BW_TRY(alloc((void**)&Gam, sizeof(double2) * nv2));
  BW_TRY(alloc((void**)&Gp, sizeof(double2) * nc * nc));
  BW_TRY(alloc((void**)&Gc, sizeof(double2) * ns * ns));
  BW_TRY(alloc((void**)&T, sizeof(double2) * nc * no * nc * nv));
  BW_TRY(alloc((void**)&scr, sizeof(double2) * scr_n));
  const Scratch S{scr, scr_n};
  BW_HIP(hipMemsetAsync(hvo, 0, sizeof(double2) * o * naux * nv, st));
  BW_HIP(hipMemsetAsync(gvv, 0, sizeof(double2) * naux * nv2, st));
  BW_HIP(hipMemsetAsync(goo, 0, sizeof(double2) * naux * o * o, st));

  // gamma and its contractions
  BW_TRY(fgemm((int)ns, (int)ns, m, 1, SrcWr1c{X, dim, wts}, SrcR1{X, dim}, EpStore{gam, ns}, S, st));
  k_gamma_sums<<<grid1(nv2 + nc * nc), 256, 0, st>>>(gam, nc, nv, Gam, Gp);
  BW_HIP(hipGetLastError());
  k_gc<<<grid1(ns * ns), 256, 0, st>>>(gam, Gp, nc, nv, Gc);
  BW_HIP(hipGetLastError());

  // ---- first-order singles block ----
  BW_TRY(fgemm(naux, (int)ns, (int)ns, 1, SrcLvo{h->Lvo, naux, nv}, SrcMatK{gam, ns}, EpHvoIa{hvo, naux, nv, 2.0},
               S, st));
  BW_TRY(fgemm(naux, (int)nv2, nc * nc, 1, SrcLooIJ{h->Loo, o, nc}, SrcGamIJ_ab{gam, nc, nv},
               EpAdd{gvv, nv2, -1.0}, S, st));
  BW_TRY(fgemm(naux, nc * nc, (int)nv2, 1, SrcLvvFlat{h->Lvv, nv2}, SrcGam_ba_JI{gam, nc, nv},
               EpGooJI{goo, o, nc, -1.0}, S, st));

  // ---- coupling ----
  // weighted unpacks, Y-build
  BW_TRY(unpack_weighted(h, m, X, wts, st));
  BW_TRY(ybuild_fp64(h, m, st));
  const long ldrt = (long)m * nc * nv;
  // T[I][j][K][a]
  BW_TRY(fgemm(nv, nc, m * nv, nc * no, SrcRtc{h->Zb, ldrt, nc, nv, no}, SrcR1kb{X, dim, nv}, EpT{T, nc, nv}, S,
               st));
  // gvv += 2 Y conj(r1)
  BW_TRY(fgemm((int)((long)naux * nv), nv, m * nc, 1, SrcYk{h->Y, (long)naux * nv}, SrcR1cK{X, dim, nc, nv},
               EpAdd{gvv, nv, 2.0}, S, st));
  // light coupling terms
  BW_TRY(fgemm(naux, nv, nc * nc, no, SrcLooKI{h->Loo, o, nc}, SrcTcKI{T, nc, no, nv},
               EpHvo{hvo, nc, naux, nv, 2.0}, S, st));
  BW_TRY(fgemm(naux, nv, nc * no, nc, SrcLooKj{h->Loo, o, nc, no}, SrcTcKj{T, nc, no, nv},
               EpHvo{hvo, 0, naux, nv, -2.0}, S, st));
  BW_TRY(fgemm(naux, nc * nc, no * nv, 1, SrcLvoc{h->Lvo, nc, naux, nv}, SrcTc_ja_KI{T, nc, no, nv},
               EpGooKI{goo, o, nc, 2.0}, S, st));
  BW_TRY(fgemm(naux, nc * no, (int)ns, 1, SrcLvoc{h->Lvo, 0, naux, nv}, SrcTc_Ia_Kj{T, nc, no, nv},
               EpGooKj{goo, o, nc, no, -2.0}, S, st));
  // X^T (conjugated) into the sigma X workspace, Rn, then the heavy GEMM
  //   hvo[nc+j][P][b] += 2 sum_{(mI,a)} conj(X^P_{mI,a}) R~_{mIj}[a][b]
  {
    double2* XT = h->X;
    BW_TRY(fgemm(m * nc, (int)((long)naux * nv), nv, 1, SrcR1rows{X, dim, nc, nv}, SrcLvvRows{h->Lvv, nv},
                 EpXT{XT, nv, naux}, S, st));
    double2 *Rn = nullptr, *C = nullptr;
    const long K = (long)m * nc * nv;
    BW_TRY(alloc((void**)&Rn, sizeof(double2) * K * no * nv));
    const int nb = cdv(nv, AT);
    k_unpack_rows<<<(unsigned)((long)m * nc * no * (nb * (nb + 1) / 2)), 256, 0, st>>>(X, dim, nc, no, nv, wts, Rn);
    BW_HIP(hipGetLastError());
    const int M = naux, N = no * nv;
    const long tiles = (long)cdv(M, BT) * cdv(N, BT);
    const int nsplit = (int)std::max<long>(1, std::min<long>(8, (512 + tiles - 1) / tiles));
    BW_TRY(alloc((void**)&C, sizeof(double2) * nsplit * (long)M * N));
    SrcGroupedK<8> A{XT, 0, naux, naux, naux, (int)K};
    SrcGroupedK<8> B{Rn, 0, (long)N, N, N, (int)K};
    k_bgemm<<<dim3((unsigned)tiles, nsplit), 256, 0, st>>>(A, B, M, N, (int)K, C);
    BW_HIP(hipGetLastError());
    k_scatter_add<<<grid1((long)M * N), 256, 0, st>>>(C, nsplit, M, N, nv, (long)naux * nv, nv, 2.0,
                                                      hvo + (long)nc * naux * nv);
    BW_HIP(hipGetLastError());
    BW_HIP(hipStreamSynchronize(st));
    dfree(h, Rn);
    dfree(h, C);
    owned.erase(std::remove(owned.begin(), owned.end(), (void*)Rn), owned.end());
    owned.erase(std::remove(owned.begin(), owned.end(), (void*)C), owned.end());
  }

  // ---- second order (W) ----
  {
    double2 *WT, *PQ, *PQG, *Ef, *C;
    double *hr, *Sv;
    BW_TRY(alloc((void**)&WT, sizeof(double2) * 2 * npairs * nv2));
    BW_TRY(alloc((void**)&PQ, sizeof(double2) * 2 * npairs * nv2));
    BW_TRY(alloc((void**)&PQG, sizeof(double2) * 2 * ns * o * nv));
    BW_TRY(alloc((void**)&hr, sizeof(double) * npairs * nv));
    BW_TRY(alloc((void**)&Sv, sizeof(double) * nc * no * (nv + 1)));
    BW_TRY(wbuild(h, WT, st));
    k_tau<<<dim3(grid1(nv2, 256, 64), (unsigned)npairs), 256, 0, st>>>(WT, npairs, h->eps, o, nv);
    BW_HIP(hipGetLastError());
    BW_TRY(fgemm(nv, (int)(2 * npairs * nv), nv, 1, SrcGam4{Gam, nv}, SrcWT{WT, nv}, EpPQ{PQ, nv}, S, st));
    BW_TRY(fgemm((int)ns, o * nv, (int)ns, 2, SrcMatK{Gc, ns}, SrcWcore{WT, npairs, nv, o},
                 EpPQG{PQG, ns, (long)o * nv}, S, st));
    BW_TRY(alloc((void**)&Ef, sizeof(double2) * (long)o * o * nv2));
    k_zero_diag_blocks<<<grid1((long)o * nv2), 256, 0, st>>>(Ef, o, nv);
    BW_HIP(hipGetLastError());
    k_efill<<<(unsigned)(npairs * cdv(nv, ET)), 256, 0, st>>>(WT, PQ, PQG, h->eps, nc, o, nv, npairs, Ef, hr);
    BW_HIP(hipGetLastError());
    BW_HIP(hipStreamSynchronize(st));
    dfree(h, WT);
    dfree(h, PQ);
    owned.erase(std::remove(owned.begin(), owned.end(), (void*)WT), owned.end());
    owned.erase(std::remove(owned.begin(), owned.end(), (void*)PQ), owned.end());
    // hvo[k][P][a] += 8 sum_{(l,c)} LoT[(l,c)][P] Ef[k][l][c][a]
    const int M = naux, N = o * nv, K = o * nv;
    const long tiles = (long)cdv(M, BT) * cdv(N, BT);
    const int nsplit = (int)std::max<long>(1, std::min<long>(8, (512 + tiles - 1) / tiles));
    BW_TRY(alloc((void**)&C, sizeof(double2) * nsplit * (long)M * N));
    SrcGroupedK<8> A{h->LoT, 0, naux, naux, naux, K};
    SrcGroupedK<8> B{Ef, (long)o * nv2, nv, nv, N, K};
    k_bgemm<<<dim3((unsigned)tiles, nsplit), 256, 0, st>>>(A, B, M, N, K, C);
    BW_HIP(hipGetLastError());
    k_scatter_add<<<grid1((long)M * N), 256, 0, st>>>(C, nsplit, M, N, nv, (long)naux * nv, nv, 8.0, hvo);
    BW_HIP(hipGetLastError());
    // eps
    k_rho<<<nc * no, 256, sizeof(double) * 5 * nv, st>>>(X, dim, m, nc, no, nv, wts, Sv);
    BW_HIP(hipGetLastError());
    k_eps_final<<<cdv(d.n, 128), 128, 0, st>>>(gam, Sv, hr, nc, no, nv, deps);
    BW_HIP(hipGetLastError());
  }

  // ---- Hermitian projection into dL ----
  {
    const int nt = cdv(d.n, DT);
    k_dl_assemble<<<dim3((unsigned)(nt * nt), naux), 256, 0, st>>>(gvv, goo, hvo, o, nv, naux, dL);
    BW_HIP(hipGetLastError());
  }
  BW_HIP(hipStreamSynchronize(st));
  release();
#undef BW_TRY
#undef BW_HIP
  return ADC2_OK;
}

}  // namespace adc2
