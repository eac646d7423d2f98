// adc2x.hip -- the extended scheme ADC(2)-x: the first-order doubles-doubles
// block of the intermediate-state matrix (the truncation of Eq. 12 carried one
// order further on the doubles; named in the Conclusions as the next step).
//
// With the doubles |Ijab> = a+_a a+_b a_j a_I |Phi0> (I core, j valence,
// a<b) and R^{cd}_{Kk} the full-index amplitudes (antisymmetric in c, d) of a
// vector's doubles, the block adds to sigma2
//   sum_{c<d} <ab||cd> r^{cd}_{Ij}                                (particle ladder)
// + sum_{K,k} <Kk||Ij> r^{ab}_{Kk}                                 (hole ladder)
// + P(ab) [ sum_{k,c} <kb||cj> R^{ac}_{Ik} + sum_{K,c} <Kb||cI> R^{ac}_{Kj} ]   (rings)
// with P(ab) f = f - f(a<->b), k valence and K core in the rings (the two
// hole pairs the core-valence separation leaves).
//
// The four integral blocks (the particle ladder's with four virtual
// indices) are formed once per handle when the method is selected and kept
// in HBM, in layouts that make each term one GEMM on the doubles of the
// vectors:
//   Vpp [(a<b)][(c<d)] = <ab||cd>       from blocks of (ac|bd) = sum_P L^P_ac L^P_bd
//                                        (FP64 MFMA, a few a-values per block)
//   Hh  [(I,j)][(K,k)] = <Kk||Ij>        from the occupied Cholesky block
//   WvT [(j,b)][(k,c)] = <kb||cj>        (k, j valence)
//   WcT [(I,b)][(K,c)] = <Kb||cI>        (K, I core)
// npair^2 complex values for Vpp (32 GB at nv = 300); the rings no^2 nv^2 and
// nc^2 nv^2.  The contractions run in FP64 whatever the handle's precision.
#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "internal.h"
#include "tile.h"

namespace adc2 {

namespace {

__host__ __device__ inline long cdl(long a, long b) { return (a + b - 1) / b; }
inline unsigned grid1(long n, long per = 256, long cap = 16384) {
  return (unsigned)std::max<long>(1, std::min<long>((n + per - 1) / per, cap));
}
__device__ __forceinline__ long pair_q(int a, int b, int nv) {   // a < b
  return (long)a * nv - (long)a * (a + 1) / 2 + (b - a - 1);
}

// Vpp rows of the a-values [a0, a0 + na): V holds (ac|bd) at [(a - a0, c)][(b, d)].
__global__ void k_vpp_rows(const double2* __restrict__ V, int a0, int na, int nv, long npair,
                           double2* __restrict__ Vpp) {
  const long nv2 = (long)nv * nv;
  const long total = (long)na * nv * npair;       // (a local, b, q') with b > a checked inside
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long qp = e % npair;
    const long ab = e / npair;
    const int b = (int)(ab % nv), al = (int)(ab / nv);
    const int a = a0 + al;
    if (b <= a) continue;
    // q' = (c < d): invert the row-major strict upper triangle
    int c = 0;
    {
      long rem = qp;
      while (rem >= nv - 1 - c) {
        rem -= nv - 1 - c;
        ++c;
      }
      const int d = c + 1 + (int)rem;
      const double2 acbd = V[((long)al * nv + c) * nv2 + (long)b * nv + d];
      const double2 adbc = V[((long)al * nv + d) * nv2 + (long)b * nv + c];
      Vpp[pair_q(a, b, nv) * npair + qp] = make_double2(acbd.x - adbc.x, acbd.y - adbc.y);
    }
  }
}

// Hh[(I,j)][(K,k)] = <Kk||Ij> = (KI|kj) - (Kj|kI), Loo [P][o][o] = L^P_pq.
__global__ void k_hole_ladder_ints(const double2* __restrict__ Loo, int naux, int o, int nc, int no,
                                   double2* __restrict__ Hh) {
  const long n2 = (long)nc * no;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n2 * n2; e += (long)gridDim.x * blockDim.x) {
    const long r = e / n2, cidx = e % n2;
    const int I = (int)(r / no), j = nc + (int)(r % no);
    const int K = (int)(cidx / no), k = nc + (int)(cidx % no);
    double2 s = czero();
    for (int P = 0; P < naux; ++P) {
      const double2* Lp = Loo + (long)P * o * o;
      s = cadd(s, csub(cmul(Lp[K * o + I], Lp[k * o + j]), cmul(Lp[K * o + j], Lp[k * o + I])));
    }
    Hh[e] = s;
  }
}

// W[(j,b)][(k,c)] -= G[(k,j)][(b,c)] over the hole block of size nh (the
// exchange part (kj|bc) of the ring integrals, permuted into place).
__global__ void k_ring_exchange(const double2* __restrict__ G, int nh, int nv, double2* __restrict__ W) {
  const long n = (long)nh * nv;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n * n; e += (long)gridDim.x * blockDim.x) {
    const long r = e / n, cc = e % n;
    const int j = (int)(r / nv), b = (int)(r % nv), k = (int)(cc / nv), c = (int)(cc % nv);
    const double2 g = G[((long)k * nh + j) * nv * nv + (long)b * nv + c];
    W[e] = csub(W[e], g);
  }
}

// Unpacked full-index doubles of m vectors (x [m][dim], doubles packed after
// ns singles) in two layouts:
//   Ru[(m, I, a)][(k, c)] = R^{ac}_{Ik}     (k valence)
//   Rc[(m, j, a)][(K, c)] = R^{ac}_{Kj}     (K core)
// R^{ac} = r^{ac} for a < c, -r^{ca} for a > c, 0 on the diagonal.
__global__ void k_x_unpack(const double2* __restrict__ x, long dim, long ns, int m, int nc, int no, int nv,
                           long npair, double2* __restrict__ Ru, double2* __restrict__ Rc) {
  const long per = (long)nc * no * nv * nv;
  const long total = (long)m * per;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int mv = (int)(e / per);
    long r = e % per;
    const int c = (int)(r % nv);
    r /= nv;
    const int a = (int)(r % nv);
    r /= nv;
    const int k = (int)(r % no);
    const int I = (int)(r / no);
    double2 v = czero();
    if (a != c) {
      const int lo = a < c ? a : c, hi = a < c ? c : a;
      v = x[(long)mv * dim + ns + ((long)I * no + k) * npair + pair_q(lo, hi, nv)];
      if (a > c) v = cneg(v);
    }
    Ru[((((long)mv * nc + I) * nv + a) * no + k) * nv + c] = v;
    Rc[((((long)mv * no + k) * nv + a) * nc + I) * nv + c] = v;
  }
}

// sigma2 += Gv[(m,I,a)][(j,b)] - Gv[(m,I,b)][(j,a)] + Gc[(m,j,a)][(I,b)] - Gc[(m,j,b)][(I,a)]  (a < b)
__global__ void k_x_ring_pack(const double2* __restrict__ Gv, const double2* __restrict__ Gc, long dim, long ns,
                              int m, int nc, int no, int nv, long npair, double2* __restrict__ s) {
  const long per = (long)nc * no * npair;
  const long total = (long)m * per;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int mv = (int)(e / per);
    const long r = e % per;
    const long q = r % npair;
    const int j = (int)((r / npair) % no), I = (int)(r / npair / no);
    int a = 0;
    long rem = q;
    while (rem >= nv - 1 - a) {
      rem -= nv - 1 - a;
      ++a;
    }
    const int b = a + 1 + (int)rem;
    const long gv = (long)no * nv, gc = (long)nc * nv;
    const double2 t1 = Gv[(((long)mv * nc + I) * nv + a) * gv + (long)j * nv + b];
    const double2 t2 = Gv[(((long)mv * nc + I) * nv + b) * gv + (long)j * nv + a];
    const double2 t3 = Gc[(((long)mv * no + j) * nv + a) * gc + (long)I * nv + b];
    const double2 t4 = Gc[(((long)mv * no + j) * nv + b) * gc + (long)I * nv + a];
    double2* p = s + (long)mv * dim + ns + r;
    *p = cadd(*p, cadd(csub(t1, t2), csub(t3, t4)));
  }
}

// C[i][j] += sum_k A[i*lda + k] B[k*ldb + j]   (A row-major, B K-major), one vector's block
__global__ __launch_bounds__(256) void k_gemm_rk_acc(int M, int N, int K, const double2* __restrict__ A, long lda,
                                                      const double2* __restrict__ B, long ldb,
                                                      double2* __restrict__ C, long ldc) {
  __shared__ TileSmem s;
  const int nbj = (int)cdl(N, TN);
  const int i0 = (blockIdx.x / nbj) * TM, j0 = (blockIdx.x % nbj) * TN;
  SrcR<false> sa{A + (long)i0 * lda, lda, K, M - i0, 1.0};
  SrcK<false> sb{B + j0, ldb, K, N - j0, 1.0};
  Acc acc;
  acc.zero();
  mainloop(s, sa, sb, 0, (int)cdl(K, TK), acc);
  for_each_acc(acc, [&](int r, int c, double2 v) {
    const int i = i0 + r, j = j0 + c;
    if (i < M && j < N) {
      double2* p = C + (long)i * ldc + j;
      *p = cadd(*p, v);
    }
  });
}

// diagonal of the first-order doubles block, added to the ADC(2) diagonal:
// <ab||ab> + <Ij||Ij> + <jb||bj> + <ja||aj> + <Ib||bI> + <Ia||aI>
__global__ void k_x_diag(const double* __restrict__ d0, const double2* __restrict__ Vpp,
                         const double2* __restrict__ Hh, const double2* __restrict__ WvT,
                         const double2* __restrict__ WcT, long ns, int nc, int no, int nv, long npair,
                         double* __restrict__ dx) {
  const long nd = (long)nc * no * npair;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < ns + nd; e += (long)gridDim.x * blockDim.x) {
    if (e < ns) {
      dx[e] = d0[e];
      continue;
    }
    const long r = e - ns;
    const long q = r % npair;
    const int j = (int)((r / npair) % no), I = (int)(r / npair / no);
    int a = 0;
    long rem = q;
    while (rem >= nv - 1 - a) {
      rem -= nv - 1 - a;
      ++a;
    }
    const int b = a + 1 + (int)rem;
    const long nvv = (long)no * nv, ncv = (long)nc * nv;
    const long ij = (long)I * no + j;
    double v = d0[e] + Vpp[q * npair + q].x + Hh[ij * (nc * no) + ij].x;
    v += WvT[((long)j * nv + b) * nvv + (long)j * nv + b].x + WvT[((long)j * nv + a) * nvv + (long)j * nv + a].x;
    v += WcT[((long)I * nv + b) * ncv + (long)I * nv + b].x + WcT[((long)I * nv + a) * ncv + (long)I * nv + a].x;
    dx[e] = v;
  }
}

}  // namespace

// Bytes of the ADC(2)-x integral blocks of a handle.
static size_t adc2x_bytes(const Dims& d) {
  return sizeof(double2) * ((size_t)d.npair * d.npair + (size_t)d.nc * d.no * d.nc * d.no +
                            (size_t)d.no * d.nv * d.no * d.nv + (size_t)d.nc * d.nv * d.nc * d.nv);
}

adc2_status build_adc2x(adc2_handle h, hipStream_t st) {
  if (h->Vpp) return ADC2_OK;
  const Dims& d = h->d;
  const int nc = d.nc, no = d.no, nv = d.nv, naux = d.naux, o = d.o;
  const long nv2 = (long)nv * nv, npair = d.npair;
  const size_t need = adc2x_bytes(d);
  if (need > ADC2X_MAX_BYTES) {
    char buf[240];
    snprintf(buf, sizeof buf,
             "adc2_set_method: the ADC(2)-x integral blocks need %.1f GB (the <ab||cd> block grows as nv^4), above "
             "the %.0f GB limit",
             need / 1e9, ADC2X_MAX_BYTES / 1e9);
    set_error(buf);
    return ADC2_ERR_OOM;
  }
  std::vector<void*> tmp;
  auto release_tmp = [&]() {
    hipStreamSynchronize(st);
    for (void* p : tmp) dfree(h, p);
    tmp.clear();
  };
  auto fail_all = [&](adc2_status r) {
    release_tmp();
    dfree(h, h->Vpp);
    dfree(h, h->Hh);
    dfree(h, h->WvT);
    dfree(h, h->WcT);
    dfree(h, h->diagx);
    h->Vpp = h->Hh = h->WvT = h->WcT = nullptr;
    h->diagx = nullptr;
    return r;
  };
#define X_TRY(call)                                                           \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      set_error(std::string("adc2_set_method: ") + #call + ": " + hipGetErrorString(e_)); \
      return fail_all(e_ == hipErrorOutOfMemory ? ADC2_ERR_OOM : ADC2_ERR_HIP); \
    }                                                                         \
  } while (0)
#define X_RC(call)                      \
  do {                                  \
    const adc2_status r_ = (call);      \
    if (r_ != ADC2_OK) return fail_all(r_); \
  } while (0)
  X_TRY(dmalloc(h, &h->Vpp, sizeof(double2) * npair * npair));
  X_TRY(dmalloc(h, &h->Hh, sizeof(double2) * (size_t)nc * no * nc * no));
  X_TRY(dmalloc(h, &h->WvT, sizeof(double2) * (size_t)no * nv * no * nv));
  X_TRY(dmalloc(h, &h->WcT, sizeof(double2) * (size_t)nc * nv * nc * nv));
  X_TRY(dmalloc(h, &h->diagx, sizeof(double) * (size_t)d.dim));
  // particle ladder: (ac|bd) for blocks of a-values (each block at most 2 GiB), then <ab||cd> rows
  {
    const long per_a = (long)nv * nv2 * (long)sizeof(double2);
    const int ab = (int)std::max<long>(1, std::min<long>(nv, (2L << 30) / per_a));
    double2* V = nullptr;
    X_TRY(dmalloc(h, &V, sizeof(double2) * (size_t)ab * nv * nv2));
    tmp.push_back(V);
    for (int a0 = 0; a0 < nv; a0 += ab) {
      const int na = std::min(ab, nv - a0);
      X_RC(bgemm_kmajor(h->Lvv + (long)a0 * nv, 0, nv2, na * nv, h->Lvv, 0, nv2, (int)nv2, na * nv, (int)nv2, naux, 1,
                        V, st));
      k_vpp_rows<<<grid1((long)na * nv * npair), 256, 0, st>>>(V, a0, na, nv, npair, h->Vpp);
      X_TRY(hipGetLastError());
    }
    release_tmp();
  }
  // hole ladder
  k_hole_ladder_ints<<<grid1((long)nc * no * nc * no), 256, 0, st>>>(h->Loo, naux, o, nc, no, h->Hh);
  X_TRY(hipGetLastError());
  // rings: direct part (kc|bj) = sum_P L^P_kc L^P_bj from the transposed occupied block
  // LoT[(l,d)][P] = L^P_ld, then the exchange part (kj|bc) from (occupied block) x (Lvv)
  {
    const double2* LvT = h->LoT + (long)nc * nv * naux;   // valence rows
    const double2* LcT = h->LoT;                          // core rows
    X_RC(gemm_rr(no * nv, no * nv, naux, LvT, naux, true, LvT, naux, false, h->WvT, (long)no * nv, 1.0, false, st));
    X_RC(gemm_rr(nc * nv, nc * nv, naux, LcT, naux, true, LcT, naux, false, h->WcT, (long)nc * nv, 1.0, false, st));
    double2* G = nullptr;
    X_TRY(dmalloc(h, &G, sizeof(double2) * (size_t)std::max(no, nc) * std::max(no, nc) * nv2));
    tmp.push_back(G);
    // G[(k,j)][(b,c)] = sum_P L^P_kj L^P_bc over the valence block, then the core block
    X_RC(bgemm_kmajor(h->Loo + (long)nc * o + nc, o, (long)o * o, no, h->Lvv, 0, nv2, (int)nv2, no * no, (int)nv2,
                      naux, 1, G, st));
    k_ring_exchange<<<grid1((long)no * nv * no * nv), 256, 0, st>>>(G, no, nv, h->WvT);
    X_TRY(hipGetLastError());
    X_RC(bgemm_kmajor(h->Loo, o, (long)o * o, nc, h->Lvv, 0, nv2, (int)nv2, nc * nc, (int)nv2, naux, 1, G, st));
    k_ring_exchange<<<grid1((long)nc * nv * nc * nv), 256, 0, st>>>(G, nc, nv, h->WcT);
    X_TRY(hipGetLastError());
    release_tmp();
  }
  k_x_diag<<<grid1(d.dim), 256, 0, st>>>(h->diag, h->Vpp, h->Hh, h->WvT, h->WcT, d.ns, nc, no, nv, npair, h->diagx);
  X_TRY(hipGetLastError());
  X_TRY(hipStreamSynchronize(st));
  return ADC2_OK;
#undef X_TRY
#undef X_RC
}

adc2_status ensure_ws_x(adc2_handle h, int m) {
  if (h->wsx_m >= m) return ADC2_OK;
  dfree(h, h->Xw);
  h->Xw = nullptr;
  h->wsx_m = 0;
  const Dims& d = h->d;
  const size_t blk = (size_t)m * d.nc * d.no * d.nv * d.nv;   // each of Ru, Rc, Gv, Gc
  ADC2_HIP(dmalloc(h, &h->Xw, sizeof(double2) * 4 * blk));
  h->wsx_m = m;
  return ADC2_OK;
}

// sigma2 += (first-order doubles block) r2 for m vectors (FP64).
adc2_status adc2x_apply(adc2_handle h, int m, const double2* x, double2* s, hipStream_t st) {
  const Dims& d = h->d;
  const int nc = d.nc, no = d.no, nv = d.nv;
  const long npair = d.npair, dim = d.dim, ns = d.ns;
  adc2_status rc = ensure_ws_x(h, m);
  if (rc != ADC2_OK) return rc;
  const int nco = nc * no;
  for (int v = 0; v < m; ++v) {
    const double2* xv = x + (long)v * dim + ns;
    double2* sv = s + (long)v * dim + ns;
    // particle ladder: s[(I,j)][q] += sum_q' r[(I,j)][q'] Vpp[q][q']
    if ((rc = gemm_rr(nco, (int)npair, (int)npair, xv, npair, false, h->Vpp, npair, false, sv, npair, 1.0, true, st)) !=
        ADC2_OK)
      return rc;
    // hole ladder: s[(I,j)][q] += sum_(K,k) Hh[(I,j)][(K,k)] r[(K,k)][q]
    const long tiles = cdl(nco, TM) * cdl(npair, TN);
    k_gemm_rk_acc<<<(unsigned)tiles, 256, 0, st>>>(nco, (int)npair, nco, h->Hh, nco, xv, npair, sv, npair);
    ADC2_CHECK_LAUNCH();
  }
  // rings
  const size_t blk = (size_t)m * nc * no * nv * nv;
  double2* Ru = h->Xw;
  double2* Rc = Ru + blk;
  double2* Gv = Rc + blk;
  double2* Gc = Gv + blk;
  k_x_unpack<<<grid1((long)blk), 256, 0, st>>>(x, dim, ns, m, nc, no, nv, npair, Ru, Rc);
  ADC2_CHECK_LAUNCH();
  if ((rc = gemm_rr(m * nc * nv, no * nv, no * nv, Ru, (long)no * nv, false, h->WvT, (long)no * nv, false, Gv,
                    (long)no * nv, 1.0, false, st)) != ADC2_OK)
    return rc;
  if ((rc = gemm_rr(m * no * nv, nc * nv, nc * nv, Rc, (long)nc * nv, false, h->WcT, (long)nc * nv, false, Gc,
                    (long)nc * nv, 1.0, false, st)) != ADC2_OK)
    return rc;
  k_x_ring_pack<<<grid1((long)m * d.nd), 256, 0, st>>>(Gv, Gc, dim, ns, m, nc, no, nv, npair, s);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

}  // namespace adc2

extern "C" adc2_status adc2_set_method(adc2_handle h, int method, void* stream) {
  using namespace adc2;
  if (!h) {
    set_error("adc2_set_method: NULL handle");
    return ADC2_ERR_ARG;
  }
  if (method != ADC2_METHOD_ADC2 && method != ADC2_METHOD_ADC2X) {
    set_error("adc2_set_method: unknown method");
    return ADC2_ERR_ARG;
  }
  if (method == ADC2_METHOD_ADC2X) {
    const adc2_status rc = build_adc2x(h, (hipStream_t)stream);
    if (rc != ADC2_OK) return rc;
  }
  h->method = method;
  return ADC2_OK;
}
