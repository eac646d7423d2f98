// k_setup.hip -- setup kernels: Cholesky-block repack, MP2 amplitudes and the
// dense CVS singles block through second order.
//
// Storage split (Implementation section): setup keeps only integrals with up
// to two virtual indices; contractions that carry three or four virtual
// indices are formed from L inside the sigma GEMMs.  The setup forms
//   W^{kl}_{ac} = <ac||kl> = (ak|cl) - (al|ck)   for every occupied pair k<l,
//   tau = W / D^{ac}_{kl},  D = e_a + e_c - e_k - e_l   (Eq. 15 denominators),
// the MP2 energy, and the singles block
//   M11[(I,a),(J,b)] = d_IJ d_ab (e_a - e_I) + <aJ||Ib>
//      + 1/2 d_IJ (B + B^H)_ab,  B = sum_{k<l} tau^{kl} (W^{kl})^H
//      + d_ab Q_IJ,  Q_IJ = 1/4 sum_{k,cd} conj(W_{cd,Jk}) W_{cd,Ik} (1/D_Ik + 1/D_Jk)
//      - 1/2 (E + E^H),  E_{(Ia),(Jb)} = sum_{k,c} tau_{ac,Ik} conj(W_{bc,Jk})
// which is the second-order truncation (Eq. 12) of the intermediate-state
// matrix (Eq. 9) on the core-excited singles.
#include <vector>
#include <cmath>
#include <algorithm>

#include "internal.h"
#include "tile.h"

namespace adc2 {

// ---------------------------------------------------------------------------
// Repack L[P][p][q] into the Lvv / Lvo / Loo blocks and check Hermiticity.
// One workgroup per (P, 32x32 tile (pb, qb)); the mirror tile (qb, pb) is
// staged in LDS so that both reads are coalesced.
// ---------------------------------------------------------------------------
constexpr int RT = 32;

__global__ __launch_bounds__(256) void k_repack(const double2* __restrict__ L, int naux, int n, int o,
                                                 int nv, double2* __restrict__ Lvv,
                                                 double2* __restrict__ Lvo, double2* __restrict__ Loo,
                                                 double* __restrict__ pmax) {
  __shared__ double2 tA[RT][RT + 1];
  __shared__ double2 tB[RT][RT + 1];
  __shared__ double red[2][256];
  const int nt = (n + RT - 1) / RT;
  const int tile = blockIdx.x, P = blockIdx.y;
  const int pb = tile / nt, qb = tile % nt;
  const double2* LP = L + (long)P * n * n;
  const int tid = threadIdx.x;
  for (int e = tid; e < RT * RT; e += 256) {
    int r = e / RT, c = e % RT;
    int p = pb * RT + r, q = qb * RT + c;
    tA[r][c] = (p < n && q < n) ? LP[(long)p * n + q] : make_double2(0, 0);
    int p2 = qb * RT + r, q2 = pb * RT + c;
    tB[r][c] = (p2 < n && q2 < n) ? LP[(long)p2 * n + q2] : make_double2(0, 0);
  }
  __syncthreads();
  double dmax = 0.0, amax = 0.0;
  for (int e = tid; e < RT * RT; e += 256) {
    int r = e / RT, c = e % RT;
    int p = pb * RT + r, q = qb * RT + c;
    if (p >= n || q >= n) continue;
    double2 v = tA[r][c];
    double2 w = tB[c][r];      // L[q][p]
    double dx = v.x - w.x, dy = v.y + w.y;
    double dd = sqrt(dx * dx + dy * dy);
    double av = sqrt(v.x * v.x + v.y * v.y);
    if (!isfinite(av)) { av = INFINITY; dd = INFINITY; }
    dmax = fmax(dmax, dd);
    amax = fmax(amax, av);
    if (p >= o && q >= o) {
      Lvv[((long)P * nv + (p - o)) * nv + (q - o)] = v;
    } else if (p < o && q >= o) {
      // L^P_{a k} = conj(L^P_{k a})
      Lvo[((long)p * naux + P) * nv + (q - o)] = make_double2(v.x, -v.y);
    } else if (p < o && q < o) {
      Loo[((long)P * o + p) * o + q] = v;
    }
  }
  red[0][tid] = dmax;
  red[1][tid] = amax;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      red[0][tid] = fmax(red[0][tid], red[0][tid + s]);
      red[1][tid] = fmax(red[1][tid], red[1][tid + s]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    long b = (long)blockIdx.y * gridDim.x + blockIdx.x;
    pmax[2 * b] = red[0][0];
    pmax[2 * b + 1] = red[1][0];
  }
}

adc2_status launch_repack(const double2* L, const double* eps, adc2_handle h, double* herm_out,
                          hipStream_t st) {
  const Dims& d = h->d;
  const int nt = (d.n + RT - 1) / RT;
  const long nblk = (long)nt * nt * d.naux;
  double* pmax = nullptr;
  ADC2_HIP(hipMallocAsync((void**)&pmax, sizeof(double) * 2 * nblk, st));
  dim3 grid(nt * nt, d.naux);
  k_repack<<<grid, 256, 0, st>>>(L, d.naux, d.n, d.o, d.nv, h->Lvv, h->Lvo, h->Loo, pmax);
  ADC2_CHECK_LAUNCH();
  std::vector<double> hp(2 * nblk);
  ADC2_HIP(hipMemcpyAsync(hp.data(), pmax, sizeof(double) * 2 * nblk, hipMemcpyDeviceToHost, st));
  ADC2_HIP(hipStreamSynchronize(st));
  ADC2_HIP(hipFreeAsync(pmax, st));
  double dm = 0, am = 0;
  for (long b = 0; b < nblk; ++b) {
    dm = std::max(dm, hp[2 * b]);
    am = std::max(am, hp[2 * b + 1]);
  }
  herm_out[0] = dm;
  herm_out[1] = am;
  (void)eps;
  return ADC2_OK;
}

// ---------------------------------------------------------------------------
// MP2: W^{kl}[a][c] = sum_P (L^P_{ak} L^P_{cl} - L^P_{al} L^P_{ck}) for k<l.
// Antisymmetric rank-2K product on the upper tile pairs (a-blk <= c-blk);
// the epilogue writes W and its negative mirror and accumulates
// -|W|^2 / D with D from energies staged in LDS.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tile_pair(int t, int nb, int& ab, int& cb) {
  // upper-triangular enumeration of (ab <= cb)
  int r = 0;
  while (t >= nb - r) {
    t -= nb - r;
    ++r;
  }
  ab = r;
  cb = r + t;
}

__global__ __launch_bounds__(256) void k_wbuild(const double2* __restrict__ Lvo, const double* __restrict__ eps,
                                                 const int2* __restrict__ pairs, int npairs, int naux, int nv,
                                                 int o, double2* __restrict__ W, double* __restrict__ epart) {
  __shared__ TileSmem s;
  __shared__ double ea[TM], ec[TN];
  __shared__ double red[256];
  const int nb = (nv + TM - 1) / TM;
  const int ntp = nb * (nb + 1) / 2;
  const long nblocks = (long)npairs * ntp;
  const long lid = xcd_remap(blockIdx.x, nblocks);
  const int p = (int)(lid / ntp);
  const int t = (int)(lid % ntp);
  int abk, cbk;
  tile_pair(t, nb, abk, cbk);
  const int a0 = abk * TM, c0 = cbk * TN;
  const int2 kl = pairs[p];
  const long lds = (long)naux * nv;
  const double2* Lk = Lvo + (long)kl.x * lds;
  const double2* Ll = Lvo + (long)kl.y * lds;
  const int tid = threadIdx.x;
  if (tid < TM) ea[tid] = (a0 + tid < nv) ? eps[o + a0 + tid] : 0.0;
  else if (tid < TM + TN) ec[tid - TM] = (c0 + tid - TM < nv) ? eps[o + c0 + tid - TM] : 0.0;

  Acc acc;
  acc.zero();
  const int nkc = (naux + TK - 1) / TK;
  {
    SrcK<false> A{Lk + a0, nv, naux, nv - a0, 1.0};
    SrcK<false> B{Ll + c0, nv, naux, nv - c0, 1.0};
    mainloop(s, A, B, 0, nkc, acc);
  }
  {
    SrcK<false> A{Ll + a0, nv, naux, nv - a0, 1.0};
    SrcK<false> B{Lk + c0, nv, naux, nv - c0, -1.0};
    mainloop(s, A, B, 0, nkc, acc);
  }
  __syncthreads();
  const double ekl = eps[kl.x] + eps[kl.y];
  double2* Wp = W + (long)p * nv * nv;
  double e = 0.0;
  for_each_acc(acc, [&](int r, int c, double2 v) {
    const int a = a0 + r, cc = c0 + c;
    if (a >= nv || cc >= nv) return;
    if (a < cc) {
      Wp[(long)a * nv + cc] = v;
      Wp[(long)cc * nv + a] = make_double2(-v.x, -v.y);
      const double D = ea[r] + ec[c] - ekl;
      e -= (v.x * v.x + v.y * v.y) / D;
    } else if (a == cc) {
      Wp[(long)a * nv + a] = make_double2(0.0, 0.0);
    }
  });
  red[tid] = e;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0) epart[lid] = red[0];
}

// ---------------------------------------------------------------------------
// Pair contraction  C_b[a][x] = sum_t s_t sum_c W[pA_t][a][c] / D(a,c;kA_t,lA_t)
//                                          * conj(W[pB_t][x][c])
// over the term list of batch b, split over K.  Each list entry is
// int4 (pA, pB, kA, lA) with sign in a parallel array.
// K is padded per entry to a multiple of TK so that chunks never straddle.
// ---------------------------------------------------------------------------
struct SrcTau {
  static constexpr int MAP = RMAJOR;
  const double2* W;
  const int4* ent;
  const double* sgn;
  const double* eps;
  int o, nv, a0, cpe;  // cpe = chunks per entry
  long nv2;
  __device__ __forceinline__ double2 get(int k, int i) const {
    const int chunk = k / TK;
    const int t = chunk / cpe;
    const int c = (chunk - t * cpe) * TK + (k % TK);
    const int a = a0 + i;
    if (c >= nv || a >= nv) return czero();
    const int4 en = ent[t];
    const double2 w = W[(long)en.x * nv2 + (long)a * nv + c];
    const double D = eps[o + a] + eps[o + c] - eps[en.z] - eps[en.w];
    const double f = sgn[t] / D;
    return make_double2(w.x * f, w.y * f);
  }
};

struct SrcWc {
  static constexpr int MAP = RMAJOR;
  const double2* W;
  const int4* ent;
  int nv, b0, cpe;
  long nv2;
  __device__ __forceinline__ double2 get(int k, int i) const {
    const int chunk = k / TK;
    const int t = chunk / cpe;
    const int c = (chunk - t * cpe) * TK + (k % TK);
    const int b = b0 + i;
    if (c >= nv || b >= nv) return czero();
    const double2 w = W[(long)ent[t].y * nv2 + (long)b * nv + c];
    return make_double2(w.x, -w.y);
  }
};

__global__ __launch_bounds__(256) void k_pairc(const double2* __restrict__ W, const double* __restrict__ eps,
                                                const int4* __restrict__ ent, const double* __restrict__ sgn,
                                                const int* __restrict__ ent_off, int o, int nv, int nsplit,
                                                double2* __restrict__ part) {
  __shared__ TileSmem s;
  const int nb = (nv + TM - 1) / TM;
  const int tile = blockIdx.x % (nb * nb);
  const int split = blockIdx.x / (nb * nb);
  const int batch = blockIdx.y;
  const int ab = tile / nb, xb = tile % nb;
  const int a0 = ab * TM, b0 = xb * TN;
  const int cpe = (nv + TK - 1) / TK;
  const int e0 = ent_off[batch], e1 = ent_off[batch + 1];
  const int nchunks = (e1 - e0) * cpe;
  const int per = (nchunks + nsplit - 1) / nsplit;
  const int kc0 = split * per, kc1 = min(nchunks, kc0 + per);
  const long nv2 = (long)nv * nv;
  SrcTau A{W, ent + e0, sgn + e0, eps, o, nv, a0, cpe, nv2};
  SrcWc B{W, ent + e0, nv, b0, cpe, nv2};
  Acc acc;
  acc.zero();
  mainloop(s, A, B, kc0, kc1, acc);
  double2* out = part + ((long)batch * nsplit + split) * nv2;
  for_each_acc(acc, [&](int r, int c, double2 v) {
    const int a = a0 + r, b = b0 + c;
    if (a < nv && b < nv) out[(long)a * nv + b] = v;
  });
}

__global__ void k_sum_splits(const double2* __restrict__ part, int nsplit, long len, int nbatch,
                             double2* __restrict__ out) {
  long total = len * nbatch;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    long b = e / len, r = e % len;
    double2 acc = make_double2(0, 0);
    for (int sidx = 0; sidx < nsplit; ++sidx) acc = cadd(acc, part[((long)b * nsplit + sidx) * len + r]);
    out[e] = acc;
  }
}

// ---------------------------------------------------------------------------
// Term (ii):  Q_IJ = 1/4 sum_k s sum_cd conj(W[pJ][c][d]) W[pI][c][d] (1/D^{cd}_{Ik} + 1/D^{cd}_{Jk})
// one workgroup per (I, J, k); partials summed on the host side of assembly.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_qterm(const double2* __restrict__ W, const double* __restrict__ eps,
                                                const int* __restrict__ pidx, int nc, int o, int nv,
                                                double2* __restrict__ qpart) {
  __shared__ double2 red[256];
  const int k = blockIdx.x % o;
  const int J = (blockIdx.x / o) % nc;
  const int I = blockIdx.x / (o * nc);
  const int tid = threadIdx.x;
  double2 acc = make_double2(0, 0);
  if (k != I && k != J) {
    const int pI = pidx[I * o + k], pJ = pidx[J * o + k];
    const double sI = (I < k) ? 1.0 : -1.0, sJ = (J < k) ? 1.0 : -1.0;
    const double2* WI = W + (long)pI * nv * nv;
    const double2* WJ = W + (long)pJ * nv * nv;
    const double eIk = eps[I] + eps[k], eJk = eps[J] + eps[k];
    for (long e = tid; e < (long)nv * nv; e += 256) {
      const int c = (int)(e / nv), dd = (int)(e % nv);
      const double ecd = eps[o + c] + eps[o + dd];
      const double f = 1.0 / (ecd - eIk) + 1.0 / (ecd - eJk);
      const double2 t = cdotc(WJ[e], WI[e]);
      acc = cadd(acc, cscale(t, f));
    }
    acc = cscale(acc, 0.25 * sI * sJ);
  }
  red[tid] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) red[tid] = cadd(red[tid], red[tid + st]);
    __syncthreads();
  }
  if (tid == 0) qpart[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// <Ka||Ij> = (KI|aj) - (Kj|aI)  stored as Vt[I][j][K][a]
// ---------------------------------------------------------------------------
__global__ void k_vint(const double2* __restrict__ Lvo, const double2* __restrict__ Loo, int nc, int no,
                       int nv, int naux, int o, double2* __restrict__ Vt) {
  const long total = (long)nc * no * nc * nv;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int a = (int)(e % nv);
    const int K = (int)((e / nv) % nc);
    const int j = (int)((e / ((long)nv * nc)) % no);
    const int I = (int)(e / ((long)nv * nc * no));
    const int jo = nc + j;
    double2 acc = make_double2(0, 0);
    for (int P = 0; P < naux; ++P) {
      const double2 lKI = Loo[((long)P * o + K) * o + I];
      const double2 laj = Lvo[((long)jo * naux + P) * nv + a];
      const double2 lKj = Loo[((long)P * o + K) * o + jo];
      const double2 laI = Lvo[((long)I * naux + P) * nv + a];
      acc = cadd(acc, csub(cmul(lKI, laj), cmul(lKj, laI)));
    }
    Vt[e] = acc;
  }
}

// ---------------------------------------------------------------------------
// First order:  F1[(I,a)][(J,b)] = sum_P Lvo[I][P][a] conj(Lvo[J][P][b]) = (aI|Jb)
// batched over (I,J), written straight into M11.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_first_aIJb(const double2* __restrict__ Lvo, int nc, int nv, int naux,
                                                     double2* __restrict__ M11) {
  __shared__ TileSmem s;
  const int nb = (nv + TM - 1) / TM;
  const int tile = blockIdx.x % (nb * nb);
  const int IJ = blockIdx.x / (nb * nb);
  const int I = IJ / nc, J = IJ % nc;
  const int a0 = (tile / nb) * TM, b0 = (tile % nb) * TN;
  const long lds = (long)naux * nv;
  SrcK<false> A{Lvo + I * lds + a0, nv, naux, nv - a0, 1.0};
  SrcK<true> B{Lvo + J * lds + b0, nv, naux, nv - b0, 1.0};
  Acc acc;
  acc.zero();
  mainloop(s, A, B, 0, (naux + TK - 1) / TK, acc);
  const long ns = (long)nc * nv;
  for_each_acc(acc, [&](int r, int c, double2 v) {
    const int a = a0 + r, b = b0 + c;
    if (a < nv && b < nv) M11[((long)I * nv + a) * ns + (long)J * nv + b] = v;
  });
}

// (ab|JI) = sum_P Lvv[P][a][b] Loo[P][J][I]:  rows (a,b) flattened, columns (J,I)
struct SrcLooCore {
  static constexpr int MAP = KMAJOR;
  const double2* Loo;
  int o, nc, naux, j0;
  __device__ __forceinline__ double2 get(int k, int i) const {
    const int jj = j0 + i;
    if (k >= naux || jj >= nc * nc) return czero();
    const int J = jj / nc, I = jj % nc;
    return Loo[((long)k * o + J) * o + I];
  }
};

__global__ __launch_bounds__(256) void k_first_abJI(const double2* __restrict__ Lvv,
                                                     const double2* __restrict__ Loo, int nc, int nv, int naux,
                                                     int o, double2* __restrict__ G2) {
  __shared__ TileSmem s;
  const long nv2 = (long)nv * nv;
  const int ncc = nc * nc;
  const int nbj = (ncc + TN - 1) / TN;
  const long i0 = (long)(blockIdx.x / nbj) * TM;
  const int j0 = (blockIdx.x % nbj) * TN;
  SrcK<false> A{Lvv + i0, nv2, naux, (int)min((long)TM, nv2 - i0), 1.0};
  SrcLooCore B{Loo, o, nc, naux, j0};
  Acc acc;
  acc.zero();
  mainloop(s, A, B, 0, (naux + TK - 1) / TK, acc);
  for_each_acc(acc, [&](int r, int c, double2 v) {
    const long ab = i0 + r;
    const int jj = j0 + c;
    if (ab < nv2 && jj < ncc) G2[(long)jj * nv2 + ab] = v;   // G2[(J,I)][(a,b)]
  });
}

// ---------------------------------------------------------------------------
// Assembly of M11 and the diagonal of M.
// ---------------------------------------------------------------------------
__global__ void k_assemble(double2* __restrict__ M11, const double* __restrict__ eps,
                           const double2* __restrict__ G2, const double2* __restrict__ Bm,
                           const double2* __restrict__ Q, const double2* __restrict__ E, int nc, int nv,
                           int o) {
  const long ns = (long)nc * nv;
  const long nv2 = (long)nv * nv;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < ns * ns; e += (long)gridDim.x * blockDim.x) {
    const long row = e / ns, col = e % ns;
    const int I = (int)(row / nv), a = (int)(row % nv);
    const int J = (int)(col / nv), b = (int)(col % nv);
    double2 v = M11[e];                                   // (aI|Jb)
    v = csub(v, G2[(long)(J * nc + I) * nv2 + (long)a * nv + b]);   // -(ab|JI)
    if (I == J) {
      const double2 bab = Bm[(long)a * nv + b], bba = Bm[(long)b * nv + a];
      v = cadd(v, make_double2(0.5 * (bab.x + bba.x), 0.5 * (bab.y - bba.y)));
      if (a == b) v.x += eps[o + a] - eps[I];
    }
    if (a == b) v = cadd(v, Q[I * nc + J]);
    const double2 eIJ = E[((long)(I * nc + J)) * nv2 + (long)a * nv + b];
    const double2 eJI = E[((long)(J * nc + I)) * nv2 + (long)b * nv + a];
    v = csub(v, make_double2(0.5 * (eIJ.x + eJI.x), 0.5 * (eIJ.y - eJI.y)));
    M11[e] = v;
  }
}

__global__ void k_diag(const double2* __restrict__ M11, const double* __restrict__ eps, int nc, int no,
                       int nv, double* __restrict__ diag) {
  const long ns = (long)nc * nv;
  const long npair = (long)nv * (nv - 1) / 2;
  const long dim = ns + (long)nc * no * npair;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < dim; e += (long)gridDim.x * blockDim.x) {
    if (e < ns) {
      diag[e] = M11[e * ns + e].x;
    } else {
      const long q = e - ns;
      const long ij = q / npair;
      long pr = q % npair;
      const int I = (int)(ij / no), j = (int)(ij % no);
      // invert the row-major upper-triangle pair index
      int a = (int)((2.0 * nv - 1.0 - sqrt((2.0 * nv - 1.0) * (2.0 * nv - 1.0) - 8.0 * pr)) / 2.0);
      if (a < 0) a = 0;
      while ((long)(a + 1) * nv - (long)(a + 1) * (a + 2) / 2 <= pr) ++a;
      while ((long)a * nv - (long)a * (a + 1) / 2 > pr) --a;
      const long base = (long)a * nv - (long)a * (a + 1) / 2;
      const int b = (int)(pr - base) + a + 1;
      const int o = nc + no;
      diag[e] = eps[o + a] + eps[o + b] - eps[I] - eps[nc + j];
    }
  }
}

static inline int grid_for(long n, int per = 256, int cap = 8192) {
  long g = (n + per - 1) / per;
  return (int)std::max<long>(1, std::min<long>(g, cap));
}

// W for every occupied pair (k<l), in the same pair order as build_m11.
// W for the npairs occupied pairs listed (device int2 (k, l), k < l) into
// W[t][a][c]; epart: npairs * nb(nb+1)/2 doubles of MP2 energy partials.
adc2_status wbuild_pairs(adc2_handle h, const int2* dpairs, int npairs, double2* W, double* epart,
                         hipStream_t st) {
  const Dims& d = h->d;
  const int nb = (d.nv + TM - 1) / TM;
  const long nwblk = (long)npairs * (nb * (nb + 1) / 2);
  if (nwblk == 0) return ADC2_OK;
  k_wbuild<<<(unsigned)nwblk, 256, 0, st>>>(h->Lvo, h->eps, dpairs, npairs, d.naux, d.nv, d.o, W, epart);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

adc2_status wbuild(adc2_handle h, double2* W, hipStream_t st) {
  const Dims& d = h->d;
  const int o = d.o, nv = d.nv;
  std::vector<int2> pairs;
  for (int k = 0; k < o; ++k)
    for (int l = k + 1; l < o; ++l) pairs.push_back(make_int2(k, l));
  const int npairs = (int)pairs.size();
  if (npairs == 0) return ADC2_OK;
  const int nb = (nv + TM - 1) / TM;
  const long nwblk = (long)npairs * (nb * (nb + 1) / 2);
  int2* dpairs = nullptr;
  double* epart = nullptr;
  hipError_t e = dmalloc(h, &dpairs, sizeof(int2) * npairs);
  if (e == hipSuccess) e = dmalloc(h, &epart, sizeof(double) * nwblk);
  if (e == hipSuccess) e = hipMemcpyAsync(dpairs, pairs.data(), sizeof(int2) * npairs, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    k_wbuild<<<(unsigned)nwblk, 256, 0, st>>>(h->Lvo, h->eps, dpairs, npairs, d.naux, nv, o, W, epart);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dfree(h, dpairs);
  dfree(h, epart);
  if (e != hipSuccess) {
    set_error(std::string("wbuild: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? ADC2_ERR_OOM : ADC2_ERR_HIP;
  }
  return ADC2_OK;
}

adc2_status build_m11(adc2_handle h, hipStream_t st) {
  const Dims& d = h->d;
  const int nc = d.nc, o = d.o, nv = d.nv, naux = d.naux;
  const long nv2 = (long)nv * nv;
  const long ns = d.ns;

  // occupied pairs k<l and the pair index lookup
  std::vector<int2> pairs;
  std::vector<int> pidx(o * o, -1);
  for (int k = 0; k < o; ++k)
    for (int l = k + 1; l < o; ++l) {
      pidx[k * o + l] = pidx[l * o + k] = (int)pairs.size();
      pairs.push_back(make_int2(k, l));
    }
  const int npairs = (int)pairs.size();

  // term (i) list: all pairs; term (iii) lists per (I,J): k != I, J
  std::vector<int4> ent;
  std::vector<double> sgn;
  std::vector<int> off;
  off.push_back(0);
  for (int p = 0; p < npairs; ++p) {
    ent.push_back(make_int4(p, p, pairs[p].x, pairs[p].y));
    sgn.push_back(1.0);
  }
  off.push_back((int)ent.size());
  for (int I = 0; I < nc; ++I)
    for (int J = 0; J < nc; ++J) {
      for (int k = 0; k < o; ++k) {
        if (k == I || k == J) continue;
        const double s = ((I < k) ? 1.0 : -1.0) * ((J < k) ? 1.0 : -1.0);
        ent.push_back(make_int4(pidx[I * o + k], pidx[J * o + k], I, k));
        sgn.push_back(s);
      }
      off.push_back((int)ent.size());
    }

  // device scratch for the setup
  int2* dpairs = nullptr;
  int* dpidx = nullptr;
  int4* dent = nullptr;
  double* dsgn = nullptr;
  int* doff = nullptr;
  double2 *W = nullptr, *part = nullptr, *Bm = nullptr, *E = nullptr, *G2 = nullptr, *qpart = nullptr;
  double* epart = nullptr;
  const int nb = (nv + TM - 1) / TM;
  const int ntp = nb * (nb + 1) / 2;
  const long nwblk = (long)npairs * ntp;
  const int nsplit_i = std::max(1, std::min(128, (int)((long)npairs * ((nv + TK - 1) / TK) / 64)));
  const int nsplit_iii = 4;
  const size_t part_len = std::max((size_t)nsplit_i, (size_t)(nc * nc * nsplit_iii)) * nv2;

  auto cleanup = [&]() {
    dfree(h, dpairs); dfree(h, dpidx); dfree(h, dent); dfree(h, dsgn); dfree(h, doff);
    dfree(h, W); dfree(h, part); dfree(h, Bm); dfree(h, E); dfree(h, G2); dfree(h, qpart); dfree(h, epart);
  };
#define SETUP_HIP(call)                                                            \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));                \
      hipStreamSynchronize(st);                                                    \
      cleanup();                                                                   \
      return e_ == hipErrorOutOfMemory ? ADC2_ERR_OOM : ADC2_ERR_HIP;              \
    }                                                                              \
  } while (0)

  SETUP_HIP(dmalloc(h, &dpairs, sizeof(int2) * std::max(1, npairs)));
  SETUP_HIP(dmalloc(h, &dpidx, sizeof(int) * o * o));
  SETUP_HIP(dmalloc(h, &dent, sizeof(int4) * std::max<size_t>(1, ent.size())));
  SETUP_HIP(dmalloc(h, &dsgn, sizeof(double) * std::max<size_t>(1, sgn.size())));
  SETUP_HIP(dmalloc(h, &doff, sizeof(int) * off.size()));
  SETUP_HIP(dmalloc(h, &W, sizeof(double2) * std::max<long>(1, (long)npairs * nv2)));
  SETUP_HIP(dmalloc(h, &part, sizeof(double2) * part_len));
  SETUP_HIP(dmalloc(h, &Bm, sizeof(double2) * nv2));
  SETUP_HIP(dmalloc(h, &E, sizeof(double2) * nc * nc * nv2));
  SETUP_HIP(dmalloc(h, &G2, sizeof(double2) * nc * nc * nv2));
  SETUP_HIP(dmalloc(h, &qpart, sizeof(double2) * nc * nc * o));
  SETUP_HIP(dmalloc(h, &epart, sizeof(double) * std::max<long>(1, nwblk)));
  SETUP_HIP(hipMemcpyAsync(dpairs, pairs.data(), sizeof(int2) * npairs, hipMemcpyHostToDevice, st));
  SETUP_HIP(hipMemcpyAsync(dpidx, pidx.data(), sizeof(int) * o * o, hipMemcpyHostToDevice, st));
  SETUP_HIP(hipMemcpyAsync(dent, ent.data(), sizeof(int4) * ent.size(), hipMemcpyHostToDevice, st));
  SETUP_HIP(hipMemcpyAsync(dsgn, sgn.data(), sizeof(double) * sgn.size(), hipMemcpyHostToDevice, st));
  SETUP_HIP(hipMemcpyAsync(doff, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice, st));

  // MP2 amplitudes / W for every occupied pair
  if (npairs > 0) {
    k_wbuild<<<(unsigned)nwblk, 256, 0, st>>>(h->Lvo, h->eps, dpairs, npairs, naux, nv, o, W, epart);
    SETUP_HIP(hipGetLastError());
  }
  // term (i): B = sum_{k<l} tau^{kl} W^{kl H}
  if (npairs > 0) {
    dim3 g(nb * nb * nsplit_i, 1);
    k_pairc<<<g, 256, 0, st>>>(W, h->eps, dent, dsgn, doff, o, nv, nsplit_i, part);
    SETUP_HIP(hipGetLastError());
    k_sum_splits<<<grid_for(nv2), 256, 0, st>>>(part, nsplit_i, nv2, 1, Bm);
    SETUP_HIP(hipGetLastError());
  } else {
    SETUP_HIP(hipMemsetAsync(Bm, 0, sizeof(double2) * nv2, st));
  }
  // term (iii): E^{IJ} = sum_k tau^{Ik} W^{Jk H}
  {
    dim3 g(nb * nb * nsplit_iii, nc * nc);
    k_pairc<<<g, 256, 0, st>>>(W, h->eps, dent, dsgn, doff + 1, o, nv, nsplit_iii, part);
    SETUP_HIP(hipGetLastError());
    k_sum_splits<<<grid_for(nv2 * nc * nc), 256, 0, st>>>(part, nsplit_iii, nv2, nc * nc, E);
    SETUP_HIP(hipGetLastError());
  }
  // term (ii)
  k_qterm<<<nc * nc * o, 256, 0, st>>>(W, h->eps, dpidx, nc, o, nv, qpart);
  SETUP_HIP(hipGetLastError());
  // first order
  k_first_aIJb<<<nc * nc * nb * nb, 256, 0, st>>>(h->Lvo, nc, nv, naux, h->M11);
  SETUP_HIP(hipGetLastError());
  {
    const int nbi = (int)((nv2 + TM - 1) / TM);
    const int nbj = (nc * nc + TN - 1) / TN;
    k_first_abJI<<<nbi * nbj, 256, 0, st>>>(h->Lvv, h->Loo, nc, nv, naux, o, G2);
    SETUP_HIP(hipGetLastError());
  }
  k_vint<<<grid_for((long)nc * d.no * nc * nv), 256, 0, st>>>(h->Lvo, h->Loo, nc, d.no, nv, naux, o, h->Vt);
  SETUP_HIP(hipGetLastError());

  // Q and E_MP2 reductions on the host (small)
  std::vector<double2> hq(nc * nc * o);
  std::vector<double> he(std::max<long>(1, nwblk));
  SETUP_HIP(hipMemcpyAsync(hq.data(), qpart, sizeof(double2) * hq.size(), hipMemcpyDeviceToHost, st));
  if (npairs > 0)
    SETUP_HIP(hipMemcpyAsync(he.data(), epart, sizeof(double) * nwblk, hipMemcpyDeviceToHost, st));
  SETUP_HIP(hipStreamSynchronize(st));
  double emp2 = 0.0;
  for (long b = 0; b < (npairs > 0 ? nwblk : 0); ++b) emp2 += he[b];
  h->e_mp2 = emp2;
  std::vector<double2> Q(nc * nc);
  for (int IJ = 0; IJ < nc * nc; ++IJ) {
    double2 a = make_double2(0, 0);
    for (int k = 0; k < o; ++k) {
      a.x += hq[IJ * o + k].x;
      a.y += hq[IJ * o + k].y;
    }
    Q[IJ] = a;
  }
  double2* dQ = qpart;  // reuse
  SETUP_HIP(hipMemcpyAsync(dQ, Q.data(), sizeof(double2) * nc * nc, hipMemcpyHostToDevice, st));
  k_assemble<<<grid_for(ns * ns), 256, 0, st>>>(h->M11, h->eps, G2, Bm, dQ, E, nc, nv, o);
  SETUP_HIP(hipGetLastError());
  k_diag<<<grid_for(d.dim, 256, 16384), 256, 0, st>>>(h->M11, h->eps, nc, d.no, nv, h->diag);
  SETUP_HIP(hipGetLastError());
  SETUP_HIP(hipStreamSynchronize(st));
  cleanup();
#undef SETUP_HIP
  return ADC2_OK;
}

}  // namespace adc2
