// transition.hip -- modified transition moments and oscillator strengths
// (paper, Theory section, transition properties): T_n = X_n^H F with
// F_I = <Psi~_I| D |Psi0> for the three Cartesian components of a dipole
// operator D = sum_pq d_pq a+_p a_q, and f_n = (2/3) omega_n |T_n|^2.
//
// F in the Moller-Plesset expansion (the paper builds the transition density
// through second order and prints no expressions; these are the orders of the
// definition):
//   singles (I, a):  F = d_aI - sum_{j in O, b} tau^{ab}_{Ij} d_jb  (+ F2, order 2)
//   doubles (I, j, a<b) in the basis a+_a a+_b a_j a_I |Phi0>, first order
//   (their second order reaches T only at third order):
//     F = -[ (d_vv tau_Ij - (d_vv tau_Ij)^T)_{ab}
//            - sum_{k in O} (d_kI tau^{ab}_{kj} + d_kj tau^{ab}_{Ik}) ]
// (tau_Ij antisymmetric, so tau_Ij d_vv^T = -(d_vv tau_Ij)^T), with the MP2
// amplitudes tau of every occupied pair from the setup's W-build.  The
// second-order singles F2 (tm_second_order below):
//   F2_Ia = sum_b d_ab s_Ib - sum_j d_jI s_ja + sum_{jb} d_jb u^{ab}_{Ij}
//           - 1/4 sum_c rho_ac d_cI - 1/4 sum_k d_ak sigma_Ik
//           + 1/2 sum_{lb} tau^{ab}_{Il} h_lb,   h_lb = sum_{kc} conj(tau^{cb}_{kl}) d_ck,
// s and u the second-order singles and doubles amplitudes of the ground state,
//   s_ia = (N1_ia - N2_ia) / (e_a - e_i),
//     N1_ia = sum_{P,b} Z^P_ib L^P_ab,  N2_ia = sum_{P,j} L^P_ji Z^P_ja,
//     Z^P_ib = sum_{jc} tau^{bc}_{ij} L^P_jc,
//   u^{ab}_{Ij} = [ sum_{c,d} (ac|bd) tau^{cd}_{Ij}               (particle ladder)
//                 + sum_{k<l} <kl||Ij> tau^{ab}_{kl}            (hole ladder)
//                 + P(Ij) P(ab) r^{ab}_{Ij} ] / D^{ab}_{Ij},
//     r^{ab}_{ij} = sum_P Z^P_ia L^P_bj - sum_{kc} tau^{ac}_{ik} (kj|bc),
// and the pair densities rho_ac = sum_{klb} tau^{ab}_{kl} conj(tau^{cb}_{kl}),
// sigma_ik = sum_{lcd} tau^{cd}_{il} conj(tau^{cd}_{kl}); j, k, l over every
// occupied spinor.
#include <algorithm>
#include <string>
#include <vector>

#include "internal.h"
#include "tile.h"

namespace adc2 {
namespace {

// pair (k < l) of occupied spinors -> its row-major index
__device__ __forceinline__ long pair_of(int k, int l, int o) { return (long)k * o - (long)k * (k + 1) / 2 + (l - k - 1); }

// tau^{..}_{kl} as a signed pair: +tau of (k, l) for k < l, -tau of (l, k) for k > l; 0 for k == l
__device__ __forceinline__ double2 tau_at(const double2* __restrict__ tau, int k, int l, int o, long nv2, long ab) {
  if (k == l) return make_double2(0.0, 0.0);
  if (k < l) return tau[pair_of(k, l, o) * nv2 + ab];
  const double2 v = tau[pair_of(l, k, o) * nv2 + ab];
  return make_double2(-v.x, -v.y);
}

// singles: one workgroup per (component, I, a)
__global__ __launch_bounds__(256) void k_tm_singles(const double2* __restrict__ tau, const double2* __restrict__ dip,
                                                     int nc, int o, int nv, int n, long dim, double2* __restrict__ F) {
  __shared__ double2 red[256];
  const int blk = blockIdx.x;
  const int comp = blk / (nc * nv), r = blk - comp * nc * nv;
  const int I = r / nv, a = r - I * nv;
  const long nv2 = (long)nv * nv;
  const double2* d = dip + (long)comp * n * n;
  double2 acc = make_double2(0.0, 0.0);
  for (long e = threadIdx.x; e < (long)o * nv; e += 256) {
    const int j = (int)(e / nv), b = (int)(e - (long)j * nv);
    const double2 t = tau_at(tau, I, j, o, nv2, (long)a * nv + b);
    acc = cadd(acc, cmul(t, d[(long)j * n + o + b]));
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double2 daI = d[(long)(o + a) * n + I];
    F[(long)comp * dim + (long)I * nv + a] = make_double2(daI.x - red[0].x, daI.y - red[0].y);
  }
}

// doubles of one (component, I) and every valence j = nc + blockIdx.y:
// A_j[a][b] = (d_vv tau_Ij)[a][b] at Ab[a * lda + j' * nv + b] (j' = blockIdx.y),
// out = F blocks of (I, nc..o-1) in order, a < b packed
__global__ __launch_bounds__(256) void k_tm_doubles(const double2* __restrict__ Ab, long lda,
                                                     const double2* __restrict__ tau,
                                                     const double2* __restrict__ d, int I, int nc, int o, int nv,
                                                     int n, long npair, double2* __restrict__ out0) {
  const long nv2 = (long)nv * nv;
  const int jv = blockIdx.y, jg = nc + jv;
  const double2* A = Ab + (long)jv * nv;
  double2* out = out0 + (long)jv * npair;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < nv2; e += (long)gridDim.x * 256) {
    const int a = (int)(e / nv), b = (int)(e - (long)a * nv);
    if (a >= b) continue;
    const long ab = (long)a * nv + b;
    const double2 x = A[(long)a * lda + b], y = A[(long)b * lda + a];
    double2 s = make_double2(x.x - y.x, x.y - y.y);
    for (int k = 0; k < o; ++k) {
      const double2 t1 = cmul(d[(long)k * n + I], tau_at(tau, k, jg, o, nv2, ab));
      const double2 t2 = cmul(d[(long)k * n + jg], tau_at(tau, I, k, o, nv2, ab));
      s.x -= t1.x + t2.x;
      s.y -= t1.y + t2.y;
    }
    const long q = (long)a * nv - (long)a * (a + 1) / 2 + (b - a - 1);
    out[q] = make_double2(-s.x, -s.y);
  }
}


// dst[b][a][c] = src[a][b][c] (conjugated if CONJ); A, B, C the extents of src
template <bool CONJ>
__global__ void k_swap12(const double2* __restrict__ src, long A, long B, long C, double2* __restrict__ dst) {
  const long total = A * B * C;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const long c = e % C, ba = e / C;
    const long a = ba % A, b = ba / A;
    double2 v = src[(a * B + b) * C + c];
    if (CONJ) v.y = -v.y;
    dst[e] = v;
  }
}

// dst[c][r] = src[r][c] for an R x Cc matrix, 32 x 32 tiles through LDS
__global__ __launch_bounds__(256) void k_transpose(const double2* __restrict__ src, long R, long Cc,
                                                    double2* __restrict__ dst) {
  __shared__ double2 t[32][33];
  const long tilesC = (Cc + 31) / 32;
  const long tr = blockIdx.x / tilesC, tc = blockIdx.x - tr * tilesC;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const long r = tr * 32 + k, c = tc * 32 + tx;
    t[k][tx] = (r < R && c < Cc) ? src[r * Cc + c] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const long c = tc * 32 + k, r = tr * 32 + tx;
    if (r < R && c < Cc) dst[c * R + r] = t[tx][k];
  }
}

// Tph[j][a][k][c] = tau^{ac}_{jk} over every ordered occupied pair (0 for j == k)
__global__ void k_build_tph(const double2* __restrict__ tau, int o, int nv, double2* __restrict__ Tph) {
  const long nv2 = (long)nv * nv, total = (long)o * nv * o * nv;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const int c = (int)(e % nv);
    long r = e / nv;
    const int k = (int)(r % o);
    r /= o;
    const int a = (int)(r % nv), j = (int)(r / nv);
    Tph[e] = tau_at(tau, j, k, o, nv2, (long)a * nv + c);
  }
}

// G[p][(I, j)] = <kl||Ij> = sum_P (L^P_kI L^P_lj - L^P_kj L^P_lI) for the pair p = (k < l)
__global__ void k_oooo(const double2* __restrict__ Loo, int naux, int o, int nc, const int2* __restrict__ pairs,
                       int npairs, double2* __restrict__ G) {
  const long total = (long)npairs * nc * o;
  const long oo = (long)o * o;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const int j = (int)(e % o);
    const long t = e / o;
    const int I = (int)(t % nc), p = (int)(t / nc);
    const int k = pairs[p].x, l = pairs[p].y;
    double2 acc = make_double2(0.0, 0.0);
    for (int P = 0; P < naux; ++P) {
      const double2* L = Loo + (long)P * oo;
      const double2 x = cmul(L[(long)k * o + I], L[(long)l * o + j]);
      const double2 y = cmul(L[(long)k * o + j], L[(long)l * o + I]);
      acc.x += x.x - y.x;
      acc.y += x.y - y.y;
    }
    G[e] = acc;
  }
}

// dst[e] += alpha * sum_s part[s][e], e < n
__global__ void k_sum_parts(const double2* __restrict__ part, int nsplit, long n, double alpha,
                            double2* __restrict__ dst) {
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
    double2 a = make_double2(0.0, 0.0);
    for (int q = 0; q < nsplit; ++q) a = cadd(a, part[(long)q * n + e]);
    dst[e].x += alpha * a.x;
    dst[e].y += alpha * a.y;
  }
}

// Nt[j][a][b] += R[a][j][b] - R[b][j][a] - Rp[j][a][b] + Rp[j][b][a]  (one core I)
__global__ void k_ring_add(const double2* __restrict__ R, const double2* __restrict__ Rp, int o, int nv,
                           double2* __restrict__ Nt) {
  const long nv2 = (long)nv * nv, total = (long)o * nv2, onv = (long)o * nv;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const int b = (int)(e % nv);
    const long r = e / nv;
    const int a = (int)(r % nv), j = (int)(r / nv);
    const double2 x1 = R[(long)a * onv + (long)j * nv + b], x2 = R[(long)b * onv + (long)j * nv + a];
    const double2 y1 = Rp[((long)j * nv + a) * nv + b], y2 = Rp[((long)j * nv + b) * nv + a];
    Nt[e].x += x1.x - x2.x - y1.x + y2.x;
    Nt[e].y += x1.y - x2.y - y1.y + y2.y;
  }
}

// u[I][j][a][b] = Nt / (e_a + e_b - e_I - e_j), 0 for j == I
__global__ void k_u_divide(double2* __restrict__ Nt, const double* __restrict__ eps, int nc, int o, int nv) {
  const long nv2 = (long)nv * nv, total = (long)nc * o * nv2;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const int b = (int)(e % nv);
    const long r = e / nv;
    const int a = (int)(r % nv);
    const long q = r / nv;
    const int j = (int)(q % o), I = (int)(q / o);
    if (j == I) {
      Nt[e] = make_double2(0.0, 0.0);
      continue;
    }
    const double w = 1.0 / (eps[o + a] + eps[o + b] - eps[I] - eps[j]);
    Nt[e].x *= w;
    Nt[e].y *= w;
  }
}

// s[i][a] = (N1[i][a] - N2T[a][i]) / (e_a - e_i)
__global__ void k_singles_amp(const double2* __restrict__ N1, const double2* __restrict__ N2T,
                              const double* __restrict__ eps, int o, int nv, double2* __restrict__ s) {
  const long total = (long)o * nv;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const int a = (int)(e % nv), i = (int)(e / nv);
    const double w = 1.0 / (eps[o + a] - eps[i]);
    const double2 x = N1[e], y = N2T[(long)a * o + i];
    s[e] = make_double2((x.x - y.x) * w, (x.y - y.y) * w);
  }
}

// wdc[comp][(k, c)] = d^comp_{ck}
__global__ void k_dvo_rows(const double2* __restrict__ dip, int o, int nv, int n, double2* __restrict__ wdc) {
  const long onv = (long)o * nv, total = 3 * onv;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const int comp = (int)(e / onv);
    const long r = e - comp * onv;
    const int k = (int)(r / nv), c = (int)(r % nv);
    wdc[e] = dip[(long)comp * n * n + (long)(o + c) * n + k];
  }
}

// F2 of one (component, I, a), added to the singles row of F; one workgroup each
__global__ __launch_bounds__(256) void k_f2_assemble(const double2* __restrict__ u, const double2* __restrict__ sa,
                                                      const double2* __restrict__ rho,
                                                      const double2* __restrict__ sig,
                                                      const double2* __restrict__ f2p,
                                                      const double2* __restrict__ dip, int nc, int o, int nv, int n,
                                                      long dim, double2* __restrict__ F) {
  __shared__ double2 red[256];
  const int blk = blockIdx.x;
  const int comp = blk / (nc * nv), r = blk - comp * nc * nv;
  const int I = r / nv, a = r - I * nv;
  const long nv2 = (long)nv * nv;
  const double2* d = dip + (long)comp * n * n;
  double2 acc = make_double2(0.0, 0.0);
  // sum_{jb} d_jb u^{ab}_{Ij}
  for (long e = threadIdx.x; e < (long)o * nv; e += 256) {
    const int j = (int)(e / nv), b = (int)(e - (long)j * nv);
    acc = cadd(acc, cmul(d[(long)j * n + o + b], u[((long)I * o + j) * nv2 + (long)a * nv + b]));
  }
  // sum_b d_ab s_Ib - 1/4 sum_c rho_ac d_cI
  for (int b = threadIdx.x; b < nv; b += 256) {
    acc = cadd(acc, cmul(d[(long)(o + a) * n + o + b], sa[(long)I * nv + b]));
    const double2 t = cmul(rho[(long)a * nv + b], d[(long)(o + b) * n + I]);
    acc.x -= 0.25 * t.x;
    acc.y -= 0.25 * t.y;
  }
  // - sum_j d_jI s_ja - 1/4 sum_k d_ak sigma_Ik
  for (int j = threadIdx.x; j < o; j += 256) {
    const double2 t = cmul(d[(long)j * n + I], sa[(long)j * nv + a]);
    const double2 q = cmul(d[(long)(o + a) * n + j], sig[(long)I * o + j]);
    acc.x -= t.x + 0.25 * q.x;
    acc.y -= t.y + 0.25 * q.y;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double2 t = f2p[((long)I * nv + a) * 3 + comp];
    double2* out = F + (long)comp * dim + (long)I * nv + a;
    out->x += red[0].x + t.x;
    out->y += red[0].y + t.y;
  }
}

// part[sl][I][k] = sum over slice sl of e < K of Tph[I][e] conj(Tph[k][e]) (rows of length K);
// grid (o, nsl), one workgroup per (k, slice)
__global__ __launch_bounds__(256) void k_sigma_part(const double2* __restrict__ Tph, long K, int nc, int o, int nsl,
                                                     double2* __restrict__ part) {
  __shared__ double2 red[8][256];
  const int k = blockIdx.x, sl = blockIdx.y;
  const long per = (K + nsl - 1) / nsl;
  const long e0 = (long)sl * per, e1 = e0 + per < K ? e0 + per : K;
  const double2* rk = Tph + (long)k * K;
  for (int I0 = 0; I0 < nc; I0 += 8) {
    double2 acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = make_double2(0.0, 0.0);
    for (long e = e0 + threadIdx.x; e < e1; e += 256) {
      const double2 v = rk[e];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (I0 + q >= nc) break;
        const double2 u = Tph[(long)(I0 + q) * K + e];
        acc[q].x += u.x * v.x + u.y * v.y;   // u conj(v)
        acc[q].y += u.y * v.x - u.x * v.y;
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st)
#pragma unroll
        for (int q = 0; q < 8; ++q) red[q][threadIdx.x] = cadd(red[q][threadIdx.x], red[q][threadIdx.x + st]);
      __syncthreads();
    }
    if (threadIdx.x < 8 && I0 + (int)threadIdx.x < nc)
      part[((long)sl * nc + I0 + threadIdx.x) * o + k] = red[threadIdx.x][0];
    __syncthreads();
  }
}

// dst[e] = conj(src[e])
__global__ void k_conj(const double2* __restrict__ src, long n, double2* __restrict__ dst) {
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
    const double2 v = src[e];
    dst[e] = make_double2(v.x, -v.y);
  }
}

unsigned grid_for(long n) { return (unsigned)std::max<long>(1, std::min<long>(8192, (n + 255) / 256)); }

adc2_status tfail(adc2_status s, const std::string& m) {
  set_error("adc2_transition: " + m);
  return s;
}

}  // namespace

// Second-order singles F2 of the three components, added to the singles rows
// of F (expressions in the file header).  tau: the pair amplitudes of every
// occupied pair (k < l) in row-major pair order, dpairs their (k, l) list.
// Work space (freed here): Tph and (kj|bc) twice, o^2 nv^2 complex each, the
// Lvv transpose naux nv^2, two (ac|bd) blocks of up to 32 a-values (each at
// most 16 GiB), the pair amplitudes and u of the pairs (I, j), nc o nv^2 each.
adc2_status tm_second_order(adc2_handle h, const double2* tau, const int2* dpairs, int npairs,
                            const double2* dip, double2* F, hipStream_t st) {
  const Dims& d = h->d;
  const int nc = d.nc, o = d.o, nv = d.nv, n = d.n, naux = d.naux;
  const long nv2 = (long)nv * nv, onv = (long)o * nv, dim = d.dim;
  std::vector<void*> bufs;
  auto release = [&]() {
    hipStreamSynchronize(st);
    for (void* q : bufs) dfree(h, q);
    bufs.clear();
  };
  auto alloc = [&](double2** q, long count) -> adc2_status {
    const hipError_t e = dmalloc(h, (void**)q, sizeof(double2) * std::max<long>(count, 1));
    if (e != hipSuccess) {
      set_error(std::string("adc2_transition: hipMalloc: ") + hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? ADC2_ERR_OOM : ADC2_ERR_HIP;
    }
    bufs.push_back(*q);
    return ADC2_OK;
  };
  auto drop = [&](double2* q) {   // free one buffer early (after the stream has finished with it)
    hipStreamSynchronize(st);
    dfree(h, q);
    bufs.erase(std::remove(bufs.begin(), bufs.end(), (void*)q), bufs.end());
  };
  auto launched = [&](const char* what) -> adc2_status {
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return ADC2_OK;
    set_error(std::string("adc2_transition: ") + what + ": " + hipGetErrorString(e));
    return ADC2_ERR_HIP;
  };
  auto hip_ok = [&](hipError_t e) -> adc2_status {
    if (e == hipSuccess) return ADC2_OK;
    set_error(std::string("adc2_transition: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? ADC2_ERR_OOM : ADC2_ERR_HIP;
  };
#define T2_TRY(x)                    \
  do {                               \
    const adc2_status r_ = (x);      \
    if (r_ != ADC2_OK) {             \
      release();                     \
      return r_;                     \
    }                                \
  } while (0)

  // tau over every ordered pair, [j][a][k][c]
  double2 *Tph, *LovP, *ZT;
  T2_TRY(alloc(&Tph, onv * onv));
  k_build_tph<<<grid_for(onv * onv), 256, 0, st>>>(tau, o, nv, Tph);
  T2_TRY(launched("k_build_tph"));
  // Z^P_ib at ZT[i][b][P] = sum_{(j,c)} Tph[i][b][(j,c)] L^P_jc, L^P_jc = conj(Lvo[j][P][c]) at LovP[P][(j,c)]
  T2_TRY(alloc(&LovP, (long)naux * onv));
  T2_TRY(alloc(&ZT, onv * naux));
  k_swap12<true><<<grid_for((long)naux * onv), 256, 0, st>>>(h->Lvo, o, naux, nv, LovP);
  T2_TRY(launched("k_swap12"));
  T2_TRY(gemm_rr((int)onv, naux, (int)onv, Tph, onv, false, LovP, onv, false, ZT, naux, 1.0, false, st));
  drop(LovP);
  // second-order singles amplitudes
  double2 *LvvT, *N1, *ZA, *LooK, *N2T, *sa;
  T2_TRY(alloc(&LvvT, nv2 * naux));      // [a][b][P] = L^P_ab
  T2_TRY(alloc(&N1, onv));
  T2_TRY(alloc(&ZA, onv * naux));
  T2_TRY(alloc(&LooK, (long)o * o * naux));   // [k][j][P] = L^P_kj
  T2_TRY(alloc(&N2T, onv));
  T2_TRY(alloc(&sa, onv));
  const long lvv_tiles = ((naux + 31) / 32) * ((nv2 + 31) / 32);
  k_transpose<<<(unsigned)lvv_tiles, 256, 0, st>>>(h->Lvv, naux, nv2, LvvT);
  T2_TRY(launched("k_transpose"));
  const long loo_tiles = ((naux + 31) / 32) * (((long)o * o + 31) / 32);
  k_transpose<<<(unsigned)loo_tiles, 256, 0, st>>>(h->Loo, naux, (long)o * o, LooK);
  T2_TRY(launched("k_transpose"));
  T2_TRY(gemm_rr(o, nv, (int)(nv * (long)naux), ZT, nv * (long)naux, false, LvvT, nv * (long)naux, false, N1, nv,
                 1.0, false, st));
  k_swap12<false><<<grid_for(onv * naux), 256, 0, st>>>(ZT, o, nv, naux, ZA);
  T2_TRY(launched("k_swap12"));
  T2_TRY(gemm_rr(nv, o, (int)((long)o * naux), ZA, (long)o * naux, false, LooK, (long)o * naux, true, N2T, o, 1.0,
                 false, st));
  k_singles_amp<<<grid_for(onv), 256, 0, st>>>(N1, N2T, h->eps, o, nv, sa);
  T2_TRY(launched("k_singles_amp"));
  drop(ZA);
  drop(N1);
  drop(N2T);
  // (kj|bc) at P1[(j,b)][(k,c)]
  double2 *Koovv, *P1;
  T2_TRY(alloc(&Koovv, (long)o * o * nv2));
  T2_TRY(gemm_rr(o * o, (int)nv2, naux, LooK, naux, false, LvvT, naux, false, Koovv, nv2, 1.0, false, st));
  drop(LvvT);
  drop(LooK);
  T2_TRY(alloc(&P1, (long)o * o * nv2));
  k_swap12<false><<<grid_for((long)o * o * nv2), 256, 0, st>>>(Koovv, o, onv, nv, P1);
  T2_TRY(launched("k_swap12"));
  drop(Koovv);
  // numerators of u for the pairs (I, j): hole ladder first (it writes Nt)
  double2 *Nt, *G;
  T2_TRY(alloc(&Nt, (long)nc * o * nv2));
  T2_TRY(alloc(&G, (long)npairs * nc * o));
  k_oooo<<<grid_for((long)npairs * nc * o), 256, 0, st>>>(h->Loo, naux, o, nc, dpairs, npairs, G);
  T2_TRY(launched("k_oooo"));
  T2_TRY(bgemm_kmajor(G, 0, (long)nc * o, nc * o, tau, 0, nv2, (int)nv2, nc * o, (int)nv2, npairs, 1, Nt, st));
  drop(G);
  // ring terms, one core I at a time
  double2 *R, *Rp;
  T2_TRY(alloc(&R, nv * onv));
  T2_TRY(alloc(&Rp, onv * nv));
  for (int I = 0; I < nc; ++I) {
    T2_TRY(gemm_rr(nv, (int)onv, naux, ZT + (long)I * nv * naux, naux, false, h->LoT, naux, true, R, onv, 1.0, false,
                   st));
    T2_TRY(gemm_rr(nv, (int)onv, (int)onv, Tph + (long)I * nv * onv, onv, false, P1, onv, false, R, onv, -1.0, true,
                   st));
    T2_TRY(gemm_rr((int)onv, nv, naux, ZT, naux, false, h->LoT + (long)I * nv * naux, naux, true, Rp, nv, 1.0, false,
                   st));
    T2_TRY(gemm_rr((int)onv, nv, (int)onv, Tph, onv, false, P1 + (long)I * nv * onv, onv, false, Rp, nv, -1.0, true,
                   st));
    k_ring_add<<<grid_for((long)o * nv2), 256, 0, st>>>(R, Rp, o, nv, Nt + (long)I * o * nv2);
    T2_TRY(launched("k_ring_add"));
  }
  drop(R);
  drop(Rp);
  drop(P1);
  drop(ZT);
  // particle ladder sum_{c,d} (ac|bd) tau^{cd}_{Ij} for every pair (I, j), in blocks of ab a-values:
  //   V[(a,c)][(b,d)] = sum_P L^P_ac L^P_bd   (K-major GEMM over P)
  //   W[a][b][(c,d)]  = V[a][c][b][d]          (per-a swap of c and b)
  //   Nt[(I,j)][a][b] += sum_{(c,d)} tau^{cd}_{Ij} W[(a,b)][(c,d)]
  // with the signed amplitudes of the pairs (I, j) gathered as TIj[(I,j)][(c,d)] from Tph.
  {
    double2 *TIj, *V, *W;
    // a-values per block: up to 32, each of V and W under 16 GiB
    const long per_a = (long)nv * nv2 * (long)sizeof(double2);
    const int ab = (int)std::max<long>(1, std::min<long>(std::min(nv, 32), (16L << 30) / per_a));
    T2_TRY(alloc(&TIj, (long)nc * o * nv2));
    for (int I = 0; I < nc; ++I) {
      k_swap12<false><<<grid_for(onv * nv), 256, 0, st>>>(Tph + (long)I * nv * onv, nv, o, nv,
                                                          TIj + (long)I * o * nv2);
      T2_TRY(launched("k_swap12"));
    }
    T2_TRY(alloc(&V, (long)ab * nv * nv2));
    T2_TRY(alloc(&W, (long)ab * nv * nv2));
    for (int a0 = 0; a0 < nv; a0 += ab) {
      const int na = std::min(ab, nv - a0);
      T2_TRY(bgemm_kmajor(h->Lvv + (long)a0 * nv, 0, nv2, na * nv, h->Lvv, 0, nv2, (int)nv2, na * nv, (int)nv2, naux,
                          1, V, st));
      k_swap12<false><<<grid_for((long)na * nv * nv2), 256, 0, st>>>(V, (long)na * nv, nv, nv, W);
      T2_TRY(launched("k_swap12"));
      // W as [a][c][b][d] -> [a][b][c][d]: the swap above exchanged (a,c) with b; restore a as the outer index
      k_swap12<false><<<grid_for((long)na * nv * nv2), 256, 0, st>>>(W, nv, na, nv * (long)nv, V);
      T2_TRY(launched("k_swap12"));
      T2_TRY(gemm_rr(nc * o, na * nv, (int)nv2, TIj, nv2, false, V, nv2, false, Nt + (long)a0 * nv, nv2, 1.0, true,
                     st));
    }
    drop(TIj);
    drop(V);
    drop(W);
  }
  k_u_divide<<<grid_for((long)nc * o * nv2), 256, 0, st>>>(Nt, h->eps, nc, o, nv);
  T2_TRY(launched("k_u_divide"));
  // pair densities and the particle-hole term
  double2 *rho, *sig, *wdc, *hb, *f2p;
  T2_TRY(alloc(&rho, nv2));
  T2_TRY(alloc(&sig, (long)nc * o));
  T2_TRY(alloc(&wdc, 3 * onv));
  T2_TRY(alloc(&hb, 3 * onv));
  T2_TRY(alloc(&f2p, (long)nc * nv * 3));
  {
    // rho_ac = 2 sum_{(p, b)} tau_p[b][a] conj(tau_p[b][c]) over the pairs p = (k < l): split-K GEMM of
    // the K-major rows (p, b) against their conjugate
    double2 *tc, *rpart;
    const long Kr = (long)npairs * nv;
    const int nsr = (int)std::max<long>(1, std::min<long>(std::max(1, 1024 / (((nv + 127) / 128) * ((nv + 127) / 128))),
                                                          Kr / 256));
    T2_TRY(alloc(&tc, (long)npairs * nv2));
    T2_TRY(alloc(&rpart, (long)nsr * nv2));
    k_conj<<<grid_for((long)npairs * nv2), 256, 0, st>>>(tau, (long)npairs * nv2, tc);
    T2_TRY(launched("k_conj"));
    T2_TRY(bgemm_kmajor(tau, 0, nv, nv, tc, 0, nv, nv, nv, nv, (int)Kr, nsr, rpart, st));
    T2_TRY(hip_ok(hipMemsetAsync(rho, 0, sizeof(double2) * nv2, st)));
    k_sum_parts<<<grid_for(nv2), 256, 0, st>>>(rpart, nsr, nv2, 2.0, rho);
    T2_TRY(launched("k_sum_parts"));
    drop(tc);
    drop(rpart);
    // sigma_Ik over slices of the rows of Tph
    double2* spart;
    const long Ks = nv * onv;
    const int nsl = (int)std::max<long>(1, std::min<long>(64, Ks / 4096));
    T2_TRY(alloc(&spart, (long)nsl * nc * o));
    k_sigma_part<<<dim3(o, nsl), 256, 0, st>>>(Tph, Ks, nc, o, nsl, spart);
    T2_TRY(launched("k_sigma_part"));
    T2_TRY(hip_ok(hipMemsetAsync(sig, 0, sizeof(double2) * nc * o, st)));
    k_sum_parts<<<grid_for((long)nc * o), 256, 0, st>>>(spart, nsl, (long)nc * o, 1.0, sig);
    T2_TRY(launched("k_sum_parts"));
    drop(spart);
  }
  k_dvo_rows<<<grid_for(3 * onv), 256, 0, st>>>(dip, o, nv, n, wdc);
  T2_TRY(launched("k_dvo_rows"));
  T2_TRY(gemm_rr(3, (int)onv, (int)onv, wdc, onv, false, Tph, onv, true, hb, onv, 1.0, false, st));
  T2_TRY(gemm_rr(nc * nv, 3, (int)onv, Tph, onv, false, hb, onv, false, f2p, 3, 0.5, false, st));
  k_f2_assemble<<<(unsigned)(3 * nc * nv), 256, 0, st>>>(Nt, sa, rho, sig, f2p, dip, nc, o, nv, n, dim, F);
  T2_TRY(launched("k_f2_assemble"));
  release();
#undef T2_TRY
  return ADC2_OK;
}
}  // namespace adc2

using namespace adc2;

extern "C" ADC2_API adc2_status adc2_transition(adc2_handle h, const void* dip, int nroots, const void* X,
                                                const double* omega, int order, void* T, double* f, void* stream) {
  if (!h || !dip || !X || !omega || !T || !f) return tfail(ADC2_ERR_ARG, "NULL argument");
  if (order != 1 && order != 2) return tfail(ADC2_ERR_ARG, "order must be 1 or 2");
  if (nroots < 1 || nroots > ADC2_MAX_ROOTS) return tfail(ADC2_ERR_ARG, "nroots must be in 1..ADC2_MAX_ROOTS");
  hipStream_t st = (hipStream_t)stream;
  const Dims& d = h->d;
  const int nc = d.nc, no = d.no, nv = d.nv, o = d.o, n = d.n;
  const long nv2 = (long)nv * nv, dim = d.dim, ns = d.ns;
  std::vector<int2> pairs;
  for (int k = 0; k < o; ++k)
    for (int l = k + 1; l < o; ++l) pairs.push_back(make_int2(k, l));
  const int npairs = (int)pairs.size();
  int2* dpairs = nullptr;
  double2 *tau = nullptr, *F = nullptr, *Ab = nullptr, *G = nullptr, *scr = nullptr;
  adc2_status rc = ADC2_OK;
  std::string msg;
  auto hip = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && rc == ADC2_OK) {
      rc = e == hipErrorOutOfMemory ? ADC2_ERR_OOM : ADC2_ERR_HIP;
      msg = std::string(what) + ": " + hipGetErrorString(e);
    }
    return rc == ADC2_OK;
  };
  auto status = [&](adc2_status r) {
    if (r != ADC2_OK && rc == ADC2_OK) {
      rc = r;
      msg = adc2_last_error();
    }
    return rc == ADC2_OK;
  };
  const int nblk = dav_nblk(dim);
  const int ntile = ((nroots + 15) / 16) * 1;
  hip(dmalloc(h, &F, sizeof(double2) * 3 * dim), "hipMalloc");
  if (npairs > 0) {
    hip(dmalloc(h, &tau, sizeof(double2) * npairs * nv2), "hipMalloc");
    hip(dmalloc(h, &dpairs, sizeof(int2) * npairs), "hipMalloc");
  }
  hip(dmalloc(h, &Ab, sizeof(double2) * nv * (long)no * nv), "hipMalloc");
  hip(dmalloc(h, &G, sizeof(double2) * nroots * 3), "hipMalloc");
  hip(dmalloc(h, &scr, sizeof(double2) * 256 * (long)nblk * ntile), "hipMalloc");
  if (rc == ADC2_OK && npairs > 0) {
    hip(hipMemcpyAsync(dpairs, pairs.data(), sizeof(int2) * npairs, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    if (status(wbuild(h, tau, st))) status(tau_from_w(tau, dpairs, npairs, h->eps, o, nv, st));
  } else if (rc == ADC2_OK) {
    hip(hipMemsetAsync(F, 0, sizeof(double2) * 3 * dim, st), "hipMemsetAsync");
  }
  const double2* dp = (const double2*)dip;
  if (rc == ADC2_OK && npairs > 0) {
    k_tm_singles<<<(unsigned)(3 * nc * nv), 256, 0, st>>>(tau, dp, nc, o, nv, n, dim, F);
    hip(hipGetLastError(), "k_tm_singles");
  }
  if (rc == ADC2_OK && npairs > 0 && order == 2) status(tm_second_order(h, tau, dpairs, npairs, dp, F, st));
  const unsigned gd = (unsigned)std::min<long>(4096, (nv2 + 255) / 256);
  const long lda = (long)no * nv;
  for (int c = 0; c < 3 && rc == ADC2_OK && npairs > 0; ++c) {
    const double2* dc = dp + (long)c * n * n;
    for (int I = 0; I < nc && rc == ADC2_OK; ++I) {
      // the pairs (I, j) of the valence j > I follow each other in pair order:
      // Ab[a][(j', b)] = sum_c d_ac tau^{cb}_{Ij} for all of them in one GEMM
      // (B given transposed: tau_Ij^T = -tau_Ij)
      const double2* tI = tau + ((long)I * o - (long)I * (I + 1) / 2 + (nc - I - 1)) * nv2;
      if (!status(gemm_rr(nv, (int)lda, nv, dc + (long)o * n + o, n, false, tI, nv, false, Ab, lda, -1.0, false,
                          st)))
        break;
      k_tm_doubles<<<dim3(gd, no), 256, 0, st>>>(Ab, lda, tau, dc, I, nc, o, nv, n, d.npair,
                                                 F + (long)c * dim + ns + (long)I * no * d.npair);
      hip(hipGetLastError(), "k_tm_doubles");
    }
  }
  // T[k][c] = X_k^H F_c
  if (rc == ADC2_OK) status(dav_gram((const double2*)X, nroots, F, 3, dim, G, 3, scr, st));
  std::vector<double2> hT(nroots * 3);
  if (rc == ADC2_OK) hip(hipMemcpyAsync(hT.data(), G, sizeof(double2) * nroots * 3, hipMemcpyDeviceToHost, st),
                         "hipMemcpyAsync");
  if (hipStreamSynchronize(st) != hipSuccess && rc == ADC2_OK) {
    rc = ADC2_ERR_HIP;
    msg = "hipStreamSynchronize";
  }
  dfree(h, F);
  dfree(h, tau);
  dfree(h, dpairs);
  dfree(h, Ab);
  dfree(h, G);
  dfree(h, scr);
  if (rc != ADC2_OK) return tfail(rc, msg);
  double2* To = (double2*)T;
  for (int k = 0; k < nroots; ++k) {
    double s2 = 0.0;
    for (int c = 0; c < 3; ++c) {
      To[k * 3 + c] = hT[k * 3 + c];
      s2 += hT[k * 3 + c].x * hT[k * 3 + c].x + hT[k * 3 + c].y * hT[k * 3 + c].y;
    }
    f[k] = (2.0 / 3.0) * omega[k] * s2;
  }
  return ADC2_OK;
}
