// transition.hip -- modified transition moments and oscillator strengths
// (paper, Theory section, transition properties): T_n = X_n^H F with
// F_I = <Psi~_I| D |Psi0> for the three Cartesian components of a dipole
// operator D = sum_pq d_pq a+_p a_q, and f_n = (2/3) omega_n |T_n|^2.
//
// F is built through first order in the Moller-Plesset expansion:
//   singles (I, a):  F = d_aI - sum_{j in O, b} tau^{ab}_{Ij} d_jb
//   doubles (I, j, a<b) in the basis a+_a a+_b a_j a_I |Phi0>:
//     F = -[ (d_vv tau_Ij - (d_vv tau_Ij)^T)_{ab}
//            - sum_{k in O} (d_kI tau^{ab}_{kj} + d_kj tau^{ab}_{Ik}) ]
// (tau_Ij antisymmetric, so tau_Ij d_vv^T = -(d_vv tau_Ij)^T), with the MP2
// amplitudes tau of every occupied pair from the setup's W-build.  The
// second-order terms of F are not included.
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

// doubles of one (component, I, j): A = d_vv tau_Ij, out = F block of (I, j), a < b packed
__global__ __launch_bounds__(256) void k_tm_doubles(const double2* __restrict__ A, const double2* __restrict__ tau,
                                                     const double2* __restrict__ d, int I, int jg, int o, int nv,
                                                     int n, double2* __restrict__ out) {
  const long nv2 = (long)nv * nv;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < nv2; e += (long)gridDim.x * 256) {
    const int a = (int)(e / nv), b = (int)(e - (long)a * nv);
    if (a >= b) continue;
    const long ab = (long)a * nv + b;
    const double2 x = A[ab], y = A[(long)b * nv + a];
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

adc2_status tfail(adc2_status s, const std::string& m) {
  set_error("adc2_transition: " + m);
  return s;
}

}  // namespace
}  // namespace adc2

using namespace adc2;

extern "C" ADC2_API adc2_status adc2_transition(adc2_handle h, const void* dip, int nroots, const void* X,
                                                const double* omega, void* T, double* f, void* stream) {
  if (!h || !dip || !X || !omega || !T || !f) return tfail(ADC2_ERR_ARG, "NULL argument");
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
  hip(hipMalloc(&F, sizeof(double2) * 3 * dim), "hipMalloc");
  if (npairs > 0) {
    hip(hipMalloc(&tau, sizeof(double2) * npairs * nv2), "hipMalloc");
    hip(hipMalloc(&dpairs, sizeof(int2) * npairs), "hipMalloc");
  }
  hip(hipMalloc(&Ab, sizeof(double2) * nv2), "hipMalloc");
  hip(hipMalloc(&G, sizeof(double2) * nroots * 3), "hipMalloc");
  hip(hipMalloc(&scr, sizeof(double2) * 256 * (long)nblk * ntile), "hipMalloc");
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
  const unsigned gd = (unsigned)std::min<long>(4096, (nv2 + 255) / 256);
  for (int c = 0; c < 3 && rc == ADC2_OK && npairs > 0; ++c) {
    const double2* dc = dp + (long)c * n * n;
    for (int I = 0; I < nc && rc == ADC2_OK; ++I)
      for (int j = 0; j < no && rc == ADC2_OK; ++j) {
        const int jg = nc + j;
        const double2* tIj = tau + ((long)I * o - (long)I * (I + 1) / 2 + (jg - I - 1)) * nv2;
        // A = d_vv tau_Ij  (B given transposed: tau_Ij^T = -tau_Ij)
        if (!status(gemm_rr(nv, nv, nv, dc + (long)o * n + o, n, false, tIj, nv, false, Ab, nv, -1.0, false, st)))
          break;
        k_tm_doubles<<<gd, 256, 0, st>>>(Ab, tau, dc, I, jg, o, nv, n,
                                         F + (long)c * dim + ns + ((long)I * no + j) * d.npair);
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
  hipFree(F);
  hipFree(tau);
  hipFree(dpairs);
  hipFree(Ab);
  hipFree(G);
  hipFree(scr);
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
