// fns.hip -- frozen natural virtual spinors from the MP2 density
// (paper, State-Average Frozen Natural Spinors: Eq. 15 and the steps of
// Eq. 17-20).
//
//   D_ab = 1/2 sum_{c,i,j} <ac||ij><ij||bc> / (e^{ac}_{ij} e^{bc}_{ij})
//        = sum_{i<j} sum_c tau^{ij}_{ac} conj(tau^{ij}_{bc}),   tau = W / D,
// built from the same W-build as the setup (occupied pairs in chunks of at
// most 2 GiB), one Hermitian rank-nv product per pair on the FP64 matrix
// cores.  The small eigenproblems (D V = V n; the kept block of the virtual
// Fock matrix) run on the host; the Cholesky vectors are rotated on the GPU,
// L'^P = W^H L^P W with W = blockdiag(1_o, U), U = V~ Z~.
//
// The state-averaged CIS(D) densities of Eq. 16 are not included (their
// expressions are not in the paper); D is the MP2 term alone.
#include <algorithm>
#include <string>
#include <vector>

#include "hostla.h"
#include "internal.h"
#include "tile.h"

namespace adc2 {
namespace {

// W[t][a][c] /= e_a + e_c - e_k - e_l for the pairs (k, l) of the chunk
__global__ void k_tau(double2* __restrict__ W, const int2* __restrict__ pairs, int npairs,
                      const double* __restrict__ eps, int o, int nv) {
  const long nv2 = (long)nv * nv, total = (long)npairs * nv2;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int t = (int)(e / nv2);
    const long r = e - t * nv2;
    const int a = (int)(r / nv), c = (int)(r - (long)a * nv);
    const int2 kl = pairs[t];
    const double D = eps[o + a] + eps[o + c] - eps[kl.x] - eps[kl.y];
    const double2 w = W[e];
    W[e] = make_double2(w.x / D, w.y / D);
  }
}

}  // namespace

// W[t][a][c] -> tau = W / (e_a + e_c - e_k - e_l) in place for the device
// pair list (k, l) of t < npairs
adc2_status tau_from_w(double2* W, const int2* dpairs, int npairs, const double* eps, int o, int nv, hipStream_t st) {
  const long tot = (long)npairs * nv * nv;
  if (tot == 0) return ADC2_OK;
  k_tau<<<(unsigned)std::min<long>(16384, (tot + 255) / 256), 256, 0, st>>>(W, dpairs, npairs, eps, o, nv);
  ADC2_CHECK_LAUNCH();
  return ADC2_OK;
}

namespace {

adc2_status ffail(adc2_status s, const std::string& m) {
  set_error("adc2_fns: " + m);
  return s;
}

}  // namespace
}  // namespace adc2

using namespace adc2;

extern "C" ADC2_API adc2_status adc2_fns(adc2_handle h, const void* L, double threshold, int* nv_out, double* occ,
                                         void* L_out, double* eps_out, void* stream) {
  if (!h || !nv_out) return ffail(ADC2_ERR_ARG, "NULL handle or nv_out");
  if ((L_out == nullptr) != (eps_out == nullptr)) return ffail(ADC2_ERR_ARG, "L_out and eps_out go together");
  if (L_out && !L) return ffail(ADC2_ERR_ARG, "L is NULL");
  *nv_out = 0;
  hipStream_t st = (hipStream_t)stream;
  const Dims& d = h->d;
  const int o = d.o, nv = d.nv, n = d.n;
  const long nv2 = (long)nv * nv;
  std::vector<int2> pairs;
  for (int k = 0; k < o; ++k)
    for (int l = k + 1; l < o; ++l) pairs.push_back(make_int2(k, l));
  const int npairs = (int)pairs.size();
  const int chunk = (int)std::max<long>(1, std::min<long>(npairs, (2L << 30) / (nv2 * (long)sizeof(double2))));
  const int nb = (nv + TM - 1) / TM;

  int2* dpairs = nullptr;
  double2 *Wc = nullptr, *Dd = nullptr, *WT = nullptr, *YT = nullptr;
  double* epart = nullptr;
  adc2_status rc = ADC2_OK;
  std::string msg;
  auto hip = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && rc == ADC2_OK) {
      rc = e == hipErrorOutOfMemory ? ADC2_ERR_OOM : ADC2_ERR_HIP;
      msg = std::string(what) + ": " + hipGetErrorString(e);
    }
    return rc == ADC2_OK;
  };
  auto cleanup = [&]() {
    dfree(h, dpairs);
    dfree(h, Wc);
    dfree(h, Dd);
    dfree(h, WT);
    dfree(h, YT);
    dfree(h, epart);
  };

  // ---- D (Eq. 15) ----
  hip(dmalloc(h, &Dd, sizeof(double2) * nv2), "hipMalloc");
  if (rc == ADC2_OK) hip(hipMemsetAsync(Dd, 0, sizeof(double2) * nv2, st), "hipMemsetAsync");
  if (npairs > 0 && rc == ADC2_OK) {
    hip(dmalloc(h, &dpairs, sizeof(int2) * npairs), "hipMalloc");
    if (rc == ADC2_OK) hip(dmalloc(h, &Wc, sizeof(double2) * chunk * nv2), "hipMalloc");
    if (rc == ADC2_OK) hip(dmalloc(h, &epart, sizeof(double) * (long)chunk * (nb * (nb + 1) / 2)), "hipMalloc");
    if (rc == ADC2_OK)
      hip(hipMemcpyAsync(dpairs, pairs.data(), sizeof(int2) * npairs, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    for (int p0 = 0; p0 < npairs && rc == ADC2_OK; p0 += chunk) {
      const int cnt = std::min(chunk, npairs - p0);
      if ((rc = wbuild_pairs(h, dpairs + p0, cnt, Wc, epart, st)) != ADC2_OK) {
        msg = adc2_last_error();
        break;
      }
      if ((rc = tau_from_w(Wc, dpairs + p0, cnt, h->eps, o, nv, st)) != ADC2_OK) {
        msg = adc2_last_error();
        break;
      }
      for (int t = 0; t < cnt && rc == ADC2_OK; ++t) {
        const double2* tp = Wc + (long)t * nv2;
        if ((rc = gemm_rr(nv, nv, nv, tp, nv, false, tp, nv, true, Dd, nv, 1.0, true, st)) != ADC2_OK)
          msg = adc2_last_error();
      }
    }
  }
  std::vector<hostla::cplx> D(nv2);
  if (rc == ADC2_OK) {
    hip(hipMemcpyAsync(D.data(), Dd, sizeof(double2) * nv2, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    hip(hipStreamSynchronize(st), "hipStreamSynchronize");
  }
  dfree(h, Wc);
  Wc = nullptr;
  if (rc != ADC2_OK) {
    cleanup();
    return ffail(rc, msg);
  }

  // ---- natural virtuals (Eq. 17), truncation, semicanonical block (Eq. 18-20) ----
  for (int a = 0; a < nv; ++a)
    for (int b = a; b < nv; ++b) {
      const hostla::cplx v = 0.5 * (D[(long)a * nv + b] + std::conj(D[(long)b * nv + a]));
      D[(long)a * nv + b] = v;
      D[(long)b * nv + a] = std::conj(v);
    }
  std::vector<double> w(nv);
  std::vector<hostla::cplx> V(nv2);
  if (hostla::herm_eig(nv, D.data(), w.data(), V.data()) != 0) {
    cleanup();
    return ffail(ADC2_ERR_NOCONV, "adc2_fns: the eigensolve of the virtual density did not converge");
  }
  // descending occupations
  std::vector<int> ord(nv);
  for (int i = 0; i < nv; ++i) ord[i] = nv - 1 - i;
  int keep = 0;
  for (int i = 0; i < nv; ++i) {
    if (occ) occ[i] = w[ord[i]];
    if (w[ord[i]] >= threshold) ++keep;
  }
  *nv_out = keep;
  if (!L_out) {
    cleanup();
    return ADC2_OK;
  }
  if (keep == 0) {
    cleanup();
    return ffail(ADC2_ERR_ARG, "no natural virtual spinor has an occupation above the threshold");
  }
  std::vector<double> ev(nv);
  hip(hipMemcpyAsync(ev.data(), h->eps + o, sizeof(double) * nv, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  hip(hipStreamSynchronize(st), "hipStreamSynchronize");
  // F_NS = V~^H diag(e_v) V~
  std::vector<hostla::cplx> F((size_t)keep * keep), Zt((size_t)keep * keep);
  for (int i = 0; i < keep; ++i)
    for (int j = 0; j < keep; ++j) {
      hostla::cplx acc = 0.0;
      for (int a = 0; a < nv; ++a) acc += std::conj(V[(long)a * nv + ord[i]]) * ev[a] * V[(long)a * nv + ord[j]];
      F[(size_t)i * keep + j] = acc;
    }
  for (int i = 0; i < keep; ++i)
    for (int j = i; j < keep; ++j) {
      const hostla::cplx v = 0.5 * (F[(size_t)i * keep + j] + std::conj(F[(size_t)j * keep + i]));
      F[(size_t)i * keep + j] = v;
      F[(size_t)j * keep + i] = std::conj(v);
    }
  std::vector<double> ep(keep);
  if (hostla::herm_eig(keep, F.data(), ep.data(), Zt.data()) != 0) {
    cleanup();
    return ffail(ADC2_ERR_NOCONV, "adc2_fns: the eigensolve of the kept Fock block did not converge");
  }
  // WT = W^T (n' x n, row-major), W = blockdiag(1_o, U), U = V~ Z~
  const int np = o + keep;
  std::vector<hostla::cplx> hWT((size_t)np * n, 0.0);
  for (int j = 0; j < o; ++j) hWT[(size_t)j * n + j] = 1.0;
  for (int j = 0; j < keep; ++j)
    for (int a = 0; a < nv; ++a) {
      hostla::cplx u = 0.0;
      for (int i = 0; i < keep; ++i) u += V[(long)a * nv + ord[i]] * Zt[(size_t)i * keep + j];
      hWT[(size_t)(o + j) * n + o + a] = u;
    }
  std::vector<double> he(np);
  hip(hipMemcpyAsync(he.data(), h->eps, sizeof(double) * o, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  hip(hipStreamSynchronize(st), "hipStreamSynchronize");
  for (int j = 0; j < keep; ++j) he[o + j] = ep[j];

  // ---- L'^P = W^H L^P W:  YT = W^T (L^P)^T,  L'^P = conj(W^T) YT^T ----
  if (rc == ADC2_OK) hip(dmalloc(h, &WT, sizeof(double2) * np * n), "hipMalloc");
  if (rc == ADC2_OK) hip(dmalloc(h, &YT, sizeof(double2) * np * n), "hipMalloc");
  if (rc == ADC2_OK)
    hip(hipMemcpyAsync(WT, hWT.data(), sizeof(double2) * np * n, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
  if (rc == ADC2_OK)
    hip(hipMemcpyAsync(eps_out, he.data(), sizeof(double) * np, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
  const double2* Lin = (const double2*)L;
  double2* Lo = (double2*)L_out;
  for (int P = 0; P < d.naux && rc == ADC2_OK; ++P) {
    if ((rc = gemm_rr(np, n, n, WT, n, false, Lin + (long)P * n * n, n, false, YT, n, 1.0, false, st)) != ADC2_OK ||
        (rc = gemm_rr(np, np, n, WT, n, true, YT, n, false, Lo + (long)P * np * np, np, 1.0, false, st)) != ADC2_OK)
      msg = adc2_last_error();
  }
  // the host arrays above are consumed by the stream before they go out of scope
  if (hipStreamSynchronize(st) != hipSuccess && rc == ADC2_OK) {
    rc = ADC2_ERR_HIP;
    msg = "hipStreamSynchronize";
  }
  cleanup();
  if (rc != ADC2_OK) return ffail(rc, msg);
  return ADC2_OK;
}
