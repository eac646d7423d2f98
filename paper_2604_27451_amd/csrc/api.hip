// api.hip -- C ABI entry points of the CVS-ADC(2) library and the host-side
// driver of the block Davidson solver.  The host only orchestrates: every
// arithmetic step runs in the kernels of k_setup / k_sigma / k_davidson; the
// host reads back the residual norms, the Ritz values and the count of new
// search directions to decide convergence and restarts.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"

namespace adc2 {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

static adc2_status fail(adc2_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

static void free_handle(adc2_handle h) {
  if (!h) return;
  dfree(h, h->Lvv);
  dfree(h, h->Lvo);
  dfree(h, h->Loo);
  dfree(h, h->Vt);
  dfree(h, h->LoT);
  dfree(h, h->Lv32);
  dfree(h, h->LvT32);
  dfree(h, h->LvB);
  dfree(h, h->LvTB);
  dfree(h, h->XB);
  dfree(h, h->RB);
  dfree(h, h->eps);
  dfree(h, h->M11);
  dfree(h, h->diag);
  dfree(h, h->X);
  dfree(h, h->Y);
  dfree(h, h->part);
  dfree(h, h->Zb);
  dfree(h, h->Tp);
  dfree(h, h->Vpp);
  dfree(h, h->Hh);
  dfree(h, h->WvT);
  dfree(h, h->WcT);
  dfree(h, h->diagx);
  dfree(h, h->Xw);
  if (h->ev0) hipEventDestroy(h->ev0);
  if (h->ev1) hipEventDestroy(h->ev1);
  for (int i = 0; i <= adc2_handle_s::NK; ++i)
    if (h->kev[i]) hipEventDestroy(h->kev[i]);
  delete h;
}

static double sigma_flops_per_vector(const Dims& d) {
  const double nc = d.nc, no = d.no, nv = d.nv, naux = d.naux;
  return 8.0 * (2.0 * nc * no * nv * nv * naux + 2.0 * nc * nv * nv * naux + (nc * nv) * (nc * nv));
}

// ---------------------------------------------------------------------------
// Small kernel: compact + scale eigenvectors of a block Gram matrix.
// Keeps columns with lambda > rel * lambda_max, scaled by lambda^-1/2.
// ---------------------------------------------------------------------------
__global__ void k_orth_coeffs(const double* __restrict__ lam, const double2* __restrict__ U, int n, int ldu,
                              double rel, double2* __restrict__ Uo, int ldo, int* __restrict__ count) {
  __shared__ int keep[64];
  __shared__ int nk;
  if (threadIdx.x == 0) {
    double lmax = 0.0;
    for (int i = 0; i < n; ++i) lmax = fmax(lmax, lam[i]);
    int c = 0;
    for (int i = n - 1; i >= 0; --i)
      if (lmax > 0.0 && lam[i] > rel * lmax && isfinite(lam[i])) keep[c++] = i;
    nk = c;
    *count = c;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * nk; e += blockDim.x) {
    const int r = e / nk, c = e % nk;
    const int src = keep[c];
    const double sc = 1.0 / sqrt(lam[src]);
    const double2 u = U[(long)r * ldu + src];
    Uo[(long)r * ldo + c] = make_double2(u.x * sc, u.y * sc);
  }
}

__global__ void k_diag_set(double2* __restrict__ G, int ldg, const double* __restrict__ w, int n) {
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    G[(long)i * ldg + j] = make_double2(i == j ? w[i] : 0.0, 0.0);
  }
}

__global__ void k_sub_scaled(double2* __restrict__ S, const double2* __restrict__ X, const double* __restrict__ w,
                             int k, long dim) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < dim * k; e += (long)gridDim.x * blockDim.x) {
    const int j = (int)(e / dim);
    S[e] = make_double2(S[e].x - w[j] * X[e].x, S[e].y - w[j] * X[e].y);
  }
}

__global__ void k_gather_theta(const double* __restrict__ th, const int* __restrict__ idx, int n,
                               double* __restrict__ out) {
  if (threadIdx.x < n) out[threadIdx.x] = th[idx[threadIdx.x]];
}

// Preconditioner of the full-space solver from the Schur complement of the
// doubles block: the correction equation (theta - M) t = r with M22 ~ diag(D)
// gives t2 = (theta - D)^-1 (r2 + M21 t1), and t1 from the singles block of
// the folded operator, approximated by its diagonal
//   t1_e = r1_e / (theta - d11_e - nu_e / (theta - Dbar_e))
// (nu_e = |column e of M21|^2, Dbar_e its weighted mean doubles energy).
// Step 1: t1 into T's singles, zero doubles (the sigma of (t1, 0) gives M21 t1).
__global__ void k_schur_singles(double2* __restrict__ T, const double* __restrict__ theta, int k, long dim, long ns,
                                const double* __restrict__ diag, const double* __restrict__ nu,
                                const double* __restrict__ dbar) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < dim * k; e += (long)gridDim.x * blockDim.x) {
    const int q = (int)(e / dim);
    const long x = e % dim;
    if (x >= ns) {
      T[e] = make_double2(0.0, 0.0);
      continue;
    }
    const double th = theta[q];
    double den = th - diag[x];
    const double gap = th - dbar[x];
    if (nu[x] > 0.0 && fabs(gap) > 1e-12) den -= nu[x] / gap;
    if (fabs(den) < 1e-8) den = den < 0.0 ? -1e-8 : 1e-8;
    T[e] = make_double2(T[e].x / den, T[e].y / den);
  }
}

// Step 2: t2 = (theta - D)^-1 (r2 + W2), r the residual of root idx[q], W = sigma of (t1, 0).
__global__ void k_schur_doubles(double2* __restrict__ T, const double2* __restrict__ W,
                                const double2* __restrict__ R, const int* __restrict__ idx,
                                const double* __restrict__ theta, int k, long dim, long ns,
                                const double* __restrict__ diag) {
  const long nd = dim - ns;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nd * k; e += (long)gridDim.x * blockDim.x) {
    const int q = (int)(e / nd);
    const long x = ns + e % nd;
    double den = theta[q] - diag[x];
    if (fabs(den) < 1e-8) den = den < 0.0 ? -1e-8 : 1e-8;
    const double2 r = R[(long)idx[q] * dim + x], wv = W[(long)q * dim + x];
    T[(long)q * dim + x] = make_double2((r.x + wv.x) / den, (r.y + wv.y) / den);
  }
}

}  // namespace adc2

using namespace adc2;

namespace adc2 {

hipError_t dmalloc_raw(adc2_handle h, void** p, size_t bytes) {
  if (!h || !h->alloc.alloc) return hipMalloc(p, bytes);
  if (bytes == 0) {          // as hipMalloc: success, no memory
    *p = nullptr;
    return hipSuccess;
  }
  *p = h->alloc.alloc(bytes, h->alloc.ctx);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

void dfree(adc2_handle h, void* p) {
  if (!p) return;
  if (!h || !h->alloc.alloc) {
    hipFree(p);
    return;
  }
  hipDeviceSynchronize();
  h->alloc.release(p, h->alloc.ctx);
}

}  // namespace adc2

extern "C" {

const char* adc2_last_error(void) { return g_last_error.c_str(); }

size_t adc2_dim(adc2_handle h) { return h ? (size_t)h->d.dim : 0; }

adc2_status adc2_destroy(adc2_handle h) {
  free_handle(h);
  return ADC2_OK;
}

adc2_status adc2_setup(const void* L, const double* eps, int nc, int no, int nv, int naux, int prec,
                       const adc2_alloc* alloc, void* stream, adc2_handle* out) {
  if (!out) return fail(ADC2_ERR_ARG, "adc2_setup: out is NULL");
  *out = nullptr;
  if (!L || !eps) return fail(ADC2_ERR_ARG, "adc2_setup: L or eps is NULL");
  if (nc <= 0 || no <= 0 || nv < 2 || naux <= 0)
    return fail(ADC2_ERR_ARG, "adc2_setup: need nc>0, no>0, nv>=2, naux>0");
  if (prec != ADC2_FP64 && prec != ADC2_C64 && prec != ADC2_BF16X3)
    return fail(ADC2_ERR_ARG, "adc2_setup: unsupported precision");
  if (nc > 64) return fail(ADC2_ERR_ARG, "adc2_setup: nc > 64 not supported");
  hipStream_t st = (hipStream_t)stream;
  adc2_handle h = new adc2_handle_s();
  Dims& d = h->d;
  d.nc = nc;
  d.no = no;
  d.nv = nv;
  d.naux = naux;
  d.o = nc + no;
  d.n = d.o + nv;
  d.ns = (long)nc * nv;
  d.npair = (long)nv * (nv - 1) / 2;
  d.nd = (long)nc * no * d.npair;
  d.dim = d.ns + d.nd;
  d.nocc_pair = (long)d.o * (d.o - 1) / 2;
  h->prec = prec;
  if (alloc && alloc->alloc) {
    if (!alloc->release) {
      delete h;
      return fail(ADC2_ERR_ARG, "adc2_setup: alloc callbacks need both alloc and release");
    }
    h->alloc = *alloc;
  }
  if (const char* v = getenv("ADC2_ZGEMM"))
    h->zgemm = strcmp(v, "3m") == 0    ? ZGEMM_3M
               : strcmp(v, "big") == 0 ? ZGEMM_BIG
               : strcmp(v, "mid") == 0 ? ZGEMM_MID
                                       : ZGEMM_WIDE;
#define SETUP_TRY(call)                                                           \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));               \
      free_handle(h);                                                             \
      return e_ == hipErrorOutOfMemory ? ADC2_ERR_OOM : ADC2_ERR_HIP;             \
    }                                                                             \
  } while (0)
  // energies must be finite
  std::vector<double> he(d.n);
  SETUP_TRY(hipMemcpyAsync(he.data(), eps, sizeof(double) * d.n, hipMemcpyDeviceToHost, st));
  SETUP_TRY(hipStreamSynchronize(st));
  for (double x : he)
    if (!std::isfinite(x)) {
      free_handle(h);
      return fail(ADC2_ERR_NONFINITE, "adc2_setup: non-finite spinor energy");
    }
  SETUP_TRY(dmalloc(h, &h->Lvv, sizeof(double2) * (size_t)naux * nv * nv));
  SETUP_TRY(dmalloc(h, &h->Lvo, sizeof(double2) * (size_t)d.o * naux * nv));
  SETUP_TRY(dmalloc(h, &h->Loo, sizeof(double2) * (size_t)naux * d.o * d.o));
  SETUP_TRY(dmalloc(h, &h->Vt, sizeof(double2) * (size_t)nc * no * nc * nv));
  SETUP_TRY(dmalloc(h, &h->eps, sizeof(double) * d.n));
  SETUP_TRY(dmalloc(h, &h->M11, sizeof(double2) * (size_t)d.ns * d.ns));
  SETUP_TRY(dmalloc(h, &h->diag, sizeof(double) * (size_t)d.dim));
  SETUP_TRY(hipEventCreate(&h->ev0));
  SETUP_TRY(hipEventCreate(&h->ev1));
  SETUP_TRY(hipMemcpyAsync(h->eps, eps, sizeof(double) * d.n, hipMemcpyDeviceToDevice, st));
  double herm[2] = {0, 0};
  adc2_status rc = launch_repack((const double2*)L, eps, h, herm, st);
  if (rc != ADC2_OK) {
    free_handle(h);
    return rc;
  }
  if (!std::isfinite(herm[0]) || !std::isfinite(herm[1])) {
    free_handle(h);
    return fail(ADC2_ERR_NONFINITE, "adc2_setup: non-finite Cholesky vector element");
  }
  if (herm[0] > 1e-12 * herm[1]) {
    char buf[160];
    snprintf(buf, sizeof buf, "adc2_setup: L not Hermitian (max |L_pq - conj L_qp| = %.3e, max |L| = %.3e)",
             herm[0], herm[1]);
    free_handle(h);
    return fail(ADC2_ERR_NOT_HERMITIAN, buf);
  }
  rc = build_m11(h, st);
  if (rc == ADC2_OK) rc = build_lvt(h, st);
  if (rc == ADC2_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(ADC2_ERR_HIP, "adc2_setup: sync failed");
  if (rc != ADC2_OK) {
    free_handle(h);
    return rc;
  }
  *out = h;
  return ADC2_OK;
#undef SETUP_TRY
}

adc2_status adc2_sigma(adc2_handle h, int m, const void* X, void* S, void* stream) {
  if (!h || !X || !S || m <= 0) return fail(ADC2_ERR_ARG, "adc2_sigma: bad arguments");
  if (X == S) return fail(ADC2_ERR_ARG, "adc2_sigma: S must not alias X");
  return sigma_fp64(h, m, (const double2*)X, (double2*)S, (hipStream_t)stream);
}

adc2_status adc2_set_precision(adc2_handle h, int prec) {
  if (!h) return fail(ADC2_ERR_ARG, "adc2_set_precision: NULL handle");
  if (prec != ADC2_FP64 && prec != ADC2_C64 && prec != ADC2_BF16X3)
    return fail(ADC2_ERR_ARG, "adc2_set_precision: unknown precision");
  h->prec = prec;
  return ADC2_OK;
}

adc2_status adc2_rayleigh(adc2_handle h, int k, const void* X, double* omega, double* resnorm, void* stream) {
  if (!h || !X || !omega || k <= 0 || k > 32) return fail(ADC2_ERR_ARG, "adc2_rayleigh: bad arguments");
  hipStream_t st = (hipStream_t)stream;
  const long dim = h->d.dim;
  const int nblk = dav_nblk(dim);
  double2 *S = nullptr, *G = nullptr, *scr = nullptr;
  double *w = nullptr, *np = nullptr;
  adc2_status rc = ADC2_OK;
  const int saved = h->prec;
  std::vector<double2> hg(32 * 32), hn(32 * 32);
  std::vector<double> hp(32 * (size_t)nblk);
  auto done = [&](adc2_status r) {
    h->prec = saved;
    dfree(h, S); dfree(h, G); dfree(h, scr); dfree(h, w); dfree(h, np);
    return r;
  };
#define RQ_TRY(call)                                                            \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) {                                                     \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));             \
      return done(e_ == hipErrorOutOfMemory ? ADC2_ERR_OOM : ADC2_ERR_HIP);     \
    }                                                                           \
  } while (0)
  RQ_TRY(dmalloc(h, &S, sizeof(double2) * k * dim));
  RQ_TRY(dmalloc(h, &G, sizeof(double2) * 2 * 32 * 32));
  RQ_TRY(dmalloc(h, &scr, sizeof(double2) * 256 * (long)nblk * 16 * 4));
  RQ_TRY(dmalloc(h, &w, sizeof(double) * 32));
  RQ_TRY(dmalloc(h, &np, sizeof(double) * 32 * nblk));
  h->prec = ADC2_FP64;
  if ((rc = sigma_fp64(h, k, (const double2*)X, S, st)) != ADC2_OK) return done(rc);
  if ((rc = dav_gram((const double2*)X, k, S, k, dim, G, 32, scr, st)) != ADC2_OK) return done(rc);
  if ((rc = dav_gram((const double2*)X, k, (const double2*)X, k, dim, G + 32 * 32, 32, scr, st)) != ADC2_OK)
    return done(rc);
  RQ_TRY(hipMemcpyAsync(hg.data(), G, sizeof(double2) * 32 * 32, hipMemcpyDeviceToHost, st));
  RQ_TRY(hipMemcpyAsync(hn.data(), G + 32 * 32, sizeof(double2) * 32 * 32, hipMemcpyDeviceToHost, st));
  RQ_TRY(hipStreamSynchronize(st));
  std::vector<double> wn(k), nn(k);
  for (int i = 0; i < k; ++i) {
    nn[i] = hn[i * 32 + i].x;
    wn[i] = hg[i * 32 + i].x / nn[i];
    omega[i] = wn[i];
  }
  if (resnorm) {
    RQ_TRY(hipMemcpyAsync(w, wn.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
    k_sub_scaled<<<(unsigned)std::min<long>(8192, (dim * k + 255) / 256), 256, 0, st>>>(S, (const double2*)X, w, k,
                                                                                       dim);
    RQ_TRY(hipGetLastError());
    if ((rc = dav_norms(S, k, dim, np, nblk, st)) != ADC2_OK) return done(rc);
    RQ_TRY(hipMemcpyAsync(hp.data(), np, sizeof(double) * 32 * nblk, hipMemcpyDeviceToHost, st));
    RQ_TRY(hipStreamSynchronize(st));
    for (int i = 0; i < k; ++i) {
      double a = 0.0;
      for (int b = 0; b < nblk; ++b) a += hp[(size_t)b * 32 + i];
      resnorm[i] = std::sqrt(a / nn[i]);
    }
  }
#undef RQ_TRY
  return done(ADC2_OK);
}

adc2_status adc2_omega_backward(adc2_handle h, int nroots, const void* X, const double* g_omega, void* dL,
                                double* deps, void* stream) {
  if (!h || !X || !g_omega || !dL || !deps) return fail(ADC2_ERR_ARG, "adc2_omega_backward: NULL argument");
  if (nroots <= 0 || nroots > ADC2_MAX_ROOTS)
    return fail(ADC2_ERR_ARG, "adc2_omega_backward: nroots must be in 1..ADC2_MAX_ROOTS");
  for (int k = 0; k < nroots; ++k)
    if (!std::isfinite(g_omega[k])) return fail(ADC2_ERR_ARG, "adc2_omega_backward: non-finite g_omega");
  if (h->method != ADC2_METHOD_ADC2)
    return fail(ADC2_ERR_ARG, "adc2_omega_backward: the adjoint covers the ADC(2) matrix only");
  return omega_backward(h, nroots, (const double2*)X, g_omega, (double2*)dL, deps, (hipStream_t)stream);
}

adc2_status adc2_get_m11(adc2_handle h, void* dst, void* stream) {
  if (!h || !dst) return fail(ADC2_ERR_ARG, "adc2_get_m11: bad arguments");
  ADC2_HIP(hipMemcpyAsync(dst, h->M11, sizeof(double2) * h->d.ns * h->d.ns, hipMemcpyDeviceToDevice,
                          (hipStream_t)stream));
  return ADC2_OK;
}

adc2_status adc2_get_diag(adc2_handle h, double* dst, void* stream) {
  if (!h || !dst) return fail(ADC2_ERR_ARG, "adc2_get_diag: bad arguments");
  ADC2_HIP(hipMemcpyAsync(dst, cur_diag(h), sizeof(double) * h->d.dim, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return ADC2_OK;
}

adc2_status adc2_profile(adc2_handle h, int enable) {
  if (!h) return fail(ADC2_ERR_ARG, "adc2_profile: NULL handle");
  for (int i = 0; i <= adc2_handle_s::NK; ++i)
    if (!h->kev[i]) ADC2_HIP(hipEventCreate(&h->kev[i]));
  for (int i = 0; i < adc2_handle_s::NK; ++i) {
    h->k_launches[i] = 0;
    h->k_ms[i] = 0.0;
    h->k_flops[i] = 0.0;
  }
  h->profiling = enable ? 1 : 0;
  return ADC2_OK;
}

int adc2_kernel_stats(adc2_handle h, adc2_kstat* out, int max) {
  if (!h) return -1;
  static const char* names[adc2_handle_s::NK] = {"unpack", "ybuild", "light1", "xbuild",
                                                 "sigma2", "pack2", "backc", "m11mv"};
  for (int i = 0; i < adc2_handle_s::NK && i < max && out; ++i) {
    memset(&out[i], 0, sizeof(out[i]));
    strncpy(out[i].name, names[i], sizeof(out[i].name) - 1);
    out[i].launches = h->k_launches[i];
    out[i].ms = h->k_ms[i];
    out[i].flops = h->k_flops[i];
  }
  return adc2_handle_s::NK;
}

adc2_status adc2_mp2_energy(adc2_handle h, double* e) {
  if (!h || !e) return fail(ADC2_ERR_ARG, "adc2_mp2_energy: bad arguments");
  *e = h->e_mp2;
  return ADC2_OK;
}

// ---------------------------------------------------------------------------
// Block Davidson
// ---------------------------------------------------------------------------
namespace {

struct DavWork {
  adc2_handle h = nullptr;   // owner of the allocations (its callbacks, if any)
  double2 *V = nullptr, *S = nullptr, *Xb = nullptr, *R = nullptr, *T = nullptr, *T2 = nullptr;
  double2 *Vn = nullptr, *Sn = nullptr, *Ref = nullptr, *P = nullptr;
  double2 *G = nullptr, *Z = nullptr, *Gt = nullptr, *Ut = nullptr, *Cc = nullptr, *scratch = nullptr;
  double *theta = nullptr, *lam = nullptr, *npart = nullptr, *thact = nullptr, *pnu = nullptr, *pdb = nullptr;
  int *idx = nullptr, *count = nullptr;
  ~DavWork() {
    dfree(h, V); dfree(h, S); dfree(h, Xb); dfree(h, R); dfree(h, T); dfree(h, T2); dfree(h, Vn); dfree(h, Sn);
    dfree(h, Ref); dfree(h, P); dfree(h, pnu); dfree(h, pdb);
    dfree(h, G); dfree(h, Z); dfree(h, Gt); dfree(h, Ut); dfree(h, Cc); dfree(h, scratch);
    dfree(h, theta); dfree(h, lam); dfree(h, npart); dfree(h, thact); dfree(h, idx); dfree(h, count);
  }
};

constexpr int LDG = 64;

// Orthonormalise the na vectors in T against V[0..s) (two passes of
// projection + symmetric orthonormalisation of the block).  Returns the
// number of surviving vectors (left in T) or -1 on error.
int orth_block(DavWork& w, const double2* V, int s, int na, long dim, int nblk, hipStream_t st,
               adc2_status& rc) {
  (void)nblk;
  for (int pass = 0; pass < 2 && na > 0; ++pass) {
    if (s > 0) {
      if ((rc = dav_gram(V, s, w.T, na, dim, w.Cc, 32, w.scratch, st)) != ADC2_OK) return -1;
      if ((rc = dav_combine(V, s, w.Cc, 32, na, dim, w.T, -1.0, true, st)) != ADC2_OK) return -1;
    }
    if ((rc = dav_gram(w.T, na, w.T, na, dim, w.Gt, LDG, w.scratch, st)) != ADC2_OK) return -1;
    if ((rc = dav_heevj(w.Gt, na, LDG, w.lam, w.Ut, LDG, st)) != ADC2_OK) return -1;
    k_orth_coeffs<<<1, 256, 0, st>>>(w.lam, w.Ut, na, LDG, 1e-14, w.Cc, 32, w.count);
    int cnt = 0;
    if (hipMemcpyAsync(&cnt, w.count, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = fail(ADC2_ERR_HIP, "orth_block: count readback failed");
      return -1;
    }
    if (cnt > 0) {
      if ((rc = dav_combine(w.T, na, w.Cc, 32, cnt, dim, w.T2, 1.0, false, st)) != ADC2_OK) return -1;
      std::swap(w.T, w.T2);
    }
    na = cnt;
  }
  return na;
}

}  // namespace

adc2_status adc2_davidson(adc2_handle h, int nroots, const adc2_dav_opts* opt, const void* guess,
                          double* omega, void* Xout, adc2_dav_info* info, void* stream) {
  const auto t_start = std::chrono::steady_clock::now();
  if (!h || !omega) return fail(ADC2_ERR_ARG, "adc2_davidson: bad arguments");
  if (opt && opt->mixed_tol > 0.0) {
    // two stages: split-BF16 sigma builds to mixed_tol, then FP64 from those vectors
    const double tol = opt->tol > 0 ? opt->tol : 1e-8;
    if (opt->follow) return fail(ADC2_ERR_ARG, "adc2_davidson: the two-stage solve does not follow roots");
    if (!(opt->mixed_tol > tol)) return fail(ADC2_ERR_ARG, "adc2_davidson: mixed_tol must exceed tol");
    if (h->prec != ADC2_FP64) return fail(ADC2_ERR_ARG, "adc2_davidson: the two-stage solve needs an FP64 handle");
    if (nroots <= 0 || nroots > ADC2_MAX_ROOTS) return fail(ADC2_ERR_ARG, "adc2_davidson: nroots must be in 1..32");
    hipStream_t st = (hipStream_t)stream;
    double2* Xm = nullptr;
    if (dmalloc(h, &Xm, sizeof(double2) * (size_t)nroots * h->d.dim) != hipSuccess)
      return fail(ADC2_ERR_OOM, "adc2_davidson: no memory for the first-stage vectors");
    adc2_dav_opts o1 = *opt;
    o1.mixed_tol = 0.0;
    o1.tol = opt->mixed_tol;
    adc2_dav_info i1{}, i2{};
    h->prec = ADC2_BF16X3;
    adc2_status r = adc2_davidson(h, nroots, &o1, guess, omega, Xm, &i1, stream);
    h->prec = ADC2_FP64;
    if (r == ADC2_OK || r == ADC2_ERR_NOCONV) {   // a first stage short of mixed_tol still seeds the second
      adc2_dav_opts o2 = *opt;
      o2.mixed_tol = 0.0;
      o2.nguess = nroots;
      r = adc2_davidson(h, nroots, &o2, Xm, omega, Xout, &i2, stream);
    }
    const std::string msg = r == ADC2_OK ? std::string() : std::string(adc2_last_error());
    (void)hipStreamSynchronize(st);
    dfree(h, Xm);
    if (info) {
      *info = i2;
      info->iters = i1.iters + i2.iters;
      info->n_sigma = i1.n_sigma + i2.n_sigma;
      info->ms_sigma = i1.ms_sigma + i2.ms_sigma;
      info->sigma_flops = i1.sigma_flops + i2.sigma_flops;
      info->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    if (r != ADC2_OK) return fail(r, msg);
    return ADC2_OK;
  }
  if (opt && opt->solver == ADC2_SOLVER_FOLDED) {
    if (nroots <= 0 || nroots > ADC2_MAX_ROOTS) return fail(ADC2_ERR_ARG, "adc2_davidson: nroots must be in 1..32");
    if (h->method != ADC2_METHOD_ADC2)
      return fail(ADC2_ERR_ARG, "adc2_davidson: the folded solver needs the diagonal doubles block of ADC(2); "
                                "use the full-space solver for ADC(2)-x");
    return fold_davidson(h, nroots, opt, guess, omega, Xout, info, (hipStream_t)stream);
  }
  if (opt && opt->solver != ADC2_SOLVER_FULL) return fail(ADC2_ERR_ARG, "adc2_davidson: unknown solver");
  const int k = nroots;
  if (k <= 0 || k > ADC2_MAX_ROOTS || 3 * k > LDG)
    return fail(ADC2_ERR_ARG, "adc2_davidson: nroots must be in 1..21");
  hipStream_t st = (hipStream_t)stream;
  const Dims& d = h->d;
  const long dim = d.dim;
  if (dim < k) return fail(ADC2_ERR_ARG, "adc2_davidson: nroots exceeds the matrix dimension");
  double tol = (opt && opt->tol > 0) ? opt->tol : 1e-8;
  int max_iter = (opt && opt->max_iter > 0) ? opt->max_iter : 300;
  int max_sub = (opt && opt->max_subspace > 0) ? opt->max_subspace : std::max(6 * k, 3 * k);
  max_sub = std::min<long>(std::min(max_sub, LDG), dim);
  if (max_sub < std::min<long>(3 * k, dim))
    return fail(ADC2_ERR_ARG, "adc2_davidson: max_subspace must be >= 3*nroots");
  int nguess = (opt && opt->nguess > 0) ? opt->nguess : (k <= 8 ? 2 * k : k);
  nguess = (int)std::min<long>(nguess, max_sub - k);
  nguess = (int)std::min<long>(nguess, d.ns);
  nguess = std::max(nguess, k);
  const int verbose = opt ? opt->verbose : 0;
  const bool follow = opt && opt->follow != 0;
  if (follow && (!guess || nguess < k))
    return fail(ADC2_ERR_ARG, "adc2_davidson: root following needs at least nroots guess vectors");
  const int keep_max = std::min(std::min(2 * k, 32), max_sub - k);
  const int nblk = dav_nblk(dim);
  // preconditioner: the Schur form above (default), or the plain diagonal
  bool schur = true;
  if (const char* v = getenv("ADC2_FULL_PRECOND")) schur = strcmp(v, "diag") != 0;
  hipStream_t st0 = (hipStream_t)stream;
  if (schur) {
    adc2_status r0 = build_fold_precond(h, st0);
    if (r0 != ADC2_OK) return r0;
  }

  DavWork w;
  w.h = h;
#define DAV_TRY(call) ADC2_HIP(call)
  DAV_TRY(dmalloc(h, &w.V, sizeof(double2) * max_sub * dim));
  DAV_TRY(dmalloc(h, &w.S, sizeof(double2) * max_sub * dim));
  DAV_TRY(dmalloc(h, &w.Xb, sizeof(double2) * k * dim));
  DAV_TRY(dmalloc(h, &w.R, sizeof(double2) * k * dim));
  DAV_TRY(dmalloc(h, &w.T, sizeof(double2) * std::max(k, nguess) * dim));
  DAV_TRY(dmalloc(h, &w.T2, sizeof(double2) * std::max(k, nguess) * dim));
  DAV_TRY(dmalloc(h, &w.Vn, sizeof(double2) * keep_max * dim));
  DAV_TRY(dmalloc(h, &w.Sn, sizeof(double2) * keep_max * dim));
  DAV_TRY(dmalloc(h, &w.G, sizeof(double2) * LDG * LDG));
  DAV_TRY(dmalloc(h, &w.Z, sizeof(double2) * LDG * LDG));
  DAV_TRY(dmalloc(h, &w.Gt, sizeof(double2) * LDG * LDG));
  DAV_TRY(dmalloc(h, &w.Ut, sizeof(double2) * LDG * LDG));
  DAV_TRY(dmalloc(h, &w.Cc, sizeof(double2) * LDG * 32));
  DAV_TRY(dmalloc(h, &w.scratch, sizeof(double2) * 256 * (long)nblk * 16 * 4));
  DAV_TRY(dmalloc(h, &w.theta, sizeof(double) * LDG));
  DAV_TRY(dmalloc(h, &w.lam, sizeof(double) * LDG));
  DAV_TRY(dmalloc(h, &w.npart, sizeof(double) * 32 * nblk));
  DAV_TRY(dmalloc(h, &w.thact, sizeof(double) * 32));
  DAV_TRY(dmalloc(h, &w.idx, sizeof(int) * LDG));
  DAV_TRY(dmalloc(h, &w.count, sizeof(int)));
  if (schur) {
    DAV_TRY(dmalloc(h, &w.pnu, sizeof(double) * d.ns));
    DAV_TRY(dmalloc(h, &w.pdb, sizeof(double) * d.ns));
    DAV_TRY(hipMemcpyAsync(w.pnu, h->pre_nu.data(), sizeof(double) * d.ns, hipMemcpyHostToDevice, st));
    DAV_TRY(hipMemcpyAsync(w.pdb, h->pre_dbar.data(), sizeof(double) * d.ns, hipMemcpyHostToDevice, st));
    DAV_TRY(hipStreamSynchronize(st));
  }
  if (follow) {
    // reference vectors of the followed roots: the first nroots guess vectors as given
    DAV_TRY(dmalloc(h, &w.Ref, sizeof(double2) * k * dim));
    DAV_TRY(dmalloc(h, &w.P, sizeof(double2) * LDG * LDG));
    DAV_TRY(hipMemcpyAsync(w.Ref, guess, sizeof(double2) * k * dim, hipMemcpyDeviceToDevice, st));
  }

  double ms_sigma = 0.0;
  int n_sigma = 0;
  long n_half = 0;   // half sigma products (one of the two heavy GEMMs) of the preconditioner
  auto run_sigma = [&](const double2* x, double2* s_out, int m) -> adc2_status {
    DAV_TRY(hipEventRecord(h->ev0, st));
    adc2_status r = sigma_call(h, m, x, s_out, SIGMA_SINGLES_IN | SIGMA_DOUBLES_IN, st);
    if (r != ADC2_OK) return r;
    DAV_TRY(hipEventRecord(h->ev1, st));
    DAV_TRY(hipEventSynchronize(h->ev1));
    float ms = 0.f;
    DAV_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    ms_sigma += ms;
    n_sigma += m;
    return ADC2_OK;
  };

  // initial guess into T, then orthonormalise
  adc2_status rc = ADC2_OK;
  if (guess) {
    DAV_TRY(hipMemcpyAsync(w.T, guess, sizeof(double2) * nguess * dim, hipMemcpyDeviceToDevice, st));
  } else {
    std::vector<double> hd(d.ns);
    DAV_TRY(hipMemcpyAsync(hd.data(), h->diag, sizeof(double) * d.ns, hipMemcpyDeviceToHost, st));
    DAV_TRY(hipStreamSynchronize(st));
    std::vector<int> ord(d.ns);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return hd[a] < hd[b]; });
    ord.resize(nguess);
    DAV_TRY(hipMemcpyAsync(w.idx, ord.data(), sizeof(int) * nguess, hipMemcpyHostToDevice, st));
    if ((rc = dav_unit_guess(w.T, nguess, dim, w.idx, st)) != ADC2_OK) return rc;
    DAV_TRY(hipStreamSynchronize(st));   // ord (pageable, block-local) consumed before it is freed
  }
  int g = orth_block(w, w.V, 0, nguess, dim, nblk, st, rc);
  if (g < 0) return rc;
  if (g < k) return fail(ADC2_ERR_ARG, "adc2_davidson: guess vectors are linearly dependent");
  DAV_TRY(hipMemcpyAsync(w.V, w.T, sizeof(double2) * g * dim, hipMemcpyDeviceToDevice, st));
  if ((rc = run_sigma(w.V, w.S, g)) != ADC2_OK) return rc;
  if ((rc = dav_gram(w.V, g, w.S, g, dim, w.G, LDG, w.scratch, st)) != ADC2_OK) return rc;
  int s = g;

  std::vector<double> th(LDG), np(32 * nblk), rn(k);
  std::vector<double2> hz((size_t)LDG * LDG), hp((size_t)LDG * LDG);
  // Root following (root-specific Davidson of Hirao and Nakatsuji): root j is
  // the Ritz pair whose vector overlaps most with reference vector j, taken
  // greedily in decreasing order of overlap; the chosen columns of Z (and
  // their Ritz values) are moved to the front in reference order, so the
  // residual, restart and convergence steps below act on the followed roots.
  auto follow_select = [&](int s_) -> adc2_status {
    if ((rc = dav_gram(w.Ref, k, w.V, s_, dim, w.P, LDG, w.scratch, st)) != ADC2_OK) return rc;
    DAV_TRY(hipMemcpyAsync(hz.data(), w.Z, sizeof(double2) * LDG * s_, hipMemcpyDeviceToHost, st));
    DAV_TRY(hipMemcpyAsync(hp.data(), w.P, sizeof(double2) * LDG * k, hipMemcpyDeviceToHost, st));
    DAV_TRY(hipMemcpyAsync(th.data(), w.theta, sizeof(double) * s_, hipMemcpyDeviceToHost, st));
    DAV_TRY(hipStreamSynchronize(st));
    std::vector<double> ov((size_t)k * s_);
    for (int j = 0; j < k; ++j)
      for (int l = 0; l < s_; ++l) {
        double re = 0.0, im = 0.0;
        for (int i = 0; i < s_; ++i) {
          const double2 a = hp[(size_t)j * LDG + i], z = hz[(size_t)i * LDG + l];
          re += a.x * z.x - a.y * z.y;
          im += a.x * z.y + a.y * z.x;
        }
        ov[(size_t)j * s_ + l] = re * re + im * im;
      }
    std::vector<int> sel(k, -1);
    std::vector<char> used(s_, 0);
    for (int n = 0; n < k; ++n) {
      int bj = -1, bl = -1;
      double best = -1.0;
      for (int j = 0; j < k; ++j) {
        if (sel[j] >= 0) continue;
        for (int l = 0; l < s_; ++l)
          if (!used[l] && ov[(size_t)j * s_ + l] > best) {
            best = ov[(size_t)j * s_ + l];
            bj = j;
            bl = l;
          }
      }
      sel[bj] = bl;
      used[bl] = 1;
    }
    std::vector<int> order(sel);
    for (int l = 0; l < s_; ++l)
      if (!used[l]) order.push_back(l);
    std::vector<double2> z2((size_t)LDG * s_);
    std::vector<double> th2(s_);
    for (int c = 0; c < s_; ++c) {
      th2[c] = th[order[c]];
      for (int i = 0; i < s_; ++i) z2[(size_t)i * LDG + c] = hz[(size_t)i * LDG + order[c]];
    }
    DAV_TRY(hipMemcpyAsync(w.Z, z2.data(), sizeof(double2) * LDG * s_, hipMemcpyHostToDevice, st));
    DAV_TRY(hipMemcpyAsync(w.theta, th2.data(), sizeof(double) * s_, hipMemcpyHostToDevice, st));
    DAV_TRY(hipStreamSynchronize(st));   // host copies consumed before they go out of scope
    return ADC2_OK;
  };
  int it = 0;
  bool conv = false, nonfinite = false, stalled = false;
  for (it = 1; it <= max_iter; ++it) {
    if ((rc = dav_heevj(w.G, s, LDG, w.theta, w.Z, LDG, st)) != ADC2_OK) return rc;
    if (follow && (rc = follow_select(s)) != ADC2_OK) return rc;
    if ((rc = dav_residual(w.V, w.S, s, w.Z, LDG, w.theta, k, dim, w.Xb, w.R, w.npart, nblk, st)) != ADC2_OK)
      return rc;
    DAV_TRY(hipMemcpyAsync(th.data(), w.theta, sizeof(double) * s, hipMemcpyDeviceToHost, st));
    DAV_TRY(hipMemcpyAsync(np.data(), w.npart, sizeof(double) * 32 * nblk, hipMemcpyDeviceToHost, st));
    DAV_TRY(hipStreamSynchronize(st));
    double rmax = 0.0;
    for (int j = 0; j < k; ++j) {
      double a = 0.0;
      for (int b = 0; b < nblk; ++b) a += np[(long)b * 32 + j];
      rn[j] = std::sqrt(a);
      if (!std::isfinite(rn[j]) || !std::isfinite(th[j])) nonfinite = true;
      rmax = std::max(rmax, rn[j]);
    }
    if (verbose) {
      fprintf(stderr, "[adc2 davidson] it %3d  s %2d  w0 %.12f  max|r| %.3e\n", it, s, th[0], rmax);
    }
    if (nonfinite) break;
    std::vector<int> act;
    for (int j = 0; j < k; ++j)
      if (rn[j] > tol) act.push_back(j);
    if (act.empty()) {
      conv = true;
      break;
    }
    if (it == max_iter) break;
    const int na = (int)act.size();
    for (int q = 0; q < na; ++q)
      DAV_TRY(hipMemcpyAsync(w.T + (long)q * dim, w.R + (long)act[q] * dim, sizeof(double2) * dim,
                             hipMemcpyDeviceToDevice, st));
    DAV_TRY(hipMemcpyAsync(w.idx, act.data(), sizeof(int) * na, hipMemcpyHostToDevice, st));
    DAV_TRY(hipStreamSynchronize(st));   // act (pageable, loop-local) consumed before it is freed
    k_gather_theta<<<1, 64, 0, st>>>(w.theta, w.idx, na, w.thact);
    if (schur) {
      const unsigned gb = (unsigned)std::min<long>(16384, (dim * na + 255) / 256);
      k_schur_singles<<<gb, 256, 0, st>>>(w.T, w.thact, na, dim, d.ns, cur_diag(h), w.pnu, w.pdb);
      DAV_TRY(hipGetLastError());
      // M21 t1: the singles-input half of a sigma (ADC(2)-x needs the whole product of (t1, 0))
      const int parts = h->method == ADC2_METHOD_ADC2 ? SIGMA_SINGLES_IN : (SIGMA_SINGLES_IN | SIGMA_DOUBLES_IN);
      DAV_TRY(hipEventRecord(h->ev0, st));
      if ((rc = sigma_call(h, na, w.T, w.T2, parts, st)) != ADC2_OK) return rc;
      DAV_TRY(hipEventRecord(h->ev1, st));
      DAV_TRY(hipEventSynchronize(h->ev1));
      float ms = 0.f;
      DAV_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
      ms_sigma += ms;
      n_half += parts == SIGMA_SINGLES_IN ? na : 2 * na;
      k_schur_doubles<<<gb, 256, 0, st>>>(w.T, w.T2, w.R, w.idx, w.thact, na, dim, d.ns, cur_diag(h));
      DAV_TRY(hipGetLastError());
    } else if ((rc = dav_precondition(w.T, w.thact, cur_diag(h), na, dim, st)) != ADC2_OK) {
      return rc;
    }
    int na_use = na;
    if (s + na > max_sub && keep_max >= k && keep_max < s) {
      const int keep = keep_max;
      if ((rc = dav_combine(w.V, s, w.Z, LDG, keep, dim, w.Vn, 1.0, false, st)) != ADC2_OK) return rc;
      if ((rc = dav_combine(w.S, s, w.Z, LDG, keep, dim, w.Sn, 1.0, false, st)) != ADC2_OK) return rc;
      DAV_TRY(hipMemcpyAsync(w.V, w.Vn, sizeof(double2) * keep * dim, hipMemcpyDeviceToDevice, st));
      DAV_TRY(hipMemcpyAsync(w.S, w.Sn, sizeof(double2) * keep * dim, hipMemcpyDeviceToDevice, st));
      k_diag_set<<<1, 256, 0, st>>>(w.G, LDG, w.theta, keep);
      s = keep;
    }
    // tiny problems: the subspace cannot restart below nroots; take what fits
    if (s + na_use > max_sub) na_use = max_sub - s;
    if (na_use <= 0) {
      stalled = true;
      break;
    }
    const int nt = orth_block(w, w.V, s, na_use, dim, nblk, st, rc);
    if (nt < 0) return rc;
    if (nt == 0) {
      stalled = true;
      break;
    }
    DAV_TRY(hipMemcpyAsync(w.V + (long)s * dim, w.T, sizeof(double2) * nt * dim, hipMemcpyDeviceToDevice, st));
    if ((rc = run_sigma(w.V + (long)s * dim, w.S + (long)s * dim, nt)) != ADC2_OK) return rc;
    if ((rc = dav_gram(w.V, s + nt, w.S + (long)s * dim, nt, dim, w.G + s, LDG, w.scratch, st)) != ADC2_OK)
      return rc;
    s += nt;
  }
  if (it > max_iter) it = max_iter;
  for (int j = 0; j < k; ++j) omega[j] = th[j];
  if (Xout) DAV_TRY(hipMemcpyAsync(Xout, w.Xb, sizeof(double2) * k * dim, hipMemcpyDeviceToDevice, st));
  DAV_TRY(hipStreamSynchronize(st));
  if (info) {
    memset(info, 0, sizeof(*info));
    info->iters = it;
    info->n_sigma = n_sigma;
    info->converged = conv ? 1 : 0;
    info->subspace = s;
    for (int j = 0; j < k; ++j) info->resnorm[j] = rn[j];
    info->ms_sigma = ms_sigma;
    info->sigma_flops = sigma_flops_per_vector(d) * (n_sigma + 0.5 * n_half);
    info->ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  }
#undef DAV_TRY
  if (nonfinite) return fail(ADC2_ERR_NONFINITE, "adc2_davidson: non-finite residual or Ritz value");
  if (!conv) {
    return fail(ADC2_ERR_NOCONV, stalled ? "adc2_davidson: subspace stalled before convergence"
                                         : "adc2_davidson: max_iter reached");
  }
  return ADC2_OK;
}

}  // extern "C"
