// internal.h -- handle layout and kernel launchers of the CVS-ADC(2) library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>
#include <functional>
#include <vector>

#include "../../include/adc2.h"

namespace adc2 {

void set_error(const std::string& msg);

#define ADC2_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::adc2::set_error(std::string(#call) + ": " + hipGetErrorString(e_));         \
      return e_ == hipErrorOutOfMemory ? ADC2_ERR_OOM : ADC2_ERR_HIP;               \
    }                                                                               \
  } while (0)

#define ADC2_CHECK_LAUNCH() ADC2_HIP(hipGetLastError())

// Device memory of a handle: through its callbacks when set, else hipMalloc / hipFree
// (dfree waits for the device first, as hipFree does; NULL is ignored).
hipError_t dmalloc_raw(adc2_handle h, void** p, size_t bytes);
void dfree(adc2_handle h, void* p);
template <class T>
inline hipError_t dmalloc(adc2_handle h, T** p, size_t bytes) {
  return dmalloc_raw(h, reinterpret_cast<void**>(p), bytes);
}

// Sizes of one system.
// Engines of the FP64 heavy GEMMs (zgemm.h): 128 x 128 four-multiplication
// on four waves, 128 x 64 three-multiplication, 128 x 64 four-multiplication
// at two workgroups per CU, 128 x 128 four-multiplication on eight waves (the
// default).  Chosen per handle at setup (environment ADC2_ZGEMM = big, 3m,
// mid or wide) or by adc2_autotune.
constexpr int ZGEMM_BIG = 0, ZGEMM_3M = 1, ZGEMM_MID = 2, ZGEMM_WIDE = 3;

struct Dims {
  int nc, no, nv, naux;
  int o, n;               // o = nc + no, n = o + nv
  long ns;                // singles nc*nv
  long npair;             // nv*(nv-1)/2
  long nd;                // doubles nc*no*npair
  long dim;               // ns + nd
  long nocc_pair;         // o*(o-1)/2 pairs k<l of occupied spinors
};

// Device buffers owned by a handle.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace adc2

struct adc2_handle_s {
  adc2::Dims d;
  int prec = 0;
  adc2_alloc alloc{};       // device-memory callbacks (alloc == NULL: hipMalloc / hipFree)
  // integral blocks
  double2* Lvv = nullptr;   // [naux][nv][nv]      L^P_{ac}
  double2* Lvo = nullptr;   // [o][naux][nv]       L^P_{a k}  (k occupied)
  double2* Loo = nullptr;   // [naux][o][o]        L^P_{k l}
  double2* Vt = nullptr;    // [nc][no][nc][nv]    <Ka||Ij> at [I][j][K][a]
  double2* LoT = nullptr;   // [o*nv][naux]        conj(L^P_{dl}) at [(l,d)][P] (every occupied l)
  double2* LvT = nullptr;   // LoT + nc*nv*naux:   its valence rows (not a separate allocation)
  float2* Lv32 = nullptr;   // precision form: complex64 copy of the valence rows of Lvo
  float2* LvT32 = nullptr;  // precision form: complex64 copy of LvT
  void* LvB = nullptr;      // split-BF16 variant: Lv32 and LvT32 in the blocked split layout (zgemmb.h)
  void* LvTB = nullptr;
  void* XB = nullptr;       // split-BF16 workspace: X and the unpacked doubles in the blocked split layout
  void* RB = nullptr;
  int wsb_m = 0;
  double* eps = nullptr;    // [n]
  double2* M11 = nullptr;   // [ns][ns]
  double* diag = nullptr;   // [dim]
  double e_mp2 = 0.0;
  // sigma workspace (grown on demand)
  int ws_m = 0;
  double2* X = nullptr;     // [m*nc][naux][nv]      X^P_{Ia}
  double2* Y = nullptr;     // [m*nc][naux][nv]      Y^P_{Ic}
  double2* Zb = nullptr;    // unpacked doubles [(j,d)][(mI,c)], then the sigma2 core product [mI][j][a][b]
  double2* Tp = nullptr;    // light sigma1 partials [m*nc][no/4][nc][nv]
  double2* part = nullptr;  // split-K partials of the back-contraction
  int nsplit = 0;
  int ysplit = 1;           // K-splits of the Y-build GEMM
  int ysplit_tuned = 0;     // K-split fixed by adc2_autotune (0: the size heuristic)
  int zgemm = adc2::ZGEMM_WIDE;  // engine of the FP64 heavy GEMMs (ZGEMM_*)
  // method: ADC2_METHOD_ADC2 or ADC2_METHOD_ADC2X (first-order doubles block, adc2x.hip)
  int method = 0;
  double2* Vpp = nullptr;   // ADC(2)-x: [(a<b)][(c<d)] <ab||cd>
  double2* Hh = nullptr;    //           [(I,j)][(K,k)] <Kk||Ij>
  double2* WvT = nullptr;   //           [(j,b)][(k,c)] <kb||cj>, k, j valence
  double2* WcT = nullptr;   //           [(I,b)][(K,c)] <Kb||cI>, K, I core
  double* diagx = nullptr;  //           diagonal of M with the first-order doubles block
  double2* Xw = nullptr;    //           sigma work space: unpacked doubles (two layouts), ring products
  int wsx_m = 0;
  // folded-solver preconditioner (host, built on first use): per singles (K,c) the coupling
  // column norm sum_d |M21_{d,(Kc)}|^2 and its |M21|^2-weighted mean doubles energy
  std::vector<double> pre_nu, pre_dbar;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // set while the handle solves inside adc2_davidson_batch: the solvers' sigma
  // requests go to the batch's rendezvous instead of running alone
  std::function<adc2_status(int m, const double2* xin, double2* sout, int parts, hipStream_t st)> sigma_hook;
  // per-kernel profiling of the sigma build
  static constexpr int NK = 8;   // unpack, ybuild, light1, xbuild, sigma2, pack2, backc, m11mv
  int profiling = 0;
  hipEvent_t kev[NK + 1] = {};
  long k_launches[NK] = {};
  double k_ms[NK] = {};
  double k_flops[NK] = {};
};

namespace adc2 {

// ---- setup kernels (k_setup.hip) ----
adc2_status launch_repack(const double2* L, const double* eps, adc2_handle h, double* herm_out,
                          hipStream_t st);
adc2_status build_m11(adc2_handle h, hipStream_t st);

// ---- sigma kernels (k_sigma.hip) ----
adc2_status sigma_fp64(adc2_handle h, int m, const double2* X, double2* S, hipStream_t st);
constexpr int SIGMA_SINGLES_IN = 1;   // (r1, 0) -> (M11 r1, M21 r1)
constexpr int SIGMA_DOUBLES_IN = 2;   // (0, r2) -> singles M12 r2 only
adc2_status sigma_parts(adc2_handle h, int m, const double2* X, double2* S, int parts, hipStream_t st);
// One sigma request: m vectors of system h, parts as above.
struct SigReq {
  adc2_handle h;
  int m;
  const double2* xin;
  double2* sout;
  int parts;
};
adc2_status sigma_multi(int nreq, const SigReq* rq, hipStream_t st);
// A solver's sigma: through h->sigma_hook when set, else sigma_parts.
adc2_status sigma_call(adc2_handle h, int m, const double2* X, double2* S, int parts, hipStream_t st);
adc2_status build_lvt(adc2_handle h, hipStream_t st);
adc2_status build_c64(adc2_handle h, hipStream_t st);
adc2_status build_b3(adc2_handle h, hipStream_t st);
adc2_status ensure_ws_b3(adc2_handle h, int m);
adc2_status ensure_ws(adc2_handle h, int m);
// K-split count of the Y-build by the size rule for h's form and engine at block size m
int ysplit_rule(adc2_handle h, int m);
adc2_status unpack_weighted(adc2_handle h, int m, const double2* xin, const double* wts, hipStream_t st);
adc2_status ybuild_fp64(adc2_handle h, int m, hipStream_t st);
// Y-build GEMM of one request in the handle's form (h->ysplit partials) and the partial sum
adc2_status ybuild_launch(adc2_handle h, int m, hipStream_t st);
adc2_status ybuild_sum(adc2_handle h, int m, hipStream_t st);
// MP2 amplitudes in place: W[t][a][c] /= e_a + e_c - e_k - e_l for the device pair list (k, l) (fns.hip)
adc2_status tau_from_w(double2* W, const int2* dpairs, int npairs, const double* eps, int o, int nv, hipStream_t st);
// bytes of an R x K operand in the blocked split-BF16 layout
long split_bytes(long R, long K);
adc2_status pack_valence_b3(adc2_handle h, __bf16* dst, hipStream_t st);
adc2_status schur_gemm_b3(adc2_handle h, int c0, int nck, const __bf16* LvB, __bf16* Ab, float2* Z, hipStream_t st);

// ---- setup pieces reused by the adjoint (k_setup.hip) ----
// W[p][a][c] = <ac||kl> for every occupied pair p = (k<l) in row-major pair order.
adc2_status wbuild(adc2_handle h, double2* W, hipStream_t st);
// the same for a device list of pairs (k, l); epart holds npairs * nb(nb+1)/2 doubles, nb = ceil(nv / 64)
adc2_status wbuild_pairs(adc2_handle h, const int2* dpairs, int npairs, double2* W, double* epart,
                         hipStream_t st);

// ---- large-tile FP64 GEMM of two K-major grouped operands (k_adjoint.hip) ----
// C[s][i][j] = sum_{k in split s} A(k, i) B(k, j), A(k, i) = A[g*a_gstride + x + k*a_ld] with
// i = g*a_inner + x (likewise B); gridDim.y = nsplit K-splits, C holds nsplit partials.
adc2_status bgemm_kmajor(const double2* A, long a_gstride, long a_ld, int a_inner, const double2* B, long b_gstride,
                         long b_ld, int b_inner, int M, int N, int K, int nsplit, double2* C, hipStream_t st);

// ---- ADC(2)-x (adc2x.hip) ----
constexpr size_t ADC2X_MAX_BYTES = size_t(64) << 30;   // integral blocks of the first-order doubles block
adc2_status build_adc2x(adc2_handle h, hipStream_t st);
// sigma2 += (first-order doubles block) r2 for m full vectors (FP64)
adc2_status adc2x_apply(adc2_handle h, int m, const double2* x, double2* s, hipStream_t st);
// diagonal of M for the handle's method
inline const double* cur_diag(adc2_handle h) { return h->method == ADC2_METHOD_ADC2X ? h->diagx : h->diag; }

// ---- folded solver (fold.hip) ----
// per singles (K,c): nu = squared norm of column (K,c) of M21 and its |M21|^2-weighted
// mean doubles energy, into h->pre_nu / h->pre_dbar (built once per handle)
adc2_status build_fold_precond(adc2_handle h, hipStream_t st);
adc2_status fold_davidson(adc2_handle h, int k, const adc2_dav_opts* opt, const void* guess, double* omega,
                          void* Xout, adc2_dav_info* info, hipStream_t st);

// ---- adjoint (k_adjoint.hip) ----
adc2_status omega_backward(adc2_handle h, int m, const double2* X, const double* g, double2* dL, double* deps,
                           hipStream_t st);

// ---- generic GEMM helpers (k_sigma.hip) ----
// C[i][j] = alpha * sum_k A(i,k) B(k,j) (+ beta C), A row-major (k contiguous,
// lda), B given as B^T row-major (element (k,j) at B[j*ldb + k]), optional conj.
adc2_status gemm_rr(int M, int N, int K, const double2* A, long lda, bool conjA, const double2* B,
                    long ldb, bool conjB, double2* C, long ldc, double alpha, bool accumulate,
                    hipStream_t st);

// ---- Davidson kernels (k_davidson.hip) ----
adc2_status dav_gram(const double2* V, int s, const double2* W, int m, long dim, double2* G, int ldg,
                     double2* scratch, hipStream_t st);
adc2_status dav_combine(const double2* V, int s, const double2* C, int ldc, int m, long dim,
                        double2* out, double alpha, bool accumulate, hipStream_t st);
adc2_status dav_residual(const double2* V, const double2* Sg, int s, const double2* Yc, int ldy,
                         const double* theta, int k, long dim, double2* Xout, double2* R,
                         double* norms2_partial, int nblk, hipStream_t st);
adc2_status dav_precondition(double2* T, const double* theta, const double* diag, int k, long dim,
                             hipStream_t st);
adc2_status dav_heevj(const double2* G, int n, int ldg, double* w, double2* Z, int ldz,
                      hipStream_t st);
adc2_status dav_scale_columns(double2* T, int k, long dim, const double* s, hipStream_t st);
adc2_status dav_norms(const double2* T, int k, long dim, double* partial, int nblk, hipStream_t st);
adc2_status dav_unit_guess(double2* V, int g, long dim, const int* idx, hipStream_t st);
int dav_nblk(long dim);

}  // namespace adc2
