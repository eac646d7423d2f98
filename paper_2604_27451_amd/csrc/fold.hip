// fold.hip -- folded (doubles-free) Davidson solver for the lowest roots of
// the CVS-ADC(2) secular matrix (paper Eq. 11-12, CVS section).
//
// The doubles block is diagonal at second order, M22 = diag(D), so for an
// eigenvalue omega below min D the doubles are eliminated exactly:
//   x2 = (omega - D)^-1 M21 x1,
//   [M11 + M12 (omega - D)^-1 M21] x1 = omega x1.
// The search space is kept in singles only, V = {v_i}, with U_i = M21 v_i
// stored on the GPU.  The projected problem
//   G(omega) = V^H M11 V + U^H (omega - D)^-1 U
// is expanded in Chebyshev polynomials of tau(D), an affine image of
// 1/(D - w0) with w0 below the roots (or of D itself):
//   (omega - D)^-1 = sum_m g_m(omega) T_m(tau(D)),
// so that K_m = U^H T_m U is computed once per basis vector on the GPU and
// G(omega) for any omega < min D costs only host arithmetic.  Each root j
// solves lambda_j(G(omega)) = omega by safeguarded Newton steps
// (d lambda_j / d omega = -|x2|^2); the Newton update
// (lambda + omega |x2|^2) / (1 + |x2|^2) is the Rayleigh quotient of the Ritz
// vector built at omega and is the value returned.  New directions are the
// singles residuals divided by an approximate diagonal of the folded
// operator, omega - d11_e - nu_e / (omega - Dbar_e), with nu_e the squared
// norm of column e of M21 and Dbar_e its weighted mean doubles energy.
// The residual of the Ritz pair
// (x1, x2) is r1 = M11 x1 + M12 x2 - omega x1 (the doubles residual vanishes
// by construction), so each iteration applies M21 to the new directions and
// M12 to the Ritz doubles: one sigma build's worth of GEMMs per root, as in
// the full-space solver, with the doubles never entering the search space.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "hostla.h"
#include "internal.h"
#include "tile.h"

namespace adc2 {

using hostla::cplx;

namespace {

constexpr int FMM = 128;    // Chebyshev moments stored (computed on demand, 8 at a time)
constexpr int FGB = 16;     // Gram tile edge
constexpr int FCH = 32;     // doubles per LDS chunk
constexpr int FMB = 8;      // moments are held in blocks of 8
constexpr int FSMAX = 64;   // largest search space
constexpr int FCLAMP = 25;  // iterations a projected root may stay at the expansion limit
constexpr int FSTALL = 40;  // iterations without a 20% drop of the largest residual before giving up

__host__ __device__ inline int cdf(long a, long b) { return (int)((a + b - 1) / b); }

// Chebyshev moments on the FP64 matrix cores.  The weights T_m(t_d) are
// real, so with P_ij(d) = conj(U_i[d]) U_j[d]
//   Re K_m[i][j] = sum_d Re P_ij(d) T_m(t_d),  Im K_m[i][j] = sum_d Im P_ij(d) T_m(t_d)
// is a real GEMM: rows (pair, re|im), columns m, contraction over the doubles
// d.  The pairs p = i qc + jq (i < s, jq < qc) are enumerated densely, 16 per
// matrix-instruction row block; a wave owns RB row blocks, a workgroup 64 RB
// pairs x 16 NCB moments and one slice of the doubles (split-K).  A fragments
// are the products P formed in registers from the staged U rows (lane l:
// pair 16 rb + l % 16, d = 4 kstep + l / 16), so P never touches LDS or HBM;
// B fragments are T_m(t_d) of the staged chunk (cos(m arccos t_d) for the
// first two m of the slice, the three-term recurrence after).  The next
// chunk's U values are loaded into registers while the current chunk's
// matrix instructions run.  Per 4 doubles a wave issues 2 RB NCB
// v_mfma_f64_16x16x4_f64.
//   part[((tile * nz + z) * nchb + chb)][pl * NM + mm] (complex),
//   pl < 64 RB the pair within the tile, mm < NM = 16 NCB, moment m = z NM + mm.
constexpr int MKC = 32;   // doubles per staged chunk
constexpr int MPF = (FSMAX + FGB) * MKC / 256;   // staged complex values per thread and chunk (upper bound)
template <int NCB, int RB>
__global__ __launch_bounds__(256) void k_cheb_mfma(const double2* __restrict__ U, long ldu, long nd, int s, int jc0,
                                                    int qc, const double* __restrict__ D, double c, double ih,
                                                    int inv, double w0, int nchb, int nz,
                                                    double2* __restrict__ part) {
  constexpr int NM = 16 * NCB;
  constexpr int TP = 64 * RB;   // pairs per workgroup
  __shared__ double2 ui[FSMAX][MKC + 1];
  __shared__ double2 uj[FGB][MKC + 1];
  __shared__ double tb[MKC][NM + 1];
  const int tile = blockIdx.y, z = blockIdx.z;
  const int m0 = z * NM;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int jl = lane & 15, kq = lane >> 4;
  const int npair = s * qc;
  const int p0 = tile * TP;
  const int ilo = p0 / qc, ihi = min(s - 1, (min(npair, p0 + TP) - 1) / qc);
  const int nrow = ihi - ilo + 1;
  const int nstage = (nrow + qc) * MKC;
  // this lane's pair in each of its row blocks (a pair beyond the last reads zeros)
  int pi_[RB], pj_[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int p = p0 + (w * RB + rb) * 16 + jl;
    pi_[rb] = p < npair ? p / qc - ilo : -1;
    pj_[rb] = p < npair ? p % qc : 0;
  }
  d4 acc[RB][2][NCB];
#pragma unroll
  for (int a = 0; a < RB; ++a)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int b = 0; b < NCB; ++b) acc[a][q][b] = d4{0.0, 0.0, 0.0, 0.0};
  const long nch = (nd + MKC - 1) / MKC;
  // the next chunk's U values and doubles energy, loaded into registers ahead of use
  double2 pf[MPF];
  double dnext = 0.0;
  auto load = [&](long ch) {
    const long e0 = ch * MKC;
#pragma unroll
    for (int k = 0; k < MPF; ++k) {
      const int t = tid + 256 * k;
      double2 v = make_double2(0.0, 0.0);
      if (t < nstage) {
        const int row = t / MKC, e = t - row * MKC;
        const long ge = e0 + e;
        if (ge < nd) v = row < nrow ? U[(long)(ilo + row) * ldu + ge] : U[(long)(jc0 + row - nrow) * ldu + ge];
      }
      pf[k] = v;
    }
    if (tid < MKC) dnext = e0 + tid < nd ? D[e0 + tid] : 0.0;
  };
  long ch = blockIdx.x;
  if (ch < nch) load(ch);
  for (; ch < nch; ch += nchb) {
    const long e0 = ch * MKC;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < MPF; ++k) {
      const int t = tid + 256 * k;
      if (t < nstage) {
        const int row = t / MKC, e = t - row * MKC;
        if (row < nrow) ui[row][e] = pf[k];
        else uj[row - nrow][e] = pf[k];
      }
    }
    if (tid < MKC) {   // T_m(t_d), m0 <= m < m0 + NM: two cosines, then the three-term recurrence
      double tv[NM];
      if (e0 + tid < nd) {
        const double x = fmin(1.0, fmax(-1.0, ((inv ? 1.0 / (dnext - w0) : dnext) - c) * ih));
        const double th = acos(x);
        tv[0] = cos((double)m0 * th);
        tv[1] = cos((double)(m0 + 1) * th);
#pragma unroll
        for (int q = 2; q < NM; ++q) tv[q] = 2.0 * x * tv[q - 1] - tv[q - 2];
      } else {
#pragma unroll
        for (int q = 0; q < NM; ++q) tv[q] = 0.0;
      }
#pragma unroll
      for (int q = 0; q < NM; ++q) tb[tid][q] = tv[q];
    }
    __syncthreads();
    if (ch + nchb < nch) load(ch + nchb);
#pragma unroll
    for (int ks = 0; ks < MKC / 4; ++ks) {
      const int dl = ks * 4 + kq;
      double bf[NCB];
#pragma unroll
      for (int b = 0; b < NCB; ++b) bf[b] = tb[dl][b * 16 + jl];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        double pr = 0.0, pim = 0.0;
        if (pi_[rb] >= 0) {
          const double2 u = ui[pi_[rb]][dl];
          const double2 v = uj[pj_[rb]][dl];
          pr = u.x * v.x + u.y * v.y;   // conj(u) v
          pim = u.x * v.y - u.y * v.x;
        }
#pragma unroll
        for (int b = 0; b < NCB; ++b) {
          acc[rb][0][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(pr, bf[b], acc[rb][0][b], 0, 0, 0);
          acc[rb][1][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(pim, bf[b], acc[rb][1][b], 0, 0, 0);
        }
      }
    }
  }
  // accumulator (row = pair kq + 4 r of the block, column mm = 16 b + jl) -> this workgroup's partial
  double2* out = part + ((long)(tile * nz + z) * nchb + blockIdx.x) * (TP * NM);
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int b = 0; b < NCB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int pl = (w * RB + rb) * 16 + kq + 4 * r, mm = b * 16 + jl;
        out[(long)pl * NM + mm] = make_double2(acc[rb][0][b][r], acc[rb][1][b][r]);
      }
}

// K[m][i][jq] = sum_chb part of k_cheb_mfma   for m < MM, i < s, jq < qc
__global__ void k_cheb_mfma_reduce(const double2* __restrict__ part, int s, int qc, int TP, int NM, int nz, int nchb,
                                   int MM, double2* __restrict__ K) {
  const long total = (long)MM * s * qc;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int m = (int)(e / ((long)s * qc));
    const int p = (int)(e % ((long)s * qc));          // i * qc + jq
    const int tile = p / TP, pl = p % TP;
    const int z = m / NM, mm = m % NM;
    const double2* src = part + (long)(tile * nz + z) * nchb * ((long)TP * NM) + (long)pl * NM + mm;
    double2 a = make_double2(0.0, 0.0);
    for (int b = 0; b < nchb; ++b) a = cadd(a, src[(long)b * TP * NM]);
    K[e] = a;
  }
}

// out_j[d] = f_j(d) sum_{i<s} U_i[d] Y[i][j],  f_j(d) = 1 / (om_j - D_d), j < q <= 32, s <= 64
__global__ __launch_bounds__(256) void k_fold_x2(const double2* __restrict__ U, long ldu, long nd, int s,
                                                  const double2* __restrict__ Y, int q,
                                                  const double* __restrict__ om, const double* __restrict__ D,
                                                  double2* __restrict__ out, long ldo) {
  __shared__ double2 ys[FSMAX * 32];
  __shared__ double oms[32];
  for (int t = threadIdx.x; t < s * q; t += blockDim.x) ys[(t / q) * 32 + t % q] = Y[t];
  if (threadIdx.x < q) oms[threadIdx.x] = om[threadIdx.x];
  __syncthreads();
  for (long d = blockIdx.x * (long)blockDim.x + threadIdx.x; d < nd; d += (long)gridDim.x * blockDim.x) {
    const double Dd = D[d];
    // 16 roots per pass: one read of U for up to 16 roots
    for (int jb = 0; jb < q; jb += 16) {
      double2 acc[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) acc[k] = make_double2(0.0, 0.0);
      for (int i = 0; i < s; ++i) {
        const double2 u = U[(long)i * ldu + d];
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (jb + k < q) acc[k] = cadd(acc[k], cmul(u, ys[i * 32 + jb + k]));
      }
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (jb + k < q) out[(long)(jb + k) * ldo + d] = cscale(acc[k], 1.0 / (oms[jb + k] - Dd));
    }
  }
}

// In place U_j <- sum_{i<s} U_i C[i][j] for j < q <= s <= 64; one workgroup
// per 64 doubles, the block of U staged in LDS before any row is rewritten.
// C (s x q, row-major) is read with wave-uniform addresses, so only the U
// block occupies LDS (two workgroups per CU fit).
__global__ __launch_bounds__(256) void k_fold_rotate(double2* __restrict__ U, long ldu, long nd, int s,
                                                      const double2* __restrict__ C, int q) {
  __shared__ double2 us[FSMAX][65];
  const long d0 = (long)blockIdx.x * 64;
  for (int t = threadIdx.x; t < s * 64; t += blockDim.x) {
    const int i = t / 64, e = t % 64;
    us[i][e] = (d0 + e < nd) ? U[(long)i * ldu + d0 + e] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const int e = threadIdx.x & 63, jg = threadIdx.x >> 6;
  if (d0 + e < nd) {
    for (int j = jg; j < q; j += 4) {
      double2 a = make_double2(0.0, 0.0);
      for (int i = 0; i < s; ++i) a = cadd(a, cmul(us[i][e], C[i * q + j]));
      U[(long)j * ldu + d0 + e] = a;
    }
  }
}

// dst[r * ldd + e] = src[r * lds + e] for r < q, e < n  (row gather / scatter)
__global__ void k_rows_copy(const double2* __restrict__ src, long lds, double2* __restrict__ dst, long ldd, int q,
                            long n) {
  const long total = (long)q * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long r = e / n, c = e - r * n;
    dst[r * ldd + c] = src[r * lds + c];
  }
}

// min / max of D (per-block partials)
__global__ void k_minmax(const double* __restrict__ D, long n, double* __restrict__ out) {
  __shared__ double lo[256], hi[256];
  double a = 1e300, b = -1e300;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    a = fmin(a, D[e]);
    b = fmax(b, D[e]);
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + st]);
      hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = lo[0];
    out[2 * blockIdx.x + 1] = hi[0];
  }
}

// Main coupling term of the preconditioner for one virtual c = c0 + cc and
// one valence j (workgroup (cc, j)):
//   part[j][c] = ( sum_{a<b} |V_ab|^2,  sum_{a<b} |V_ab|^2 (e_a + e_b - e_j) ),
//   V_ab = <ab||cj> = Z[cc][j][a][b] - Z[cc][j][b][a],  Z[cc][j][x][y] = (x c|y j).
// 32x32 tile pairs (a-block <= b-block) through LDS so that both Z reads are
// coalesced.  Every (j, c) entry is written once: no clearing, and the sums
// over j are taken afterwards in a fixed order.
__global__ __launch_bounds__(256) void k_schur_red(const float2* __restrict__ Z, int no, int nv, int c0,
                                                    const double* __restrict__ ev, const double* __restrict__ ej,
                                                    double* __restrict__ part) {
  __shared__ float2 t1[32][33];
  __shared__ float2 t2[32][33];
  __shared__ double red[2][256];
  const int cc = blockIdx.x, j = blockIdx.y;
  const float2* C = Z + ((long)cc * no + j) * nv * nv;
  const double e_j = ej[j];
  const int tid = threadIdx.x;
  const int nb = (nv + 31) / 32;
  double s0 = 0.0, s1 = 0.0;
  for (int ab = 0; ab < nb; ++ab) {
    for (int bb = ab; bb < nb; ++bb) {
      const int a0 = ab * 32, b0 = bb * 32;
      __syncthreads();
      for (int e = tid; e < 1024; e += 256) {
        const int r = e / 32, q = e % 32;
        const int a = a0 + r, b = b0 + q;
        t1[r][q] = (a < nv && b < nv) ? C[(long)a * nv + b] : make_float2(0.f, 0.f);
        const int b2 = b0 + r, a2 = a0 + q;
        t2[r][q] = (a2 < nv && b2 < nv) ? C[(long)b2 * nv + a2] : make_float2(0.f, 0.f);
      }
      __syncthreads();
      for (int e = tid; e < 1024; e += 256) {
        const int r = e / 32, q = e % 32;
        const int a = a0 + r, b = b0 + q;
        if (a < nv && b < nv && a < b) {
          const double vx = (double)t1[r][q].x - (double)t2[q][r].x;
          const double vy = (double)t1[r][q].y - (double)t2[q][r].y;
          const double w2 = vx * vx + vy * vy;
          s0 += w2;
          s1 += w2 * (ev[a] + ev[b] - e_j);
        }
      }
    }
  }
  red[0][tid] = s0;
  red[1][tid] = s1;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
      red[0][tid] += red[0][tid + st];
      red[1][tid] += red[1][tid + st];
    }
    __syncthreads();
  }
  if (tid == 0) {
    double* o = part + ((long)j * nv + c0 + cc) * 2;
    o[0] = red[0][0];
    o[1] = red[1][0];
  }
}

// f(0..n-1) on up to 16 host threads
template <class F>
static void par_for(int n, F&& f) {
  const int nt = std::min(n, (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency())));
  if (nt <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int> next(0);
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      int i;
      while ((i = next++) < n) f(i);
    });
  for (auto& x : th) x.join();
}

struct FoldRoot {
  double omega = 0.0;            // evaluation point: x2 = (omega - D)^-1 U y
  double rq = 0.0;               // Rayleigh quotient of that (x1, x2): (lambda + omega |x2|^2) / (1 + |x2|^2)
  double n2 = 0.0;               // |x2|^2 for the unit-norm y
  std::vector<cplx> y;           // eigenvector of G(omega) for this root
  std::vector<cplx> Z;           // all eigenvectors of G(omega) (columns)
  int status = 0;                // 0 ok, 1 root not below the doubles threshold, 2 expansion too long,
                                 // 3 more moments needed (need), 4 below the shifted map's range,
                                 // 5 projected eigensolve did not converge
  int need = 0;
  int clamped = 0;               // consecutive iterations with status 1 (held at the expansion limit)
  int branch = 0;                // eigenvalue index j of lambda_j(G(omega)) = omega this entry solves
};

}  // namespace

// Diagonal of the folded operator without the omega dependence of each
// doubles energy: per singles e = (K,c), nu_e = sum_d |M21_{d,e}|^2 and the
// weighted mean Dbar_e = sum_d |M21_{d,e}|^2 D_d / nu_e, so that
//   diag[M11 + M12 (omega - D)^-1 M21]_e ~ d11_e + nu_e / (omega - Dbar_e).
// The dominant three-virtual column  <ab||cj> (same for every K) comes from
// split-BF16 GEMMs over chunks of c, Z[cc][j][a][b] = sum_P L^P_{a,c} L^P_{b,j}
// (8 nv^3 no naux flops in all, on the BF16 matrix cores; the ~1e-6 relative
// error of the split form is immaterial for a preconditioner); the light
// columns -d_ac <Kb||Ij> + d_bc <Ka||Ij> from the stored <Ka||Ij> (their
// interference with the main term is left out: this is a preconditioner).
adc2_status build_fold_precond(adc2_handle h, hipStream_t st) {
  if (!h->pre_nu.empty()) return ADC2_OK;
  const Dims& d = h->d;
  const int nc = d.nc, no = d.no, nv = d.nv, naux = d.naux, o = d.o;
  const long nvo = (long)no * nv;
  // chunk of virtuals c per GEMM: Z (complex64, nck no nv^2) within about 2 GB
  const int nck = (int)std::max<long>(1, std::min<long>(nv, (2L << 30) / (8L * nvo * nv)));
  __bf16 *Ab = nullptr, *Bown = nullptr;
  float2* Z = nullptr;
  double* part = nullptr;
  std::vector<double> eps(d.n);
  std::vector<double2> Vt((size_t)nc * no * nc * nv);
  std::vector<double> hpart((size_t)no * nv * 2);
  hipError_t e = dmalloc(h, &Ab, split_bytes((long)nck * nv, naux));
  if (e == hipSuccess) e = dmalloc(h, &Z, sizeof(float2) * nck * nvo * nv);
  if (e == hipSuccess) e = dmalloc(h, &part, sizeof(double) * 2 * nvo);
  if (e == hipSuccess && !h->LvB) e = dmalloc(h, &Bown, split_bytes(nvo, naux));
  if (e == hipSuccess) e = hipMemcpy(eps.data(), h->eps, sizeof(double) * d.n, hipMemcpyDeviceToHost);
  adc2_status rc = ADC2_OK;
  const __bf16* LvB = h->LvB ? (const __bf16*)h->LvB : Bown;
  if (e == hipSuccess && Bown) rc = pack_valence_b3(h, Bown, st);
  for (int c0 = 0; c0 < nv && e == hipSuccess && rc == ADC2_OK; c0 += nck) {
    const int nk = std::min(nck, nv - c0);
    rc = schur_gemm_b3(h, c0, nk, LvB, Ab, Z, st);
    if (rc != ADC2_OK) break;
    k_schur_red<<<dim3(nk, no), 256, 0, st>>>(Z, no, nv, c0, h->eps + o, h->eps + nc, part);
    e = hipGetLastError();
  }
  if (e == hipSuccess && rc == ADC2_OK) e = hipStreamSynchronize(st);
  if (e == hipSuccess && rc == ADC2_OK)
    e = hipMemcpy(hpart.data(), part, sizeof(double) * hpart.size(), hipMemcpyDeviceToHost);
  if (e == hipSuccess && rc == ADC2_OK)
    e = hipMemcpy(Vt.data(), h->Vt, sizeof(double2) * Vt.size(), hipMemcpyDeviceToHost);
  dfree(h, Ab);
  dfree(h, Bown);
  dfree(h, Z);
  dfree(h, part);
  if (rc != ADC2_OK) return rc;
  if (e != hipSuccess) {
    set_error(std::string("adc2_davidson: preconditioner: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? ADC2_ERR_OOM : ADC2_ERR_HIP;
  }
  // sums over j in a fixed order
  std::vector<double> hnm(2 * nv, 0.0);
  for (int j = 0; j < no; ++j)
    for (int c = 0; c < nv; ++c) {
      hnm[c] += hpart[((size_t)j * nv + c) * 2];
      hnm[nv + c] += hpart[((size_t)j * nv + c) * 2 + 1];
    }
  const double* ev = eps.data() + o;
  std::vector<double> nu((size_t)nc * nv), db((size_t)nc * nv);
  for (int K = 0; K < nc; ++K) {
    // light columns: sum over I, j and x != c of |<Kx||Ij>|^2, weighted by D = e_c + e_x - e_I - e_j
    std::vector<double> lnu(nv, 0.0), lmu(nv, 0.0);
    for (int I = 0; I < nc; ++I)
      for (int j = 0; j < no; ++j) {
        const double2* V = &Vt[(((size_t)I * no + j) * nc + K) * nv];
        double T0 = 0.0, T1 = 0.0;
        for (int x = 0; x < nv; ++x) {
          const double w2 = V[x].x * V[x].x + V[x].y * V[x].y;
          T0 += w2;
          T1 += w2 * ev[x];
        }
        const double eIj = eps[I] + eps[nc + j];
        for (int c = 0; c < nv; ++c) {
          const double wc = V[c].x * V[c].x + V[c].y * V[c].y;
          lnu[c] += T0 - wc;
          lmu[c] += (ev[c] - eIj) * (T0 - wc) + (T1 - wc * ev[c]);
        }
      }
    for (int c = 0; c < nv; ++c) {
      const double n0 = hnm[c], m0 = hnm[nv + c] - eps[K] * hnm[c];
      const double nn = n0 + lnu[c], mm = m0 + lmu[c];
      nu[(size_t)K * nv + c] = nn;
      db[(size_t)K * nv + c] = nn > 0.0 ? mm / nn : 0.0;
    }
  }
  h->pre_nu.swap(nu);
  h->pre_dbar.swap(db);
  return ADC2_OK;
}

adc2_status fold_davidson(adc2_handle h, int k, const adc2_dav_opts* opt, const void* guess, double* omega,
                          void* Xout, adc2_dav_info* info, hipStream_t st) {
  if (h->method != ADC2_METHOD_ADC2) {
    set_error("adc2_davidson (folded): needs the diagonal doubles block of ADC(2)");
    return ADC2_ERR_ARG;
  }
  const bool follow = opt && opt->follow != 0;
  const Dims& dd = h->d;
  const long ns = dd.ns, nd = dd.nd, dim = dd.dim;
  const double tol = (opt && opt->tol > 0) ? opt->tol : 1e-8;
  const int max_iter = (opt && opt->max_iter > 0) ? opt->max_iter : 300;
  const int verbose = opt ? opt->verbose : 0;
  int smax = (opt && opt->max_subspace > 0) ? opt->max_subspace : FSMAX;
  smax = std::min(smax, FSMAX);
  smax = std::max(smax, 2 * k);            // room for k Ritz vectors plus k new directions
  smax = (int)std::min<long>(smax, ns);
  if (k > smax) {
    set_error("adc2_davidson (folded): nroots exceeds the singles dimension or the search-space limit");
    return ADC2_ERR_ARG;
  }
  const int keep_max = std::max(k, std::min(2 * k, smax - k));   // vectors kept at a restart
  int nguess = (opt && opt->nguess > 0) ? opt->nguess : (k <= 8 ? 2 * k : k);
  nguess = (int)std::min<long>(std::min(nguess, smax), ns);
  const int qmax = std::max(nguess, k);
  if (follow && (!guess || nguess < k)) {
    set_error("adc2_davidson: root following needs at least nroots guess vectors");
    return ADC2_ERR_ARG;
  }
  // root following: every branch lambda_b(G(omega)) = omega of the search
  // space (b < s; the b-th root below min D is branch b) is solved and root j
  // is the one whose Ritz vector overlaps most with guess j
  const int nbr = follow ? smax : k;

  // ---- device buffers ----
  std::vector<void*> owned;
  std::vector<void*>* pinned_list = nullptr;
  auto release = [&]() {
    for (void* p : owned) dfree(h, p);
    owned.clear();
    if (pinned_list) {
      for (void* p : *pinned_list) hipHostFree(p);
      pinned_list->clear();
    }
  };
  auto dalloc = [&](void** p, size_t bytes) -> adc2_status {
    hipError_t e = dmalloc(h, p, std::max<size_t>(bytes, 16));
    if (e != hipSuccess) {
      set_error(std::string("adc2_davidson (folded): hipMalloc: ") + hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? ADC2_ERR_OOM : ADC2_ERR_HIP;
    }
    owned.push_back(*p);
    return ADC2_OK;
  };
#define FD_TRY(expr)            \
  do {                          \
    adc2_status r_ = (expr);    \
    if (r_ != ADC2_OK) {        \
      hipStreamSynchronize(st); \
      release();                \
      return r_;                \
    }                           \
  } while (0)
#define FD_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) {                                                               \
      set_error(std::string("adc2_davidson (folded): ") + #call + ": " + hipGetErrorString(e_)); \
      hipStreamSynchronize(st);                                                           \
      release();                                                                          \
      return e_ == hipErrorOutOfMemory ? ADC2_ERR_OOM : ADC2_ERR_HIP;                     \
    }                                                                                     \
  } while (0)

  double2 *Sb, *Tin, *X2, *Sx, *Kd, *part, *Yd, *Cd;
  double *omd, *mm;
  int nchb = (int)std::max<long>(1, std::min<long>(512, nd / 4096));
  if (const char* v = getenv("ADC2_CHEB_NCHB")) nchb = (int)std::max<long>(1, std::min<long>(1024, atol(v)));
  const int nmb = FMM / FMB;
  const long part_len = (long)((FSMAX + FGB - 1) / FGB) * nmb * nchb * FMB * 256;   // split-K partials of the moments
  FD_TRY(dalloc((void**)&Sb, sizeof(double2) * smax * dim));
  FD_TRY(dalloc((void**)&Tin, sizeof(double2) * qmax * dim));
  FD_TRY(dalloc((void**)&X2, sizeof(double2) * k * dim));
  FD_TRY(dalloc((void**)&Sx, sizeof(double2) * k * dim));
  FD_TRY(dalloc((void**)&Kd, sizeof(double2) * FMM * smax * FGB));
  FD_TRY(dalloc((void**)&part, sizeof(double2) * part_len));
  FD_TRY(dalloc((void**)&Yd, sizeof(double2) * FSMAX * FSMAX));
  FD_TRY(dalloc((void**)&Cd, sizeof(double2) * FSMAX * FSMAX));
  FD_TRY(dalloc((void**)&omd, sizeof(double) * 32));
  FD_TRY(dalloc((void**)&mm, sizeof(double) * 2 * 256));
  // Host <-> device traffic goes through pinned staging and contiguous device
  // rows only; strided rows are gathered / scattered by k_rows_copy.
  double2* Rowc;
  FD_TRY(dalloc((void**)&Rowc, sizeof(double2) * qmax * ns));
  std::vector<void*> pinned;
  auto release_pinned = [&]() {
    for (void* p : pinned) hipHostFree(p);
    pinned.clear();
  };
  auto palloc = [&](void** p, size_t bytes) -> adc2_status {
    hipError_t e = hipHostMalloc(p, std::max<size_t>(bytes, 16), hipHostMallocDefault);
    if (e != hipSuccess) {
      set_error(std::string("adc2_davidson (folded): hipHostMalloc: ") + hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? ADC2_ERR_OOM : ADC2_ERR_HIP;
    }
    pinned.push_back(*p);
    return ADC2_OK;
  };
  pinned_list = &pinned;
  cplx *hRow, *hK, *hY;
  double* hD;
  {
    adc2_status r = palloc((void**)&hRow, sizeof(cplx) * qmax * ns);
    if (r == ADC2_OK) r = palloc((void**)&hK, sizeof(cplx) * FMM * smax * FGB);
    if (r == ADC2_OK) r = palloc((void**)&hY, sizeof(cplx) * FSMAX * FSMAX);
    if (r == ADC2_OK) r = palloc((void**)&hD, sizeof(double) * std::max<long>(512 + 32, ns));
    if (r != ADC2_OK) {
      release_pinned();
      release();
      return r;
    }
  }
  const unsigned rgrid = (unsigned)std::min<long>(4096, ((long)qmax * ns + 255) / 256);
  // host rows (q x ns) -> device rows with stride dim
  auto h2d_rows = [&](const cplx* host, int q, double2* dst) -> adc2_status {
    memcpy(hRow, host, sizeof(cplx) * q * ns);
    ADC2_HIP(hipMemcpyAsync(Rowc, hRow, sizeof(double2) * q * ns, hipMemcpyHostToDevice, st));
    k_rows_copy<<<rgrid, 256, 0, st>>>(Rowc, ns, dst, dim, q, ns);
    ADC2_CHECK_LAUNCH();
    ADC2_HIP(hipStreamSynchronize(st));
    return ADC2_OK;
  };
  // device rows with stride dim (singles block) -> host rows (q x ns)
  auto d2h_rows = [&](const double2* src, int q, cplx* host) -> adc2_status {
    k_rows_copy<<<rgrid, 256, 0, st>>>(src, dim, Rowc, ns, q, ns);
    ADC2_CHECK_LAUNCH();
    ADC2_HIP(hipMemcpyAsync(hRow, Rowc, sizeof(double2) * q * ns, hipMemcpyDeviceToHost, st));
    ADC2_HIP(hipStreamSynchronize(st));
    memcpy(host, hRow, sizeof(cplx) * q * ns);
    return ADC2_OK;
  };
  // small host array -> device, through pinned staging
  auto h2d_small = [&](void* dst, const void* src, size_t bytes) -> adc2_status {
    memcpy(hY, src, bytes);
    ADC2_HIP(hipMemcpyAsync(dst, hY, bytes, hipMemcpyHostToDevice, st));
    ADC2_HIP(hipStreamSynchronize(st));
    return ADC2_OK;
  };
  const double* Ddev = h->diag + ns;       // doubles diagonal D
  const double2* Uro = nullptr;            // doubles part of Sb rows
  double2* Urw = Sb + ns;
  Uro = Urw;

  FD_TRY(build_fold_precond(h, st));
  const std::vector<double>& pnu = h->pre_nu;
  const std::vector<double>& pdb = h->pre_dbar;

  // ---- Chebyshev interval ----
  k_minmax<<<256, 256, 0, st>>>(Ddev, nd, mm);
  FD_HIP(hipGetLastError());
  std::vector<double> hm(512), d11(ns);
  FD_HIP(hipMemcpyAsync(hD, mm, sizeof(double) * 512, hipMemcpyDeviceToHost, st));
  FD_HIP(hipStreamSynchronize(st));
  memcpy(hm.data(), hD, sizeof(double) * 512);
  FD_HIP(hipMemcpyAsync(hD, h->diag, sizeof(double) * ns, hipMemcpyDeviceToHost, st));
  FD_HIP(hipStreamSynchronize(st));
  memcpy(d11.data(), hD, sizeof(double) * ns);
  double Dmin = 1e300, Dmax = -1e300;
  for (int b = 0; b < 256; ++b) {
    Dmin = std::min(Dmin, hm[2 * b]);
    Dmax = std::max(Dmax, hm[2 * b + 1]);
  }
  // Expansion variable of the moments: the shifted inverse 1/(D - w0), with
  // w0 below an estimate of the lowest root (the lower solution of
  // omega = d11_e + nu_e / (omega - Dbar_e) over the singles e), needs far
  // fewer terms than D itself; w0 is lowered, with all moments recomputed, if
  // a root falls below w0 + 0.1 (Dmin - w0).  The linear variable remains
  // for an estimate that is not below Dmin.
  hostla::ResolventMap rmap = hostla::ResolventMap::linear(Dmin, Dmax);
  double west = 1e300;
  for (long e = 0; e < ns; ++e) {
    const double a = d11[e], bb = pdb[e], nu = pnu[e];
    const double r = nu > 0.0 ? 0.5 * ((a + bb) - std::sqrt((a - bb) * (a - bb) + 4.0 * nu)) : a;
    west = std::min(west, r);
  }
  if (west < Dmin && std::isfinite(west))
    rmap = hostla::ResolventMap::shifted_inverse(Dmin, Dmax, west - std::max(1.0, 0.5 * (Dmin - west)));

  // ---- host state ----
  std::vector<cplx> Vs((size_t)smax * ns), S1((size_t)smax * ns), H11((size_t)smax * smax);
  std::vector<cplx> K((size_t)FMM * smax * smax);
  int s = 0;
  long n21 = 0, n12 = 0;
  double ms_sigma = 0.0;
  hipEvent_t e0, e1;
  FD_HIP(hipEventCreate(&e0));
  FD_HIP(hipEventCreate(&e1));
  auto sig_time = [&](int m, const double2* xin, double2* sout, int parts) -> adc2_status {
    ADC2_HIP(hipEventRecord(e0, st));
    adc2_status r = sigma_call(h, m, xin, sout, parts, st);
    if (r != ADC2_OK) return r;
    ADC2_HIP(hipEventRecord(e1, st));
    ADC2_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    ADC2_HIP(hipEventElapsedTime(&ms, e0, e1));
    ms_sigma += ms;
    return ADC2_OK;
  };
  auto cleanup_events = [&]() {
    hipEventDestroy(e0);
    hipEventDestroy(e1);
  };

  // Chebyshev moments K_m[i][j] for rows i < srows and columns [j0, j0 + q), m < 16 * mblocks
  // moment blocks held for every basis vector: with the shifted map, enough
  // for the root estimate plus two terms (more are added on demand)
  int mcomp = 3;
  if (rmap.inv) {
    std::vector<double> b(FMM), e(FMM), g(FMM), hq(FMM);
    const int M = rmap.coeffs(west, FMM, b.data(), e.data(), g.data(), hq.data());
    if (M > 0) mcomp = std::min(nmb, std::max(1, (M + 2 + FMB - 1) / FMB));
  }
  if (verbose)
    fprintf(stderr, "[adc2 folded no=%d nv=%d] D in [%.6f, %.6f], root estimate %.6f, %s map w0 %.6f, %d moments\n",
            dd.no, dd.nv, Dmin, Dmax, west, rmap.inv ? "shifted-inverse" : "linear", rmap.w0, FMB * mcomp);
  cplx* Kh = hK;
  double tm_cheb = 0.0;
  auto cheb_cols = [&](int srows, int j0, int q, int mblocks) -> adc2_status {
    const auto tc0 = std::chrono::steady_clock::now();
    for (int c0 = j0; c0 < j0 + q; c0 += FGB) {
      const int qc = std::min(FGB, j0 + q - c0);
      const int mm_ = mblocks * FMB;
      const long tot = (long)mm_ * srows * qc;
      // 16 or 32 moments per pass (z-slices for more); 128 or 256 pairs per workgroup
      const int ncb = mm_ > 16 ? 2 : 1;
      const int nm = 16 * ncb;
      const int nz = (mm_ + nm - 1) / nm;
      const int npair = srows * qc;
      const int rb = npair > 128 ? 4 : 2;
      const int tp = 64 * rb;
      const int ntile = (npair + tp - 1) / tp;
      int nch_m = (int)std::max<long>(1, std::min<long>(nchb, (nd + MKC - 1) / MKC));
      while (nch_m > 1 && (long)ntile * nz * nch_m * tp * nm > part_len) nch_m /= 2;
      dim3 g(nch_m, ntile, nz);
#define CHEB_MFMA(NCB_, RB_)                                                                              \
  k_cheb_mfma<NCB_, RB_><<<g, 256, 0, st>>>(Uro, dim, nd, srows, c0, qc, Ddev, rmap.c, rmap.ih, rmap.inv, \
                                           rmap.w0, nch_m, nz, part)
      if (ncb == 1 && rb == 4) CHEB_MFMA(1, 4);
      else if (ncb == 1) CHEB_MFMA(1, 2);
      else if (rb == 4) CHEB_MFMA(2, 4);
      else CHEB_MFMA(2, 2);
#undef CHEB_MFMA
      ADC2_CHECK_LAUNCH();
      k_cheb_mfma_reduce<<<(unsigned)std::min<long>(4096, (tot + 255) / 256), 256, 0, st>>>(part, srows, qc, tp,
                                                                                            nm, nz, nch_m, mm_, Kd);
      ADC2_CHECK_LAUNCH();
      ADC2_HIP(hipMemcpyAsync(Kh, Kd, sizeof(double2) * tot, hipMemcpyDeviceToHost, st));
      ADC2_HIP(hipStreamSynchronize(st));
      for (int m = 0; m < mm_; ++m)
        for (int i = 0; i < srows; ++i)
          for (int j = 0; j < qc; ++j) {
            const cplx v = Kh[((size_t)m * srows + i) * qc + j];
            K[((size_t)m * smax + i) * smax + c0 + j] = v;
            K[((size_t)m * smax + c0 + j) * smax + i] = std::conj(v);
          }
    }
    tm_cheb += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tc0).count();
    return ADC2_OK;
  };

  // append q orthonormal singles vectors T (host, q x ns): sigma of (v, 0), moments
  auto add_vectors = [&](const std::vector<cplx>& T, int q) -> adc2_status {
    adc2_status r = h2d_rows(T.data(), q, Tin);
    if (r != ADC2_OK) return r;
    r = sig_time(q, Tin, Sb + (long)s * dim, SIGMA_SINGLES_IN);
    if (r != ADC2_OK) return r;
    n21 += q;
    r = d2h_rows(Sb + (long)s * dim, q, S1.data() + (size_t)s * ns);
    if (r != ADC2_OK) return r;
    for (int j = 0; j < q; ++j)
      std::copy(T.begin() + (size_t)j * ns, T.begin() + (size_t)(j + 1) * ns, Vs.begin() + (size_t)(s + j) * ns);
    const int snew = s + q;
    r = cheb_cols(snew, s, q, mcomp);
    if (r != ADC2_OK) return r;
    par_for(snew, [&](int i) {
      for (int j = s; j < snew; ++j) {
        cplx a = 0.0;
        const cplx* vi = &Vs[(size_t)i * ns];
        const cplx* sj = &S1[(size_t)j * ns];
        for (long e = 0; e < ns; ++e) a += std::conj(vi[e]) * sj[e];
        H11[(size_t)i * smax + j] = a;
      }
    });
    for (int i = 0; i < snew; ++i)
      for (int j = s; j < snew; ++j) H11[(size_t)j * smax + i] = std::conj(H11[(size_t)i * smax + j]);
    for (int j = s; j < snew; ++j) H11[(size_t)j * smax + j] = H11[(size_t)j * smax + j].real();
    s = snew;
    return ADC2_OK;
  };

  // orthonormalise rows of T against Vs[0..s) and among themselves; returns the kept count
  auto orthonormalise = [&](std::vector<cplx>& T, int q) -> int {
    std::vector<double> n0(q);
    // against the space (two classical Gram-Schmidt passes, rows in parallel)
    par_for(q, [&](int r) {
      cplx* t = &T[(size_t)r * ns];
      double a0 = 0.0;
      for (long e = 0; e < ns; ++e) a0 += std::norm(t[e]);
      n0[r] = std::sqrt(a0);
      for (int pass = 0; pass < 2; ++pass) {
        std::vector<cplx> a(s);
        for (int i = 0; i < s; ++i) {
          const cplx* v = &Vs[(size_t)i * ns];
          cplx acc = 0.0;
          for (long e = 0; e < ns; ++e) acc += std::conj(v[e]) * t[e];
          a[i] = acc;
        }
        for (int i = 0; i < s; ++i) {
          const cplx* v = &Vs[(size_t)i * ns];
          for (long e = 0; e < ns; ++e) t[e] -= a[i] * v[e];
        }
      }
    });
    // among themselves (modified Gram-Schmidt, two passes)
    int kept = 0;
    for (int r = 0; r < q; ++r) {
      cplx* t = &T[(size_t)r * ns];
      if (!(n0[r] > 0.0) || !std::isfinite(n0[r])) continue;
      for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i < kept; ++i) {
          const cplx* v = &T[(size_t)i * ns];
          cplx a = 0.0;
          for (long e = 0; e < ns; ++e) a += std::conj(v[e]) * t[e];
          for (long e = 0; e < ns; ++e) t[e] -= a * v[e];
        }
      double n1 = 0.0;
      for (long e = 0; e < ns; ++e) n1 += std::norm(t[e]);
      n1 = std::sqrt(n1);
      if (n1 <= 1e-10 * n0[r]) continue;
      for (long e = 0; e < ns; ++e) t[e] /= n1;
      if (kept != r) std::copy(t, t + ns, &T[(size_t)kept * ns]);
      ++kept;
    }
    return kept;
  };

  // ---- initial space ----
  std::vector<cplx> gref;   // singles of the followed guess vectors, as given
  {
    std::vector<cplx> T((size_t)nguess * ns, cplx(0.0, 0.0));
    if (guess) {
      FD_TRY(d2h_rows((const double2*)guess, nguess, T.data()));
      if (follow) gref.assign(T.begin(), T.begin() + (size_t)k * ns);
    } else {
      std::vector<int> idx(ns);
      for (long i = 0; i < ns; ++i) idx[i] = (int)i;
      std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return d11[a] < d11[b]; });
      for (int g = 0; g < nguess; ++g) T[(size_t)g * ns + idx[g]] = 1.0;
    }
    const int q = orthonormalise(T, nguess);
    if (q < k) {
      cleanup_events();
      release();
      set_error("adc2_davidson (folded): the initial space has fewer vectors than roots");
      return ADC2_ERR_ARG;
    }
    adc2_status r = add_vectors(T, q);
    if (r != ADC2_OK) {
      cleanup_events();
      hipStreamSynchronize(st);
      release();
      return r;
    }
  }

  std::vector<FoldRoot> roots(nbr);
  for (int b = 0; b < nbr; ++b) roots[b].branch = b;
  std::vector<char> prov(k, 0);   // root held at the expansion limit this iteration
  std::vector<double> res(k, 1e300);
  bool have_omega = false, converged = false;
  int it = 0;
  // stagnation: the largest residual has not dropped below 0.8 of its best
  // value for FSTALL iterations (the precision form's noise floor)
  double best_rmax = 1e300;
  int best_it = 0;
  std::vector<cplx> x1((size_t)k * ns), r1((size_t)k * ns), mx2((size_t)k * ns);
  std::vector<double> nrm(k);
  const auto t_start = std::chrono::steady_clock::now();
  adc2_status final_rc = ADC2_OK;
  double tm_proj = 0.0, tm_res = 0.0, tm_new = 0.0;   // host-side phases (ms)
  auto now = []() { return std::chrono::steady_clock::now(); };
  auto ms_since = [](std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  };

  for (it = 1; it <= max_iter; ++it) {
    // ---- projected nonlinear problem, one thread per root ----
    const auto tp0 = now();
    double lam_min;
    {
      std::vector<double> w(s);
      std::vector<cplx> Z((size_t)s * s), Hs((size_t)s * s);
      for (int i = 0; i < s; ++i)
        for (int j = 0; j < s; ++j) Hs[(size_t)i * s + j] = H11[(size_t)i * smax + j];
      if (hostla::herm_eig(s, Hs.data(), w.data(), Z.data()) != 0) {
        set_error("adc2_davidson (folded): the eigensolve of the projected singles block did not converge");
        final_rc = ADC2_ERR_NOCONV;
        break;
      }
      lam_min = w[0];
    }
    double T0 = 0.0;
    for (int i = 0; i < s; ++i) T0 += K[(size_t)i * smax + i].real();
    const double zb = 0.5 * (-(lam_min - Dmin) + std::sqrt((lam_min - Dmin) * (lam_min - Dmin) + 4.0 * std::max(T0, 0.0))) + 1.0;
    const double lo0 = Dmin - zb;
    // a pole at |x| >= 1.05 has r = |x| - sqrt(x^2 - 1) < 0.73 and r^126 < 1e-17,
    // so at most 126 Chebyshev terms: with the shifted inverse, roots closer
    // to min D than about 0.025 (min D - w0) are out of reach of this solver
    double hi0 = rmap.reach(1.05);
    double wlo = rmap.inv ? std::max(lo0, rmap.w0 + 0.1 * (Dmin - rmap.w0)) : lo0;   // lowest omega evaluated
    auto solve_root = [&](int idx) {
      FoldRoot& R = roots[idx];
      const int j = R.branch;
      if (j >= s) {   // fewer basis vectors than this branch index
        R.status = 6;
        return;
      }
      double wv = have_omega ? R.omega : wlo;
      if (!(wv > wlo && wv < hi0)) wv = have_omega ? std::min(std::max(wv, wlo), hi0 - 1e-9 * std::fabs(hi0)) : wlo;
      double lo = wlo, hi = hi0;
      std::vector<double> b(FMM), e(FMM), w(s), gco(FMM), eco(FMM);
      std::vector<cplx> G((size_t)s * s), Z((size_t)s * s), Zp;
      // warm start from this root's last eigenvector basis, padded with the identity for the new vectors
      const int zs = R.Z.empty() ? 0 : (int)std::lround(std::sqrt((double)R.Z.size()));
      if (zs > 0 && zs <= s) {
        Zp.assign((size_t)s * s, cplx(0.0, 0.0));
        for (int i = 0; i < zs; ++i)
          for (int l = 0; l < zs; ++l) Zp[(size_t)i * s + l] = R.Z[(size_t)i * zs + l];
        for (int i = zs; i < s; ++i) Zp[(size_t)i * s + i] = 1.0;
      }
      R.status = 0;
      for (int nit = 0; nit < 80; ++nit) {
        // G = H11 + sum_m gco_m K_m,  |x2|^2 = y^H (sum_m eco_m K_m) y
        const int M = rmap.coeffs(wv, FMM, b.data(), e.data(), gco.data(), eco.data());
        if (M < 0) {
          R.status = 2;
          return;
        }
        if (M > FMB * mcomp) {
          R.status = 3;
          R.need = M;
          return;
        }
        for (int i = 0; i < s; ++i)
          for (int l = 0; l < s; ++l) {
            cplx a = H11[(size_t)i * smax + l];
            for (int m = 0; m < M; ++m) a += gco[m] * K[((size_t)m * smax + i) * smax + l];
            G[(size_t)i * s + l] = a;
          }
        for (int i = 0; i < s; ++i) {
          G[(size_t)i * s + i] = G[(size_t)i * s + i].real();
          for (int l = i + 1; l < s; ++l) {
            const cplx a = 0.5 * (G[(size_t)i * s + l] + std::conj(G[(size_t)l * s + i]));
            G[(size_t)i * s + l] = a;
            G[(size_t)l * s + i] = std::conj(a);
          }
        }
        const int bad = Zp.empty() ? hostla::herm_eig(s, G.data(), w.data(), Z.data())
                                   : hostla::herm_eig_warm(s, G.data(), Zp.data(), w.data(), Z.data());
        if (bad != 0) {
          R.status = 5;
          return;
        }
        Zp = Z;
        // |x2|^2 = y^H E y,  E = sum eco_m K_m
        double n2 = 0.0;
        {
          std::vector<cplx> y(s);
          for (int i = 0; i < s; ++i) y[i] = Z[(size_t)i * s + j];
          cplx acc = 0.0;
          for (int i = 0; i < s; ++i) {
            cplx row = 0.0;
            for (int l = 0; l < s; ++l) {
              cplx kk = 0.0;
              for (int m = 0; m < M; ++m) kk += eco[m] * K[((size_t)m * smax + i) * smax + l];
              row += kk * y[l];
            }
            acc += std::conj(y[i]) * row;
          }
          n2 = acc.real();
        }
        const double f = w[j] - wv;
        if (f > 0.0) lo = std::max(lo, wv);
        else hi = std::min(hi, wv);
        double wn = wv + f / (1.0 + std::max(n2, 0.0));
        if (!(wn > lo && wn < hi)) wn = 0.5 * (lo + hi);
        // (wv, y) is an exact eigenpair of G(wv); its distance to the root is ~|wn - wv|, which only has
        // to stay well below the residual tolerance of the outer iteration
        const double wtol = std::min(1e-10, 1e-3 * tol) * std::max(1.0, std::fabs(wv));
        const bool done = std::fabs(wn - wv) <= wtol || (hi - lo) <= 1e-15 * std::max(1.0, std::fabs(wv));
        R.omega = wv;
        R.rq = (w[j] + wv * std::max(n2, 0.0)) / (1.0 + std::max(n2, 0.0));
        R.n2 = n2;
        R.y.assign(s, 0.0);
        for (int i = 0; i < s; ++i) R.y[i] = Z[(size_t)i * s + j];
        R.Z = Z;
        if (done) break;
        wv = wn;
      }
      if (!(R.omega < hi0 - 1e-12 * std::fabs(hi0))) R.status = 1;
      // the root lies below the lowest point the shifted map may evaluate
      if (rmap.inv && wlo > lo0 && R.omega <= wlo + 1e-9 * std::max(1.0, std::fabs(wlo))) R.status = 4;
    };
    for (int attempt = 0; attempt < 4; ++attempt) {
      {
        std::vector<std::thread> th;
        for (int j = 1; j < nbr; ++j) th.emplace_back(solve_root, j);
        solve_root(0);
        for (auto& t : th) t.join();
      }
      int need = 0;
      bool below = false;
      for (int j = 0; j < nbr; ++j) {
        if (roots[j].status == 3) need = std::max(need, roots[j].need);
        if (roots[j].status == 4) below = true;
      }
      if (below) {
        // a root below the shifted map's range: move the shift down (twice as
        // far from min D) and recompute the moments of the whole space
        rmap = hostla::ResolventMap::shifted_inverse(Dmin, Dmax, Dmin - 3.0 * (Dmin - rmap.w0));
        hi0 = rmap.reach(1.05);
        wlo = std::max(lo0, rmap.w0 + 0.1 * (Dmin - rmap.w0));
        have_omega = false;
        FD_TRY(cheb_cols(s, 0, s, mcomp));
        continue;
      }
      if (need == 0) break;
      // more Chebyshev moments: recompute them for the whole space
      mcomp = std::min(nmb, (need + FMB - 1) / FMB);
      FD_TRY(cheb_cols(s, 0, s, mcomp));
    }
    if (follow) {
      // root j = the branch whose Ritz vector (x1 = V y, |x|^2 = 1 + |x2|^2)
      // overlaps most with the singles of guess j, assigned greedily in
      // decreasing order of overlap; the chosen entries move to the front
      std::vector<cplx> pg((size_t)k * s);
      std::vector<double> gn(k, 0.0);
      par_for(k, [&](int j) {
        const cplx* g = &gref[(size_t)j * ns];
        for (long e = 0; e < ns; ++e) gn[j] += std::norm(g[e]);
        for (int i = 0; i < s; ++i) {
          const cplx* v = &Vs[(size_t)i * ns];
          cplx a = 0.0;
          for (long e = 0; e < ns; ++e) a += std::conj(v[e]) * g[e];
          pg[(size_t)j * s + i] = a;
        }
      });
      std::vector<double> ov((size_t)k * nbr, -1.0);
      for (int b = 0; b < nbr; ++b) {
        const FoldRoot& R = roots[b];
        if ((R.status != 0 && R.status != 1) || (int)R.y.size() != s) continue;
        for (int j = 0; j < k; ++j) {
          cplx a = 0.0;
          for (int i = 0; i < s; ++i) a += std::conj(pg[(size_t)j * s + i]) * R.y[i];
          ov[(size_t)j * nbr + b] = std::norm(a) / ((1.0 + std::max(R.n2, 0.0)) * std::max(gn[j], 1e-300));
        }
      }
      std::vector<int> sel(k, -1);
      std::vector<char> used(nbr, 0);
      for (int n = 0; n < k; ++n) {
        int bj = -1, bb = -1;
        double best = -2.0;
        for (int j = 0; j < k; ++j) {
          if (sel[j] >= 0) continue;
          for (int b = 0; b < nbr; ++b)
            if (!used[b] && ov[(size_t)j * nbr + b] > best) {
              best = ov[(size_t)j * nbr + b];
              bj = j;
              bb = b;
            }
        }
        sel[bj] = bb;
        used[bb] = 1;
      }
      std::vector<FoldRoot> re;
      re.reserve(nbr);
      for (int j = 0; j < k; ++j) re.push_back(roots[sel[j]]);
      for (int b = 0; b < nbr; ++b)
        if (!used[b]) re.push_back(roots[b]);
      roots.swap(re);
    }
    // A projected root that is not below the limit of the resolvent expansion
    // (status 1) is held there, as an unconverged Ritz pair of G at that
    // point, while the search space grows: with a poor early space the
    // projected root lies above the true one (interlacing).  It fails only if
    // it stays there for FCLAMP iterations in a row.
    for (int j = 0; j < k; ++j) {
      if (roots[j].status == 1 && ++roots[j].clamped <= FCLAMP) {
        roots[j].status = 0;
        prov[j] = 1;
        continue;
      }
      if (roots[j].status == 0) {
        roots[j].clamped = 0;
        prov[j] = 0;
      }
    }
    for (int j = 0; j < k; ++j) {
      if (roots[j].status != 0) {
        char buf[200];
        if (roots[j].status == 5)
          snprintf(buf, sizeof buf, "adc2_davidson (folded): the projected eigensolve of root %d did not converge",
                   j);
        else
          snprintf(buf, sizeof buf,
                   "adc2_davidson (folded): root %d is not below the doubles threshold min D = %.6f (use the "
                   "full-space solver)",
                   j, Dmin);
        set_error(buf);
        final_rc = ADC2_ERR_NOCONV;
        break;
      }
    }
    if (final_rc != ADC2_OK) break;
    have_omega = true;
    tm_proj += ms_since(tp0);
    const auto tr0 = now();

    // ---- Ritz vectors and residuals ----
    std::vector<cplx> Yc((size_t)s * k);
    std::vector<double> om(k);
    for (int j = 0; j < k; ++j) {
      om[j] = roots[j].omega;
      for (int i = 0; i < s; ++i) Yc[(size_t)i * k + j] = roots[j].y[i];
      nrm[j] = std::sqrt(1.0 + std::max(roots[j].n2, 0.0));
    }
    FD_TRY(h2d_small(Yd, Yc.data(), sizeof(double2) * s * k));
    FD_TRY(h2d_small(omd, om.data(), sizeof(double) * k));
    k_fold_x2<<<(unsigned)std::min<long>(16384, (nd + 255) / 256), 256, 0, st>>>(Uro, dim, nd, s, Yd, k, omd, Ddev,
                                                                                X2 + ns, dim);
    FD_HIP(hipGetLastError());
    FD_TRY(sig_time(k, X2, Sx, SIGMA_DOUBLES_IN));
    n12 += k;
    FD_TRY(d2h_rows(Sx, k, mx2.data()));
    double rmax = 0.0;
    par_for(k, [&](int j) {
      cplx* xj = &x1[(size_t)j * ns];
      cplx* rj = &r1[(size_t)j * ns];
      for (long e = 0; e < ns; ++e) {
        xj[e] = 0.0;
        rj[e] = mx2[(size_t)j * ns + e];
      }
      for (int i = 0; i < s; ++i) {
        const cplx y = roots[j].y[i];
        const cplx* v = &Vs[(size_t)i * ns];
        const cplx* sv = &S1[(size_t)i * ns];
        for (long e = 0; e < ns; ++e) {
          xj[e] += y * v[e];
          rj[e] += y * sv[e];
        }
      }
      double rr = 0.0;
      for (long e = 0; e < ns; ++e) {
        rj[e] -= om[j] * xj[e];
        rr += std::norm(rj[e]);
      }
      res[j] = std::sqrt(rr) / nrm[j];
    });
    for (int j = 0; j < k; ++j) rmax = std::max(rmax, res[j]);
    tm_res += ms_since(tr0);
    if (verbose) {
      fprintf(stderr, "[adc2 folded no=%d nv=%d] it %3d  space %2d  max|r| %.3e  omega0 %.12f\n", dd.no, dd.nv, it,
              s, rmax, om[0]);
    }
    bool any_prov = false;
    for (int j = 0; j < k; ++j) any_prov = any_prov || prov[j];
    if (rmax <= tol && !any_prov) {
      converged = true;
      break;
    }
    if (it == max_iter) break;
    if (rmax < 0.8 * best_rmax) {
      best_rmax = rmax;
      best_it = it;
    } else if (!any_prov && it - best_it >= FSTALL) {
      char buf[320];
      snprintf(buf, sizeof buf,
               "adc2_davidson (folded): residual stagnated at %.3e for %d iterations (tolerance %.1e is below "
               "the noise floor of the sigma arithmetic, or a requested root lies too close to min D = %.6f for "
               "the folded solver: use the full-space solver)",
               rmax, FSTALL, tol, Dmin);
      set_error(buf);
      final_rc = ADC2_ERR_NOCONV;
      break;
    }

    // ---- new directions: diagonal preconditioner on the singles ----
    const auto tn0 = now();
    std::vector<cplx> T((size_t)k * ns);
    int q = 0;
    for (int j = 0; j < k; ++j) {
      if (res[j] <= tol && !prov[j]) continue;
      cplx* t = &T[(size_t)q * ns];
      for (long e = 0; e < ns; ++e) {
        // approximate diagonal of the folded operator minus omega
        double den = om[j] - d11[e];
        const double gap = om[j] - pdb[e];
        if (pnu[e] > 0.0 && std::fabs(gap) > 1e-12) den -= pnu[e] / gap;
        if (std::fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
        t[e] = r1[(size_t)j * ns + e] / den;
      }
      ++q;
    }
    // ---- restart: keep the Ritz singles of every root and the next ones of the highest root ----
    if (s + q > smax) {
      const int nk = std::min(keep_max, s);
      std::vector<cplx> C((size_t)s * nk, 0.0);
      for (int j = 0; j < k && j < nk; ++j)
        for (int i = 0; i < s; ++i) C[(size_t)i * nk + j] = roots[j].y[i];
      for (int c = k; c < nk; ++c)
        for (int i = 0; i < s; ++i) C[(size_t)i * nk + c] = roots[k - 1].Z[(size_t)i * s + c];
      // orthonormalise the columns of C (modified Gram-Schmidt, two passes)
      int kc = 0;
      for (int c = 0; c < nk; ++c) {
        for (int pass = 0; pass < 2; ++pass)
          for (int p = 0; p < kc; ++p) {
            cplx a = 0.0;
            for (int i = 0; i < s; ++i) a += std::conj(C[(size_t)i * nk + p]) * C[(size_t)i * nk + c];
            for (int i = 0; i < s; ++i) C[(size_t)i * nk + c] -= a * C[(size_t)i * nk + p];
          }
        double nn = 0.0;
        for (int i = 0; i < s; ++i) nn += std::norm(C[(size_t)i * nk + c]);
        nn = std::sqrt(nn);
        if (nn < 1e-8) continue;
        for (int i = 0; i < s; ++i) C[(size_t)i * nk + kc] = C[(size_t)i * nk + c] / nn;
        ++kc;
      }
      std::vector<cplx> Cc((size_t)s * kc);
      for (int i = 0; i < s; ++i)
        for (int c = 0; c < kc; ++c) Cc[(size_t)i * kc + c] = C[(size_t)i * nk + c];
      FD_TRY(h2d_small(Cd, Cc.data(), sizeof(double2) * s * kc));
      k_fold_rotate<<<(unsigned)((nd + 63) / 64), 256, 0, st>>>(Urw, dim, nd, s, Cd, kc);
      FD_HIP(hipGetLastError());
      // Cc is pageable host memory local to this block: the copy must have
      // consumed it before the block ends
      FD_HIP(hipStreamSynchronize(st));
      // host side: V, S1, H11, K
      auto rot_rows = [&](std::vector<cplx>& A) {
        std::vector<cplx> out((size_t)kc * ns, 0.0);
        for (int c = 0; c < kc; ++c)
          for (int i = 0; i < s; ++i) {
            const cplx w = Cc[(size_t)i * kc + c];
            if (w == cplx(0.0, 0.0)) continue;
            for (long e = 0; e < ns; ++e) out[(size_t)c * ns + e] += w * A[(size_t)i * ns + e];
          }
        std::copy(out.begin(), out.end(), A.begin());
      };
      rot_rows(Vs);
      rot_rows(S1);
      auto rot_mat = [&](cplx* A) {   // A (s x s, ld smax) <- C^H A C
        std::vector<cplx> T1((size_t)s * kc, 0.0), T2((size_t)kc * kc, 0.0);
        for (int i = 0; i < s; ++i)
          for (int c = 0; c < kc; ++c) {
            cplx a = 0.0;
            for (int l = 0; l < s; ++l) a += A[(size_t)i * smax + l] * Cc[(size_t)l * kc + c];
            T1[(size_t)i * kc + c] = a;
          }
        for (int r = 0; r < kc; ++r)
          for (int c = 0; c < kc; ++c) {
            cplx a = 0.0;
            for (int i = 0; i < s; ++i) a += std::conj(Cc[(size_t)i * kc + r]) * T1[(size_t)i * kc + c];
            T2[(size_t)r * kc + c] = a;
          }
        for (int r = 0; r < kc; ++r)
          for (int c = 0; c < kc; ++c) A[(size_t)r * smax + c] = T2[(size_t)r * kc + c];
      };
      rot_mat(H11.data());
      for (int m = 0; m < FMB * mcomp; ++m) rot_mat(&K[(size_t)m * smax * smax]);
      for (int j = 0; j < nbr; ++j) {
        roots[j].y.clear();
        roots[j].Z.clear();   // the basis changed: next solve starts cold
      }
      s = kc;
    }
    const int qk = orthonormalise(T, q);
    if (qk == 0) {
      set_error("adc2_davidson (folded): no new search directions (stagnation)");
      final_rc = ADC2_ERR_NOCONV;
      break;
    }
    tm_new += ms_since(tn0);
    FD_TRY(add_vectors(T, qk));
  }
  if (verbose)
    fprintf(stderr,
            "[adc2 folded] host ms: projected problem %.0f, residuals (incl. M12 sigma) %.0f, new directions + "
            "restarts %.0f; moments %.0f; sigma %.0f; total %.0f\n",
            tm_proj, tm_res, tm_new, tm_cheb, ms_sigma, ms_since(t_start));

  // ---- outputs ----
  if (final_rc == ADC2_OK || final_rc == ADC2_ERR_NOCONV) {
    for (int j = 0; j < k; ++j) omega[j] = roots[j].rq;
    if (Xout && have_omega && !roots[0].y.empty() && (int)roots[0].y.size() == s) {
      double2* X = (double2*)Xout;
      std::vector<cplx> Yc((size_t)s * k), xs((size_t)k * ns);
      std::vector<double> om(k);
      for (int j = 0; j < k; ++j) {
        om[j] = roots[j].omega;
        for (int i = 0; i < s; ++i) Yc[(size_t)i * k + j] = roots[j].y[i] / nrm[j];
        for (long e = 0; e < ns; ++e) xs[(size_t)j * ns + e] = x1[(size_t)j * ns + e] / nrm[j];
      }
      FD_TRY(h2d_small(Yd, Yc.data(), sizeof(double2) * s * k));
      FD_TRY(h2d_small(omd, om.data(), sizeof(double) * k));
      k_fold_x2<<<(unsigned)std::min<long>(16384, (nd + 255) / 256), 256, 0, st>>>(Uro, dim, nd, s, Yd, k, omd, Ddev,
                                                                                  X + ns, dim);
      FD_HIP(hipGetLastError());
      FD_TRY(h2d_rows(xs.data(), k, X));
    }
  }
  if (info) {
    memset(info, 0, sizeof(*info));
    info->iters = std::min(it, max_iter);
    info->n_sigma = (int)((n21 + n12 + 1) / 2);
    info->converged = converged ? 1 : 0;
    info->subspace = s;
    for (int j = 0; j < k && j < ADC2_MAX_ROOTS; ++j) info->resnorm[j] = res[j];
    info->ms_sigma = ms_sigma;
    info->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    const double nc_ = dd.nc, no_ = dd.no, nv_ = dd.nv, na_ = dd.naux;
    const double heavy = 8.0 * nc_ * no_ * nv_ * nv_ * na_, light = 8.0 * nc_ * nv_ * nv_ * na_;
    info->sigma_flops = (double)n21 * (heavy + light + 8.0 * (nc_ * nv_) * (nc_ * nv_)) + (double)n12 * (heavy + light);
  }
  cleanup_events();
  FD_HIP(hipStreamSynchronize(st));
  release();
#undef FD_TRY
#undef FD_HIP
  if (final_rc != ADC2_OK) return final_rc;
  return converged ? ADC2_OK : ADC2_ERR_NOCONV;
}

}  // namespace adc2
