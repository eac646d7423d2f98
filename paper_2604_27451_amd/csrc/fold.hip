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
// so that K_m = U^H T_m U is computed once per basis vector and G(omega)
// for any omega < min D costs only small matrix arithmetic.  Each root j
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
// All of the subspace work (the projected eigensolves, Gram-Schmidt, Ritz
// vectors, residuals, restarts) runs in FP64 on the GPU (fold_la.hip); the
// host reads status words and residual norms to steer the iteration.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "fold_la.h"
#include "hostla.h"
#include "internal.h"
#include "jacobi.h"
#include "tile.h"

namespace adc2 {

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
// B fragments are T_m(t_d) of the staged chunk (each thread forms NM/8
// consecutive moments of one d: the first two from T_0 = 1, T_1 = t_d by the
// doubling identities, the rest by the three-term recurrence).  The next
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
  // the next chunk's U values and doubles energies, loaded into registers ahead of use
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
    dnext = e0 + tid % MKC < nd ? D[e0 + tid % MKC] : 0.0;   // every thread: the energy of its weight column
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
    {  // T_m(t_d), m0 <= m < m0 + NM: thread (d, g) writes the NM/8 moments from n = m0 + g NM/8
      constexpr int PER = NM / 8;
      const int dl = tid % MKC, grp = tid / MKC;
      const double dd = dnext;
      double tv[PER];
      if (e0 + dl < nd) {
        const double x = fmin(1.0, fmax(-1.0, ((inv ? 1.0 / (dd - w0) : dd) - c) * ih));
        // (T_n, T_n+1) from (T_0, T_1) = (1, x) by the doubling identities over the bits of n:
        // T_2k = 2 T_k^2 - 1, T_2k+1 = 2 T_k T_k+1 - x, T_2k+2 = 2 T_k+1^2 - 1
        const int n = m0 + grp * PER;
        double a = 1.0, b = x;
        for (int bit = 7; bit >= 0; --bit) {
          if ((n >> bit) == 0) continue;
          const double ab = 2.0 * a * b - x;
          if ((n >> bit) & 1) {
            a = ab;
            b = 2.0 * b * b - 1.0;
          } else {
            b = ab;
            a = 2.0 * a * a - 1.0;
          }
        }
        tv[0] = a;
        tv[1] = b;
#pragma unroll
        for (int q = 2; q < PER; ++q) tv[q] = 2.0 * x * tv[q - 1] - tv[q - 2];
      } else {
#pragma unroll
        for (int q = 0; q < PER; ++q) tv[q] = 0.0;
      }
#pragma unroll
      for (int q = 0; q < PER; ++q) tb[dl][grp * PER + q] = tv[q];
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
  static_assert(FSMAX == JMAX, "search space and subspace eigensolver sizes");
  static_assert(FMM == FOLD_MM, "moment counts");
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
  if (k > smax || smax > FSMAX) {
    set_error("adc2_davidson (folded): nroots exceeds the singles dimension or the search-space limit");
    return ADC2_ERR_ARG;
  }
  const int keep_max = std::max(k, std::min(2 * k, smax - k));   // vectors kept at a restart
  int nguess = (opt && opt->nguess > 0) ? opt->nguess : (k <= 8 ? 2 * k : k);
  nguess = (int)std::min<long>(std::min(nguess, smax), ns);
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
  void* hsm = nullptr;   // pinned staging of the small host <-> device records
  auto release = [&]() {
    for (void* p : owned) dfree(h, p);
    owned.clear();
    if (hsm) hipHostFree(hsm);
    hsm = nullptr;
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

  int nchb = (int)std::max<long>(1, std::min<long>(512, nd / 4096));
  if (const char* v = getenv("ADC2_CHEB_NCHB")) nchb = (int)std::max<long>(1, std::min<long>(1024, atol(v)));
  const int nmb = FMM / FMB;
  const long part_len = (long)((FSMAX + FGB - 1) / FGB) * nmb * nchb * FMB * 256;   // split-K partials of the moments
  const int nrb = fold_resid_blocks(ns);
  // sigma rows: Sb = sigma of the basis (v, 0), singles part S1 and doubles part U = M21 v
  double2 *Sb, *Tin, *X2, *Sx, *Kt, *part, *Yd, *Cd;
  FD_TRY(dalloc((void**)&Sb, sizeof(double2) * smax * dim));
  // One block of full-length rows serves three roles in disjoint parts: the
  // singles of the new directions (input of the singles-in sigma, which does
  // not read input doubles), the Ritz doubles x2 (input of the doubles-in
  // sigma, which does not read input singles) and its output M12 x2 (singles
  // only: the doubles-in sigma writes no output doubles).
  const int qmax = std::max(nguess, k);   // rows of one sigma input block (new directions never exceed it)
  FD_TRY(dalloc((void**)&Tin, sizeof(double2) * qmax * dim));
  X2 = Tin;
  Sx = Tin;
  FD_TRY(dalloc((void**)&Kt, sizeof(double2) * FMM * smax * FGB));
  FD_TRY(dalloc((void**)&part, sizeof(double2) * part_len));
  FD_TRY(dalloc((void**)&Yd, sizeof(double2) * FSMAX * FSMAX));
  FD_TRY(dalloc((void**)&Cd, sizeof(double2) * FSMAX * FSMAX));
  // search-space state: singles basis V, S1, H11 = V^H S1, moments K_m, per-root eigenvectors
  double2 *Vd, *S1d, *Hd, *Kall, *Td, *T2d, *Gw, *Cg, *Ybr, *Zbr, *X1d, *R1d, *PG, *gref, *gsc;
  FD_TRY(dalloc((void**)&Vd, sizeof(double2) * FSMAX * ns));
  FD_TRY(dalloc((void**)&S1d, sizeof(double2) * FSMAX * ns));
  FD_TRY(dalloc((void**)&Hd, sizeof(double2) * JMAX * JMAX));
  FD_TRY(dalloc((void**)&Kall, sizeof(double2) * FMM * JMAX * JMAX));
  FD_TRY(dalloc((void**)&Td, sizeof(double2) * FSMAX * ns));
  FD_TRY(dalloc((void**)&T2d, sizeof(double2) * FSMAX * ns));
  FD_TRY(dalloc((void**)&Gw, sizeof(double2) * JMAX * JMAX));
  FD_TRY(dalloc((void**)&Cg, sizeof(double2) * JMAX * JMAX));
  FD_TRY(dalloc((void**)&Ybr, sizeof(double2) * nbr * JMAX));
  FD_TRY(dalloc((void**)&Zbr, sizeof(double2) * nbr * JMAX * JMAX));
  FD_TRY(dalloc((void**)&X1d, sizeof(double2) * k * ns));
  FD_TRY(dalloc((void**)&R1d, sizeof(double2) * k * ns));
  FD_TRY(dalloc((void**)&PG, sizeof(double2) * JMAX * k));
  FD_TRY(dalloc((void**)&gref, sizeof(double2) * k * ns));
  FD_TRY(dalloc((void**)&gsc, sizeof(double2) * 16L * dav_nblk(ns) * 256));
  double *hw, *lam, *npart, *ov, *gnd, *omd, *scd, *pnu_d, *pdb_d, *mm;
  FD_TRY(dalloc((void**)&hw, sizeof(double) * JMAX));
  FD_TRY(dalloc((void**)&lam, sizeof(double) * JMAX));
  FD_TRY(dalloc((void**)&npart, sizeof(double) * k * nrb));
  FD_TRY(dalloc((void**)&ov, sizeof(double) * k * nbr));
  FD_TRY(dalloc((void**)&gnd, sizeof(double) * k));
  FD_TRY(dalloc((void**)&omd, sizeof(double) * FSMAX));
  FD_TRY(dalloc((void**)&scd, sizeof(double) * FSMAX));
  FD_TRY(dalloc((void**)&pnu_d, sizeof(double) * ns));
  FD_TRY(dalloc((void**)&pdb_d, sizeof(double) * ns));
  FD_TRY(dalloc((void**)&mm, sizeof(double) * 2 * 256));
  int *icount, *ibuf;
  FD_TRY(dalloc((void**)&icount, sizeof(int) * 4));
  FD_TRY(dalloc((void**)&ibuf, sizeof(int) * 2 * FSMAX));
  FoldEntry* entd;
  FoldResult* resd;
  FoldBounds* bndd;
  FD_TRY(dalloc((void**)&entd, sizeof(FoldEntry) * nbr));
  FD_TRY(dalloc((void**)&resd, sizeof(FoldResult) * nbr));
  FD_TRY(dalloc((void**)&bndd, sizeof(FoldBounds)));
  const size_t hsm_bytes = std::max<size_t>(
      {sizeof(double) * 512, sizeof(double) * k * nrb, sizeof(double) * k * nbr, sizeof(FoldEntry) * nbr,
       sizeof(FoldResult) * nbr, sizeof(double2) * JMAX * JMAX, sizeof(double) * ns});
  FD_HIP(hipHostMalloc(&hsm, hsm_bytes, hipHostMallocDefault));
  // small records through the pinned staging block (each transfer completes before the block is reused)
  auto up = [&](void* dst, const void* src, size_t bytes) -> adc2_status {
    memcpy(hsm, src, bytes);
    ADC2_HIP(hipMemcpyAsync(dst, hsm, bytes, hipMemcpyHostToDevice, st));
    ADC2_HIP(hipStreamSynchronize(st));
    return ADC2_OK;
  };
  auto down = [&](void* dst, const void* src, size_t bytes) -> adc2_status {
    ADC2_HIP(hipMemcpyAsync(hsm, src, bytes, hipMemcpyDeviceToHost, st));
    ADC2_HIP(hipStreamSynchronize(st));
    memcpy(dst, hsm, bytes);
    return ADC2_OK;
  };
  // out[j] (+)= alpha sum_i V[i] C[i][j] over rows of length n, in blocks of 32 columns
  auto combine = [&](const double2* V, int s_, const double2* C, int ldc, int m, long n, double2* out, double alpha,
                     bool acc) -> adc2_status {
    for (int c0 = 0; c0 < m; c0 += 32) {
      adc2_status r = dav_combine(V, s_, C + c0, ldc, std::min(32, m - c0), n, out + (long)c0 * n, alpha, acc, st);
      if (r != ADC2_OK) return r;
    }
    return ADC2_OK;
  };
  const unsigned rgrid = (unsigned)std::min<long>(4096, ((long)FSMAX * ns + 255) / 256);
  const double* Ddev = h->diag + ns;       // doubles diagonal D
  const double* d11d = h->diag;            // singles diagonal of M11
  double2* Urw = Sb + ns;                  // doubles part of the Sb rows
  const double2* Uro = Urw;

  FD_TRY(build_fold_precond(h, st));
  FD_TRY(up(pnu_d, h->pre_nu.data(), sizeof(double) * ns));
  FD_TRY(up(pdb_d, h->pre_dbar.data(), sizeof(double) * ns));
  const std::vector<double>& pnu = h->pre_nu;
  const std::vector<double>& pdb = h->pre_dbar;

  // ---- Chebyshev interval ----
  k_minmax<<<256, 256, 0, st>>>(Ddev, nd, mm);
  FD_HIP(hipGetLastError());
  std::vector<double> hm(512), d11(ns);
  FD_TRY(down(hm.data(), mm, sizeof(double) * 512));
  FD_TRY(down(d11.data(), d11d, sizeof(double) * ns));
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
  // per singles e, the lower root of omega = d11_e + nu_e / (omega - Dbar_e): the
  // folded diagonal's estimate of the root that single e dominates
  std::vector<double> rest(ns);
  double west = 1e300;
  for (long e = 0; e < ns; ++e) {
    const double a = d11[e], bb = pdb[e], nu = pnu[e];
    const double r = nu > 0.0 ? 0.5 * ((a + bb) - std::sqrt((a - bb) * (a - bb) + 4.0 * nu)) : a;
    rest[e] = std::isfinite(r) ? r : 1e300;
    west = std::min(west, r);
  }
  if (west < Dmin && std::isfinite(west))
    rmap = hostla::ResolventMap::shifted_inverse(Dmin, Dmax, west - std::max(1.0, 0.5 * (Dmin - west)));
  // Truncation of the resolvent expansion: to FP64 rounding for the FP64
  // sigma; with the complex64 and split-BF16 contractions (relative sigma
  // noise ~1e-7 and ~1e-6, residual tolerances 1e-3 .. 1e-5) 1e-10 is far
  // below that noise and needs about 0.6 times the terms.
  const double exp_tol = h->prec == ADC2_FP64 ? 1e-17 : 1e-10;
  rmap.tol = exp_tol;
  auto fmap = [&]() { return FoldMap{rmap.inv ? 1 : 0, rmap.c, rmap.ih, rmap.w0, rmap.tol}; };

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

  // Chebyshev moments K_m[i][j] for rows i < srows and columns [j0, j0 + q), m < 8 * mblocks
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
                                                                                            nm, nz, nch_m, mm_, Kt);
      ADC2_CHECK_LAUNCH();
      adc2_status r = fold_cheb_scatter(Kt, mm_, srows, c0, qc, Kall, st);
      if (r != ADC2_OK) return r;
    }
    if (verbose) ADC2_HIP(hipStreamSynchronize(st));
    tm_cheb += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tc0).count();
    return ADC2_OK;
  };

  // append the q orthonormal singles vectors in rows 0..q-1 of Td: sigma of (v, 0), moments, H11 columns
  auto add_vectors = [&](int q) -> adc2_status {
    if (q > qmax) {
      set_error("adc2_davidson (folded): more new directions than the input block holds");
      return ADC2_ERR_ARG;
    }
    k_rows_copy<<<rgrid, 256, 0, st>>>(Td, ns, Tin, dim, q, ns);
    ADC2_CHECK_LAUNCH();
    adc2_status r = sig_time(q, Tin, Sb + (long)s * dim, SIGMA_SINGLES_IN);
    if (r != ADC2_OK) return r;
    n21 += q;
    k_rows_copy<<<rgrid, 256, 0, st>>>(Sb + (long)s * dim, dim, S1d + (long)s * ns, ns, q, ns);
    ADC2_CHECK_LAUNCH();
    ADC2_HIP(hipMemcpyAsync(Vd + (long)s * ns, Td, sizeof(double2) * q * ns, hipMemcpyDeviceToDevice, st));
    const int snew = s + q;
    if ((r = cheb_cols(snew, s, q, mcomp)) != ADC2_OK) return r;
    if ((r = dav_gram(Vd, snew, S1d + (long)s * ns, q, ns, Hd + s, JMAX, gsc, st)) != ADC2_OK) return r;
    if ((r = fold_herm_fill(Hd, s, snew, st)) != ADC2_OK) return r;
    s = snew;
    return ADC2_OK;
  };

  // orthonormalise rows 0..q-1 of Td against V[0..s) (two classical Gram-Schmidt passes, all rows at once)
  // and among themselves (modified Gram-Schmidt, two passes, in row order); a row whose norm falls to
  // 1e-10 of its initial norm is dropped; returns the kept count (rows 0..kept-1 of Td)
  auto orthonormalise = [&](int q, int& kept) -> adc2_status {
    kept = 0;
    if (q <= 0) return ADC2_OK;
    adc2_status r = fold_rownorm(Td, q, ns, lam, st);
    if (r != ADC2_OK) return r;
    for (int pass = 0; pass < 2 && s > 0; ++pass) {
      if ((r = dav_gram(Vd, s, Td, q, ns, Cg, JMAX, gsc, st)) != ADC2_OK) return r;
      if ((r = combine(Vd, s, Cg, JMAX, q, ns, Td, -1.0, true)) != ADC2_OK) return r;
    }
    if ((r = fold_mgs(Td, q, ns, lam, icount, st)) != ADC2_OK) return r;
    return down(&kept, icount, sizeof(int));
  };

  // ---- initial space ----
  std::vector<double> gn(k, 0.0);
  {
    if (guess) {
      k_rows_copy<<<rgrid, 256, 0, st>>>((const double2*)guess, dim, Td, ns, nguess, ns);
      FD_HIP(hipGetLastError());
      if (follow) {
        // singles of the followed guess vectors, as given, and their squared norms
        k_rows_copy<<<rgrid, 256, 0, st>>>((const double2*)guess, dim, gref, ns, k, ns);
        FD_HIP(hipGetLastError());
        FD_TRY(dav_gram(gref, k, gref, k, ns, Gw, JMAX, gsc, st));
        std::vector<double2> g2((size_t)JMAX * JMAX);
        FD_TRY(down(g2.data(), Gw, sizeof(double2) * JMAX * JMAX));
        for (int j = 0; j < k; ++j) gn[j] = g2[(size_t)j * JMAX + j].x;
        FD_TRY(up(gnd, gn.data(), sizeof(double) * k));
      }
    } else {
      std::vector<int> idx(ns);
      for (long i = 0; i < ns; ++i) idx[i] = (int)i;
      // unit vectors on the singles of lowest folded-diagonal root estimate
      std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return rest[a] < rest[b]; });
      FD_TRY(up(ibuf, idx.data(), sizeof(int) * nguess));
      FD_TRY(fold_unit(Td, nguess, ns, ibuf, st));
    }
    int q = 0;
    FD_TRY(orthonormalise(nguess, q));
    if (q < k) {
      cleanup_events();
      hipStreamSynchronize(st);
      release();
      set_error("adc2_davidson (folded): the initial space has fewer vectors than roots");
      return ADC2_ERR_ARG;
    }
    adc2_status r = add_vectors(q);
    if (r != ADC2_OK) {
      cleanup_events();
      hipStreamSynchronize(st);
      release();
      return r;
    }
  }

  // projected roots (host side: the steering data; the vectors live in the device slots)
  struct Root {
    int branch = 0, slot = 0;   // eigenvalue index j of lambda_j(G(omega)) = omega; storage slot
    int ysize = 0, zsize = 0;   // basis size of the vector / eigenvectors in the slot (0: none)
    int status = 0, need = 0;
    int clamped = 0;            // consecutive iterations with status 1 (held at the expansion limit)
    double omega = 0.0, rq = 0.0, n2 = 0.0;
  };
  std::vector<Root> roots(nbr);
  for (int b = 0; b < nbr; ++b) roots[b].branch = roots[b].slot = b;
  std::vector<char> prov(k, 0);   // root held at the expansion limit this iteration
  std::vector<double> res(k, 1e300), nrm(k, 1.0);
  bool res_valid = false;   // res holds an evaluation for every root
  bool have_omega = false, converged = false;
  int it = 0;
  // stagnation: the largest residual has not dropped below 0.8 of its best
  // value for FSTALL iterations (the precision form's noise floor)
  double best_rmax = 1e300;
  int best_it = 0;
  const auto t_start = std::chrono::steady_clock::now();
  adc2_status final_rc = ADC2_OK;
  double tm_proj = 0.0, tm_res = 0.0, tm_new = 0.0;   // host-side phases (ms)
  auto now = []() { return std::chrono::steady_clock::now(); };
  auto ms_since = [](std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  };
  std::vector<FoldEntry> ent(nbr);
  std::vector<FoldResult> rres(nbr);
  std::vector<double> hnp((size_t)k * nrb), hov((size_t)k * nbr);
  std::vector<int> ib(FSMAX);
  std::vector<double> hd(FSMAX);

  for (it = 1; it <= max_iter; ++it) {
    // ---- projected nonlinear problem: one workgroup per root, lowest eigenvalue of H11 first ----
    const auto tp0 = now();
    FD_TRY(dav_heevj(Hd, s, JMAX, hw, Gw, JMAX, st));
    // a pole at |x| >= 1.05 has r = |x| - sqrt(x^2 - 1) < 0.73 and r^126 < 1e-17,
    // so at most 126 Chebyshev terms: with the shifted inverse, roots closer
    // to min D than about 0.025 (min D - w0) are out of reach of this solver
    double hi0 = rmap.reach(1.05);
    for (int attempt = 0; attempt < 4; ++attempt) {
      for (int b = 0; b < nbr; ++b) {
        const Root& R = roots[b];
        ent[b] = FoldEntry{R.branch, R.slot, R.zsize, have_omega ? 1 : 0, R.omega};
      }
      FD_TRY(up(entd, ent.data(), sizeof(FoldEntry) * nbr));
      FD_TRY(fold_solve_launch(Hd, Kall, s, FMB * mcomp, fmap(), Dmin, hi0, tol, hw, entd, nbr, resd, Ybr, Zbr, bndd,
                               st));
      FD_TRY(down(rres.data(), resd, sizeof(FoldResult) * nbr));
      int need = 0;
      bool below = false;
      for (int b = 0; b < nbr; ++b) {
        Root& R = roots[b];
        const FoldResult& q = rres[b];
        R.status = q.status;
        R.need = q.need;
        if (q.ysize == s) {
          R.omega = q.omega;
          R.rq = q.rq;
          R.n2 = q.n2;
          R.ysize = s;
        }
        if (q.zsize > 0) R.zsize = q.zsize;
        if (R.status == 3) need = std::max(need, R.need);
        if (R.status == 4) below = true;
      }
      if (below) {
        // a root below the shifted map's range: move the shift down (twice as
        // far from min D) and recompute the moments of the whole space
        rmap = hostla::ResolventMap::shifted_inverse(Dmin, Dmax, Dmin - 3.0 * (Dmin - rmap.w0));
        rmap.tol = exp_tol;
        hi0 = rmap.reach(1.05);
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
      FD_TRY(dav_gram(Vd, s, gref, k, ns, PG, k, gsc, st));
      FD_TRY(fold_overlap(PG, s, k, Ybr, entd, resd, nbr, gnd, ov, st));
      FD_TRY(down(hov.data(), ov, sizeof(double) * k * nbr));
      for (int b = 0; b < nbr; ++b) {
        const Root& R = roots[b];
        if ((R.status != 0 && R.status != 1) || R.ysize != s)
          for (int j = 0; j < k; ++j) hov[(size_t)j * nbr + b] = -1.0;
      }
      std::vector<int> sel(k, -1);
      std::vector<char> used(nbr, 0);
      for (int n = 0; n < k; ++n) {
        int bj = -1, bb = -1;
        double best = -2.0;
        for (int j = 0; j < k; ++j) {
          if (sel[j] >= 0) continue;
          for (int b = 0; b < nbr; ++b)
            if (!used[b] && hov[(size_t)j * nbr + b] > best) {
              best = hov[(size_t)j * nbr + b];
              bj = j;
              bb = b;
            }
        }
        sel[bj] = bb;
        used[bb] = 1;
      }
      std::vector<Root> re;
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
    // Residuals are evaluated for the roots not converged at their last
    // evaluation (M12 x2, the expensive half, only for those); when all of
    // those converge, the rest are evaluated at once with the same Ritz
    // vectors, so convergence is always declared on a pass over every root.
    // Root following re-selects roots each iteration: every root, always.
    for (int j = 0; j < k; ++j) nrm[j] = std::sqrt(1.0 + std::max(roots[j].n2, 0.0));
    auto eval_res = [&](const std::vector<int>& sel) -> adc2_status {
      const int qa = (int)sel.size();
      if (qa == 0) return ADC2_OK;
      std::vector<int> sl(qa);
      for (int c = 0; c < qa; ++c) {
        sl[c] = roots[sel[c]].slot;
        hd[c] = roots[sel[c]].omega;
      }
      adc2_status r = up(ibuf, sl.data(), sizeof(int) * qa);
      if (r == ADC2_OK) r = up(ibuf + FSMAX, sel.data(), sizeof(int) * qa);
      if (r == ADC2_OK) r = up(omd, hd.data(), sizeof(double) * qa);
      if (r == ADC2_OK) r = fold_gather_y(Ybr, ibuf, nullptr, s, qa, Yd, st);
      if (r != ADC2_OK) return r;
      k_fold_x2<<<(unsigned)std::min<long>(16384, (nd + 255) / 256), 256, 0, st>>>(Uro, dim, nd, s, Yd, qa, omd,
                                                                                  Ddev, X2 + ns, dim);
      ADC2_CHECK_LAUNCH();
      if ((r = sig_time(qa, X2, Sx, SIGMA_DOUBLES_IN)) != ADC2_OK) return r;
      n12 += qa;
      if ((r = fold_resid(Vd, S1d, s, ns, Yd, qa, omd, Sx, dim, ibuf + FSMAX, X1d, R1d, npart, st)) != ADC2_OK)
        return r;
      if ((r = down(hnp.data(), npart, sizeof(double) * qa * nrb)) != ADC2_OK) return r;
      for (int c = 0; c < qa; ++c) {
        double a = 0.0;
        for (int b = 0; b < nrb; ++b) a += hnp[(size_t)c * nrb + b];
        res[sel[c]] = std::sqrt(a) / nrm[sel[c]];
      }
      return ADC2_OK;
    };
    std::vector<int> act, rest;
    for (int j = 0; j < k; ++j) {
      if (follow || !res_valid || res[j] > tol || prov[j]) act.push_back(j);
      else rest.push_back(j);
    }
    if (act.empty()) act.swap(rest);
    FD_TRY(eval_res(act));
    res_valid = true;
    {
      bool act_ok = true;
      for (int j : act) act_ok = act_ok && res[j] <= tol && !prov[j];
      if (act_ok && !rest.empty()) FD_TRY(eval_res(rest));   // certificate pass over the converged ones
    }
    double rmax = 0.0;
    for (int j = 0; j < k; ++j) rmax = std::max(rmax, res[j]);
    tm_res += ms_since(tr0);
    if (verbose) {
      fprintf(stderr, "[adc2 folded no=%d nv=%d] it %3d  space %2d  max|r| %.3e  omega0 %.12f  (%d evaluated)\n",
              dd.no, dd.nv, it, s, rmax, roots[0].omega, (int)act.size());
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
    int q = 0;
    for (int j = 0; j < k; ++j) {
      if (res[j] <= tol && !prov[j]) continue;
      ib[q] = j;
      hd[q] = roots[j].omega;
      ++q;
    }
    FD_TRY(up(ibuf, ib.data(), sizeof(int) * q));
    FD_TRY(up(scd, hd.data(), sizeof(double) * q));
    FD_TRY(fold_newdir(R1d, ns, ibuf, scd, q, d11d, pnu_d, pdb_d, Td, st));
    // ---- restart: keep the Ritz singles of every root and the next ones of the highest root ----
    if (s + q > smax) {
      const int nk = std::min(keep_max, s);
      for (int j = 0; j < k; ++j) ib[j] = roots[j].slot;
      FD_TRY(up(ibuf, ib.data(), sizeof(int) * k));
      FD_TRY(fold_restart_basis(Ybr, Zbr, ibuf, k, roots[k - 1].slot, s, nk, Cd, icount, st));
      int kc = 0;
      FD_TRY(down(&kc, icount, sizeof(int)));
      // V, S1 (rows), H11 and every held K_m (C^H A C), the doubles parts U (in place)
      FD_TRY(combine(Vd, s, Cd, kc, kc, ns, T2d, 1.0, false));
      FD_HIP(hipMemcpyAsync(Vd, T2d, sizeof(double2) * kc * ns, hipMemcpyDeviceToDevice, st));
      FD_TRY(combine(S1d, s, Cd, kc, kc, ns, T2d, 1.0, false));
      FD_HIP(hipMemcpyAsync(S1d, T2d, sizeof(double2) * kc * ns, hipMemcpyDeviceToDevice, st));
      FD_TRY(fold_rot_small(Hd, 0, 1, s, Cd, kc, st));
      FD_TRY(fold_rot_small(Kall, (long)JMAX * JMAX, FMB * mcomp, s, Cd, kc, st));
      k_fold_rotate<<<(unsigned)((nd + 63) / 64), 256, 0, st>>>(Urw, dim, nd, s, Cd, kc);
      FD_HIP(hipGetLastError());
      for (int j = 0; j < nbr; ++j) roots[j].ysize = roots[j].zsize = 0;   // the basis changed: next solve starts cold
      s = kc;
    }
    int qk = 0;
    FD_TRY(orthonormalise(q, qk));
    if (qk == 0) {
      set_error("adc2_davidson (folded): no new search directions (stagnation)");
      final_rc = ADC2_ERR_NOCONV;
      break;
    }
    tm_new += ms_since(tn0);
    FD_TRY(add_vectors(qk));
  }
  if (verbose)
    fprintf(stderr,
            "[adc2 folded] host ms: projected problem %.0f, residuals (incl. M12 sigma) %.0f, new directions + "
            "restarts %.0f; moments %.0f; sigma %.0f; total %.0f\n",
            tm_proj, tm_res, tm_new, tm_cheb, ms_sigma, ms_since(t_start));

  // ---- outputs ----
  if (final_rc == ADC2_OK || final_rc == ADC2_ERR_NOCONV) {
    for (int j = 0; j < k; ++j) omega[j] = roots[j].rq;
    if (Xout && have_omega && roots[0].ysize == s) {
      double2* X = (double2*)Xout;
      for (int j = 0; j < k; ++j) {
        ib[j] = roots[j].slot;
        hd[j] = roots[j].omega;
      }
      std::vector<double> sc(k);
      for (int j = 0; j < k; ++j) sc[j] = 1.0 / nrm[j];
      FD_TRY(up(ibuf, ib.data(), sizeof(int) * k));
      FD_TRY(up(omd, hd.data(), sizeof(double) * k));
      FD_TRY(up(scd, sc.data(), sizeof(double) * k));
      FD_TRY(fold_gather_y(Ybr, ibuf, scd, s, k, Yd, st));
      k_fold_x2<<<(unsigned)std::min<long>(16384, (nd + 255) / 256), 256, 0, st>>>(Uro, dim, nd, s, Yd, k, omd, Ddev,
                                                                                  X + ns, dim);
      FD_HIP(hipGetLastError());
      // singles x1 / |x| = V y / |x| of the final Ritz vectors
      FD_TRY(combine(Vd, s, Yd, k, k, ns, T2d, 1.0, false));
      k_rows_copy<<<rgrid, 256, 0, st>>>(T2d, ns, X, dim, k, ns);
      FD_HIP(hipGetLastError());
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
