// jacobi.h -- one-workgroup parallel cyclic Jacobi eigensolver for a complex
// Hermitian n x n matrix (n <= 64) held in LDS, FP64.  Used for the
// subspace eigenproblems of both Davidson solvers (the projected matrix
// V^H M V of the full-space solver, the projected singles blocks and the
// folded matrices G(omega) of the folded solver).
//
// Pair (p,q) rotation J = [[c, s e], [-s conj(e), c]], e = a_pq/|a_pq|,
// t = sign(tau)/(|tau| + sqrt(1+tau^2)), tau = (a_qq - a_pp)/(2|a_pq|),
// zeroes a_pq of J^H A J; all n/2 disjoint pairs of a round-robin round are
// applied together.  Sweeps stop when the off-diagonal Frobenius norm is
// below 1e-15 of the whole (squared: 1e-30).
#pragma once
#include <hip/hip_runtime.h>

#include "tile.h"

namespace adc2 {

constexpr int JMAX = 64;
constexpr int JSWEEPS = 40;

struct JacobiSmem {
  double ar[JMAX][JMAX];    // real and imaginary parts of A (both triangles)
  double ai[JMAX][JMAX];
  double2 zs[JMAX][JMAX];   // accumulated rotations: eigenvectors as columns
  double rc[JMAX / 2], rs[JMAX / 2];
  double2 re[JMAX / 2];
  int rp[JMAX / 2], rq[JMAX / 2];
  double red[256];
  int perm[JMAX];           // ascending order of the eigenvalues ar[perm[i]][perm[i]]
  int done;                 // 1 once the sweeps converged
};

// A (n x n, both triangles consistent) in S.ar / S.ai; blockDim.x == 256.
// On return (after a barrier): S.zs holds the eigenvectors as columns in the
// unsorted order of the diagonal of S.ar, S.perm the ascending order, S.done
// whether the sweeps converged within JSWEEPS.
__device__ inline void jacobi_lds(JacobiSmem& S, int n) {
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += 256) {
    const int i = e / n, j = e % n;
    S.zs[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  if (tid == 0) S.done = 0;
  __syncthreads();
  const int N = (n + 1) & ~1;   // even number of players (player n is a dummy if n is odd)
  const int npair = N / 2;
  for (int sweep = 0; sweep <= JSWEEPS; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n * n; e += 256) {
      const int i = e / n, j = e % n;
      const double v = S.ar[i][j] * S.ar[i][j] + S.ai[i][j] * S.ai[i][j];
      tot += v;
      if (i != j) off += v;
    }
    S.red[tid] = off;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) S.red[tid] += S.red[tid + st];
      __syncthreads();
    }
    const double offs = S.red[0];
    __syncthreads();
    S.red[tid] = tot;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) S.red[tid] += S.red[tid + st];
      __syncthreads();
    }
    if (tid == 0) S.done = (offs <= 1e-30 * S.red[0] || offs == 0.0) ? 1 : 0;
    __syncthreads();
    if (S.done || sweep == JSWEEPS) break;
    for (int round = 0; round < N - 1; ++round) {
      if (tid < npair) {
        // round-robin: player 0 fixed, players 1..N-1 rotate
        int a, b;
        if (tid == 0) {
          a = 0;
          b = 1 + (round % (N - 1));
        } else {
          a = 1 + ((round + tid) % (N - 1));
          b = 1 + ((round + N - 1 - tid) % (N - 1));
        }
        const int p = min(a, b), q = max(a, b);
        double c = 1.0, s = 0.0;
        double2 ee = make_double2(1.0, 0.0);
        if (q < n) {
          const double br = S.ar[p][q], bi = S.ai[p][q];
          const double mag = sqrt(br * br + bi * bi);
          const double app = S.ar[p][p], aqq = S.ar[q][q];
          if (mag > 1e-300 && mag > 1e-18 * (fabs(app) + fabs(aqq))) {
            const double tau = (aqq - app) / (2.0 * mag);
            const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            ee = make_double2(br / mag, bi / mag);
          }
        }
        S.rp[tid] = p;
        S.rq[tid] = q;
        S.rc[tid] = c;
        S.rs[tid] = s;
        S.re[tid] = ee;
      }
      __syncthreads();
      // column update A <- A J and Z <- Z J
      for (int it = tid; it < npair * n; it += 256) {
        const int pr = it / n, r = it % n;
        const int p = S.rp[pr], q = S.rq[pr];
        if (q >= n || S.rs[pr] == 0.0) continue;
        const double c = S.rc[pr], s = S.rs[pr];
        const double2 e = S.re[pr];
        const double2 x = make_double2(S.ar[r][p], S.ai[r][p]);
        const double2 y = make_double2(S.ar[r][q], S.ai[r][q]);
        // new_p = c x - s conj(e) y ; new_q = s e x + c y
        const double2 ny = cmul(cconj(e), y);
        const double2 nx = cmul(e, x);
        S.ar[r][p] = c * x.x - s * ny.x;
        S.ai[r][p] = c * x.y - s * ny.y;
        S.ar[r][q] = s * nx.x + c * y.x;
        S.ai[r][q] = s * nx.y + c * y.y;
        const double2 zx = S.zs[r][p], zy = S.zs[r][q];
        const double2 zny = cmul(cconj(e), zy);
        const double2 znx = cmul(e, zx);
        S.zs[r][p] = make_double2(c * zx.x - s * zny.x, c * zx.y - s * zny.y);
        S.zs[r][q] = make_double2(s * znx.x + c * zy.x, s * znx.y + c * zy.y);
      }
      __syncthreads();
      // row update A <- J^H A : new_p = c x - s e y ; new_q = s conj(e) x + c y
      for (int it = tid; it < npair * n; it += 256) {
        const int pr = it / n, r = it % n;
        const int p = S.rp[pr], q = S.rq[pr];
        if (q >= n || S.rs[pr] == 0.0) continue;
        const double c = S.rc[pr], s = S.rs[pr];
        const double2 e = S.re[pr];
        const double2 x = make_double2(S.ar[p][r], S.ai[p][r]);
        const double2 y = make_double2(S.ar[q][r], S.ai[q][r]);
        const double2 ey = cmul(e, y);
        const double2 cx = cmul(cconj(e), x);
        S.ar[p][r] = c * x.x - s * ey.x;
        S.ai[p][r] = c * x.y - s * ey.y;
        S.ar[q][r] = s * cx.x + c * y.x;
        S.ai[q][r] = s * cx.y + c * y.y;
      }
      __syncthreads();
      if (tid < npair) {
        const int p = S.rp[tid], q = S.rq[tid];
        if (q < n && S.rs[tid] != 0.0) {
          S.ar[p][q] = S.ai[p][q] = S.ar[q][p] = S.ai[q][p] = 0.0;
          S.ai[p][p] = S.ai[q][q] = 0.0;
        }
      }
      __syncthreads();
    }
  }
  // ascending order (selection by one thread; n <= 64)
  if (tid == 0) {
    for (int i = 0; i < n; ++i) S.perm[i] = i;
    for (int i = 0; i < n; ++i) {
      int best = i;
      for (int j = i + 1; j < n; ++j)
        if (S.ar[S.perm[j]][S.perm[j]] < S.ar[S.perm[best]][S.perm[best]]) best = j;
      const int t = S.perm[i];
      S.perm[i] = S.perm[best];
      S.perm[best] = t;
    }
  }
  __syncthreads();
}

}  // namespace adc2
