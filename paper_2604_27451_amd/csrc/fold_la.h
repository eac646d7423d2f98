// fold_la.h -- device-side subspace linear algebra of the folded solver
// (fold_la.hip): the records exchanged with the host and the launchers.
// Matrices of the search space (H11, the moments K_m, eigenvector slots)
// are s x s blocks with leading dimension JMAX = 64; singles vectors are
// contiguous rows of ns = nc nv complex128 values.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace adc2 {

constexpr int FOLD_MM = 128;   // largest number of Chebyshev terms of the resolvent

// Expansion variable of the moments (see hostla::ResolventMap): linear
// t = (D - c) ih, or shifted inverse t = (1/(D - w0) - c) ih.
struct FoldMap {
  int inv;
  double c, ih, w0;
  double tol;   // truncation of the expansion (terms until r^m < tol)
};

// One projected root to solve (host -> device): branch index, storage slot of
// its eigenvectors, the size of the eigenvector block already in the slot (0:
// start cold) and the previous omega (has_prev).
struct FoldEntry {
  int branch, slot, zwarm, has_prev;
  double omega;
};

// Result of one projected root (device -> host); omega, rq, n2 and w are
// those of the last Newton step; ysize (zsize) the basis size of the vector
// (eigenvectors) it wrote to its slot, 0 if none.
struct FoldResult {
  double omega, rq, n2, w;
  int status, need, ysize, zsize;
};

struct FoldBounds {
  double lam_min, lo0, wlo, hi0;
};

adc2_status fold_solve_launch(const double2* H, const double2* K, int s, int Mmax, const FoldMap& map, double Dmin,
                              double hi0, double tol, const double* hw, const FoldEntry* ent, int n,
                              FoldResult* res, double2* Ybr, double2* Zbr, FoldBounds* bnd, hipStream_t st);
adc2_status fold_gather_y(const double2* Ybr, const int* slot, const double* scale, int s, int q, double2* Y,
                          hipStream_t st);
int fold_resid_blocks(long ns);
adc2_status fold_resid(const double2* V, const double2* S1, int s, long ns, const double2* Y, int q, const double* om,
                       const double2* Sx, long ldx, const int* row, double2* X1, double2* R1, double* npart,
                       hipStream_t st);
adc2_status fold_newdir(const double2* R1, long ns, const int* root, const double* om, int q, const double* d11,
                        const double* pnu, const double* pdb, double2* T, hipStream_t st);
adc2_status fold_unit(double2* T, int q, long ns, const int* idx, hipStream_t st);
adc2_status fold_herm_fill(double2* H, int s, int snew, hipStream_t st);
adc2_status fold_cheb_scatter(const double2* Kt, int mm, int srows, int c0, int qc, double2* K, hipStream_t st);
adc2_status fold_overlap(const double2* PG, int s, int k, const double2* Ybr, const FoldEntry* ent,
                         const FoldResult* res, int nbr, const double* gn, double* ov, hipStream_t st);
adc2_status fold_restart_basis(const double2* Ybr, const double2* Zbr, const int* rs, int k, int zslot, int s, int nk,
                               double2* C, int* count, hipStream_t st);
adc2_status fold_rot_small(double2* base, long stride, int nmat, int s, const double2* C, int kc, hipStream_t st);
adc2_status fold_rownorm(const double2* T, int q, long ns, double* n2, hipStream_t st);
adc2_status fold_mgs(double2* T, int q, long ns, const double* n2, int* count, hipStream_t st);

}  // namespace adc2
