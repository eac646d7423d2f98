/*
 * adc2.h -- C ABI of the MI355X (gfx950) two-component CVS-ADC(2) library.
 *
 * The library computes core-excitation energies of the two-component
 * core-valence-separated ADC(2) method: the lowest eigenvalues of the
 * Hermitian intermediate-state secular matrix M (paper, Theory section,
 * Eq. 11: M X = X Omega, X^H X = 1), with M expanded to second order in the
 * Moller-Plesset partitioning (Eq. 12) and restricted to the core-valence
 * separated manifold a+_a a_I, a+_a a+_b a_I a_j with I core, j valence
 * (CVS section).  Two-electron integrals are never stored with more than two
 * virtual indices: they are generated on the fly from complex Cholesky
 * vectors (Implementation section), <pq||rs> = (pr|qs) - (ps|qr) with
 * (pq|rs) = sum_P L^P_pq L^P_rs.
 *
 * Conventions shared by every entry point
 *   - Spinors are ordered [core nc | valence no | virtual nv], n = nc+no+nv.
 *   - Complex data are interleaved (re, im) doubles, the layout of
 *     torch.complex128 (C99 double _Complex).
 *   - An ADC vector has dim = nc*nv + nc*no*nv*(nv-1)/2 entries: singles
 *     (I, a) at I*nv + a, then doubles packed lexicographically over
 *     (I, j, a<b) with the pair (a,b) at a*nv - a*(a+1)/2 + (b-a-1).
 *     The doubles basis state is a+_a a+_b a_j a_I |Phi0>, orthonormal, so
 *     plain complex inner products of vectors are the correct metric.
 *   - "dev" pointers are HIP device pointers; "host" pointers are host memory.
 *     The caller owns every pointer it passes; the library never frees them.
 *   - stream is a hipStream_t (may be NULL for the default stream).  Calls
 *     are stream-ordered; adc2_setup and adc2_davidson synchronise the stream
 *     before returning because they hand scalars back on the host.
 *   - A handle is not thread-safe.  Errors never throw across the ABI: every
 *     call returns an adc2_status and records a message for adc2_last_error.
 */
#ifndef ADC2_H
#define ADC2_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define ADC2_API __attribute__((visibility("default")))
#else
#define ADC2_API
#endif

typedef struct adc2_handle_s* adc2_handle;

typedef enum {
  ADC2_OK = 0,
  ADC2_ERR_ARG = 1,            /* bad size, null pointer, unsupported option   */
  ADC2_ERR_NOT_HERMITIAN = 2,  /* some L^P is not Hermitian beyond 1e-12*max|L| */
  ADC2_ERR_OOM = 3,            /* device allocation failed                      */
  ADC2_ERR_HIP = 4,            /* a HIP runtime call failed                     */
  ADC2_ERR_NOCONV = 5,         /* Davidson hit max_iter; best results written   */
  ADC2_ERR_NONFINITE = 6       /* NaN/Inf in inputs or in the iteration         */
} adc2_status;

typedef enum {
  ADC2_FP64 = 0,               /* complex FP64 contractions on the FP64 MFMA     */
  ADC2_C64 = 1                 /* precision form: the two heavy sigma
                                  contractions on complex64 operands with the
                                  FP32 MFMA and FP32 accumulation; setup,
                                  denominators, packing, Davidson and subspace
                                  eigensolver stay FP64                          */
  ,
  ADC2_BF16X3 = 2              /* precision form, split-BF16 variant: the same
                                  two contractions on the BF16 MFMA with each
                                  complex64 operand split into hi = bf16(x),
                                  lo = bf16(x - hi); hi*hi + hi*lo + lo*hi
                                  accumulated in FP32 (relative error ~1e-5)     */
} adc2_precision;

#define ADC2_MAX_ROOTS 32

typedef struct {
  double tol;          /* converged when every ||M x_k - w_k x_k||_2 <= tol  */
  int max_iter;        /* Davidson iterations (0 -> 300)                      */
  int max_subspace;    /* subspace cap before restart (0 -> max(6k, 2k+k))   */
  int nguess;          /* initial guess vectors (0 -> 2k if k <= 8 else k)    */
  int verbose;         /* print one line per iteration to stderr              */
  int solver;          /* ADC2_SOLVER_FULL (0) or ADC2_SOLVER_FOLDED (1)      */
  int follow;          /* 1: root following (full-space solver only), below  */
  double mixed_tol;    /* > 0: two-stage solve through split-BF16, below     */
} adc2_dav_opts;

/* Eigensolvers of adc2_davidson.
 * ADC2_SOLVER_FULL: block Davidson in the full singles+doubles space.
 * ADC2_SOLVER_FOLDED: the doubles block M22 = diag(D) is eliminated exactly,
 *   [M11 + M12 (omega - D)^-1 M21] x1 = omega x1, x2 = (omega - D)^-1 M21 x1,
 *   and the search space holds singles only; valid for roots below the
 *   lowest doubles energy (min D minus 0.2 times half the width of the D
 *   range); otherwise it returns ADC2_ERR_NOCONV with a message naming the
 *   root.  The returned vectors are the full (x1, x2), unit norm. */
#define ADC2_SOLVER_FULL 0
#define ADC2_SOLVER_FOLDED 1

typedef struct {
  int iters;                        /* Davidson iterations performed          */
  int n_sigma;                      /* sigma vectors computed                  */
  int converged;                    /* 1 if every root met tol                 */
  int subspace;                     /* final subspace size                     */
  double resnorm[ADC2_MAX_ROOTS];   /* final residual 2-norms                 */
  double ms_sigma;                  /* HIP-event time inside sigma builds     */
  double ms_total;                  /* wall time of the adc2_davidson call     */
  double sigma_flops;               /* algorithmic flops of those sigma builds */
} adc2_dav_info;

/*
 * Device-memory callbacks, optional in adc2_setup / adc2_setup_batch.  With
 * them, every device buffer of a handle -- its integral blocks and sigma work
 * spaces, and the per-call work spaces of the entry points that take the
 * handle (solvers, adjoint, transition moments, natural spinors, autotuner)
 * -- comes from alloc(bytes, ctx) and goes back through release(ptr, ctx), so
 * that a caching allocator (PyTorch's, for instance) can back it.  alloc
 * returns NULL when it cannot serve the request (reported as ADC2_ERR_OOM);
 * the returned memory must be device memory of the current device, aligned
 * to 256 bytes.  The library waits for the device to be idle before each
 * release, as hipFree does.  NULL, or alloc == NULL, selects hipMalloc and
 * hipFree.  The struct is copied at setup; ctx must stay valid for the
 * handle's lifetime.  Pinned host staging buffers and the handle-free
 * adc2_peak_probe still use the HIP allocators.
 */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*release)(void* ptr, void* ctx);
  void* ctx;
} adc2_alloc;

/*
 * adc2_setup -- build a handle for one system.
 *   L     dev, complex128 [naux][n][n]; each L[P] must be Hermitian
 *         (L[P][q][p] = conj(L[P][p][q])); read only during the call.
 *   eps   dev, float64 [n]: canonical spinor energies (diagonal Fock matrix),
 *         core < valence < virtual is not required but every virtual minus
 *         occupied denominator must be nonzero.
 *   nc, no, nv, naux  > 0 (nv >= 2).
 *   prec  adc2_precision: arithmetic of the sigma build (setup is always FP64).
 *   alloc optional device-memory callbacks (above), NULL for hipMalloc.
 * Work done (stream-ordered, then synchronised): slicing L into the
 * virtual-virtual, virtual-occupied and occupied-occupied blocks; the MP2
 * amplitudes tau = <ac||kl> / D^{ac}_{kl} over all occupied k,l (denominators
 * of Eq. 15) and the MP2 energy; the dense CVS singles block through second
 * order; the diagonal of M used by the preconditioner.
 * Errors: ADC2_ERR_ARG (sizes, null pointers), ADC2_ERR_NOT_HERMITIAN,
 * ADC2_ERR_NONFINITE (NaN/Inf in L or eps), ADC2_ERR_OOM, ADC2_ERR_HIP.
 * On error *out is set to NULL and nothing is leaked.
 */
ADC2_API adc2_status adc2_setup(const void* L, const double* eps, int nc, int no, int nv,
                       int naux, int prec, const adc2_alloc* alloc, void* stream, adc2_handle* out);

/* Vector length nc*nv + nc*no*nv*(nv-1)/2 (0 for a NULL handle). */
ADC2_API size_t adc2_dim(adc2_handle h);

/*
 * adc2_sigma -- S = M X for a block of m vectors (Eq. 11 operator).
 *   X  dev complex128 [m][dim]; S dev complex128 [m][dim] (overwritten;
 *   must not alias X).  m >= 1.  Stream-ordered, asynchronous.
 * Errors: ADC2_ERR_ARG, ADC2_ERR_OOM (workspace growth), ADC2_ERR_HIP.
 */
ADC2_API adc2_status adc2_sigma(adc2_handle h, int m, const void* X, void* S, void* stream);

/*
 * adc2_sigma_noalloc -- adc2_sigma (FP64 form) that allocates nothing.
 * For callers that cannot allocate device memory during the call: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The caller passes X and S as for adc2_sigma; the sigma's work
 * spaces (the X-build output, the Y-build partials, the unpacked doubles and
 * the light and back-contraction partials) come from one static device
 * array of 128 MiB that the library holds on every device it runs on until
 * the process ends, instead of the handle's buffers.  No hipMalloc, hipFree
 * or other allocating call is made.  The array is shared by every call on a
 * device and keeps the last call's contents; no kernel of the sigma reads
 * scratch memory it has not written in the same call.  Calls that overlap on
 * one device (concurrent streams or threads) race on the array and must not
 * be issued.  Results equal adc2_sigma's in the FP64 form: the same kernels
 * with the same split counts.
 *   m  >= 1; the work spaces of m vectors must fit the array: about
 *      16 m nc (naux nv (1 + ysplit) + no nv^2) bytes (c1: nc=6, no=10,
 *      nv=40, naux=150 fits m up to about 16).
 * Errors: ADC2_ERR_ARG (NULL, m < 1, S aliasing X, a handle in a precision
 * form, sizes above the maximum, with the bytes needed in the message),
 * ADC2_ERR_HIP.  Stream-ordered, asynchronous.
 */
ADC2_API adc2_status adc2_sigma_noalloc(adc2_handle h, int m, const void* X, void* S, void* stream);

/*
 * adc2_davidson -- lowest nroots eigenpairs of M by block Davidson (FP64).
 *   nroots   1..ADC2_MAX_ROOTS.
 *   opt      may be NULL (tol 1e-8, defaults above).
 *   guess    dev complex128 [g][dim] or NULL (NULL: unit vectors on the
 *            lowest singles diagonal elements of M); g = opt->nguess or the
 *            default count.
 *   omega    host float64 [nroots], ascending.
 *   X        dev complex128 [nroots][dim] or NULL: normalised eigenvectors.
 *   info     host, may be NULL.
 * Two-stage solve (opt->mixed_tol > 0, handle in ADC2_FP64): the roots are
 * first solved with split-BF16 sigma builds to residual mixed_tol, then by
 * the FP64 solver to tol started from those vectors; the results are FP64
 * roots (the precision form's arithmetic never reaches them).  info sums
 * both stages; the handle is left in ADC2_FP64.  mixed_tol must exceed
 * tol (ADC2_ERR_ARG otherwise, and with root following).
 * Root following (opt->follow = 1): the root-specific Davidson the paper
 * uses to keep each root matched to its guess (Hirao and Nakatsuji, cited in
 * the Computational details).  Root j is, at every iteration, the Ritz pair
 * whose unit vector overlaps most (|<g_j|x>|^2 / |g_j|^2) with guess vector
 * g_j, assigned greedily in decreasing order of overlap; omega and X are
 * then in guess order, not ascending.  The folded solver solves every branch
 * of its projected problem (one per search-space vector) and measures the
 * overlap on the singles (the doubles of its Ritz vectors follow from their
 * singles).
 * Needs guess with at least nroots vectors (ADC2_ERR_ARG otherwise).
 * Returns ADC2_ERR_NOCONV (with the best omega/X/info written) when max_iter
 * is reached; ADC2_ERR_NONFINITE when the iteration produced NaN/Inf.
 * Synchronises the stream.
 */
ADC2_API adc2_status adc2_davidson(adc2_handle h, int nroots, const adc2_dav_opts* opt,
                          const void* guess, double* omega, void* X,
                          adc2_dav_info* info, void* stream);

/*
 * adc2_set_precision -- switch the arithmetic of subsequent sigma builds
 * (adc2_sigma, adc2_davidson) on an existing handle.  ADC2_C64 builds its
 * complex64 operand copies on first use (stream-ordered).  ADC2_ERR_ARG for an
 * unknown precision.
 */
ADC2_API adc2_status adc2_set_precision(adc2_handle h, int prec);

/*
 * adc2_set_method -- the scheme of M for subsequent sigma builds, solves and
 * diagonals of the handle.
 *   ADC2_METHOD_ADC2   (default) CVS-ADC(2): doubles block diag(D), zeroth order.
 *   ADC2_METHOD_ADC2X  CVS-ADC(2)-x, the extended scheme the paper's
 *     Conclusions name as the next step: the doubles block also carries its
 *     first-order part, the fluctuation potential between the doubly excited
 *     determinants (particle ladder <ab||cd>, hole ladder <Kk||Ij>, and the
 *     ring terms <kb||cj> (k, j valence) and <Kb||cI> (K, I core) that the
 *     core-valence separation leaves).  The singles block and the coupling
 *     are those of ADC(2).
 * Selecting ADC(2)-x forms its integral blocks once (FP64, stream-ordered,
 * then synchronised): npair^2 + (nc no)^2 + (no nv)^2 + (nc nv)^2 complex
 * values, npair = nv(nv-1)/2 (32 GB at nv = 300); ADC2_ERR_OOM with the size
 * in the message above 64 GiB.  Its sigma terms run in FP64 on the MFMA
 * whatever the precision form.  Under ADC(2)-x the folded solver (which needs
 * a diagonal doubles block) and adc2_omega_backward return ADC2_ERR_ARG; the
 * full-space solver and adc2_rayleigh apply the ADC(2)-x matrix.
 * Errors: ADC2_ERR_ARG (NULL handle, unknown method), ADC2_ERR_OOM, ADC2_ERR_HIP.
 */
#define ADC2_METHOD_ADC2 0
#define ADC2_METHOD_ADC2X 1
ADC2_API adc2_status adc2_set_method(adc2_handle h, int method, void* stream);

/*
 * adc2_rayleigh -- FP64 Rayleigh quotients and residual norms of k vectors:
 *   omega[i] = x_i^H M x_i / x_i^H x_i,  resnorm[i] = ||M x_i - omega_i x_i|| / ||x_i||
 * computed with an FP64 sigma build whatever the handle's precision (the
 * final polish of the precision form, and an a-posteriori certificate: for
 * Hermitian M an eigenvalue lies within resnorm of omega).
 *   X dev complex128 [k][dim]; omega, resnorm host float64 [k] (resnorm may be
 *   NULL).  Synchronises the stream.
 */
ADC2_API adc2_status adc2_rayleigh(adc2_handle h, int k, const void* X, double* omega, double* resnorm,
                                   void* stream);

/*
 * adc2_omega_backward -- adjoint of the eigenvalues (differentiation form;
 * Hellmann-Feynman theorem applied to the Hermitian eigenproblem of
 * Eq. 11 with M through second order, Eq. 12).  For vectors x_k and weights
 * g_k it returns the gradient of
 *     f(L, eps) = sum_k g_k x_k^H M(L, eps) x_k / (x_k^H x_k)
 * with the x_k held fixed, which is the vector-Jacobian product
 * sum_k g_k d omega_k when the x_k are eigenvectors (e.g. the X of
 * adc2_davidson).  All arithmetic is FP64 on the GPU whatever the handle's
 * precision.
 *   nroots   number of vectors, 1..ADC2_MAX_ROOTS
 *   X        dev complex128 [nroots][dim], each with non-zero norm
 *   g_omega  host float64 [nroots], the upstream gradient d(loss)/d omega_k
 *   dL       dev complex128 [naux][n][n], overwritten with G^P_pq: the
 *            Hermitian projection of df/dRe L + i df/dIm L, so that
 *            df = Re sum conj(G) dL for every Hermitian perturbation dL
 *            (torch's complex-gradient convention restricted to Hermitian L)
 *   deps     dev float64 [n], overwritten with df/d eps_p
 * The Cholesky blocks and energies are those the handle was set up with.
 * Device workspace of the order of o^2 nv^2 + 2 nroots nc no nv^2 complex
 * values is allocated for the call and freed before it returns (about 30 GB
 * at nc=6, no=60, nv=300, 10 roots).  Synchronises the stream.  Errors:
 * ADC2_ERR_ARG (NULL pointers, nroots out of range, non-finite g_omega, a
 * zero vector), ADC2_ERR_OOM, ADC2_ERR_HIP; dL and deps are then undefined.
 */
ADC2_API adc2_status adc2_omega_backward(adc2_handle h, int nroots, const void* X, const double* g_omega,
                                         void* dL, double* deps, void* stream);

/*
 * Batching form: several independent systems (molecules) of uneven size
 * solved together.  Each system keeps its own handle; what is shared is the
 * launch sequence.  In a batched sigma every phase of the sigma build runs for
 * all systems before the next phase, and the two heavy contractions (the
 * sigma2 product and the Y-build of the Cholesky-vector-driven sigma) of all
 * systems in the complex64 or split-BF16 form are ONE launch each, whose
 * workgroups walk a ragged list of (system, K-split, output tile) work items.
 */
typedef struct {
  const void* L;        /* dev complex128 [naux][n][n], Hermitian per P (as adc2_setup) */
  const double* eps;    /* dev float64 [n] */
  int nc, no, nv, naux;
} adc2_mol;

/*
 * adc2_setup_batch -- adc2_setup for nmol systems (1..64) with one precision.
 *   alloc  optional device-memory callbacks shared by every handle (NULL: hipMalloc).
 *   mols   host [nmol]; out host [nmol] receives the handles (each released
 *          with adc2_destroy).  On error every handle already built is
 *          destroyed, out[] is set to NULL and the failing system's index is
 *          named in adc2_last_error.  Synchronises the stream.
 */
ADC2_API adc2_status adc2_setup_batch(int nmol, const adc2_mol* mols, int prec, const adc2_alloc* alloc,
                                      void* stream, adc2_handle* out);

/*
 * adc2_sigma_batch -- S_i = M_i X_i for nmol systems in one batched launch
 * sequence (stream-ordered, asynchronous).
 *   hs host [nmol] distinct handles; m host [nmol] (>= 1); X, S host arrays
 *   [nmol] of dev pointers, complex128 [m_i][dim_i] as adc2_sigma.
 * Results equal nmol separate adc2_sigma calls: the same kernels compute the
 * same tiles in the same order.  Errors: ADC2_ERR_ARG (NULL, m < 1, a handle
 * repeated), ADC2_ERR_OOM, ADC2_ERR_HIP.
 */
ADC2_API adc2_status adc2_sigma_batch(int nmol, const adc2_handle* hs, const int* m, const void* const* X,
                                      void* const* S, void* stream);

/*
 * adc2_davidson_batch -- adc2_davidson for nmol systems solved concurrently.
 * Each system runs its own solver (opt->solver, same options for all) on its
 * own host thread and HIP stream.
 *   mode ADC2_BATCH_ROUNDS:  whenever the solvers need sigma builds they meet
 *        at a rendezvous and the pending requests of all systems still
 *        iterating run as one batched sigma (adc2_sigma_batch) on the given
 *        stream; a system that converges (or fails) leaves the rendezvous.
 *   mode ADC2_BATCH_STREAMS: no rendezvous; every system's sigma builds run
 *        on its own stream and the GPU overlaps the streams (and one system's
 *        host work with the others' kernels).
 * In both modes each system's iterates, and so its roots, equal those of a
 * separate adc2_davidson call.
 *   omega  host float64 [nmol][nroots];  X host [nmol] of dev pointers
 *   (complex128 [nroots][dim_i]) or NULL;  info host [nmol] or NULL.
 * Returns the first non-OK status in system order (every system's results
 * are still written; adc2_last_error names the system).  Synchronises the
 * stream; guesses are the default ones.
 */
#define ADC2_BATCH_ROUNDS 0
#define ADC2_BATCH_STREAMS 1
ADC2_API adc2_status adc2_davidson_batch(int nmol, const adc2_handle* hs, int nroots, const adc2_dav_opts* opt,
                                         int mode, double* omega, void* const* X, adc2_dav_info* info,
                                         void* stream);

/*
 * Graph-captured batched sigma (batching form): the whole launch sequence of
 * one adc2_sigma_batch call (every phase of every system, the grouped heavy
 * GEMMs included) recorded once as a HIP graph and replayed with one launch.
 * A replay reads X_i and writes S_i at the device addresses given at capture,
 * so a caller refills X_i in place between replays.
 *
 * adc2_graph_sigma_batch -- arguments as adc2_sigma_batch.  Runs the batched
 *   sigma once eagerly on `stream` (so S_i = M_i X_i on return, and every
 *   work space is sized), synchronises it, then captures the same sequence on
 *   an internal stream and instantiates it into *out.  Per-kernel profiling
 *   is suspended during the capture.  Errors: those of adc2_sigma_batch, and
 *   ADC2_ERR_ARG for a handle in the ADC(2)-x method (its doubles block is
 *   outside the captured sequence).
 * adc2_graph_launch -- replays the graph on `stream` (asynchronous).  The
 *   handles must still exist, and every one must still hold the work spaces
 *   (addresses and capacities), operand copies, precision form, method,
 *   engine and split counts the graph recorded: a sigma call with a larger
 *   block, a change of precision or method, or adc2_autotune re-sizes or
 *   changes them, and the launch then returns ADC2_ERR_ARG (capture again)
 *   instead of replaying.  A replay shares the
 *   handles' work spaces with every other sigma on them: calls that overlap
 *   in time race.
 * adc2_graph_destroy -- releases the graph (NULL is accepted).
 */
typedef struct adc2_graph_s* adc2_graph;
ADC2_API adc2_status adc2_graph_sigma_batch(int nmol, const adc2_handle* hs, const int* m, const void* const* X,
                                            void* const* S, void* stream, adc2_graph* out);
ADC2_API adc2_status adc2_graph_launch(adc2_graph g, void* stream);
ADC2_API adc2_status adc2_graph_destroy(adc2_graph g);

/* Copy the dense singles block M11 (complex128 [nc*nv][nc*nv], row (I,a),
 * column (J,b)) into dev buffer dst.  Stream-ordered. */
ADC2_API adc2_status adc2_get_m11(adc2_handle h, void* dst, void* stream);

/* Copy the real diagonal of M (float64 [dim]) into dev buffer dst. */
ADC2_API adc2_status adc2_get_diag(adc2_handle h, double* dst, void* stream);

/* MP2 correlation energy -1/4 sum |<ab||ij>|^2 / D^{ab}_{ij} (host scalar). */
ADC2_API adc2_status adc2_mp2_energy(adc2_handle h, double* e_mp2);

/*
 * Per-kernel timing of the sigma build (for roofline reporting).
 * adc2_profile(h, 1) resets the counters and brackets every sigma kernel
 * launch with HIP events on the launch stream (each sigma call then
 * synchronises its stream once); adc2_profile(h, 0) stops it.
 * adc2_kernel_stats fills up to max entries and returns how many kernels are
 * tracked (or -1 for a NULL handle).  flops are the algorithmic flops of the
 * recorded launches (8 per complex multiply-add).
 */
typedef struct {
  char name[24];
  long launches;
  double ms;        /* summed event time of those launches */
  double flops;     /* summed algorithmic flops */
} adc2_kstat;

ADC2_API adc2_status adc2_profile(adc2_handle h, int enable);
ADC2_API int adc2_kernel_stats(adc2_handle h, adc2_kstat* out, int max);

/*
 * adc2_transition -- transition dipole moments and oscillator strengths
 * (paper, Theory section, transition properties):
 *   T_n = X_n^H F,  F_I = <Psi~_I| D |Psi0>,  f_n = (2/3) omega_n sum_x |T_n^x|^2,
 * for the three Cartesian components of a one-particle operator
 * D = sum_pq d_pq a+_p a_q.  F in the Moller-Plesset expansion of that
 * definition: singles through `order` (1: zeroth and first; 2: also the
 * second, the order of the paper's transition density), doubles through
 * first order (their second order reaches T only at third order).  The
 * second-order singles hold the second-order ground-state singles and
 * doubles amplitudes (particle and hole ladders, ring terms) and the pair
 * densities; the intermediate states are the core rows of the full singles
 * class.
 *   dip    dev complex128 [3][n][n], d^x, d^y, d^z (Hermitian), spinor order
 *          of the setup.
 *   X      dev complex128 [nroots][dim], normalised eigenvectors (e.g. from
 *          adc2_davidson); omega host float64 [nroots].
 *   order  1 or 2.
 *   T      host complex128 [nroots][3]; f host float64 [nroots].
 * Work space: the MP2 amplitudes of every occupied pair (o(o-1)/2 nv^2
 * complex), F (3 dim complex) and small buffers; order 2 adds up to three
 * o^2 nv^2 arrays (amplitudes of every ordered pair, (kj|bc) twice), the
 * (ac|bd) integrals of up to 32 a-values twice (at most 2 x 16 GiB) and
 * naux nv^2 + 2 nc o nv^2; all allocated and freed here (about 35 GB at
 * nc=6, no=60, nv=300; ADC2_ERR_OOM where it does not fit).  The particle
 * ladder costs naux nv^4 + nc o nv^4 complex multiply-adds (FP64 MFMA).
 * Synchronises the stream.  Errors: ADC2_ERR_ARG (NULL argument, nroots out
 * of 1..ADC2_MAX_ROOTS, order not 1 or 2), ADC2_ERR_OOM, ADC2_ERR_HIP.
 */
ADC2_API adc2_status adc2_transition(adc2_handle h, const void* dip, int nroots, const void* X, const double* omega,
                                     int order, void* T, double* f, void* stream);

/*
 * adc2_fns -- frozen natural virtual spinors (paper, State-Average Frozen
 * Natural Spinors: Eq. 15 and Eq. 17-20) from the MP2 virtual density of the
 * system h was set up for:
 *   D_ab = 1/2 sum_{c,i,j} <ac||ij><ij||bc> / (e^{ac}_{ij} e^{bc}_{ij}),
 *   D V = V n;  V~ = natural virtuals with n >= threshold;
 *   F_NS = V~^H diag(e_virt) V~ = Z~ e' Z~^H;  U = V~ Z~.
 * The occupied spinors stay canonical.  The CIS(D) state average of Eq. 16
 * is not included: D is its MP2 term.
 *   L         dev complex128 [naux][n][n], the Cholesky vectors h was set up
 *             with (the handle keeps only blocks of them).
 *   threshold occupation cut (the paper's production value is 10^-4.5).
 *   nv_out    host: the number nv' of kept virtual spinors.
 *   occ       host float64 [nv] or NULL: all occupations n, descending.
 *   L_out     dev complex128 with room for [naux][n'][n'] (n' = nc+no+nv' <=
 *             n): the rotated vectors L'^P = W^H L^P W, W = blockdiag(1, U),
 *             packed with stride n'; eps_out dev float64 with room for n':
 *             occupied energies unchanged, then e'.  Both NULL: only nv_out
 *             and occ are computed.
 * A handle set up on (L_out, eps_out, nc, no, nv', naux) is the truncated
 * problem; with every natural virtual kept its roots equal those of h.
 * Synchronises the stream.  Errors: ADC2_ERR_ARG (NULL handle or nv_out,
 * only one of L_out / eps_out, nothing above the threshold), ADC2_ERR_OOM,
 * ADC2_ERR_HIP.  Work space: up to 2 GiB plus nv^2 and 2 n'n complex.
 */
ADC2_API adc2_status adc2_fns(adc2_handle h, const void* L, double threshold, int* nv_out, double* occ,
                              void* L_out, double* eps_out, void* stream);

/*
 * Autotuner of the sigma build's dominant GEMM, the Y-build (M12 half of the
 * sigma, Implementation section): its K-split count decides how many
 * workgroups a launch has against extra partial traffic and a summation
 * pass, and in the FP64 form its engine decides the tile shape (128 x 128 on
 * eight waves, 128 x 64 at two workgroups per CU, 128 x 128 on four waves, or
 * 128 x 64 three-multiplication).
 * adc2_autotune times the Y-build of h's current precision form at block size
 * m: in the FP64 form first each engine at its own size-rule K-split (unless
 * the environment variable ADC2_ZGEMM fixes the engine), then, for the
 * fastest engine (or the form's only one), the K-splits 1, 2, 3, 4, 6, 8, 12,
 * 16 (those whose partial workspace stays under 8 GiB and that leave each
 * split at least 64 of the no*nv contraction indices); one warm-up and three
 * timed launches each on uniform random operands (the matrix cores run
 * measurably faster on zeros).  It fixes the fastest engine and K-split for h
 * (for every later block size too).  A choice already made for the same
 * (device, nc, no, nv, naux, m, form) in this process, or listed in the text
 * file named by the environment variable ADC2_TUNE_CACHE, is reused without
 * timing; new choices are appended to that file.  Results of sigma builds
 * differ between K-splits and engines only by rounding (the engines other than
 * the three-multiplication one give identical results at equal K-splits).
 * info (host, nullable) receives the choice, the K-splits timed and their
 * best times in ms (ncand = 0 and from_cache = 1 for a cached choice), the
 * chosen engine (zgemm: 0 = 128 x 128 on four waves, 1 =
 * three-multiplication, 2 = two per CU, 3 = 128 x 128 on eight waves) and the
 * engines timed with their best times.
 * Synchronises the stream; must not overlap other calls on h.  Errors:
 * ADC2_ERR_ARG (NULL handle, m out of 1..4096), ADC2_ERR_OOM, ADC2_ERR_HIP.
 */
typedef struct {
  int ysplit;
  int ncand;
  int cand[8];
  double ms[8];
  int from_cache;
  int zgemm;
  int nengine;
  int engine[4];
  double engine_ms[4];
} adc2_tune_info;
ADC2_API adc2_status adc2_autotune(adc2_handle h, int m, adc2_tune_info* info, void* stream);

/*
 * Peak probes: microbenchmarks of the device rates that roofline fractions
 * are quoted against, run on the device current for the calling thread, on
 * `stream`.  Not part of the method; a measurement utility.
 *   ADC2_PEAK_MFMA_F64   v_mfma_f64_16x16x4_f64 (FP64 sigma GEMMs), TFLOP/s
 *   ADC2_PEAK_MFMA_F32   v_mfma_f32_16x16x4_f32 (complex64 GEMMs), TFLOP/s
 *   ADC2_PEAK_MFMA_BF16  v_mfma_f32_16x16x32_bf16 (split-BF16 GEMMs), TFLOP/s
 *   ADC2_PEAK_VALU_F64   v_fma_f64 (folded-solver moments), TFLOP/s
 *   ADC2_PEAK_HBM_READ   streaming 16-byte loads over `bytes`, GB/s
 *   ADC2_PEAK_HBM_COPY   copy of `bytes` (read + write both counted), GB/s
 *   ADC2_PEAK_MFMA_F64_RAND, ADC2_PEAK_MFMA_BF16_RAND  the FP64 and BF16 MFMA
 *                        probes with per-lane pseudo-random operands (uniform
 *                        in [-1, 1), four registers of each side cycled):
 *                        the rate with data-like switching activity, which
 *                        the power limit may hold below the constant-operand
 *                        rate, TFLOP/s
 * bytes: buffer size of the HBM probes (0 = 2 GiB; 64 MiB .. 64 GiB),
 * ignored otherwise.  reps: timed launches (1..1000) after one warm-up; the
 * best launch (HIP events) is returned in *rate (host).  The probe allocates
 * and frees its own device buffers (up to 2 x bytes) and synchronises the
 * stream.  Errors: ADC2_ERR_ARG for a NULL rate, unknown kind or sizes out of
 * range; ADC2_ERR_OOM / ADC2_ERR_HIP from the runtime.
 */
#define ADC2_PEAK_MFMA_F64 0
#define ADC2_PEAK_MFMA_F32 1
#define ADC2_PEAK_MFMA_BF16 2
#define ADC2_PEAK_VALU_F64 3
#define ADC2_PEAK_HBM_READ 4
#define ADC2_PEAK_HBM_COPY 5
#define ADC2_PEAK_MFMA_F64_RAND 6
#define ADC2_PEAK_MFMA_BF16_RAND 7
ADC2_API adc2_status adc2_peak_probe(int kind, size_t bytes, int reps, double* rate, void* stream);

/* Release everything the handle owns.  NULL is accepted. */
ADC2_API adc2_status adc2_destroy(adc2_handle h);

/* Message of the last error on the calling thread ("" if none). */
ADC2_API const char* adc2_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ADC2_H */
