/*
 * rbicg.h -- C ABI of the MI355X recycling-BiCG library (librbicg.so).
 *
 * Method: Ahuja, de Sturler, Gugercin, Chang, "Recycling BiCG with an
 * Application to Model Reduction".  The library solves sequences of dual
 * systems (Sec. 1, eq. initialSys)
 *        A_j x_j = b_j,     A_j^H x~_j = b~_j,
 * with RBiCG (Algorithm 2), updating the recycle spaces U, U~ cycle by cycle
 * while a system is solved (Sec. 4) and carrying them to the next system.
 *
 * Conventions
 *   - Inner product (a, b) = a^H b.  The paper's A^* is written A^H.
 *   - Sparse matrices enter as CSR with int32 row pointers / column indices.
 *     Inside the library they are repacked into a wave-sliced ELL layout for
 *     the gfx950 kernels; the caller never sees it.
 *   - n-vectors are contiguous, of the handle's vector type:
 *       RBICG_F64            double
 *       RBICG_C128           complex double, interleaved (re, im)
 *       RBICG_F32_IN_F64_OUT double at the boundary (FP64 outer refinement);
 *                            the inner RBiCG stores float vectors internally
 *   - Every vector argument is a DEVICE pointer on the current HIP device,
 *     used in stream order on opts.stream; the call returns after the result
 *     is complete (it synchronizes that stream).  The library never frees
 *     caller memory.
 *   - Recycle bases are column-major n x k device arrays (leading dimension n)
 *     of the handle's storage type: double, complex double, or float for
 *     RBICG_F32_IN_F64_OUT (whose inner solver works on float copies).
 *
 * Ownership: a handle owns device copies of A and of the explicit A^H, the
 * recycle bases U, U~, C = A U, C~ = A^H U~, the cycle buffers and the
 * workspace.  They persist across systems until rbicg_destroy.  One handle
 * must not be used by two host threads at once.
 *
 * Return codes (every int function):
 *    0 RBICG_OK
 *    1 RBICG_NOT_CONVERGED  maxit or max_restarts reached; x, x~ hold the
 *                           last iterates and the stats are filled in
 *   -1 RBICG_EINVAL         bad argument (null pointer, size, k > 64, ...)
 *   -2 RBICG_ENOMEM         device allocation failed
 *   -3 RBICG_BREAKDOWN      (p~, q) or (r~, r) vanished or became NaN (Sec. 2:
 *                           serious breakdown / breakdown of the second kind;
 *                           no look-ahead is attempted)
 *   -4 RBICG_EHIP           a HIP runtime call failed
 * rbicg_last_error() returns a thread-local message for the last failure.
 */
#ifndef RBICG_H
#define RBICG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RBICG_OK 0
#define RBICG_NOT_CONVERGED 1
#define RBICG_EINVAL (-1)
#define RBICG_ENOMEM (-2)
#define RBICG_BREAKDOWN (-3)
#define RBICG_EHIP (-4)

#define RBICG_KMAX 64

typedef struct rbicg_s *rbicg_handle;

typedef enum {
  RBICG_F64 = 0,
  RBICG_C128 = 1,
  RBICG_F32_IN_F64_OUT = 2
} rbicg_precision;

/* A sparse n x n matrix in CSR form.  values is double[nnz], or double[2*nnz]
 * (interleaved complex) when values_complex = 1.  on_device = 1: the three
 * arrays are device pointers, else host pointers.  Column indices inside a
 * row need not be sorted; duplicate entries are not allowed. */
typedef struct {
  int32_t n;
  int64_t nnz;
  const int32_t *rowptr;
  const int32_t *colind;
  const void *values;
  int32_t values_complex;
  int32_t on_device;
} rbicg_csr;

/* Options (rbicg_default_opts fills them).
 *   k            recycle-space dimension (0 = plain BiCG, Algorithm 1), <= 64
 *   s            cycle length: iterations between recycle updates (Sec. 4.1)
 *   maxit        iteration cap per solve (restarts included)
 *   max_restarts restarts after a failed true-residual check
 *   update       1: update the recycle space at every completed cycle
 *   svd_tol      truncation tolerance on the cosines of the principal angles
 *                between range(C) and range(C~) (Sec. 4.3)
 *   seed         SplitMix64 seed of the x~ re-seed vector (Algorithm 2 step 3)
 *   prec         vector type / precision mode
 *   inner_tol    FP32 inner tolerance of RBICG_F32_IN_F64_OUT
 *   max_outer    outer refinement steps of RBICG_F32_IN_F64_OUT
 *   stream       hipStream_t to run on (NULL: the null stream)
 *   chunk        iterations launched between convergence polls (0: auto)
 *   profile      p > 0: time the iteration kernels of every p-th chunk of
 *                iterations with HIP events recorded between the launches
 *                (read with rbicg_profile); 0: off
 *   stall_window w > 0 (FP64 / complex solves with a recycle space; not in
 *                the paper): at every cycle end, if the smallest cycle-end
 *                value of max(||r||/||b||, ||r~||/||b~||) has not halved over
 *                the last w cycles, the solve restarts from its initial
 *                guesses without the recycle space (one of max_restarts; the
 *                restarted run builds a new space from its own cycles).
 *                0 (default): off, plain Algorithm 2.
 *   pencil_setup how the cycle-end harmonic Ritz pencil (eq. finalGenEigValue)
 *                is set up: 0 (default) from device Gram matrices of the
 *                cycle's vectors (the captured A p_i give A Phi_j); 1 by the
 *                recurrences of Sec. 4.4, which carry the blocks of
 *                Psi~^H Psi and Psi~^H Phi from cycle to cycle so that only
 *                Upsilon~_j^H U_{j-1} ((s+2) x k) is formed over the n rows
 *                (FP64 and complex handles; FP32-inner solves and the first
 *                cycle of a restarted run use 0).
 *   blocks       blocks of the iteration kernels (1024 threads each, up to 8
 *                rows per thread; 0: automatic, min(ceil(n/1024), 256) but
 *                at least ceil(n/8192)); must lie in [ceil(n/8192), 4096].
 *                The block partial sums are reduced in a fixed order, so a
 *                given value gives reproducible results; different values
 *                round the reductions differently.  Chosen by the autotuner
 *                (paper_1010_0762_amd/tune.py) or left automatic. */
typedef struct {
  int32_t k, s, maxit, max_restarts, update;
  double svd_tol;
  uint64_t seed;
  rbicg_precision prec;
  double inner_tol;
  int32_t max_outer;
  void *stream;
  int32_t chunk;
  int32_t profile;
  int32_t stall_window;
  int32_t pencil_setup;
  int32_t blocks;
} rbicg_opts;

/* A matrix repacked and resident in device memory (A and its explicit A^H),
 * so that a sequence's matrices can be uploaded once and switched without
 * host work.  It must outlive every handle that uses it. */
typedef struct rbicg_mat_s *rbicg_matrix;

/* Per-solve statistics.  relres / relres_dual are TRUE relative residuals
 * ||b - A x|| / ||b|| computed after the solve; alg_bytes counts the
 * algorithmic HBM bytes of the iterations (per-iteration model times iters). */
typedef struct {
  int32_t status, iters, restarts, outer_steps, cycles, k_used, reseeds;
  double relres, relres_dual, time_ms, alg_bytes;
} rbicg_stats;

/* Fill *opts with defaults: k=20, s=40, maxit=10000, max_restarts=2,
 * update=1, svd_tol=1e-2, seed=0, prec=RBICG_F64, inner_tol=1e-5,
 * max_outer=30, stream=NULL, chunk=0, profile=0, stall_window=0,
 * pencil_setup=0, blocks=0. */
void rbicg_default_opts(rbicg_opts *opts);

/* Repack A (and A^H, built on the host by a counting sort when AH is NULL)
 * into device memory once (a matrix of the sequence of eq. initialSys).
 * Blocks until the upload is complete. */
int rbicg_matrix_create(const rbicg_csr *A, const rbicg_csr *AH, rbicg_matrix *out);

/* Free a matrix made by rbicg_matrix_create or rbicg_matrix_pencil (no
 * handle may still use it). */
int rbicg_matrix_destroy(rbicg_matrix m);

/* Layout of a resident matrix, into info[0..4] (host array of 5 int64):
 * order n, stored entries nnz, entries of the padded sliced-ELL layout
 * (64-row slices, each as wide as its longest row), 1 if A^H shares A's
 * slice pointers and column indices (A^H has A's pattern with rows in the
 * same column order, e.g. a structurally symmetric stencil with sorted rows;
 * the iteration kernels then read the indices once per row), 1 if the values
 * are complex.  RBICG_EINVAL for null arguments; no device work. */
int rbicg_matrix_info(rbicg_matrix m, int64_t *info);

/* The pencil P = alpha E + beta A of two resident matrices, with its
 * conjugate transpose conj(alpha) E^H + conj(beta) A^H: the shifted operators
 * sigma E - A (alpha = sigma, beta = -1) of IRKA with E != I (Algorithm 3,
 * step 2).  alpha, beta: complex numbers as (re, im) pairs (host).  E must be
 * given on A's sparsity pattern (explicit zeros allowed); P is complex and
 * needs RBICG_C128 handles.
 *   *out == NULL: a new matrix with A's layout is made (the layouts are
 *     compared on the host, once) and its values are set.
 *   *out from an earlier call with the same A and E: only the values are
 *     overwritten, by one device pass on `stream` (asynchronous; the caller
 *     orders it against the handles that use *out, e.g. by using their
 *     stream or synchronizing).
 * Errors: RBICG_EINVAL for null arguments, a size or pattern mismatch, or an
 * *out that is not a pencil of A and E; RBICG_ENOMEM / RBICG_EHIP otherwise.
 * Free with rbicg_matrix_destroy. */
int rbicg_matrix_pencil(rbicg_matrix A, rbicg_matrix E, const double *alpha, const double *beta,
                        void *stream, rbicg_matrix *out);

/* Split ILU(0) preconditioning in red-black ordering (Sec. 6 solves every
 * system split-preconditioned, with recycle spaces of the preconditioned
 * systems).  The unknowns of A are coloured so that every off-diagonal entry
 * joins a red and a black unknown (5- and 7-point stencils); with P the
 * red-black permutation and P A P^T = L U + R its ILU(0) factorization, the
 * split-preconditioned operator L^{-1} P A P^T U^{-1} is block diagonal with
 * an identity red block and the black block
 *   M_B = (D_B - A_BR D_R^{-1} A_RB) S_B^{-1}
 * (S_B: the black ILU(0) pivots).  A dual pair A x = b, A^H x~ = b~ is solved
 * as M_B y_B = b^_B, M_B^H y~_B = c^_B (an ordinary handle on *black) with
 * the transforms below.
 *   rbicg_rbilu_create: host set-up from A (host or device CSR, real or
 *     complex): *out (the transforms' device data), *black (M_B and M_B^H,
 *     resident, owned by *out: valid until rbicg_rbilu_destroy, never passed
 *     to rbicg_matrix_destroy) and *nb (its order).  RBICG_EINVAL if A has a
 *     zero diagonal entry or zero pivot or its off-diagonal graph is not
 *     two-colourable.
 *   rbicg_rbilu_refresh: new values of A (A_next: same pattern, host or
 *     device CSR) -- the pivots and M_B (in place in *black) recomputed on
 *     the device on `stream`, so that a sequence of matrices on one pattern
 *     (eq. initialSys) needs one host set-up; handles on *black then take
 *     rbicg_update_recycle_on(h, black) (C = M_B U).  The pattern is compared
 *     on the host (a device A_next is copied back for that).  RBICG_EINVAL if
 *     the pattern, size or value type differ.
 *   rbicg_rbilu_refresh_values: the same from a device array of the new
 *     values alone, in the order of the CSR given at creation (the caller
 *     guarantees the pattern; nothing is checked).
 *   rbicg_rbilu_rhs: b^_B, c^_B (nb entries each) from b, b~ (n entries).
 *   rbicg_rbilu_solution: x, x~ (n entries) from y_B, y~_B and b, b~.
 * Vectors are device arrays of A's value type (double or interleaved
 * complex), used on `stream`; calls on one preconditioner must not overlap
 * (they share a scratch vector).  Free with rbicg_rbilu_destroy (which also
 * frees *black; no handle may still use it). */
typedef struct rbicg_rbilu_s *rbicg_rbilu;
int rbicg_rbilu_create(const rbicg_csr *A, rbicg_rbilu *out, rbicg_matrix *black, int32_t *nb);
int rbicg_rbilu_refresh(rbicg_rbilu P, const rbicg_csr *A_next, void *stream);
int rbicg_rbilu_refresh_values(rbicg_rbilu P, const void *values, void *stream);
int rbicg_rbilu_rhs(rbicg_rbilu P, const void *b, const void *bt, void *bB, void *btB, void *stream);
int rbicg_rbilu_solution(rbicg_rbilu P, const void *b, const void *bt, const void *yB,
                         const void *ytB, void *x, void *xt, void *stream);
int rbicg_rbilu_destroy(rbicg_rbilu P);

/* Split ILUT preconditioning (Sec. 6 solves every system of its experiments
 * split-preconditioned by an incomplete LU factorization with a drop
 * tolerance, ILUT(0.05) in Sec. 6.1).  For A = L U + E (L unit lower, U upper)
 * the dual pair A x = b, A^H x~ = b~ becomes
 *   A^ y = b^,  A^^H y~ = c^,   A^ = L^{-1} A U^{-1},  b^ = L^{-1} b,
 *   c^ = U^{-H} b~,   x = U^{-1} y,   x~ = L^{-H} y~,
 * and RBiCG (with its recycle spaces) runs on A^ without forming it: every
 * application of A^ (A^^H) is a triangular solve with U (L^H), one SpMV with
 * A (A^H) and a triangular solve with L (U^H), each triangular solve one
 * level-scheduled device kernel without barriers between levels (the
 * primal and dual directions' solves share launches).
 *   rbicg_ilut_create: host factorization of A (host or device CSR, real or
 *     complex) by ILUT(droptol, fill) -- the drop rules of rbicg_host_ilut
 *     (fill < 0: no per-row count limit) -- or, with permtol > 0, by ILUTP
 *     (column pivoting, Sec. 6.2; A Q = L U + E), level schedules of L, U,
 *     L^H, U^H, and their upload.  With pivoting the operator is
 *     A^ = L^{-1} A Q U^{-1}, c^ = U^{-H} Q^T b~ and x = Q U^{-1} y.
 *     RBICG_EINVAL on a zero pivot.
 *   rbicg_ilu_attach: h iterates with A^ of P from its next call on (NULL
 *     detaches).  P must have h's order and value type (real / complex);
 *     attach it before the rbicg_update_recycle* call that moves h to A, so
 *     that the carried space is biorthogonalized against A^ (C = A^ U).  With
 *     P attached, rbicg_solve_dual solves the
 *     preconditioned pair: b, b~ are b^, c^; x, x~ are y, y~; stats and the
 *     stopping test refer to the preconditioned residuals.  Not for
 *     RBICG_F32_IN_F64_OUT handles, shifted solves, bilinear forms or handles
 *     attached to a batch.  One handle at a time may use P.
 *   rbicg_ilu_rhs: b^, c^ from b, b~; rbicg_ilu_solution: x, x~ from y, y~.
 *     Device n-vectors, double (complex_vectors = 0; real P only) or
 *     interleaved complex; on `stream`; calls on one P must not overlap.
 *   rbicg_ilu_info: info[0..6] = n, nnz(L) (strict), nnz(U) (with the
 *     diagonal), levels of L, levels of U, 1 if a triangular solve's bounded
 *     wait ever gave up (results since are invalid), 1 if complex; info[7]
 *     = columns the pivoting moved (info: 8 int64).
 *   rbicg_ilu_set_waves: how many 64-lane waves work through the chunks of
 *     a triangular solve (default 512; [4, 65536]); fewer waves poll less,
 *     more cover wider levels.  Affects speed only, never results.
 * A triangular solve whose dependency wait exceeds its bound (it cannot in a
 * correct schedule) sets an error flag; the solve that used it returns
 * RBICG_EHIP. */
typedef struct rbicg_ilu_s *rbicg_ilu;
int rbicg_ilut_create(const rbicg_csr *A, double droptol, int32_t fill, double permtol,
                      rbicg_ilu *out);
int rbicg_ilu_attach(rbicg_handle h, rbicg_ilu P);
int rbicg_ilu_rhs(rbicg_ilu P, const void *b, const void *bt, void *bh, void *ch,
                  int32_t complex_vectors, void *stream);
int rbicg_ilu_solution(rbicg_ilu P, const void *y, const void *yt, void *x, void *xt,
                       int32_t complex_vectors, void *stream);
int rbicg_ilu_info(rbicg_ilu P, int64_t *info);
int rbicg_ilu_set_waves(rbicg_ilu P, int32_t waves);
int rbicg_ilu_destroy(rbicg_ilu P);

/* As rbicg_create, on a preloaded matrix (not owned by the handle). */
int rbicg_create_on(rbicg_matrix A, const rbicg_opts *opt, rbicg_handle *out);

/* As rbicg_update_recycle with A_next given as a preloaded matrix (NULL: keep
 * the current one): no host-side repacking or upload. */
int rbicg_update_recycle_on(rbicg_handle h, rbicg_matrix A_next);

/* A whole sequence of dual systems (eq. initialSys) in one call: for system j
 * the handle moves to mats[j] as rbicg_update_recycle_on does (the carried
 * space biorthogonalized against it; for j = 0 only when mats[0] is not the
 * handle's matrix, for j > 0 always, also when mats[j] == mats[j-1], which
 * installs the previous system's last cycle space), x[j], x~[j] are zeroed
 * first when zero_init, then rbicg_solve_dual(h, b[j], bt[j], x[j], xt[j],
 * tol, &st[j]).  The same arithmetic as those calls made one by one, without
 * a return to the caller between systems.  mats, b, bt, x, xt: host arrays
 * of nsys pointers (resident matrices; device vectors as for
 * rbicg_solve_dual); st: nsys entries (may be NULL).  Stops at the first
 * system whose call returns a negative code (an error, or RBICG_BREAKDOWN)
 * and returns that code, st filled up to that system; otherwise returns
 * RBICG_NOT_CONVERGED if any system did not converge, else RBICG_OK. */
int rbicg_solve_sequence(rbicg_handle h, int32_t nsys, const rbicg_matrix *mats,
                         const void *const *b, const void *const *bt, void *const *x,
                         void *const *xt, int32_t zero_init, double tol, rbicg_stats *st);

/* Kernel timing of the iteration kernels accumulated while opts.profile is
 * set: out[0..3] = total ms and launch count of (1) the fused direction
 * update + paired SpMV + restriction kernel and (2) the fused expansion +
 * recurrence update + norms kernel (HIP events recorded before and after
 * each launch of the sampled chunks); out[4] = algorithmic bytes of one
 * launch of kernel (1) with the current recycle dimension, out[5] =
 * algorithmic bytes of one iteration; out[6..7] = total algorithmic bytes of
 * the timed launches of kernels (1) and (2) (each launch counted with the
 * recycle dimension it ran with); out[8..12] = cycle-end telemetry (kept
 * whether or not opts.profile is set): recycle-space updates completed, total
 * host ms of their harmonic Ritz eigenproblems, total host ms of their
 * biorthogonalizations, total ms from each update's first enqueue to its
 * last, total ms the iteration launches waited for an update to release its
 * cycle buffers.  reset = 1 clears the counters after reading.  out: host
 * array of 13 doubles. */
int rbicg_profile(rbicg_handle h, int32_t reset, double *out);

/* Create a handle for matrix A (problem statement, Sec. 1).  AH may be NULL,
 * in which case the explicit conjugate transpose A^H is built on the host by
 * a counting sort; the iteration never uses atomics for A^H products.
 * Returns RBICG_OK and *out, or an error code. */
int rbicg_create(const rbicg_csr *A, const rbicg_csr *AH, const rbicg_opts *opt,
                 rbicg_handle *out);

/* Solve the dual pair A x = b, A^H x~ = b~ with RBiCG (Algorithm 2) to
 * ||b - A x|| <= tol ||b|| and ||b~ - A^H x~|| <= tol ||b~|| (relative; if b~ = 0
 * the initial dual residual replaces ||b~||).  x, xt hold x_{-1}, x~_{-1} on
 * entry and the solutions on exit.  The recycle space U, U~ of the handle is
 * used as fixed (Sec. 3); when opts.update is set, the cycle-wise update of
 * Sec. 4 builds the recycle space for the next system, installed by
 * rbicg_update_recycle.  st may be NULL.
 * RBICG_F32_IN_F64_OUT handles (not in the paper): FP64 iterative refinement
 * around the float RBiCG.  Each outer step forms r = b - A x, r~ = b~ - A^H x~
 * with the FP64 matrix, stops when both are <= tol relative, else solves
 * A d = r, A^H d~ = r~ with float matrix values and vectors (every reduction
 * in FP64) to opts.inner_tol relative and adds d, d~ to x, x~ in FP64; the
 * latest cycle's recycle space carries to the next outer step.  An inner
 * solve stops early at a cycle end without progress: near the tolerance its
 * iterate is used; otherwise it is discarded, the recycle space dropped and
 * the next outer step solves in FP64 (plain BiCG).  A correction that raises
 * the FP64 residual is taken back.  st->iters counts inner iterations,
 * st->outer_steps the refinement steps, st->restarts the FP64 inner solves;
 * st->relres is the FP64 true residual.  At most opts.max_outer steps. */
int rbicg_solve_dual(rbicg_handle h, const void *b, const void *bt, void *x, void *xt,
                     double tol, rbicg_stats *st);

/* Move to the next system of the sequence (end of Sec. 4.3): take the recycle
 * space built during the last solve (or keep the current one if no cycle
 * completed, Sec. 6.2), optionally replace the matrix by A_next (AH_next may be
 * NULL; A_next NULL keeps the matrix), recompute C = A U, C~ = A^H U~ and
 * biorthogonalize them (C~^H C = I).  A_next must have the same n. */
int rbicg_update_recycle(rbicg_handle h, const rbicg_csr *A_next, const rbicg_csr *AH_next);

/* Bilinear form u^H A^{-1} w (Sec. 1): solves A x = w and A^H x~ = u with
 * RBiCG and returns u^H x + x~^H r, r = w - A x, whose error r~^H A^{-1} r is
 * quadratic in the residuals.  *value is one double (real) or two (complex,
 * re/im) on the HOST; *err_est (host, may be NULL) receives ||r|| ||r~||, the
 * error bound without the factor ||A^{-1}||.  u, w are device vectors. */
int rbicg_bilinear(rbicg_handle h, const void *u, const void *w, double tol, void *value,
                   double *err_est, rbicg_stats *st);

/* Release every device buffer of the handle. */
int rbicg_destroy(rbicg_handle h);

/* Thread-local message of the last failure ("" if none). */
const char *rbicg_last_error(void);

/* Install U, U~ (device, column-major n x k, vector type of the handle) as the
 * recycle space and biorthogonalize C = A U, C~ = A^H U~ as in
 * rbicg_update_recycle (Algorithm 2 step 1).  k = 0 clears the space. */
int rbicg_set_recycle(rbicg_handle h, const void *U, const void *Ut, int32_t k);

/* Copy the current recycle space out: U, Ut, C, Ct (device, n x kcap each,
 * column-major; any may be NULL); *k receives the dimension.  next = 1 copies
 * the space built by the last solve's cycles instead of the installed one. */
int rbicg_get_recycle(rbicg_handle h, void *U, void *Ut, void *C, void *Ct, int32_t kcap,
                      int32_t next, int32_t *k);

/* Copy the per-iteration log of the last solve to host memory: for each
 * iteration i = 1..*count (at most cap), 10 doubles
 *   alpha_i (re, im), beta_{i-1} (re, im), rho_i = (r~_i, r_i) (re, im),
 *   ||r_i||, ||r~_i||, Re (p~_i, q_i), restart index. */
int rbicg_get_log(rbicg_handle h, double *out, int32_t cap, int32_t *count);

/* Shifted dual pairs of IRKA (Algorithm 3 steps 2-3 with E = I):
 *   (sigma_i I - A) X_i = b,   (sigma_i I - A)^H Xt_i = c,   i < S (S <= 16)
 * for a complex (RBICG_C128) handle on A (real or complex; the shift is
 * applied on the fly, no shifted matrix is formed).  All shifts share one
 * recycle space: the one built by the last update (the previous sweep's), else
 * the installed U, U~ (k <= 32).  Each shift's C_sigma = sigma U - A U and
 * C~_sigma = conj(sigma) U~ - A^H U~ is biorthogonalized on its own (Sec. 4.3,
 * from Grams of the shared basis), which is a per-shift k x k map, so one FP64
 * MFMA contraction of [U~, A^H U~, U, A U] against all shifts' vectors serves
 * every shift in each iteration; the shifts iterate in lock step in one set of
 * launches (a shift stops on its own test).  When opts.update is set, shift
 * update_from (< 0: the one of smallest |sigma|) is solved as a single pair
 * with the cycle-wise update of Sec. 4, which builds the recycle space for the
 * next sweep; every other shift runs in the batch.  No restarts in the batch:
 * a batched shift whose true residual misses tol reports NOT_CONVERGED.
 * sigma: host array of S complex values (re, im).  b, c: device n-vectors;
 * X, Xt: device n x S column-major (leading dimension n), initial guesses on
 * entry, solutions on exit.  st: host array of S stats (required).  Returns 0
 * when every shift converged, else the first failure code. */
int rbicg_solve_shifted(rbicg_handle h, int32_t S, const double *sigma, const void *b,
                        const void *c, void *X, void *Xt, double tol, int32_t update_from,
                        rbicg_stats *st);

/* Batched bilinear forms u_i^H A^{-1} w_i, i < S <= 16 (Sec. 1: bilinear
 * forms of the inverse, e.g. one per sample of a QMC estimate), on one matrix
 * and one recycle space, for a RBICG_C128 handle (real or complex A).  The S
 * dual pairs A x_i = w_i, A^H x~_i = u_i are solved by the batched shifted
 * kernels of rbicg_solve_shifted with sigma = 0: they iterate in lock step in
 * one set of launches per iteration, sharing the matrix reads and the
 * recycle space's restriction and expansion (one FP64 MFMA contraction for
 * all pairs); pair 0 is solved on its own with the cycle-wise update of
 * Sec. 4 when opts.update is set, which builds the recycle space of the next
 * batch (installed by rbicg_update_recycle).  Each value is
 * u_i^H x_i + x~_i^H r_i with r_i = w_i - A x_i, whose error r~_i^H A^{-1} r_i
 * is quadratic in the residuals.
 *   U, W     device n x S complex column-major (leading dimension n).
 *   values   host array of 2 S doubles (re, im per form).
 *   err_est  host array of S doubles (may be NULL): ||r_i|| ||r~_i||, the
 *            error bound without the factor ||A^{-1}||.
 *   st       host array of S stats (required).
 * The call allocates and frees two n x S device buffers for the solutions.
 * Returns 0 when every pair converged, else the first failure code. */
int rbicg_bilinear_batch(rbicg_handle h, int32_t S, const void *U, const void *W, double tol,
                         double *values, double *err_est, rbicg_stats *st);

/* Reduced pencil of IRKA (Algorithm 3 step 4, and step 5 with E = I):
 *   Ar = Xt^H A X,  Er = Xt^H X,  br = Xt^H b,  cr = X^H c   (m <= 32)
 * for a RBICG_C128 handle on A (the unshifted matrix, whatever shifts the
 * handle last solved with).  X, Xt: device n x m column-major complex (leading
 * dimension n, as rbicg_solve_shifted writes them); b, c: device n-vectors or
 * NULL (then br, cr are not written).  Ar, Er: host m x m complex, column-major
 * interleaved; br, cr: host m complex.  A X is formed by the SpMM kernel and
 * the projections by the FP64 MFMA Gram kernel; the call allocates and frees
 * an n x (m + 2) device buffer and returns after the results are on the
 * host.  RBICG_EINVAL for m out of range, b without c, or an m x (2m + 1) Gram
 * larger than the handle's Gram buffers (sized by its k and s). */
int rbicg_project(rbicg_handle h, int32_t m, const void *X, const void *Xt, const void *b,
                  const void *c, double *Ar, double *Er, double *br, double *cr);

/* Continuous batching of iteration launches across handles (serving several
 * requests at once).  A batch owns four HIP streams.  Every handle attached to it
 * keeps its own host thread, stream, matrix, recycle space and workspace, but
 * hands each chunk of iterations (the arguments of its iteration kernels) to
 * the batch instead of launching it; the batch launches the chunks of all
 * attached handles that are iterating in one set of launches -- per
 * iteration one k_it1_multi and one k_it2_multi covering every handle's
 * rows (each handle its own range of blocks, its own partial sums), then one
 * stopping-test launch -- once every iterating handle has handed in a chunk
 * or the oldest chunk has waited window_us microseconds.  Each handle's
 * arithmetic is that of its unbatched launches, so results are bitwise the
 * same alone and batched.  At most max_slots (<= 16) chunks per launch.
 * Handles of different vector types batch in separate launches.  Per-kernel
 * event profiling (opts.profile) is off for attached handles. */
typedef struct rbicg_batch_s *rbicg_batch;
int rbicg_batch_create(int32_t max_slots, double window_us, rbicg_batch *out);
/* Attach h to b (NULL detaches); not while h is solving.  The batch must
 * outlive the attachment. */
int rbicg_batch_attach(rbicg_handle h, rbicg_batch b);
/* out[0..5]: launches, chunks launched, handle-iterations launched, most chunks
 * in one launch, graph replays, graph captures (out: 6 doubles). */
int rbicg_batch_stats(rbicg_batch b, double *out);
/* on != 0: every launch set (the iteration kernels of one batch launch, which
 * read their arguments from device tables) is built once as a HIP graph of
 * kernel nodes (no stream capture) per table buffer and shape and replayed
 * afterwards, so that a steady mix of
 * requests is served by graph launches only (at most 64 graphs kept, least
 * recently used dropped); the tables are copied before each replay.  Results
 * are those of direct launches.  Default off. */
int rbicg_batch_use_graphs(rbicg_batch b, int32_t on);
int rbicg_batch_destroy(rbicg_batch b);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc, code that must not touch the allocator):
 * the same dual solve as rbicg_solve_dual on a handle with opts.k = 0, i.e.
 * plain BiCG (Algorithm 1; Algorithm 2 with an empty recycle space), on a
 * matrix already resident (rbicg_matrix_create), with no handle and no
 * allocation of any kind.  The kernels, their launch order and the options'
 * meaning are those of rbicg_solve_dual, so for equal inputs and options the
 * two return the same iterates, counts and residuals.
 *   A        resident matrix (real or complex values).
 *   opt      k must be 0; prec RBICG_F64 (real matrix, double vectors) or
 *            RBICG_C128 (complex vectors; real or complex matrix); maxit in
 *            [1, RBICG_NOALLOC_MAXIT]; max_restarts, seed, chunk and stream as
 *            for a handle; the other fields are ignored.
 *   b, bt    device n-vectors (caller-owned, read only).
 *   x, xt    device n-vectors: initial guesses on entry, solutions on exit.
 *   tol, st  as for rbicg_solve_dual (st may be NULL).
 * Every intermediate buffer (work vectors, block partial sums, the scalar
 * block, the iteration log) lives in one static device array of
 * RBICG_NOALLOC_SCRATCH_BYTES per GPU, held by the process until it ends:
 * n * bytes per element must be <= 2 MiB after padding n to a multiple of
 * 256 (n <= 262144 real, 131072 complex); larger inputs or maxit return
 * RBICG_EINVAL with a message, before any work.  Every call on one GPU uses
 * that GPU's one array: calls that overlap on the same GPU (two host threads,
 * or two streams) race and give wrong results; serialize them.  The first call
 * on a device looks up the array's device address once.  Host-side waits are
 * stream synchronizations (no events are created). */
#define RBICG_NOALLOC_SCRATCH_BYTES (20 * 1024 * 1024)
#define RBICG_NOALLOC_MAXIT 20000
int rbicg_solve_dual_noalloc(rbicg_matrix A, const rbicg_opts *opt, const void *b, const void *bt,
                             void *x, void *xt, double tol, rbicg_stats *st);

#ifdef __cplusplus
}
#endif
#endif /* RBICG_H */
