/*
 * polyeval: evaluation and differentiation of sparse polynomial systems on
 * MI355X (gfx950), in complex double, double double and quad double.
 *
 * The operations follow J. Verschelde and X. Yu, "GPU acceleration of
 * Newton's method for large systems of polynomial equations in double double
 * and quad double arithmetic" (2014):
 *   - a system is given in sparse distributed form: fully expanded, only
 *     monomials with a nonzero coefficient stored (Problem Statement, Sec. 1);
 *   - each monomial is split into a product of its distinct variables times a
 *     common factor of powers (Sec. 2.1, eq. (1)); the product and all its
 *     partial derivatives come from the reverse mode (Sec. 2.2); every
 *     derivative is multiplied by the common factor, the coefficient and the
 *     exponent, and the terms are summed into F and J (Sec. 2.3);
 *   - a Newton step evaluates A = J(x), b = -F(x), solves A dx = b in the
 *     least-squares sense with modified Gram-Schmidt on [A b] (Sec. 3, Fig. 4,
 *     eq. (2)) and updates x += dx (Sec. 4).
 *
 * Numbers.  A level-L number has L doubles per real part (L = 1: double,
 * L = 2: double double, L = 4: quad double), limbs most significant first,
 * forming a nonoverlapping expansion.  Complex level-L arrays are LIMB-PLANAR:
 * [2 (re, im)][L][count] doubles.  Batched arrays have a leading [P] (points).
 *   x: [P][2][L][n]      F: [P][2][L][N]      J: [P][2][L][N][n] (row-major)
 *
 * Threads and streams.  Handles are immutable after creation except where
 * noted; calls on one handle from several host threads are safe if they use
 * different output buffers.  Device work is enqueued on the given stream
 * (a hipStream_t; NULL = the default stream) and is asynchronous: outputs are
 * valid after the stream is synchronised.  Argument errors are reported
 * synchronously; device errors at the next call or at synchronisation.
 *
 * Ownership.  Host pointers passed to the create calls are read during the
 * call and not retained.  Device pointers passed to evaluation calls are
 * owned by the caller and must stay valid until the enqueued work completes.
 */
#ifndef POLYEVAL_H
#define POLYEVAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pe_status;

#define PE_OK 0
#define PE_EINVAL (-1)        /* invalid argument or malformed system */
#define PE_ENOMEM (-2)        /* device or host allocation failed */
#define PE_EUNSUPPORTED (-3)  /* valid but outside the supported sizes */
#define PE_EDEVICE (-4)       /* a HIP runtime call failed */
#define PE_ESINGULAR (-5)     /* reserved: a numerically zero Gram-Schmidt pivot is
                                 reported per point in resid_out (-1), not as
                                 the status of the call */
#define PE_ENONFINITE (-6)    /* non-finite values met where checked */

/* Level flag for real arithmetic: a level of PE_REAL | L (L = 1, 2, 4)
 * makes a system of real coefficients evaluated at real points in real
 * double, double double or quad double arithmetic.  Its arrays have one
 * component instead of two: coef [L][M], x [P][L][n], F [P][L][N],
 * J [P][L][N][n], V [P][L][M], G [P][L][nnz].  Real systems support
 * pe_eval, pe_eval_terms, pe_newton_step and the homotopy steps; pe_lstsq
 * takes the same level codes. */
#define PE_REAL 8

typedef struct pe_system pe_system;
typedef struct pe_batch pe_batch;

/* Version of this interface (increments on incompatible changes). */
int32_t pe_abi_version(void);

/* Message describing the last error on the calling host thread ("" if none).
 * The string stays valid until the next call on the same thread. */
const char* pe_last_error(void);

/* ------------------------------------------------------------------ systems
 * Load a system in sparse distributed form (Problem Statement, Sec. 1;
 * monomial split of Sec. 2.1, eq. (1)).
 *   level     1, 2 or 4 (limbs per real part), or PE_REAL | 1, 2, 4 for
 *             real arithmetic; all coefficients, points and outputs of this
 *             system are at this level.
 *   n_vars    number of variables n (1 <= n; see the size limits below).
 *   n_polys   number of polynomials N (>= 0).
 *   poly_ptr  [N+1] int64, host: monomials of polynomial p are
 *             poly_ptr[p] .. poly_ptr[p+1]-1; poly_ptr[0] = 0, nondecreasing.
 *   mon_ptr   [M+1] int64, host, M = poly_ptr[N]: occurrences of monomial t
 *             are mon_ptr[t] .. mon_ptr[t+1]-1; mon_ptr[0] = 0, nondecreasing.
 *   var_idx   [nnz] int32, host, nnz = mon_ptr[M]: variable of each
 *             occurrence, in [0, n); distinct within a monomial (any order).
 *   exps      [nnz] int32, host: exponent of each occurrence, 1..65535.
 *   coef      [2][L][M] double, host, limb-planar coefficients ([L][M]
 *             for a real system).
 *   stream    stream used for the uploads (the call synchronises it).
 * Monomials with no occurrence (constants) and polynomials with no monomial
 * are allowed; duplicate monomials are kept as given (never merged).
 * Size limits (PE_EUNSUPPORTED beyond them): n <= 65535 variables (rows of
 * J wider than 2048 columns are evaluated in tiles of 2048 columns, one
 * workgroup each; the adjoint and batches take at most 2048 variables); a
 * monomial spans at most one wavefront of 64 lanes, so it has at most
 * 64 * segment variables: 1024 in double and double double (segment 16),
 * 512 in quad double (segment 8); systems with monomials that wide get that
 * segment by default; at most 2^31 monomials and 2^32 occurrences.
 * Returns PE_EINVAL for malformed input (out-of-range index, exponent < 1,
 * duplicate variable in a monomial, non-monotone offsets), PE_EUNSUPPORTED
 * for the size limits above, PE_ENOMEM or PE_EDEVICE on allocation/copy
 * failure.  On error *out is set to NULL. */
pe_status pe_system_create(pe_system** out, int32_t level, int32_t n_vars, int32_t n_polys,
                           const int64_t* poly_ptr, const int64_t* mon_ptr, const int32_t* var_idx,
                           const int32_t* exps, const double* coef, void* stream);

/* Release a system and its device memory (NULL is allowed).  The caller must
 * make sure no enqueued work still uses it.  PE_EINVAL (nothing released)
 * while a batch that contains the system is alive. */
pe_status pe_system_destroy(pe_system* sys);

/* Sizes of a loaded system: info[0] = level (with PE_REAL if real), [1] = n, [2] = N, [3] = M,
 * [4] = nnz, [5] = largest exponent, [6] = largest monomial size k,
 * [7] = device bytes held, [8] = chunks per workgroup of the evaluation
 * launch, [9] = LDS bytes per evaluation workgroup, [10] = segment length
 * (variables per lane). */
pe_status pe_system_info(const pe_system* sys, int64_t info[11]);

/* Set the evaluation launch shape.  A monomial of k variables is handled by
 * s lanes (s the smallest power of two with s * segment >= k); the
 * monomials of a row are cut into chunks of 256 lanes, and a workgroup of
 * chunks_per_workgroup * 256 threads works on that many chunks of a row at
 * once, adding their partial rows in a fixed order.
 *   segment               variables per lane: 8 or 16 (D), 4, 6, 8 or 16
 *                         (DD), 2, 4 or 8 (QD); 0 = the default: the first of
 *                         8, 16 (D), 8, 6, 4 (DD) or 4, 2 (QD) for which the
 *                         most common monomial size k is an exact multiple of
 *                         s filling every lane (k > (segment - 1) * s), else 8
 *                         (D, DD) or 4 (QD); then widened to the shortest
 *                         compiled segment that fits the largest monomial in
 *                         64 lanes.  pe_system_create starts from the same
 *                         default.
 *   chunks_per_workgroup  1, 2 or 4 as compiled for the level and segment;
 *                         0 = the largest that fits.
 * A new segment length repacks the system (host work and a device upload
 * on `stream`, which is synchronised).  Results are bitwise reproducible for
 * a given shape; shapes differ only by rounding.  PE_EUNSUPPORTED if the
 * shape is not compiled or does not fit (LDS, column count); the previous
 * shape is then kept.  PE_EINVAL while a batch that contains the system is
 * alive (the batch uses the packed arrays).  Not to be called while work
 * using the system is enqueued. */
pe_status pe_system_set_shape(pe_system* sys, int32_t segment, int32_t chunks_per_workgroup, void* stream);

/* Evaluate F and J at P points (Sec. 2: power table, reverse-mode product
 * derivatives, coefficient/exponent multiplication and summation).
 *   x  device [P][2][L][n], read only.
 *   F  device [P][2][L][N], fully overwritten.
 *   J  device [P][2][L][N][n] row-major, fully overwritten (entries that no
 *      monomial touches are written as 0); J == NULL evaluates F only.
 * Summation order is fixed, so results are bitwise reproducible run to run.
 * Enqueues only kernels (no allocation, no host synchronisation); it may be
 * captured in a HIP graph.  PE_EINVAL for NULL x/F with P > 0 or P < 0;
 * PE_EUNSUPPORTED when P * N * (column tiles of J: ceil(n / 2048), or 1 when
 * J == NULL) exceeds 2^31 - 1 (one workgroup each). */
pe_status pe_eval(const pe_system* sys, int32_t P, const double* x, double* F, double* J,
                  void* stream);

/* Terms: the value and the gradient of every monomial, before the sum
 * reduction into F and J (the evaluation and differentiation of products of
 * variables of Sec. 2.2, Tables 1 and 2, with the coefficient, common factor
 * and exponent of Sec. 2.1 and 2.3 applied).
 *   x  device [P][2][L][n], read only.
 *   V  device [P][2][L][M]: V[t] = c_t prod_r x_{i_r}^{d_r} for input monomial
 *      t (the order of the create call's mon_ptr), fully overwritten.
 *   G  device [P][2][L][nnz]: G[o] = the partial derivative of monomial t's
 *      term with respect to its variable i_o, for input occurrence o
 *      (mon_ptr[t] <= o < mon_ptr[t+1], the order of var_idx), fully
 *      overwritten.  May be NULL when nnz = 0.
 * Summing V over a polynomial's monomials gives F, and G scattered by
 * variable gives J, up to rounding.  The first call on a system uploads a
 * map of the input order (allocates and synchronises once, until the system
 * is repacked or destroyed); later calls enqueue kernels only. */
pe_status pe_eval_terms(const pe_system* sys, int32_t P, const double* x, double* V, double* G, void* stream);

/* Adjoint: g = J(x)^H v at P points, without forming J (reverse mode with
 * the seed conj(v_p) per polynomial; the least-squares gradient of Sec. 1's
 * Gauss-Newton setting).
 *   x  device [P][2][L][n];  v  device [P][2][L][N];  g  device [P][2][L][n].
 * The first call with a given P may allocate a per-system workspace (kept
 * until destroy); later calls with P not above it allocate nothing.
 * PE_EUNSUPPORTED for a real system. */
pe_status pe_eval_adjoint(const pe_system* sys, int32_t P, const double* x, const double* v,
                          double* g, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the adjoint above with its
 * partial rows in a static device array of PE_STATIC_SCRATCH_BYTES per GPU
 * (reserved when the library's code is loaded on a GPU, held until the
 * process ends) instead of a per-system workspace.  Allocates nothing and
 * never synchronises, on every call.  Arguments, layouts and results as in
 * pe_eval_adjoint; the GPU is the calling thread's current device.  The
 * workgroups take the same groups of polynomials as pe_eval_adjoint (so the
 * results are bitwise the same) when their partial rows fit in the array,
 * otherwise fewer, larger groups (the same values up to rounding).
 * PE_EUNSUPPORTED when one partial row per point, P * 16 L * n bytes, does
 * not fit.  Every call on a GPU uses that GPU's one array: calls that overlap
 * on a GPU (different streams, or host threads) race and give wrong results;
 * serialise them.  The array needs no clearing (every call writes every
 * partial it reads). */
#define PE_STATIC_SCRATCH_BYTES ((size_t)32 << 20)
pe_status pe_eval_adjoint_static(const pe_system* sys, int32_t P, const double* x, const double* v,
                                 double* g, void* stream);

/* ------------------------------------------------------------------ batches
 * A batch evaluates S independent systems of the same level, each at the
 * same number of points, in persistent launches whose work items
 * (system, polynomial; all points) are taken from a device queue in
 * decreasing order of cost.  Systems with a row of two or more chunks form
 * one launch, the others a second one sized for their LDS; both are queued
 * on the caller's stream behind one counter-reset kernel.  The systems must
 * share the level and the segment length (pe_system_set_shape; PE_EINVAL
 * otherwise) and outlive the batch: while the batch is alive they cannot be
 * repacked (pe_system_set_shape, pe_autotune) or destroyed (PE_EINVAL).
 * Real systems are not batched (PE_EUNSUPPORTED). */
pe_status pe_batch_create(pe_batch** out, int32_t S, const pe_system* const* systems, void* stream);
pe_status pe_batch_destroy(pe_batch* batch);

/* Offsets, in doubles, of system s's blocks inside the packed batch arrays
 * for points_per_system = 1: x_off[s], F_off[s], J_off[s] (each [S+1],
 * host).  For P points per system multiply every offset by P: system s's
 * block is then [P][2][L][n_s] (x), [P][2][L][N_s] (F), [P][2][L][N_s][n_s]
 * (J). */
pe_status pe_batch_layout(const pe_batch* batch, int64_t* x_off, int64_t* F_off, int64_t* J_off);

/* Shape of the persistent launches: info[0] = S, [1] = level, [2] = segment
 * length, [3] = chunks per workgroup of the launch over the systems with
 * multi-chunk rows (2 when compiled for the level and segment and when each
 * of those systems fits in LDS with two slot regions, else 1; 1 when no
 * system has such a row).  A row evaluated in the batch gives bitwise the
 * same F and J as pe_eval on its system with that many chunks per workgroup
 * (a row of one chunk gives the same bits with any). */
pe_status pe_batch_info(const pe_batch* batch, int64_t info[4]);

/* Evaluate every system of the batch at points_per_system points each.
 * x, F, J are device arrays in the packed layout above (J may be NULL).
 * Enqueues kernels only (a counter reset and the persistent launches): no
 * allocation, no host synchronisation, capturable in a HIP graph.  Two calls
 * on the same batch must not overlap (they share the work-queue counters). */
pe_status pe_batch_eval(const pe_batch* batch, int32_t points_per_system, const double* x, double* F,
                        double* J, void* stream);

/* ------------------------------------------------------------------ Newton
 * One Gauss-Newton step at P points (Sec. 4): A = J(x), b = -F(x); modified
 * Gram-Schmidt on the augmented matrix [A b] (Fig. 4, eq. (2)) gives R and
 * y = Q^H b; back substitution solves R dx = y; x += dx.
 *   x_inout    device [P][2][L][n], updated in place.
 *   workspace  device, at least pe_newton_workspace_bytes(sys, P) bytes,
 *              256-byte aligned, owned by the caller.
 *   resid_out  device [P][2] doubles: |F(x)|_2 before the step and
 *              |dx|_inf (leading limbs), or NULL.
 * Systems with fewer than 128 variables are solved by one workgroup per
 * point; larger ones by the column-parallel solve of pe_lstsq below.
 * Requires N >= n (least squares), N <= 4096 for the column-parallel solve
 * and at most 65535 points (PE_EUNSUPPORTED otherwise).  Enqueues kernels only
 * (no allocation, no host synchronisation): capturable in a HIP graph.  A
 * numerically zero pivot (|r_kk| <= n u_L max|r|) gives dx = 0 for that point
 * and resid_out[p][1] = -1; the call itself returns PE_OK. */
size_t pe_newton_workspace_bytes(const pe_system* sys, int32_t P);
pe_status pe_newton_step(const pe_system* sys, int32_t P, double* x_inout, void* workspace,
                         double* resid_out, void* stream);

/* ------------------------------------------------------------------ Newton homotopy
 * The Newton homotopy h(x, t) = f(x) - t c with c = f(z) (Sec. 5.3): at
 * t = 1 the point z is a solution; following the solution path as t goes
 * from 1 to 0 leads to a solution of f(x) = 0.  c is device [P][2][L][N],
 * one vector per point (path); x, workspace and resid_out as in
 * pe_newton_step (the same workspace size; resid_out[p][0] is the norm of
 * the step's right-hand side).  Kernels only: capturable in a HIP graph.
 *
 * pe_homotopy_newton_step: one Gauss-Newton step on h(., t) at fixed t
 *   (A = J(x), b = -(f(x) - t c)).
 * pe_homotopy_predict: the Euler predictor from t to t + dt along the path,
 *   x += dx with J(x) dx = c dt (least squares).
 * pe_homotopy_track: t from 1 to 0 in `steps` equal steps; per step one
 *   predictor and `corrector_iters` Newton steps at the new t (t_k = 1 - k /
 *   steps, computed in double). */
pe_status pe_homotopy_newton_step(const pe_system* sys, int32_t P, double* x_inout, const double* c, double t,
                                  void* workspace, double* resid_out, void* stream);
pe_status pe_homotopy_predict(const pe_system* sys, int32_t P, double* x_inout, const double* c, double dt,
                              void* workspace, double* resid_out, void* stream);
pe_status pe_homotopy_track(const pe_system* sys, int32_t P, double* x_inout, const double* c, int32_t steps,
                            int32_t corrector_iters, void* workspace, double* resid_out, void* stream);

/* The same for every system of a batch, x in the packed batch layout;
 * resid_out is [S][P][2].  Every system is solved by one workgroup per point:
 * n + 1 <= 1024 and the largest pivot column within one workgroup's LDS. */
size_t pe_batch_newton_workspace_bytes(const pe_batch* batch, int32_t P);
pe_status pe_batch_newton_step(const pe_batch* batch, int32_t P, double* x_inout, void* workspace,
                               double* resid_out, void* stream);

/* ------------------------------------------------------------------ least squares
 * Solve A x = b in the least-squares sense by modified Gram-Schmidt on the
 * augmented matrix [A b] = [Q q][R y; 0 z] (Sec. 3, Fig. 4, eq. (2)):
 * right-looking, one workgroup per column; the inner products in rounds of
 * tiled partial sums (eq. (3)); the pivot columns normalised only when
 * needed (delayed normalisation: r_kj = a_k^H a_j / |a_k| and the update
 * divides by |a_k|^2); then the back substitution R x = y in stages of
 * blocks of 256 rows (eq. (4)).
 *   level      1, 2 or 4, or PE_REAL | 1, 2, 4 (real: one component per
 *              array below).  P points (independent problems), 0 <= P <= 65535.
 *   N, n       rows and unknowns: 1 <= n <= N <= 4096.
 *   Ab         device [P][2][L][N][n+1] row-major, column n = b; read only.
 *   x          device [P][2][L][n], the solution (written).
 *   resid_out  device [P][2] or NULL: |b|_2 (leading limbs) and |x|_inf, or
 *              -1 when a pivot was numerically zero (|r_kk| <= n u_L
 *              max |r_ii|; x is then 0).
 *   R_out      device [P][2][L][n][n+1] or NULL: R (upper triangular, real
 *              positive diagonal, zeros below) with y = Q^H b as column n.
 *   Q_out      device [P][2][L][N][n] or NULL: the orthonormal columns.
 *   workspace  device, pe_lstsq_workspace_bytes(level, P, N, n) bytes,
 *              256-byte aligned, caller-owned.
 * Enqueues kernels only (no allocation, no synchronisation): capturable. */
size_t pe_lstsq_workspace_bytes(int32_t level, int32_t P, int32_t N, int32_t n);
pe_status pe_lstsq(int32_t level, int32_t P, int32_t N, int32_t n, const double* Ab, double* x, double* resid_out,
                   double* R_out, double* Q_out, void* workspace, void* stream);

/* ------------------------------------------------------------------ tuning
 * Time the candidate launch shapes for this system at P points on the
 * current device and keep the fastest for later pe_eval calls (this call
 * allocates and synchronises).  The choice is recorded in the plan cache
 * file if one is set. */
pe_status pe_autotune(pe_system* sys, int32_t P, void* stream);

/* Use `path` (NULL to disable) as a plan cache: a text file with one line
 * per tuned system, "<key> | <segment> <chunks_per_workgroup> <microseconds>",
 * the key made of level, n, N, M, nnz, largest k and largest exponent.
 * pe_system_create uses the last matching line; pe_autotune appends. */
pe_status pe_set_plan_cache(const char* path);

#ifdef __cplusplus
}
#endif

#endif /* POLYEVAL_H */
