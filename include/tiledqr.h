/*
 * tiledqr.h -- C ABI of the MI355X tiled QR library.
 *
 * The library factors an m x n FP64 matrix A = QR (m >= n) with the tiled
 * algorithms of Bouwmeester, Jacquelin, Langou and Robert, "Tiled QR
 * factorization algorithms" (2011): the matrix is cut into p x q square tiles
 * of size nb (m = p nb, n = q nb, Remark 1 of Sec. 3.2), an elimination list
 * chosen by a reduction tree (Sec. 3) says which row zeroes which tile, and
 * the six tile kernels of Sec. 2.1 (Table 1) run on the GPU in the
 * dependency order of Algorithms 2 and 3 as soon as their inputs are ready
 * (Sec. 2.3).
 *
 * Conventions for every entry point:
 *   - Matrices are column-major with a leading dimension (LAPACK style).
 *   - "device" pointers are HIP device memory on the current device; "host"
 *     pointers are ordinary host memory.
 *   - stream is a hipStream_t passed as void*; NULL means the default stream.
 *     Device work is enqueued on it asynchronously unless stated otherwise.
 *   - Arguments are checked on the host before any launch; on an error the
 *     call returns a negative tqr_status, enqueues nothing and writes no
 *     output.  The library never aborts and never prints.
 *   - A factor handle may be used on one stream at a time; distinct handles
 *     are independent.
 */
#ifndef TILEDQR_H
#define TILEDQR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TQR_OK = 0,
  TQR_EINVAL = -1,        /* invalid argument (checked on the host)         */
  TQR_ENOMEM = -2,        /* device or host allocation failed               */
  TQR_EHIP = -3,          /* a HIP runtime call failed                      */
  TQR_ENOTCONV = -4,      /* refinement did not reach its tolerance         */
  TQR_EUNSUPPORTED = -5,  /* valid but not implemented (e.g. nb too large)  */
  TQR_EEXEC = -6          /* the device executor stopped (wait time limit)  */
} tqr_status;

/* Reduction trees (Sec. 3.1 and Sec. 3.2).  FLAT and SAMEH_KUCK produce the
 * same elimination list (the tiled Sameh-Kuck algorithm is PLASMA's
 * FlatTree); they differ only in their default kernel family.  ASAP and
 * GRASAP choose their pairs as a unit-weight execution with TT kernels and
 * the Table 1 weights runs: whenever r >= 2 rows of a column are
 * triangularized and not in a running TTQRT, the bottom r / 2 of them are
 * killed by the r / 2 rows right above them.  The pairs are computed on the
 * host before the factorization and form an ordinary elimination list, so
 * the GPU runs them like any other tree. */
typedef enum {
  TQR_TREE_FLAT = 0,
  TQR_TREE_SAMEH_KUCK = 1,
  TQR_TREE_BINARY = 2,
  TQR_TREE_FIBONACCI = 3,
  TQR_TREE_GREEDY = 4,
  TQR_TREE_PLASMA = 5,     /* needs bs in [1, p] (domain size)             */
  TQR_TREE_ASAP = 6,       /* run-time pairing of the tiled model (Sec. 3.2) */
  TQR_TREE_GRASAP = 7,     /* Greedy for the first q - bs columns, ASAP for
                              the last bs (bs in [0, q]; Sec. 3.2)         */
  TQR_TREE_HADRI = 8       /* Hadri et al.'s Semi-Parallel (TS kernels) /
                              Fully-Parallel (TT) trees: PlasmaTree with the
                              domains fixed at rows 1..bs, bs+1..2 bs, ...,
                              so the top domain shrinks (Sec. 4); bs in [1, p] */
} tqr_tree;

/* Kernel family (Sec. 2.1): TT = triangle on top of triangle (Algorithm 3),
 * TS = triangle on top of square (Algorithm 2).  DEFAULT is TS for
 * TQR_TREE_FLAT (PLASMA's algorithm, Proposition 2) and TT otherwise.  With
 * TS on a tree other than FlatTree, a killed row that is itself a pivot of
 * its column is eliminated with TT kernels (a TS kernel needs a square tile
 * under the triangle). */
typedef enum { TQR_KERN_DEFAULT = 0, TQR_KERN_TT = 1, TQR_KERN_TS = 2 } tqr_kernels;

/* Arithmetic of the trailing-update kernels (UNMQR, TSMQR, TTMQR).  Panel
 * kernels (GEQRT, TSQRT, TTQRT: norms, reflector scaling, T factors) are
 * always FP64 and tiles are always stored in FP64.  F32 / BF16 round the
 * update operands to that format, multiply on the matrix cores with FP32
 * accumulation, and subtract the FP32 result from the FP64 tile. */
typedef enum { TQR_UPD_F64 = 0, TQR_UPD_F32 = 1, TQR_UPD_BF16 = 2 } tqr_update_prec;

typedef struct {
  int64_t m, n;     /* matrix size; m % nb == 0, n % nb == 0, m >= n >= nb */
  int32_t nb;       /* tile size: 32, 64, 128 or 256 (512: TQR_EUNSUPPORTED) */
  int32_t ib;       /* inner block size: 0 = default (32); must be 32      */
  int32_t tree;     /* tqr_tree                                            */
  int32_t bs;       /* PlasmaTree / Hadri domain size; GRASAP: ASAP columns
                       k; ignored for other trees                          */
  int32_t kernels;  /* tqr_kernels                                         */
  int32_t upd;      /* tqr_update_prec                                     */
} tqr_opts;

typedef struct tqr_factors tqr_factors;   /* opaque, library-owned */

/* Human-readable name of a status code (static string). */
const char* tiledqr_strerror(int status);

/* Last HIP error code seen by the calling thread (0 if none). */
int tiledqr_last_hip_error(void);

/* ---- factorization --------------------------------------------------- */

/* Factor A (device, m x n, column-major, lda >= m) into *F.
 * Sec. 2 (the tiled algorithm), Sec. 2.3 (execution as soon as possible).
 * A is only read; the handle owns a tile-layout copy holding R, the
 * reflectors V and the compact-WY T factors.  On success *F must later be
 * released with tiledqr_destroy.  The factorization is enqueued on stream;
 * errors of the device executor are reported by tiledqr_sync.  The
 * executor runs the tasks of the DAG as subtasks: update tasks per 64-column
 * slab (128 columns for FP32 / BF16 updates at nb >= 128) and, for nb >= 128,
 * panel tasks per inner block of ib columns, block b waiting only for block b
 * of the previous panel task on the same triangle (environment
 * TQR_PANEL_SPLIT=0 keeps whole panel tasks).  A panel block subtask
 * releases its successors once it has applied its block to the next
 * block's columns and updates the rest of its tiles after that
 * (tiledqr_exec_plan; TQR_EARLY=0 releases them only when it ends).
 * FP32 / BF16 updates at nb >= 128 also stream their reflectors and C1 rows
 * block by block (TQR_STREAM=0 waits for whole predecessors).
 * Errors: TQR_EINVAL (null pointer, m % nb, n % nb, m < n, nb or ib not
 * valid, bs outside [1, p] for PlasmaTree, lda < m), TQR_EUNSUPPORTED
 * (nb = 512: a valid tile size without kernels here), TQR_ENOMEM,
 * TQR_EHIP. */
int tiledqr_factor(const tqr_opts* opts, const double* A, int64_t lda,
                   tqr_factors** F, void* stream);

/* Re-factor a new matrix of the same shape into an existing handle (no
 * allocation, no host planning).  Same errors as tiledqr_factor. */
int tiledqr_refactor(tqr_factors* F, const double* A, int64_t lda, void* stream);

/* Wait for the handle's stream and report a device executor error
 * (TQR_EEXEC) if one occurred in the last factorization. */
int tiledqr_sync(tqr_factors* F);

/* B (device, m x nrhs, ldb >= m) <- Q^T B (trans 'T') or Q B (trans 'N').
 * Q^T applies the reflector sets of the panel tasks in task order, Q in
 * reverse order (Sec. 1).  Errors: TQR_EINVAL (null, ldb < m, nrhs < 0,
 * trans), TQR_EHIP. */
int tiledqr_apply_q(const tqr_factors* F, char trans, double* B, int64_t ldb,
                    int64_t nrhs, void* stream);

/* R (device, n x n, ldr >= n) <- the upper triangular factor (zeros below
 * the diagonal).  Errors: TQR_EINVAL, TQR_EHIP. */
int tiledqr_get_r(const tqr_factors* F, double* R, int64_t ldr, void* stream);

/* Packed factor (device, m x n, ld >= m): the handle's tiles in column-major
 * matrix order, i.e. R, the GEQRT reflectors (strict lower part of each
 * triangularized tile) and the TT / TS reflectors (upper triangle or whole
 * of each zeroed tile), exactly as the kernels left them. */
int tiledqr_get_packed(const tqr_factors* F, double* out, int64_t ld, void* stream);

/* Householder scalars (device, 2 * p * q * nb doubles): tau_geqrt for tile
 * (r, c) (0-based) at ((c * p + r) * nb), then tau of the TT / TS kernel
 * that zeroed tile (i, c) at (p * q * nb + (c * p + i) * nb). */
int tiledqr_get_tau(const tqr_factors* F, double* tau, void* stream);

/* Duration in milliseconds of the last factorization's executor kernel (the
 * persistent launch, or all level launches), measured with HIP events
 * recorded on the handle's stream around the launch.  Synchronizes on the
 * end event.  Errors: TQR_EINVAL (no factorization yet), TQR_EHIP. */
int tiledqr_exec_time(tqr_factors* F, float* ms);

/* Tracing of the persistent executor.  With tracing on, every later
 * factorization records for each executor subtask (in dispatch order) the
 * wall-clock tick when its workgroup took the ticket, when its predecessors
 * were complete, when it finished, and the workgroup index.
 * tiledqr_get_trace writes 10 int64 per subtask to out (host): kind, i, piv,
 * k, j (0-based tiles), column slab (update kinds) or inner block (panel
 * kinds; -1 for a whole panel task), ticket, ready, end, workgroup; out may
 * be NULL to query *n; *ticks_per_second (may be NULL) gets the clock rate.
 * Synchronizes the handle's stream.  Errors: TQR_EINVAL, TQR_ENOMEM, TQR_EHIP. */
int tiledqr_set_trace(tqr_factors* F, int enable);
int tiledqr_get_trace(tqr_factors* F, int64_t* out, int64_t* n, double* ticks_per_second);

/* The executor's subtask table of the factorization (host copy, dispatch
 * order): sub (host, 10 int32 per subtask, may be NULL) = kind, i, piv, k, j
 * (0-based tiles), slab (column slab of an update, inner block of a panel
 * subtask or -1 for a whole panel task), dep_begin, dep_end, sdep, pdep;
 * deps (host, may be NULL) = the predecessor entries of subtask t, in
 * deps[dep_begin .. dep_end - 1]: the low 28 bits hold a predecessor index
 * smaller than t.  Bits 28-29 (stage) say when it is waited for: 0 before
 * the subtask starts; on panel block subtasks that release early, 1 before
 * the look-ahead update of the next block's columns and 2 before the
 * update of the rest of the tiles.  Bit 30 (early) asks for the
 * predecessor's early release instead of its completion.  Low-precision
 * updates at nb >= 128 also follow streamed predecessors block by block
 * while they run: sdep (or -1) is the previous writer of a pair update's C1
 * tile, and pdep (or -1) is the offset in deps of the nb/ib panel block
 * subtasks whose reflectors an update applies (block b of the update waits
 * for panel block b, its early release when bit 30 is set, and for the C1
 * writer's progress past its block b).  These are the edges of the DAG of
 * Sec. 2.3 refined to subtasks and inner blocks.  Errors: TQR_EINVAL. */
int tiledqr_exec_plan(const tqr_factors* F, int32_t* sub, int64_t* nsub, int32_t* deps, int64_t* ndeps);

/* X (device, n x nrhs, ldx >= n) <- R^{-1} X (trans 'N') or R^{-T} X (trans
 * 'T') in place, with the upper triangular factor R held in the handle
 * (Sec. 1: the back substitution of least squares).  Uses and, on the first
 * call after a factorization, forms the same diagonal-tile inverses and
 * coupling tiles as tiledqr_lstsq.  Errors: TQR_EINVAL (null, ldx < n,
 * nrhs < 0, trans), TQR_ENOMEM, TQR_EHIP; a device wait time limit is
 * reported by tiledqr_sync. */
int tiledqr_solve_r(const tqr_factors* F, char trans, double* X, int64_t ldx, int64_t nrhs, void* stream);

/* Release a handle (synchronizes its stream first).  NULL is accepted. */
int tiledqr_destroy(tqr_factors* F);

/* ---- least squares ---------------------------------------------------- */

typedef struct {
  double tol;        /* target backward error (e.g. 1e-12); <= 0: no refinement */
  int32_t max_iter;  /* refinement iterations (default 30 if <= 0)          */
  int32_t method;    /* 0 auto, 1 classical (square) / augmented (tall),
                        2 augmented system, 3 semi-normal corrections only  */
} tqr_refine;

typedef struct {      /* host memory, filled by tiledqr_lstsq */
  int32_t iters;        /* corrections computed (an undone one included)    */
  int32_t converged;
  double backward_err;  /* of the returned X, max over right-hand sides     */
  int32_t semi_normal;  /* semi-normal corrections kept                     */
  int32_t augmented;    /* augmented-system iterations                      */
} tqr_refine_info;

/* X (device, n x nrhs, ldx >= n) <- argmin ||B - A X|| using the factors F
 * (Sec. 1: x = R^{-1} (Q^T b)(1:n)).  When r != NULL and r->tol > 0 the
 * solution is refined with FP64 residuals computed on the GPU against the
 * original matrix A0 (device, m x n, lda >= m), which the caller keeps
 * unchanged until the call returns.  Square systems refine
 * x <- x + R^{-1} c with c = Q^T (b - A0 x) (classical, method 1) or
 * c = R^{-T} A0^T (b - A0 x) (semi-normal, method 3: R^{-T} A0^T equals Q^T
 * for A0 = QR and costs two products with A0 and one more triangular solve
 * instead of an application of Q^T); method 0 takes semi-normal steps
 * while each one cuts the backward error at least fourfold, then (after
 * undoing a step that raised it) classical ones.  Tall systems take the
 * same semi-normal steps (method 0 or 3), and with method 0 (or methods 1
 * and 2) then refine the augmented system [I A0; A0^T 0][r; x] = [b; 0]
 * (Bjorck 1967) with the same factors: residuals f = b - r - A0 x and
 * g = -A0^T r in FP64, corrections h = R^{-T} g, d = Q^T f,
 * dx = R^{-1}(d(1:n) - h), dr = Q [h; d(n+1:m)].  method 2 selects the
 * augmented system for square systems too.  The
 * backward error of x (r = b - A0 x, norms 2-norms per column, ||A0||_F) is
 * ||r|| / (||A0|| ||x|| + ||b||) for square systems; for tall systems the
 * smaller of that and ||A0^T r|| / (||A0|| ||r||).
 * Synchronizes the stream once per refinement iteration.  Returns
 * TQR_ENOTCONV (info filled, X holding the iterate with the smallest
 * backward error seen, info->backward_err its error) if the tolerance is not
 * reached within max_iter or the error stops halving over three
 * iterations.  The triangular solves use the inverses of the q diagonal
 * tiles of R and the coupling tiles -inv(R_ii) R_{i,i+1}, formed on the
 * first solve after a factorization (2 q nb^2 doubles of device memory
 * owned by the handle); an R^{-T} solve also keeps the tiles of R^T and
 * the transposed counterparts (q^2 + 2 q tiles of nb^2 doubles).
 * Environment TQR_TRSM_SUBST=1 solves by substitution inside the diagonal
 * tiles instead.  Errors: TQR_EINVAL, TQR_ENOMEM, TQR_EHIP, TQR_EEXEC. */
int tiledqr_lstsq(const tqr_factors* F, const double* A0, int64_t lda,
                  const double* B, int64_t ldb, int64_t nrhs,
                  double* X, int64_t ldx, const tqr_refine* r,
                  tqr_refine_info* info, void* stream);

/* Factorization and Q^T B in one executor launch: re-factor A (device,
 * lda >= m) into the existing handle F and overwrite B (device, m x nrhs,
 * ldb >= m, 1 <= nrhs <= 16) with Q^T B (Sec. 1), the application of each
 * reflector set to B running as soon as the panel task that produces it
 * (Sec. 2.3) has finished, in the same persistent launch.  The handle's
 * executor time (tiledqr_exec_time) then covers both.  The joint plan is
 * built on the first call and kept in the handle.
 * Errors: TQR_EINVAL, TQR_ENOMEM, TQR_EHIP. */
int tiledqr_refactor_qtb(tqr_factors* F, const double* A, int64_t lda, double* B, int64_t ldb,
                         int64_t nrhs, void* stream);

/* tiledqr_lstsq with Q^T B already computed (QtB: device, ldq >= n, its
 * first n rows used, e.g. from tiledqr_refactor_qtb); B (the original
 * right-hand sides) and A0 serve the refinement as in tiledqr_lstsq.
 * Errors: as tiledqr_lstsq, and TQR_EINVAL for QtB == NULL or ldq < n. */
int tiledqr_lstsq_qtb(const tqr_factors* F, const double* A0, int64_t lda,
                      const double* B, int64_t ldb, const double* QtB, int64_t ldq, int64_t nrhs,
                      double* X, int64_t ldx, const tqr_refine* r,
                      tqr_refine_info* info, void* stream);

/* ---- double complex -------------------------------------------------------- */

/* The tiled QR of a double-complex matrix (the paper's ZGEQRT family, Sec. 5)
 * with the same trees, kernel families and task graphs as tiledqr_factor,
 * on tiles of nb = 32 (other tile sizes: TQR_EUNSUPPORTED).  Each kernel uses
 * LAPACK's complex elementary reflector H = I - tau u u^H with a real beta;
 * R = H_l^H ... H_1^H A, so R's diagonal is real.
 *
 * tiledqr_zfactor: A is device memory, m x n column-major with interleaved
 *   real and imaginary parts, lda in complex elements (>= m); opts as for
 *   tiledqr_factor with nb = 32 and upd = TQR_UPD_F64 (else TQR_EINVAL).
 *   Copies A into tiles and enqueues the factorization on stream; the
 *   handle owns its storage.  Errors: TQR_EINVAL, TQR_EUNSUPPORTED,
 *   TQR_ENOMEM, TQR_EHIP.
 * tiledqr_zrefactor: factors a new matrix of the same shape and options
 *   into the handle's storage (no allocation or planning).  Errors:
 *   TQR_EINVAL, TQR_EHIP.
 * tiledqr_zapply_q: B <- Q^H B (trans 'C') or Q B ('N'); B is device
 *   memory, m x nrhs column-major complex (ldb >= m complex elements,
 *   1 <= nrhs <= 4096).  Enqueued on stream (a device scratch copy of B in
 *   row tiles is allocated and freed on it).  Errors: TQR_EINVAL,
 *   TQR_ENOMEM, TQR_EHIP.
 * tiledqr_zsolve_r: X <- R^{-1} X (X: device, n x nrhs complex, ldx >= n);
 *   back substitution, n <= 4096 (else TQR_EINVAL).  Enqueued on stream.
 * tiledqr_zlstsq: X (n x nrhs, ldx) = argmin ||B - A X||_2 column by column,
 *   X = R^{-1} (Q^H B)(1:n) (Sec. 1); B (m x nrhs, ldb) is not modified.
 *   n <= 4096.  Enqueued on stream (scratch allocated and freed on it).
 *   Errors: TQR_EINVAL, TQR_ENOMEM, TQR_EHIP.
 * tiledqr_zget_packed: the factored matrix in A's layout (R on and above
 *   the diagonal of the top n rows, the reflectors elsewhere, as LAPACK's
 *   zgeqrf would leave a tile), to device memory out (ld >= m, complex
 *   elements).  Enqueued on stream.
 * tiledqr_zget_tau: the tau of the GEQRT sets (taug) and of the TS/TT sets
 *   (taup), 32 complex values per tile, tile (r, c) at (c p + r) 32 complex
 *   elements; device memory, p q 32 complex elements each.
 * tiledqr_zsync: waits for the factorization; TQR_EEXEC if its executor
 *   stopped on a wait time limit.
 * tiledqr_zdestroy: releases the handle (NULL accepted). */
typedef struct tqr_zfactors tqr_zfactors;
int tiledqr_zfactor(const tqr_opts* opts, const double* A, int64_t lda, tqr_zfactors** F, void* stream);
int tiledqr_zrefactor(tqr_zfactors* F, const double* A, int64_t lda, void* stream);
int tiledqr_zapply_q(tqr_zfactors* F, char trans, double* B, int64_t ldb, int64_t nrhs, void* stream);
int tiledqr_zsolve_r(const tqr_zfactors* F, double* X, int64_t ldx, int64_t nrhs, void* stream);
int tiledqr_zlstsq(tqr_zfactors* F, const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx,
                   void* stream);
int tiledqr_zget_packed(const tqr_zfactors* F, double* out, int64_t ld, void* stream);
int tiledqr_zget_tau(const tqr_zfactors* F, double* taug, double* taup, void* stream);
int tiledqr_zsync(tqr_zfactors* F);
int tiledqr_zdestroy(tqr_zfactors* F);

/* ---- batched ------------------------------------------------------------ */

/* Many independent factorizations in one persistent launch.  The task
 * graphs of all problems (each built as for tiledqr_factor, Sec. 2.3) are
 * merged into one dispatch order by the executor's priority (each problem's
 * subtasks by bottom level, the longest remaining path), and one
 * persistent kernel walks them; a problem's subtasks run on its own tiles.
 * Tile sizes 32 and 64 may be mixed; all problems share upd.  The run (pack
 * every problem into tiles, reset the executor, execute) is captured once
 * as a HIP graph and replayed by every tiledqr_batch_run.
 *
 * tiledqr_batch_create: opts and lda are host arrays of nprob entries (lda
 *   is the leading dimension each run will use).  Allocates every problem's
 *   storage.  Errors: TQR_EINVAL (as tiledqr_factor per problem, differing
 *   upd), TQR_EUNSUPPORTED (nb other than 32 or 64), TQR_ENOMEM, TQR_EHIP.
 * tiledqr_batch_run: A is a host array of nprob device pointers (read by the
 *   device when the run executes; the matrices must stay unchanged until
 *   then).  Enqueued on stream.  Errors: TQR_EINVAL, TQR_EHIP.
 * tiledqr_batch_sync: waits for the last run; TQR_EEXEC if its executor
 *   stopped on a wait time limit.
 * tiledqr_batch_time: milliseconds of the last run's graph (HIP events).
 * tiledqr_batch_set_trace: with tracing on, every later run records, for
 *   each subtask of the merged dispatch order, the same four ticks as
 *   tiledqr_set_trace (ticket, ready, end, workgroup).  The captured graph
 *   is not rebuilt: the kernel reads the trace buffer's address from device
 *   memory at its start.  Synchronizes the last run's stream.  Errors:
 *   TQR_EINVAL, TQR_ENOMEM, TQR_EHIP.
 * tiledqr_batch_get_trace: 11 int64 per subtask to out (host): the ten
 *   columns of tiledqr_get_trace (tiles of the subtask's own problem), then
 *   the problem index; out may be NULL to query *n; *ticks_per_second (may
 *   be NULL) gets the clock rate.  Synchronizes the last run's stream.
 *   Errors: TQR_EINVAL (tracing off), TQR_EHIP.
 * tiledqr_batch_get: borrowed handle of problem i (valid until the batch is
 *   destroyed; not to be passed to tiledqr_destroy), usable with
 *   tiledqr_apply_q, tiledqr_get_r, tiledqr_lstsq and the other handle
 *   entry points once the run is complete.
 * tiledqr_batch_destroy: releases everything (NULL accepted). */
typedef struct tqr_batch tqr_batch;
int tiledqr_batch_create(int32_t nprob, const tqr_opts* opts, const int64_t* lda, tqr_batch** batch);
int tiledqr_batch_run(tqr_batch* batch, const double* const* A, void* stream);
int tiledqr_batch_sync(tqr_batch* batch);
int tiledqr_batch_time(tqr_batch* batch, float* ms);
int tiledqr_batch_set_trace(tqr_batch* batch, int enable);
int tiledqr_batch_get_trace(tqr_batch* batch, int64_t* out, int64_t* n, double* ticks_per_second);
int tiledqr_batch_get(tqr_batch* batch, int32_t i, tqr_factors** F);
int tiledqr_batch_destroy(tqr_batch* batch);

/* One-shot batched factorization: create a batch, run it once, wait, and
 * hand each problem's handle to the caller in F[i] (an ordinary handle,
 * released with tiledqr_destroy).  opts, A, lda and F are host arrays of
 * nprob entries; A[i] are device pointers.  Synchronizes the stream.
 * Errors: as tiledqr_batch_create / tiledqr_batch_run / tiledqr_batch_sync. */
int tiledqr_factor_batched(int32_t nprob, const tqr_opts* opts,
                           const double* const* A, const int64_t* lda,
                           tqr_factors** F, void* stream);

/* ---- makespan model of the tree / tile-size selector ---------------------- */

/* The paper chooses PlasmaTree's domain size by exhaustive search over
 * measured runs (Sec. 4); the library adds a learned model of the makespan
 * so that a tree, domain size and tile size can be picked without timing
 * every candidate.  The model is a multilayer perceptron 13 -> 64 -> 64 -> 1
 * (ReLU hidden units) mapping a candidate's features to log(makespan),
 * trained with mean squared error and Adam, all in FP32 on the GPU.
 *
 * Features (13 floats per sample): log2 p, log2 q, log2 nb; one-hot of the
 * algorithm (TS-FlatTree, TT-FlatTree, BinaryTree, Fibonacci, Greedy,
 * PlasmaTree); log2 BS for PlasmaTree, else 0; one-hot of the update
 * precision (FP64, FP32, BF16).
 *
 * Parameters: one FP32 array of tiledqr_mlp_nparam() = 5121 floats,
 * row-major, y = relu(relu(x W1 + b1) W2 + b2) W3 + b3 with W1 [13][64] at
 * 0, b1 at 832, W2 [64][64] at 896, b2 at 4992, W3 [64] at 5056, b3 at 5120.
 * All arrays are device memory; calls are enqueued on stream.
 *
 * tiledqr_mlp_forward: y[i] = model(X[13 i .. 13 i + 12]) for i < n.
 * tiledqr_mlp_loss_grad: *loss = mean_i (y_i - t_i)^2 and grad (nparam
 *   floats) its gradient; loss may be NULL.  Deterministic (fixed reduction
 *   order).  Allocates a stream-ordered workspace of about 20 KB per 64
 *   samples.
 * tiledqr_mlp_adam: one Adam step (Kingma and Ba, with bias correction; step
 *   counts from 1): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
 *   params -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).
 * Errors: TQR_EINVAL (null pointers, n < 0, bad hyper-parameters),
 *   TQR_ENOMEM, TQR_EHIP. */
int tiledqr_mlp_nparam(void);
int tiledqr_mlp_forward(const float* params, const float* X, int64_t n, float* y, void* stream);
int tiledqr_mlp_loss_grad(const float* params, const float* X, const float* t, int64_t n,
                          float* grad, float* loss, void* stream);
int tiledqr_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t nparam,
                     float lr, float beta1, float beta2, float eps, int32_t step, void* stream);

/* tiledqr_mlp_loss_grad without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight training
 * loops, harnesses that forbid hipMalloc).  Same arguments, kernels and
 * results as tiledqr_mlp_loss_grad (bit-identical), but the per-chunk partial
 * gradients live in a fixed array of the library's device memory instead of
 * a stream-ordered workspace: one array per GPU (5.2 MB, held until the
 * process ends), located on the first call on each device (make that first
 * call before any graph capture).  n is limited to
 * tiledqr_mlp_noalloc_max_samples() = 16384 samples.  Every call on one GPU
 * uses that GPU's single array, so calls that overlap on one GPU (on
 * different streams or threads without ordering) race and give wrong
 * gradients; calls ordered on one stream are safe.  No part of the array
 * needs clearing: each call writes every entry it reads.
 * Errors: TQR_EINVAL (as tiledqr_mlp_loss_grad, and n above the limit),
 * TQR_EHIP. */
int tiledqr_mlp_loss_grad_noalloc(const float* params, const float* X, const float* t, int64_t n,
                                  float* grad, float* loss, void* stream);
int tiledqr_mlp_noalloc_max_samples(void);

/* ---- host-only planning (no GPU needed) -------------------------------- */

/* Elimination list of a tree (Sec. 3): triples (i, piv, k), 1-based, in the
 * library's emission order (column by column, except Greedy, which follows
 * the rounds of Algorithm 4).  out (host, 3 * nelim int32) may be NULL to
 * query *nelim.  Errors: TQR_EINVAL (p < q, q < 1, bad tree or bs). */
int tiledqr_elim_list(int32_t p, int32_t q, int32_t tree, int32_t bs,
                      int32_t* out, int64_t* nelim);

/* Kernel tasks of the list (Algorithms 2 and 3) with their unbounded-
 * processor ASAP schedule in units of nb^3/3 flops (Table 1 weights,
 * Sec. 2.3).  tasks (host, 7 * ntasks int32) = (kind, i, piv, k, j, start,
 * finish) with kind 0 GEQRT, 1 UNMQR, 2 TSQRT, 3 TSMQR, 4 TTQRT, 5 TTMQR and
 * 0 in unused fields; may be NULL to query *ntasks.  *cp = critical path.
 * Errors: TQR_EINVAL. */
int tiledqr_schedule(int32_t p, int32_t q, int32_t tree, int32_t bs, int32_t kernels,
                     int32_t* tasks, int64_t* ntasks, int64_t* cp);

/* Predecessors of each task of tiledqr_schedule in CSR form: ptr (host,
 * ntasks + 1 int64) and idx (host, ptr[ntasks] int32, ascending per task).
 * idx may be NULL to query the sizes (ptr still filled). */
int tiledqr_task_preds(int32_t p, int32_t q, int32_t tree, int32_t bs, int32_t kernels,
                       int64_t* ptr, int32_t* idx);

#ifdef __cplusplus
}
#endif

#endif /* TILEDQR_H */
