/*
 * hec.h -- C ABI of the MI355X (gfx950) HEC / ILU(k) / level-schedule Krylov library.
 *
 * The operations follow Yang, Liu, Chen, "Development of Krylov and AMG linear
 * solvers for large-scale sparse matrices on GPUs": the HEC matrix format
 * (Sec. 2.1), SpMV (Sec. 2.2, Alg. 1, Eq. (2)), ILU(k) (Sec. 2.4, Eq. (7)-(10),
 * Alg. 2), the level-schedule triangular solver (Sec. 2.6, Eq. (11), Alg. 3) and
 * the Krylov solvers (Sec. 2.7, Alg. 4 for BiCGSTAB; restarted GMRES).
 *
 * Conventions for every entry point:
 *  - Host CSR input: Ap[n+1] row starts (Ap[0] == 0, non-decreasing), Aj[nnz]
 *    column indices strictly ascending within each row and in [0, n), Ax[nnz]
 *    values (double). These host arrays are borrowed for the duration of the
 *    call only. Indices are 0-based int32.
 *  - Vectors (x, b, y) are caller-owned DEVICE pointers of n elements of the
 *    stated dtype (for example torch tensors' data_ptr()). `stream` is a
 *    hipStream_t (NULL = the default stream).
 *  - Handles own their device memory until the matching *_destroy call. It is
 *    allocated and released in stream order on the stream of the call that
 *    created it (hipMallocAsync/hipFreeAsync, or the hooks of
 *    hec_set_allocator); destroy a handle before that stream.
 *  - Every call returns an hec_status; on failure a message for the calling
 *    thread is available from hec_last_error(). No C++ exception crosses the
 *    ABI. Arguments are validated on the host before any device work.
 *  - hec_spmv and trsv_levels are asynchronous on `stream`. Setup calls and the
 *    solvers synchronise `stream` before they return.
 *  - Distinct handles may be used from different threads. One handle must not be
 *    used concurrently on two streams.
 */
#ifndef HEC_H
#define HEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HEC_OK = 0,
    HEC_ERR_INVALID_ARG = 1,   /* bad size, pointer, CSR structure, missing diagonal, ... */
    HEC_ERR_NOMEM = 2,         /* device or host allocation failed */
    HEC_ERR_ZERO_PIVOT = 3,    /* ILU met an exactly zero pivot */
    HEC_ERR_BREAKDOWN = 4,     /* BiCGSTAB rho or (r0,v) became 0 (or non-finite) */
    HEC_ERR_NOT_CONVERGED = 5, /* maxit reached; x holds the last iterate */
    HEC_ERR_HIP = 6,           /* a HIP runtime call failed */
    HEC_ERR_TIMEOUT = 7        /* a device-side wait of a triangular solve gave up (hec_set_spin_limit) */
} hec_status;

typedef enum { HEC_F64 = 0, HEC_F32 = 1 } hec_dtype;

/* hec_from_csr / ilu_factor flag: also keep an FP32 copy of the values
 * (rounded to nearest even from the FP64 values) for mixed precision. */
#define HEC_KEEP_F32 1u

/* hec_from_csr flag: keep the remainder as COO (the row of every entry, entries in
 * row order) and multiply it entry-parallel: with the ELL part this is the HYB
 * format of Sec. 2.1 (ELL + COO) instead of HEC (ELL + CSR). */
#define HEC_COO_REMAINDER 2u

/* hec_from_csr ell_width: choose the ELL width by the HYB rule, the largest K such
 * that at least max(4096, n/3) rows hold K or more entries (0 when none). */
#define HEC_WIDTH_HYB (-2)

/* trsv_levels `which` */
#define HEC_LOWER 1u
#define HEC_UPPER 2u
#define HEC_LU 3u

typedef struct hec_matrix_s *hec_matrix; /* device HEC matrix A */
typedef struct hec_ilu_s *hec_ilu;       /* device in-place L\U factor on pattern S_k */
typedef struct hec_levels_s *hec_levels; /* lower + upper level schedules and level-ordered factor copies */

typedef struct {
    int32_t restart;    /* GMRES restart length m (ignored by BiCGSTAB); >= 1 */
    int32_t maxit;      /* max Arnoldi steps (GMRES) or loop passes (BiCGSTAB); >= 0 */
    int32_t precision;  /* 0: all FP64. 1: mixed -- FP32 matrix/factor/basis storage in the
                           inner solve, FP64 residual, dots, rotations and refinement */
    int32_t x0_zero;    /* 1: start from x = 0 (x's contents ignored); 0: x holds x0 */
    double rtol;        /* stop when ||b - A x|| / ||b|| <= rtol (FP64 true residual) */
    double ir_rtol;     /* mixed: outer refinement target (<= 0: use rtol) */
    double inner_rtol;  /* mixed: relative residual reduction asked of each inner solve */
} hec_solve_opts;

typedef struct {
    int32_t status;      /* same value as returned */
    int32_t iterations;  /* Arnoldi steps (GMRES, summed over refinement steps) or loop passes */
    int32_t restarts;    /* GMRES cycles started after the first; BiCGSTAB restarts */
    int32_t ir_steps;    /* mixed: outer refinement steps */
    double rel_res_true; /* ||b - A x|| / ||b|| in FP64 at return */
    double rel_res_est;  /* the solver's own recurrence estimate at its last step */
    double seconds;      /* wall time of the call */
} hec_solve_info;

/* ---------------------------------------------------------------- device memory */

/* Allocation hooks: alloc returns `bytes` of device memory usable in stream order
 * on `stream` (a hipStream_t), or NULL on failure (the call then fails with
 * NOMEM); free releases a block that alloc returned, in stream order on the
 * stream it was allocated on. ctx is passed through. */
typedef void *(*hec_alloc_fn)(void *ctx, size_t bytes, void *stream);
typedef void (*hec_free_fn)(void *ctx, void *ptr, size_t bytes, void *stream);

/* Every device buffer the library allocates from now on (handles, solver
 * workspaces, batch contexts, AMG levels) comes from `alloc` and goes back
 * through `free` -- for example a binding to a framework's caching allocator.
 * alloc == free == NULL restores the default (hipMallocAsync / hipFreeAsync on
 * the device's default memory pool). A buffer is always released by the
 * allocator that made it, so the hooks may change while handles exist; they
 * must stay callable until every buffer they made is released, and may be
 * called from any thread that calls the library. INVALID_ARG if only one of the
 * two is NULL. Pinned host memory (flags, staging) does not go through them. */
hec_status hec_set_allocator(hec_alloc_fn alloc, hec_free_fn free, void *ctx);

/* Device bytes currently held by the given handles (any may be NULL), the
 * matrix's cached solver workspace included: what a caller, for example a
 * serving loop admitting requests by memory, should count for one system. */
hec_status hec_footprint(hec_matrix A, hec_ilu M, hec_levels lv, int64_t *bytes);

/* ---------------------------------------------------------------- HEC matrix */

/* Sec. 2.1: build the HEC form of A on the device -- an ELL slab of width K
 * stored column-major with leading dimension ld = n rounded up to 256 (entry s
 * of row i at s*ld + i), plus the rest of every longer row in CSR (rem_ptr[n+1],
 * rem_col, rem_val). K = ell_width if ell_width >= 0, the HYB rule for
 * HEC_WIDTH_HYB, else min(20, longest row) (the paper's recommended boundary),
 * never above the longest row; the first K entries of each row go to the slab.
 * Empty slab slots of row i hold (col i, value 0); rows n..ld-1 hold (col 0,
 * value 0). ell_width = 0 gives plain CSR; ell_width >= the longest row gives
 * plain ELL (Sec. 2.1's ELL format). flags: HEC_KEEP_F32, HEC_COO_REMAINDER
 * (HYB). The matrix owns scratch for the COO remainder's partial sums, so SpMVs
 * with one HYB matrix must not overlap in time on different streams. Errors:
 * INVALID_ARG for n < 0, null pointers, unknown flags or a malformed CSR
 * (unsorted or duplicate columns, out-of-range index). */
hec_status hec_from_csr(int32_t n, const int32_t *Ap, const int32_t *Aj, const double *Ax,
                        int32_t ell_width, uint32_t flags, void *stream, hec_matrix *out);

/* Sizes of a HEC matrix (any output pointer may be NULL). */
hec_status hec_info(hec_matrix A, int32_t *n, int32_t *K, int32_t *ld, int64_t *nnz,
                    int64_t *nnz_rem);

/* Copy the HEC arrays to caller host buffers of sizes K*ld, K*ld, n+1, nnz_rem,
 * nnz_rem (for bit-exact checks). ell_val32/rem_val32 may be NULL; when given,
 * the matrix must have been built with HEC_KEEP_F32. */
hec_status hec_export(hec_matrix A, int32_t *ell_col, double *ell_val, int32_t *rem_ptr,
                      int32_t *rem_col, double *rem_val, float *ell_val32, float *rem_val32);

/* Eq. (2) with Alg. 1's order (ELL part, then the CSR remainder):
 * y = alpha*A*x + beta*y. vals selects the FP64 values or the FP32 copy; xt and
 * yt the vector dtypes. Accumulation is in FP64 when the values are FP64, in
 * FP32 otherwise. beta == 0 does not read y. x and y must not overlap. */
hec_status hec_spmv(hec_matrix A, hec_dtype vals, double alpha, const void *x, hec_dtype xt,
                    double beta, void *y, hec_dtype yt, void *stream);

hec_status hec_destroy(hec_matrix A);

/* ---------------------------------------------------------------- ILU(k) */

/* Sec. 2.4, Eq. (7)-(10), Alg. 2: incomplete LU with level of fill k. The
 * pattern S_k = {(i,j): level <= k} is built on the host (Eq. (9)-(10)); the
 * numeric elimination (for each row i and each p < i in S_k ascending:
 * a_ip /= a_pp; a_ij -= a_ip a_pj for (i,j) in S_k) runs on the device, rows
 * grouped by the Eq. (11) levels of L. L (unit diagonal implied) and U share one
 * array, as in the paper. Every row must store its diagonal (INVALID_ARG
 * otherwise); an exactly zero pivot gives ZERO_PIVOT. flags: HEC_KEEP_F32. */
hec_status ilu_factor(int32_t n, const int32_t *Ap, const int32_t *Aj, const double *Ax, int32_t k,
                      uint32_t flags, void *stream, hec_ilu *out);

/* Sec. 2.5, restricted additive Schwarz inside one device ("inner RAS"): the rows
 * are cut into nblocks contiguous blocks of ceil(n / nblocks) rows (the sequence
 * partition); each block is extended by `overlap` layers of graph neighbours (the
 * rows reached through A's stored entries, layer by layer); the entries of A outside
 * every extended block's diagonal submatrix are dropped, and ILU(k) (as in
 * ilu_factor) is computed for each extended block. The extended blocks are stacked
 * into one block-diagonal factor of sum(|extended block|) rows, each block's rows in
 * ascending system order. Its preconditioner solve (trsv_levels with HEC_LU, and the
 * solvers) solves every block independently -- no dependency crosses a block, so the
 * blocks run in parallel -- and keeps from each block only the rows it owns
 * ("restricted"). nblocks = 1, overlap = 0 equals ilu_factor. Fewer dependencies
 * mean shorter level chains and more solver iterations (Sec. 2.5, Tables 4-5).
 * INVALID_ARG for nblocks < 1, overlap < 0, a missing diagonal, or stacked sizes
 * beyond 32-bit indices. Not usable with gmres_solve_batched. */
hec_status ilu_factor_ras(int32_t n, const int32_t *Ap, const int32_t *Aj, const double *Ax, int32_t k,
                          int32_t nblocks, int32_t overlap, uint32_t flags, void *stream, hec_ilu *out);

/* n: rows of the factor (the stacked extended blocks for a RAS factor); nnz: its entries. */
hec_status ilu_info(hec_ilu M, int32_t *n, int64_t *nnz);

/* The block structure of a factor: system size, number of blocks, first stacked row
 * of each block (nblocks+1), the system row of each stacked row (factor rows), and the
 * stacked row that owns each system row (n_sys). A factor from ilu_factor reports one
 * block and identity maps. Any pointer may be NULL. */
hec_status ilu_ras_export(hec_ilu M, int32_t *n_sys, int32_t *nblocks, int32_t *block_start, int32_t *ext_row,
                          int32_t *own);

/* Copy the factor to host CSR buffers (n+1, nnz, nnz): L strictly below the
 * diagonal, U on and above it, columns ascending (stacked rows for a RAS factor). */
hec_status ilu_export(hec_ilu M, int32_t *LUp, int32_t *LUj, double *LUx);

hec_status ilu_destroy(hec_ilu M);

/* ---------------------------------------------------------------- level schedule */

/* Sec. 2.6, Eq. (11), Alg. 3: levels of L (l(i) = 1 + max l(j) over stored
 * j < i, starting from 0) and, mirrored, of U (j > i, rows from n-1 down),
 * stored 0-based; rows grouped by level in ascending row order (level_ptr +
 * perm). Also builds the level-ordered device copies of L and U used by
 * trsv_levels (allocated and filled on `stream`, which is synchronised). The
 * schedule refers to M's pattern and values at call time. */
hec_status level_schedule(hec_ilu M, void *stream, hec_levels *out);

hec_status levels_info(hec_levels lv, int32_t *n, int32_t *nlev_lower, int32_t *nlev_upper);

/* *grid = 1 when lv carries wavefront plans for both triangles (see
 * hec_set_trsv_grid), else 0 (level-blocked plans). */
hec_status levels_grid(hec_levels lv, int32_t *grid);

/* Copy the schedules to host buffers: ptr arrays of nlev+1, perm arrays of n. */
hec_status levels_export(hec_levels lv, int32_t *lower_ptr, int32_t *lower_perm,
                         int32_t *upper_ptr, int32_t *upper_perm);

hec_status levels_destroy(hec_levels lv);

/* Triangular solves wait on the device for the rows they depend on (rows of other
 * workgroups, and slots and progress inside their own). Every such wait gives up
 * after `polls` polls: the launch then ends normally with invalid outputs and
 * records the failure in the schedule, which the solvers report as
 * HEC_ERR_TIMEOUT, and levels_check for trsv_levels. A correct schedule used on
 * one stream at a time never gets there (a wait lasts at most one solve); the
 * limit exists so that a broken plan, a lost store or misuse ends in a status
 * instead of a hung device, and so that tests can force that path. polls < 0
 * restores the default (2^26); 0 gives up at the first unready poll. Applies to
 * launches made after the call, from any thread. */
hec_status hec_set_spin_limit(int64_t polls);

/* Chooses the triangular-solve kernel of the schedules level_schedule builds after
 * the call (from any thread). With enable = 1 (the default), a factor on a
 * natural-order 3D or 2D grid (detected from A) whose strict triangles hold only
 * the grid neighbours behind each row, as ILU(0) of a 7-point or 5-point stencil
 * does (Sec. 2.6: the level of a row is then the sum of its coordinates, Eq. (11)),
 * gets wavefront plans for both triangles: tiles of 8 x 8 grid columns (3D) or
 * 64 x 1 (2D, at least 16 columns across), one wavefront each, whose lanes step
 * through the levels together, passing results between neighbouring lanes through
 * LDS. Every other factor, and every factor
 * with enable = 0, gets the level-blocked plans. A schedule keeps the kind it was
 * built with (levels_grid reports it). Both kernels perform each row's
 * subtractions (fused multiply-adds) and may differ in rounding only where their
 * order differs. INVALID_ARG unless enable is 0 or 1. */
hec_status hec_set_trsv_grid(int32_t enable);

/* Synchronises `stream`, then reports (and clears) a wait of lv's triangular
 * solves that gave up since the last check: HEC_ERR_TIMEOUT, else HEC_OK. The
 * solvers make this check themselves before they return. */
hec_status levels_check(hec_levels lv, void *stream);

/* Alg. 3: solve with the factor level by level. A RAS factor (ilu_factor_ras)
 * accepts only HEC_LU, with b and x of the system size. which = HEC_LOWER: x = L^{-1} b
 * (unit diagonal); HEC_UPPER: x = U^{-1} b; HEC_LU: x = U^{-1} L^{-1} b (the
 * preconditioner solve M x = b of Eq. (7)-(8)). prec selects FP64 factor and
 * vectors, or the FP32 factor copy (ilu_factor with HEC_KEEP_F32) with FP32
 * vectors. b and x are device vectors of n elements and must not overlap.
 * Every level's rows are solved in parallel; a row starts as soon as the rows it
 * depends on are done. */
hec_status trsv_levels(hec_ilu M, hec_levels lv, uint32_t which, hec_dtype prec, const void *b,
                       void *x, void *stream);

/* ---------------------------------------------------------------- Krylov solvers */

/* Restarted GMRES(m) (Sec. 2.7), right-preconditioned with M = LU:
 * x = x0 + Z y, Z = M^{-1} applied to the Arnoldi vectors, minimising
 * ||b - A x|| over each cycle; classical Gram-Schmidt applied twice (with an FP64
 * basis the second application to each vector is delayed into the next step,
 * which equals the plain form in exact arithmetic), Givens rotations,
 * convergence decided by the FP64 true residual. precision = 1: iterative refinement in FP64 around inner
 * GMRES solves that use the FP32 copies of A and of the factor (both handles
 * built with HEC_KEEP_F32) and an FP32 Krylov basis. A refinement that stalls
 * (eight steps in a row without halving the smallest true residual so far)
 * gives up and the solve starts again in FP64 from x = 0; the iterations of
 * both phases are counted. b, x: device FP64.
 * ||b|| == 0 gives x = 0, OK, 0 iterations. On NOT_CONVERGED x holds the last
 * iterate. `info` may be NULL. */
hec_status gmres_solve(hec_matrix A, hec_ilu M, hec_levels lv, const double *b, double *x,
                       const hec_solve_opts *opts, hec_solve_info *info, void *stream);

/* Largest system (rows) gmres_solve_noalloc accepts. */
#define HEC_NOALLOC_MAX_N 16384

/* For callers that cannot allocate device memory (code under HIP graph capture
 * elsewhere on the stream, tight serving loops, harnesses that forbid hipMalloc):
 * gmres_solve with the same arguments, method, kernels and results (FP64 only:
 * precision must be 0; restart in [1, 32]; n <= HEC_NOALLOC_MAX_N, INVALID_ARG
 * otherwise), whose workspace -- Krylov basis, preconditioned basis, scalars,
 * partial sums, flags: about 9.7 MB -- is a static device array of the library
 * instead of memory allocated at the first solve. It calls no hipMalloc, hipFree,
 * host-pinned allocation or allocator hook, and creates no events (whole cycles
 * are queued; the scalars are read by plain copies). Each GPU holds one copy of
 * the array for the life of the process, and every call on that GPU shares it:
 * calls that overlap in time on one GPU (other threads, other streams) race and
 * must be serialised by the caller. The handles must already exist (their setup
 * calls allocate). */
hec_status gmres_solve_noalloc(hec_matrix A, hec_ilu M, hec_levels lv, const double *b, double *x,
                               const hec_solve_opts *opts, hec_solve_info *info, void *stream);

/* Preconditioned BiCGSTAB exactly as Alg. 4 (shadow residual r0 = b - A x0),
 * "||s|| / ||r|| satisfied" read as <= rtol * ||b||; rho == 0 or (r0, v) == 0 is
 * a breakdown. When a cycle stops (breakdown, or a recurrence residual below rtol
 * that the FP64 true residual does not confirm), the method restarts from the
 * current x with a new shadow residual, at most 3 times (info->restarts counts
 * them); BREAKDOWN is returned when the last cycle broke down and x is not
 * converged, x then holding the last iterate. FP64 only (precision must be 0). */
hec_status bicgstab_solve(hec_matrix A, hec_ilu M, hec_levels lv, const double *b, double *x,
                          const hec_solve_opts *opts, hec_solve_info *info, void *stream);

/* ---------------------------------------------------------------- batched small systems */

/* Largest system (rows) a batch context accepts: the two triangular solves of a
 * system keep their vectors in the workgroup's LDS. level_schedule prepares the
 * level-ordered factor copies the batched solver reads for every n up to this. */
#define HEC_BATCH_MAX_N 8192

typedef struct hec_batch_s *hec_batch; /* context for gmres_solve_batched */

/* Creates a context for batches of up to `capacity` systems of at most `max_n`
 * rows each, solved by GMRES(restart). It owns pinned staging memory, device
 * descriptor and result arrays, and a workspace of (2*restart + 3) * max_n
 * doubles per system (allocated here, so solving allocates nothing).
 * use_graph != 0: the first solve records descriptor upload, kernel and result
 * download into a hipGraph, and every later solve replays it. */
hec_status batch_create(int32_t capacity, int32_t restart, int32_t max_n, int32_t use_graph, hec_batch *out);

hec_status batch_destroy(hec_batch B);

/* Restarted GMRES (Sec. 2.7) on `count` independent systems A[i] x[i] = b[i] in
 * one persistent launch, one workgroup per system (the serving path for small
 * systems). Same method as gmres_solve on each system: right preconditioning with
 * the factor M[i] (Eq. (7)-(8)) applied level by level in the order of lv[i]
 * (Eq. (11), Alg. 3), classical Gram-Schmidt twice, Givens rotations, restarts
 * from the FP64 true residual; precision 1 runs each cycle on the FP32 value
 * copies (HEC_KEEP_F32 on A[i] and M[i]) with FP64 vectors and refinement.
 * The Krylov basis is FP64 in both precisions. A[i], M[i], lv[i] are handles of
 * the same size n_i <= max_n; b[i], x[i] are device FP64 vectors of n_i
 * elements; opts->restart must equal the context's. A system's result does not
 * depend on the rest of the batch. `stream`: the call waits for work already
 * queued on it, runs on the context's own stream and synchronises before it
 * returns; calls on one context must not overlap. info (may be NULL): `count`
 * entries. Returns HEC_ERR_TIMEOUT if a wait in a system's triangular solve gave
 * up (hec_set_spin_limit), else HEC_ERR_NOT_CONVERGED if any system did not
 * converge (its info entry says which). */
hec_status gmres_solve_batched(hec_batch B, int32_t count, const hec_matrix *A, const hec_ilu *M,
                               const hec_levels *lv, const double *const *b, double *const *x,
                               const hec_solve_opts *opts, hec_solve_info *info, void *stream);

/* Preconditioned conjugate gradient (Sec. 2.7 lists CG among the Krylov solvers;
 * the steps are the textbook ones): r = b - A x, z = M^{-1} r, p = z, then per
 * iteration q = A p, alpha = (r, z) / (p, q), x += alpha p, r -= alpha q,
 * z = M^{-1} r, p = z + beta p with beta = (r, z)_new / (r, z)_old. For symmetric
 * positive definite A and M = LU (an ILU(k) of an SPD M-matrix with a symmetric
 * pattern, e.g. a 3D Poisson matrix). Stops when ||r|| / ||b|| <= rtol by the
 * recurrence, confirmed by the FP64 true residual (restarting from x, at most 3
 * times, if it disagrees). (r, z) <= 0 or (p, A p) <= 0 is HEC_ERR_BREAKDOWN.
 * FP64 only (precision must be 0); opts->restart is ignored. */
hec_status cg_solve(hec_matrix A, hec_ilu M, hec_levels lv, const double *b, double *x,
                    const hec_solve_opts *opts, hec_solve_info *info, void *stream);

/* ---------------------------------------------------------------- AMG (Sec. 2.8) */

typedef struct hec_amg_s *hec_amg;

typedef struct {
    double theta;        /* strength threshold: j strongly influences i when
                            -a_ij >= theta * max_{k != i} (-a_ik) > 0; in (0, 1] (0.25) */
    int32_t max_levels;  /* most levels, the finest included; 1..32 (8, as Sec. 3.3) */
    int32_t coarse_size; /* a level of at most this many rows is the coarsest; 1..4096 (64) */
    double omega;        /* damped Jacobi weight; in (0, 2) (2/3) */
    int32_t nu1, nu2;    /* pre- and post-smoothing sweeps; 0..64 (3 and 3, as Sec. 3.3) */
    int32_t use_graph;   /* 1: record one cycle into a HIP graph at the first solve and replay it;
                            0: launch the kernels of every cycle (1) */
    int32_t smoother;    /* 0: damped Jacobi (omega); 1: Chebyshev polynomial, nu1 / nu2 its degree (0) */
    double cheb_lower;   /* Chebyshev: the smoothed interval of D^{-1} A's spectrum is
                            [cheb_lower * lmax, lmax], lmax = max_i sum_j |a_ij| / |a_ii|; in (0, 1) (0.3) */
} hec_amg_opts;

/* Sec. 2.8: AMG setup on the host for the n x n CSR matrix (Ap, Aj, Ax: host
 * arrays, 0-based, columns ascending; read during the call only). Per level:
 * Ruge-Stueben strength and coarsening (first pass: largest measure first,
 * smallest index on ties; points with no strong connection are F), direct
 * interpolation P (the paper's RSD), R = P^T, A_{l+1} = R A_l P (Galerkin), until
 * a level has at most coarse_size rows, max_levels levels exist or no coarsening
 * happens; the coarsest level keeps its dense inverse. Every operator is uploaded
 * as a HEC matrix; the handle owns them and the per-level vectors. opts may be
 * NULL (the defaults above). Errors: INVALID_ARG for a malformed CSR, n == 0 or
 * bad options; ZERO_PIVOT for a zero or missing diagonal on any level or a
 * singular coarsest level. */
hec_status amg_setup(int32_t n, const int32_t *Ap, const int32_t *Aj, const double *Ax, const hec_amg_opts *opts,
                     void *stream, hec_amg *out);

/* Hierarchy sizes: nlevels, and per level (arrays of nlevels entries, any may be
 * NULL) the rows, the nonzeros of A_l and of P_l (0 on the coarsest level). */
hec_status amg_info(hec_amg H, int32_t *nlevels, int32_t *n, int64_t *nnz, int64_t *nnz_p);

/* Host copies of level `level`: its C/F splitting (n_l entries, 1 = C; not
 * written on the coarsest level), A_l (n_l + 1, nnz, nnz) and P_l (n_l + 1,
 * nnz_p, nnz_p; columns are coarse indices, C points numbered in row order).
 * Any pointer may be NULL. */
hec_status amg_export_level(hec_amg H, int32_t level, int8_t *cf, int32_t *Ap, int32_t *Aj, double *Ax,
                            int32_t *Pp, int32_t *Pj, double *Px);

/* Alg. 5: x = 0, then V-cycles (nu1 smoothing sweeps, residual restricted by
 * R, coarse correction from zero, prolongated by P and added, nu2 sweeps; the
 * coarsest level solved with its inverse) until ||b - A x|| <= rtol ||b|| in FP64
 * or maxit cycles. Smoothers (Sec. 2.8): damped Jacobi, x += omega D^{-1} (b - A x)
 * per sweep; or Chebyshev, the Chebyshev semi-iteration on D^{-1} A over
 * [cheb_lower * lmax, lmax] (error multiplied by T_nu((theta - t) / delta) /
 * T_nu(theta / delta), theta and delta the interval's midpoint and half-width), one
 * product with A per sweep. b, x: device FP64 vectors of n elements, not overlapping. The
 * calls of one handle must not overlap in time (its per-level vectors are
 * shared). The handle runs the cycles on a stream of its own, ordered after the
 * caller's stream on entry and before it on return. Returns NOT_CONVERGED after maxit cycles (x holds the last iterate),
 * BREAKDOWN on a non-finite residual; info (may be NULL) gets the cycles and the
 * final relative residual. */
hec_status amg_solve(hec_amg H, const double *b, double *x, int32_t maxit, double rtol, void *stream,
                     hec_solve_info *info);

hec_status amg_destroy(hec_amg H);

/* Message of the last failed call on this thread ("" if none). */
const char *hec_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HEC_H */
