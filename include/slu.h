/*
 * slu.h -- C ABI of the MI355X blocked sparse LU with structure-aware
 * irregular blocking.
 *
 * The library factors a sparse matrix A (n x n, CSR) as
 *     A[perm][:, perm] = L U,
 * L unit lower triangular, U upper triangular, no row exchanges, and solves
 * A X = B and A^T X = B with the factors.  The work splits into
 *
 *   analyze (host, once per pattern): validation, fill-reducing ordering,
 *     symbolic fill to a structurally symmetric pattern S (Section 1 phase 2,
 *     Section 4.2), the diagonal block pointer (Algorithm 2), the sampled
 *     irregular blocking (Algorithm 3) or a regular blocking (Section 3.2),
 *     and the block storage plan and per-level task lists for the numeric
 *     phase;
 *   factor (device, HIP kernels for gfx950): value scatter, then for every
 *     level i of the right-looking blocked LU (Algorithm 1, Section 2.2):
 *     GETRF of the diagonal block, GESSM / TSTRF of the U and L panels and
 *     SSSSM Schur updates of the trailing blocks;
 *   solve (device): forward/backward block sweeps with L and U (or U^T, L^T).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Return value: SLU_OK (0) on success, a negative SLU_ERR_* code for an
 *   invalid argument or a runtime failure, SLU_ZERO_PIVOT (> 0) when the
 *   numeric factorization met a zero or non-finite pivot (slu_get_info then
 *   reports the permuted column).  slu_error_string() names every code.
 * - Host arrays are read during the call only; the caller keeps ownership.
 * - Device pointers are plain HIP device addresses on the current device.
 *   The library never allocates device memory: the caller provides one
 *   workspace (slu_workspace_size / slu_bind_workspace) and every value,
 *   right-hand side and solution buffer.
 * - Streams: every device entry point takes a hipStream_t (as void*, NULL
 *   meaning the legacy default stream) and is stream-ordered.  slu_factor
 *   waits for its stream once at the end to read the pivot status.
 * - A handle is not thread-safe; distinct handles are independent.
 * - Index types: rowptr int64, column / row indices int32, n < 2^31.
 */
#ifndef SLU_H
#define SLU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct slu_handle slu_handle;

/* return codes */
#define SLU_OK 0
#define SLU_ZERO_PIVOT 1          /* zero / non-finite pivot; see slu_info   */
#define SLU_NOT_CONVERGED 2       /* refinement stopped above its tolerance  */
#define SLU_ERR_ARG (-1)          /* null pointer, bad option, bad size      */
#define SLU_ERR_ROWPTR (-2)       /* rowptr[0] != 0 or not monotone          */
#define SLU_ERR_COLIDX (-3)       /* a column index outside [0, n)           */
#define SLU_ERR_UNSORTED (-4)     /* columns of a row unsorted or duplicated */
#define SLU_ERR_PERM (-5)         /* user permutation is not a permutation  */
#define SLU_ERR_STATE (-6)        /* call out of order (e.g. no workspace)   */
#define SLU_ERR_WORKSPACE (-7)    /* workspace too small or misaligned       */
#define SLU_ERR_HIP (-8)          /* a HIP runtime call failed               */
#define SLU_ERR_NOMEM (-9)        /* host allocation failed                  */
#define SLU_ERR_NOT_FACTORED (-10) /* solve before a successful factor       */
#define SLU_ERR_LIMIT (-11)       /* sizes beyond the library's index types  */

/* orderings (the paper names none; Section 1 / Section 2.1 require one) */
#define SLU_ORDER_NATURAL 0       /* identity                                */
#define SLU_ORDER_GRID_ND 1       /* geometric nested dissection of a grid   */
#define SLU_ORDER_USER 2          /* caller's permutation (new -> old)       */
#define SLU_ORDER_GRAPH_ND 3      /* graph nested dissection of A + A^T: dense
                                     vertices last, connected components
                                     apart, level-structure cuts with minimum
                                     vertex-cover separators; deterministic  */

/* schedules of the level loop */
#define SLU_SCHEDULE_WAVES 0      /* levels of equal height in the block
                                     dependency tree run together           */
#define SLU_SCHEDULE_LEVELS 1     /* strict level order of Algorithm 1       */

/* blockings */
#define SLU_BLOCK_IRREGULAR 0     /* Algorithm 3 on the sampled Algorithm 2 curve */
#define SLU_BLOCK_REGULAR 1       /* fixed block size (Section 3.2)          */

typedef struct {
    /* Algorithm 3 parameters: sample_points = 1000, step = 2, max_num = 3
     * (Section 4.3); advance = 1 follows the printed loop, advance = step
     * the "points separated by a step interval" wording. */
    int32_t sample_points;
    int32_t step;
    int32_t max_num;
    int32_t advance;
    int32_t blocking;             /* SLU_BLOCK_IRREGULAR | SLU_BLOCK_REGULAR */
    int32_t regular_block;        /* block size for SLU_BLOCK_REGULAR        */
    int32_t ordering;             /* SLU_ORDER_*                             */
    int32_t grid_dims[3];         /* nx, ny, nz for SLU_ORDER_GRID_ND; grid
                                     point x + nx*(y + ny*z) is row/column i */
    int32_t schedule;             /* SLU_SCHEDULE_WAVES | SLU_SCHEDULE_LEVELS */
    const int32_t *user_perm;     /* n entries for SLU_ORDER_USER; copied    */
} slu_options;

typedef struct {
    int64_t n;
    int64_t nnz_a;                /* entries of A                            */
    int64_t nnz_s;                /* entries of S = nnz(L + U), both triangles */
    int64_t nblocks;              /* p: blocks per dimension == levels       */
    int64_t nonempty_blocks;      /* non-empty blocks of S, both triangles   */
    int64_t ssssm_tasks;          /* (k, j) Schur-update tasks over all levels */
    double flops;                 /* sum_k (c_k - 1) + 2 (c_k - 1)^2 on S    */
    double flops_getrf;           /* part of flops inside diagonal blocks    */
    double flops_panel;           /* part in the GESSM / TSTRF panel solves  */
    double flops_ssssm;           /* part in the SSSSM Schur updates         */
    double stored_flops;          /* flops the kernels execute incl. padding */
    int64_t slab_bytes;           /* factor value storage inside the workspace */
    int64_t workspace_bytes;      /* total device workspace                  */
    int64_t zero_pivot_col;       /* permuted column of a failed pivot, or -1 */
    int32_t factored;             /* 1 after a successful slu_factor         */
    int32_t max_block;            /* largest block size                      */
    int32_t precision;            /* SLU_PRECISION_* of the next slu_factor  */
    int32_t waves;                /* launches of GETRF / panel solves        */
    int32_t rounds;               /* launches of the Schur updates           */
    int32_t reserved;
} slu_info;

/* Fill *opt with the defaults: irregular blocking, 1000 / 2 / 3 / 1,
 * natural ordering, dependency-tree waves. */
void slu_default_options(slu_options *opt);

/* Analyze the pattern of A (host).  rowptr: int64[n+1]; colidx: int32[nnz],
 * strictly increasing inside each row.  A structurally missing diagonal
 * entry is added to S as an explicit zero.  On success *out receives a new
 * handle owned by the caller (release with slu_free).  Errors:
 * SLU_ERR_ARG, SLU_ERR_ROWPTR, SLU_ERR_COLIDX, SLU_ERR_UNSORTED,
 * SLU_ERR_PERM, SLU_ERR_NOMEM, SLU_ERR_LIMIT. */
int slu_analyze(int64_t n, const int64_t *rowptr, const int32_t *colidx,
                const slu_options *opt, slu_handle **out);

/* Analysis of nsys independent systems factored together: system q has
 * order n[q] and its CSR pattern rowptr[q], colidx[q] (host arrays, copied).
 * The systems are stacked block-diagonally in the given order (rows and
 * columns of system q follow those of systems 0..q-1); each keeps its own
 * ordering (SLU_ORDER_GRID_ND with grid_dims[3q..3q+2], SLU_ORDER_GRAPH_ND or
 * SLU_ORDER_NATURAL)
 * and its own blocking (Algorithm 3 on its own block pointer, or regular
 * blocks restarting at every system).  Levels of different systems with
 * equal dependency height share the wave launches, and the Schur updates of
 * a wave run in rounds with disjoint targets, so one factorization covers
 * the whole batch.  Values, right-hand sides and solutions are the
 * systems' arrays concatenated in the same order. */
int slu_analyze_batch(int64_t nsys, const int64_t *n, const int64_t *const *rowptr,
                      const int32_t *const *colidx, const int32_t *grid_dims,
                      const slu_options *opt, slu_handle **out);

/* Host threads used by the parallel parts of slu_analyze and
 * slu_analyze_batch (the Schur-update offset tables, level by level): 0
 * (the default) takes the hardware's count, at most 16.  The analysis is the
 * same for every count.  Process-wide; SLU_ERR_ARG for a negative count. */
int slu_set_host_threads(int threads);

/* Device bytes the handle needs (factor storage + structure + scratch). */
int slu_workspace_size(const slu_handle *h, size_t *bytes);

/* Bind a caller-owned device buffer of at least slu_workspace_size bytes,
 * 256-byte aligned, and upload the structure into it on `stream`.  The
 * buffer must outlive the handle's device calls. */
int slu_bind_workspace(slu_handle *h, void *device_ptr, size_t bytes, void *stream);

/* Numeric factorization.  values: device float64[nnz_a] in the CSR order
 * given to slu_analyze.  Runs the value scatter and the level loop of
 * Algorithm 1 (GETRF, GESSM, TSTRF, SSSSM) on `stream`, then waits for the
 * stream.  Returns SLU_OK or SLU_ZERO_PIVOT. */
int slu_factor(slu_handle *h, const double *values, void *stream);

/* Solve A X = B (the system Ax = b that the factorization serves, Section 1):
 * X = perm^T U^{-1} L^{-1} perm B by a forward sweep with L and a backward
 * sweep with U over the same blocks and waves as the factorization.
 * B, X: device float64, column-major n x nrhs with leading dimension
 * ld >= n; X may alias B; both stay the caller's.  Requires a successful
 * factor (SLU_ERR_NOT_FACTORED otherwise); SLU_ERR_ARG for a null pointer
 * with nrhs > 0, nrhs < 0 or ld < n.  Stream-ordered, no host wait. */
int slu_solve(slu_handle *h, const double *B, double *X, int64_t nrhs, int64_t ld,
              void *stream);

/* Solve A^T X = B with the same factors (Section 1's Ax = b for the
 * transposed matrix, A^T = perm^T U^T L^T perm): a forward sweep with U^T,
 * then a backward sweep with L^T.  Arguments, ownership and errors as in
 * slu_solve. */
int slu_solve_transpose(slu_handle *h, const double *B, double *X, int64_t nrhs,
                        int64_t ld, void *stream);

/* Allocation-free solve, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): slu_solve (transpose = 0) or slu_solve_transpose
 * (transpose = 1) with the permuted work block held in a fixed device array
 * of the library (32 MiB per device, reserved for the life of the process)
 * instead of the workspace.  The call makes no device allocation or free.
 * Every call on one device shares that array: calls that overlap on one
 * device (two streams, two threads) race and must be serialized by the
 * caller.  Nothing in the array needs to start at zero.  Limits: n <= 4 Mi
 * rows (SLU_ERR_LIMIT otherwise, returned before any device call); the
 * right-hand sides are taken min(16, 4 Mi / n) at a time.  Other arguments,
 * ownership and errors as in slu_solve. */
int slu_solve_noalloc(slu_handle *h, const double *B, double *X, int64_t nrhs, int64_t ld,
                      int transpose, void *stream);

/* Normwise backward error per right-hand side on the device,
 * eta_c = ||b_c - op(A) x_c||_inf / (||op(A)||_inf ||x_c||_inf + ||b_c||_inf),
 * op(A) = A or A^T.  values: device float64[nnz_a]; eta: host double[nrhs].
 * Synchronizes `stream`. */
int slu_backward_error(slu_handle *h, const double *values, const double *B,
                       const double *X, int64_t nrhs, int64_t ld, int transpose,
                       double *eta, void *stream);

/* Gradient of a scalar loss with respect to the values of A for x = A^{-1} b
 * (the adjoint of the solve; no section of the paper defines it): with
 * G = A^{-T} (dloss/dx) (from slu_solve_transpose) and the solution X,
 * grad_values[q] = -sum_c G[i, c] X[j, c] for entry q = (i, j) of A in the
 * CSR order given to slu_analyze, i.e. -G X^T restricted to A's pattern.
 * G, X: device float64 column-major n x nrhs with leading dimension ld;
 * grad_values: device float64[nnz_a], overwritten.  Needs only the analysis
 * and a bound workspace. */
int slu_value_gradient(slu_handle *h, const double *G, const double *X, int64_t nrhs,
                       int64_t ld, double *grad_values, void *stream);

/* Graph mode (enable = 1): the first slu_factor afterwards captures its
 * whole launch sequence into a HIP graph on a stream of the library's own
 * (default priority); later calls copy the values into the workspace and
 * replay the graph on the caller's stream, saving the host-side launches.
 * The graph holds kernels only; it is recaptured after slu_set_precision or
 * slu_bind_workspace.  Per-kernel timing (slu_set_profiling) uses the
 * launch-by-launch path.  enable = 0 releases the graph. */
int slu_set_graph(slu_handle *h, int enable);

/* GETRF launch shape of the waves that do not take the tiled GETRF
 * (slu_set_getrf_tiled; Algorithm 1, the factorization of the diagonal
 * blocks).  A wave whose chunked diagonal blocks (more than 128 rows) include
 * one with trailing work of at least min_work, counted as the sum over its
 * column chunks of (coupled rows)^2, is factored chunk by chunk in two
 * launches per chunk: the panel of every block by one workgroup each, then
 * the trailing update spread over the GPU one 16 x 16 tile per workgroup.
 * Other waves take one launch with one workgroup per block.  Both give the
 * same factors bit for bit; the split pays on large dense diagonal blocks.
 * Default 2e5; 0 splits every wave with a chunked block.  A captured graph
 * (slu_set_graph) is released and recaptured.  SLU_ERR_ARG for a negative
 * or NaN min_work. */
int slu_set_getrf_split(slu_handle *h, double min_work);

/* Tiled GETRF (Algorithm 1's factorization of the diagonal blocks, with the
 * GESSM / TSTRF / SSSSM steps inside the block applied tile by tile): a wave
 * whose largest diagonal block has at least min_rows rows factors its blocks
 * densely in 16 x 16 tiles, one launch per tile step spread over the GPU one
 * tile per workgroup: the panel tiles are solved by products with the
 * inverted diagonal tile of the previous step and every trailing tile is
 * updated with FP64 MFMA; the diagonal tile of the step is then factored and
 * inverted.  Default 1 (every wave); min_rows = 0 keeps the one-launch or
 * split chunked GETRF (slu_set_getrf_split) on every wave whose chunks fit
 * the LDS (waves with larger dense blocks take the tiled GETRF regardless).  Same factors as the other GETRF paths up to rounding.  A captured
 * graph is released and recaptured.  SLU_ERR_ARG for a negative min_rows. */
int slu_set_getrf_tiled(slu_handle *h, int min_rows);

/* Tile edge of the tiled GETRF: 32 (the default; four waves per tile, the
 * step's 32 x 32 diagonal block factored as 2 x 2 blocks of 16) or 16 (one
 * wave per tile).  Same factors up to rounding; a captured graph is
 * recaptured.  SLU_ERR_ARG for another value. */
int slu_set_getrf_tile(slu_handle *h, int tile);

/* One row of the autotuner's table: a launch-shape setting and its median
 * factor time. */
typedef struct {
    int32_t getrf_tiled_rows;     /* slu_set_getrf_tiled                     */
    int32_t getrf_tile;           /* slu_set_getrf_tile                      */
    int32_t panel_blocked;        /* slu_set_panel_blocked                   */
    int32_t graph;                /* slu_set_graph                           */
    int32_t lookahead;            /* slu_set_lookahead                       */
    double ms;                    /* median of reps factors (HIP events)     */
} slu_tune_entry;

/* Autotuner of the launch shapes for this handle's pattern and values (the
 * batch of independent systems included): factors with each of a fixed set
 * of settings (tiled GETRF with 32- or 16-row tiles or the chunked GETRF,
 * blocked or tile-wise panel solves, launch by launch or graph replay, with
 * or without lookahead), one
 * warm-up and reps timed factors each on `stream`, keeps the setting with the
 * smallest median and factors once more with it, so the handle ends factored
 * and set to the choice.  table (capacity entries, may be NULL when capacity
 * is 0) receives the settings tried in order, *count (may be NULL) their
 * number.  values: device float64[nnz_a] as in slu_factor.  Returns SLU_OK,
 * SLU_ZERO_PIVOT, SLU_ERR_ARG (reps < 1, negative capacity, null pointers),
 * SLU_ERR_STATE (no workspace) or SLU_ERR_HIP.  Synchronizes `stream`. */
int slu_autotune(slu_handle *h, const double *values, int reps, slu_tune_entry *table, int capacity, int *count,
                 void *stream);

/* Tiled diagonal solves: in slu_solve, slu_solve_transpose and the solves
 * inside slu_solve_refined, a wave whose largest diagonal block has at least
 * min_rows rows (default 64; 0: never), whose blocks were factored by the
 * 32 x 32 tiled GETRF and are either dense (S fills at least half of every
 * block's lower triangle) or all at least min_sparse_rows rows (default 64;
 * 0: dense blocks only) solves its diagonal blocks tile by tile across the
 * GPU with the inverted diagonal tiles the factorization kept (one launch per
 * pair of 32-row tiles, b / 64 steps rounded up); otherwise, and for waves
 * with a block of 16 rows or fewer, one workgroup per block walks its column
 * chunks (b / 16 dependent steps).  Same results up to rounding.  SLU_ERR_ARG
 * for a negative argument. */
int slu_set_solve_tiled(slu_handle *h, int min_rows, int min_sparse_rows);

/* Lookahead of the Schur updates (Algorithm 1's SSSSM; the level order of
 * Section 3.2): with enable = 1 the updates of a wave whose
 * levels have pairwise disjoint targets (one launch round) are split by
 * target.  The updates of the next wave's diagonal blocks run on the
 * factor's stream as before; on a second stream of the library's own
 * (default priority) follow the updates of the next wave's panels (which its
 * panel solve waits for) and then those that reach only later waves (which
 * the next updates on the factor's stream wait for), while the next wave
 * factors its diagonal blocks and solves its panels.  Waves of several rounds run
 * their updates on the factor's stream.  max_groups (a multiple of 8; 0: one
 * workgroup per tile) caps the workgroups of a deferred launch, which then
 * walk its tiles, so that they leave room on every CU for the factor's
 * stream.  Default: disabled (512 workgroups once enabled).  The deferred
 * updates share the CUs and HBM with the next wave's latency-bound launches
 * (whose waves raise their issue priority above them), so lookahead pays
 * where those updates are large next to the diagonal work (a chain of dense
 * blocks) and can cost elsewhere; the autotuner (slu_autotune) tries both.
 * Every target receives its updates in the same order as without lookahead,
 * so the factors are the same bit for bit.  Not used under per-kernel timing
 * (slu_set_profiling).  A captured graph is recaptured (the graph then
 * holds both streams' launches).  SLU_ERR_ARG unless enable is 0 or 1 and
 * max_groups a non-negative multiple of 8. */
int slu_set_lookahead(slu_handle *h, int enable, int max_groups);

/* Blocked panel solves (Algorithm 1's GESSM / TSTRF, the panels of block
 * column i times the inverse of the coupled triangle of L_ii or U_ii): with
 * enable = 1 (the default), levels whose coupled triangles have at least 256
 * columns solve their panels in 128-column blocks across the GPU (the
 * blocks' inverted diagonal triangles, then one launch per block of
 * right-looking updates on FP64 MFMA); 0 keeps the tile-by-tile solve, one
 * workgroup per 16 or 32 panel rows, on every level.  Same results up to
 * rounding.  A captured graph is recaptured.  SLU_ERR_ARG unless 0 or 1. */
int slu_set_panel_blocked(slu_handle *h, int enable);

/* Factorization precision.  SLU_PRECISION_FP64: every step in FP64.
 * SLU_PRECISION_FP32: the Schur updates (Algorithm 1's SSSSM, nearly all of
 * the flops) take their operands rounded to FP32 and accumulate in FP32 on
 * the FP32 matrix cores; the diagonal factorizations (with their pivot
 * divisions), the panel solves and the storage stay FP64.  The factors are
 * then accurate to about FP32 precision; slu_solve_refined recovers an FP64
 * backward error by iterative refinement.  Applies to later slu_factor calls. */
#define SLU_PRECISION_FP64 0
#define SLU_PRECISION_FP32 1
int slu_set_precision(slu_handle *h, int precision);

/* Solve A X = B with FP64 iterative refinement on the current factors:
 * X <- solve(B); then repeatedly R = B - A X (FP64, original A), eta as in
 * slu_backward_error, stop when every eta <= tol, when no eta fell by half
 * (stagnation) or after maxit corrections; otherwise X += solve(R).
 * values: device float64[nnz_a] (the A that was factored); B, X as in
 * slu_solve (X must not alias B).  iters (host, may be NULL): corrections
 * applied; eta (host double[nrhs], may be NULL): final backward errors.
 * Returns SLU_OK, SLU_NOT_CONVERGED when some eta stays above tol, or an
 * error code.  Synchronizes `stream` once per iteration. */
int slu_solve_refined(slu_handle *h, const double *values, const double *B, double *X,
                      int64_t nrhs, int64_t ld, double tol, int maxit, int *iters,
                      double *eta, void *stream);

int slu_get_info(const slu_handle *h, slu_info *info);

/* Kernel classes for per-kernel timing. */
#define SLU_KERNEL_SCATTER 0      /* value scatter (and slab clear)          */
#define SLU_KERNEL_GETRF 1
#define SLU_KERNEL_PANEL 2        /* GESSM + TSTRF                           */
#define SLU_KERNEL_SSSSM 3
#define SLU_NUM_KERNELS 4

/* Enable (1) or disable (0) per-kernel timing.  While enabled, slu_factor
 * records a HIP event pair on its stream around every run of consecutive
 * launches of one kernel class (a wave's GETRF steps, its panel solves, its
 * Schur-update rounds) and adds the elapsed times and launch counts per
 * class; slu_get_kernel_times reports the totals of the last slu_factor.
 * Timing adds event work between the runs; it does not change results. */
int slu_set_profiling(slu_handle *h, int enable);
/* ms[SLU_NUM_KERNELS]: summed kernel milliseconds of the last factor;
 * launches[SLU_NUM_KERNELS]: launch counts. */
int slu_get_kernel_times(const slu_handle *h, double *ms, int64_t *launches);

/* Structure accessors (host arrays sized as stated; for parity checks). */
int slu_get_perm(const slu_handle *h, int32_t *perm);            /* n       */
int slu_get_blockptr(const slu_handle *h, int64_t *blockptr);    /* n + 1 (Algorithm 2) */
int slu_get_blocking(const slu_handle *h, int64_t *ptr);         /* p + 1 (Algorithm 3) */
/* Lower triangle of S in CSC with the diagonal first in every column:
 * colptr int64[n+1], rowidx int32[colptr[n]]. */
int slu_get_pattern(const slu_handle *h, int64_t *colptr, int32_t *rowidx);

/* Copy the factors to host arrays laid out on the lower CSC of S
 * (slu_get_pattern): for entry e of column k at row r > k,
 * lval[e] = L(r, k) and uval[e] = U(k, r); lval[colptr[k]] = U(k, k) and
 * uval[colptr[k]] = U(k, k).  Synchronizes `stream`. */
int slu_get_factors(const slu_handle *h, double *lval, double *uval, void *stream);

const char *slu_error_string(int code);

/* After a call returned SLU_ERR_HIP: the hipError_t code of the HIP call
 * that failed (the most recent such failure on the calling thread; 0 if
 * none), and its description from the HIP runtime. */
int slu_last_hip_error(void);
const char *slu_hip_error_string(int hip_code);
void slu_free(slu_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* SLU_H */
