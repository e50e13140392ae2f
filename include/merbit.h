/*
 * merbit.h -- C ABI of libmerbit.so: merge-path SpMV with bit-field lane
 * descriptors (MERBIT) for AMD Instinct MI355X (gfx950, 64-lane wavefronts).
 *
 * Method: "MERBIT: A GPU-Based SpMV Method for Iterative Workloads".
 *   - Sec. 3.3 / Algorithm 1   merge path over row ends and nonzeros, diagonal search
 *   - Sec. 4.1                 TILE storage format and its one-time generation
 *   - Sec. 4.2                 fused SpMV kernel (staged products, descriptor scan,
 *                              wavefront segmented sum, long-row fast tiles,
 *                              block-buffered commit, dual output buffers)
 *   - Sec. 4.3                 the segment length sigma
 *   - Sec. 5.5.1               PageRank by the power method
 *
 * Conventions shared by every entry point
 *   - Matrix A is n_rows x n_cols in CSR: row_ptr int32[n_rows + 1] (row_ptr[0] = 0,
 *     non-decreasing, row_ptr[n_rows] = nnz), col_ind int32[nnz] in [0, n_cols),
 *     values float or double [nnz].  Column order inside a row is free.
 *   - All array pointers are DEVICE pointers (hipMalloc or equivalent) unless
 *     the comment says "host".  The caller owns them and keeps them alive.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous on that stream unless the comment says otherwise.
 *   - Every call returns a merbit_status; nothing aborts or throws across the
 *     ABI.  On failure merbit_last_error() returns a message (thread local).
 *   - Limits: n_rows + nnz < 2^31 (32-bit coordinates and the tile_y mark bit).
 *   - A plan is not safe for concurrent use from two streams or threads.
 */
#ifndef MERBIT_H
#define MERBIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MERBIT_OK = 0,
    MERBIT_EINVAL = -1,       /* bad argument or failed CSR validation        */
    MERBIT_ENOMEM = -2,       /* device (or host) allocation failed            */
    MERBIT_EHIP = -3,         /* a HIP runtime call failed (message has it)    */
    MERBIT_EUNSUPPORTED = -4, /* dtype / sigma / block size not built          */
    MERBIT_NOT_CONVERGED = 1, /* an iterative driver reached max_iter above tol */
    MERBIT_BREAKDOWN = 2      /* BiCGSTAB: rho = (r^, r) became 0 (or the
                                 residual non-finite) before convergence       */
} merbit_status;

typedef enum { MERBIT_F32 = 0, MERBIT_F64 = 1 } merbit_dtype;

/* Granularity of the output commit (the paper's block size b, Sec. 4.2/4.3). */
typedef enum {
    MERBIT_COMMIT_AUTO = 0,  /* = MERBIT_COMMIT_WAVE                                      */
    MERBIT_COMMIT_BLOCK = 1, /* b = block_lanes: rows are buffered for a block of b/64
                                tiles and committed after one block barrier; only the
                                block's first and last rows are added atomically         */
    MERBIT_COMMIT_WAVE = 2   /* b = 64: every wavefront commits its own tile with no
                                barrier; each tile's first and last rows are added
                                atomically; blocks stay resident and stride over tiles  */
} merbit_commit;

/* Plan options; merbit_opts_init fills the defaults (every field 0 except
 * hot_columns = -1 and validate = 1). */
typedef struct {
    int32_t sigma;         /* steps per lane; 0 = 12 (F32) / 7 (F64).  Must satisfy
                              2 ceil(log2(64 sigma)) + sigma <= 32: 1..12 are built     */
    int32_t block_lanes;   /* threads per block; 0 = WAVE: 1024 (FP32, 32-bit
                              descriptors) or 512, BLOCK: 256.  Built: BLOCK 128, 256,
                              512, 1024; WAVE 256, 512, 1024 (64-bit: 256, 512)        */
    int32_t commit;        /* merbit_commit                                            */
    int32_t hot_columns;   /* LDS x cache for the most frequent columns -- an addition
                              to the paper's method: on gfx950 scattered x gathers are
                              bounded by the L2 request rate and power-law matrices
                              concentrate their nonzeros on few columns.  -1 = automatic
                              (wave commit only: largest cache that fits one block per
                              CU, kept only when the hot columns hold >= 20 % of the
                              nonzeros and the plan has at least 4 tiles per wavefront
                              of one block per CU -- a smaller plan cannot amortise the
                              copy into LDS; the block kernel gets none), 0 = off,
                              k > 0 = at most k columns (MERBIT_EUNSUPPORTED if k values
                              do not fit in LDS).  With the cache the plan owns a
                              recoded copy of col_ind (int32[nnz]) and each SpMV first
                              gathers the hot x values (one small launch); the sums and
                              their order are unchanged.                                */
    int32_t validate;      /* nonzero: check the CSR on the device first (one host
                              synchronisation); MERBIT_EINVAL if it is malformed        */
    int32_t blocks_per_cu; /* resident blocks per CU for the persistent launches;
                              0 = as many as LDS and wavefront slots allow              */
    int32_t eager_loops;   /* 0: the PageRank drivers record each chunk of iterations
                              between two convergence checks into a HIP graph on first
                              use and replay it; nonzero: launch every kernel directly  */
    int32_t desc_bits;     /* lane descriptor width: 0 or 32 (sigma <= 12), or 64
                              (2 ceil(log2(64 sigma)) + sigma <= 64, sigma <= 40; wave
                              commit only; built: FP32 sigma 16, 20, 24, 28, 32, FP64
                              14, 16, 20, 24, block_lanes 256 or 512).  SpMM and the
                              adjoint pieces need 32-bit plans.                         */
    int32_t stripes;       /* column stripes -- an addition to the paper's method for
                              gfx950's per-XCD caches: 0 or 1 = off; S = 2, 4, 8, 16 or
                              32 (wave commit only) cuts the columns into S stripes of
                              equal width and plans the stacked matrix A' whose rows
                              are the non-empty (stripe, row) pairs, stripe-major
                              (A x = sum of each row's pairs in A' x).  The tiles are
                              split into one contiguous range per XCD (8 on MI355X),
                              so an XCD gathers from about one stripe of x at a time
                              (L2-resident) and keeps the most frequent columns of its
                              own range in LDS (hot_columns then applies per range).
                              A second launch adds the stripes of each row in stripe
                              order.  The plan then owns copies of col_ind and values
                              in stacked order (values: re-copied by
                              merbit_plan_set_values, so in-place changes of the
                              array need that call) and two y' buffers [rows of A'].
                              With at least 12 tiles per wavefront the plan also owns
                              one small tile-queue line per range (each launch resets
                              it; two launches on one plan at once race, as every
                              other plan state does).  Needs nnz < 2^30.  SpMM (and
                              its dual / boundary calls), personalised PageRank,
                              transpose and SDDMM return MERBIT_EUNSUPPORTED on such a
                              plan; SpMV, PageRank, multi-graph PageRank, BiCGSTAB and
                              the adjoint fixed point run on it.                        */
    int32_t tune_rhs;      /* merbit_tune only (plans ignore it): 0 = time the SpMV;
                              k in 1..64 = time merbit_spmm with k right-hand sides    */
} merbit_opts_t;

typedef struct merbit_plan merbit_plan;

/* Read-only description of a plan (merbit_plan_info). */
typedef struct {
    int64_t n_rows, n_cols, nnz;
    int64_t tile_num;      /* ceil((nnz + n_rows) / (omega sigma))          Sec. 4.1.1 */
    int64_t lane_num;      /* ceil((nnz + n_rows) / sigma)                  Sec. 4.1.1 */
    int64_t fast_tiles;    /* tiles with the long-row mark (MSB of tile_y)  Sec. 4.2 (1) */
    int64_t chunk_num;     /* commit units (tiles for WAVE, b / 64 tiles for BLOCK)     */
    int32_t grid;          /* thread blocks of one fused launch                         */
    int32_t chunks_per_block; /* chunks each block works through (1 without hot cache) */
    int32_t hot_columns;   /* columns whose x values are served from LDS (0 = none)     */
    int32_t omega;         /* lanes per tile = wavefront size = 64                      */
    int32_t sigma;         /* merge-path steps per lane                     Sec. 4.3    */
    int32_t block_lanes;   /* lanes (threads) per block, b of Sec. 4.3                  */
    int32_t offset_bits;   /* ceil(log2(omega sigma)), width of x_offset / y_offset     */
    int32_t dtype;         /* merbit_dtype                                              */
    int32_t lds_bytes;     /* LDS per block: (b sigma + 1) values for products and row
                              partial sums (Sec. 4.3) + the hot x values               */
    int32_t commit;        /* merbit_commit of the plan                                 */
    double hot_coverage;   /* fraction of nonzeros whose column is hot (estimated from
                              a 1-in-s sample of the column stream, s <= 8, when the
                              cache holds only part of the columns; with column
                              stripes, per range: exact for a range of at most
                              64 hot_columns nonzeros, else from every 4th)             */
    int32_t desc_bits;     /* lane descriptor width: 32 or 64                           */
    int32_t stripes;       /* column stripes (1 = none)                                 */
    int32_t ranges;        /* contiguous tile ranges of the fused launch (1 = none)     */
    int32_t reserved;
    int64_t plan_rows;     /* rows of the planned matrix: n_rows, or the (stripe, row)
                              pairs of a striped plan; TILE and the exported arrays
                              are those of that matrix                                 */
    int64_t graph_captures; /* iteration chunks recorded into HIP graphs so far         */
    int64_t graph_replays;  /* iteration chunks run by replaying a recorded graph       */
} merbit_plan_info_t;

/* Fill *opts (host pointer) with the defaults. */
void merbit_opts_init(merbit_opts_t* opts);

/* Build a reusable plan (Sec. 4.1.2, Algorithm generate_tile: merge search
 * per lane, sigma-step walk, descriptor packing, long-row tile mark).
 *   n_rows, n_cols, nnz  matrix shape; n_rows + nnz < 2^31
 *   row_ptr, col_ind     device CSR arrays.  row_ptr is read only during this
 *                        call's work on `stream`; col_ind and values are
 *                        borrowed and must stay valid for the plan's life.
 *   values               device float[nnz] or double[nnz] per dtype (may be
 *                        replaced later with merbit_plan_set_values)
 *   dtype                MERBIT_F32 or MERBIT_F64
 *   opts                 host pointer to options, or NULL for the defaults
 *   out                  host pointer; receives the plan.  Free with
 *                        merbit_plan_destroy.
 * The plan owns TILE = {tile_x int32[T+1], tile_y uint32[T+1],
 * lane_desc uint32[lane_num]} and its work buffers.  Building the hot cache
 * synchronises `stream` (a column-count histogram is read back). */
int merbit_plan_create(int64_t n_rows, int64_t n_cols, int64_t nnz,
                       const int32_t* row_ptr, const int32_t* col_ind, const void* values,
                       int dtype, const merbit_opts_t* opts, void* stream, merbit_plan** out);

/* Replace the borrowed values pointer (same sparsity pattern, same dtype).
 * The TILE arrays depend only on row_ptr, so nothing is rebuilt.  A striped
 * plan copies the values into its stacked order (one gather on the plan's
 * last stream). */
int merbit_plan_set_values(merbit_plan* plan, const void* values);

/* Fill *info (host pointer).  Counts the long-row tiles on the device and
 * synchronises the plan's last stream. */
int merbit_plan_info(merbit_plan* plan, merbit_plan_info_t* info);

/* Copy TILE to host buffers (Sec. 4.1.1 layout).  Any output pointer may be
 * NULL; tile_x / tile_y need tile_num + 1 entries, lane_desc lane_num
 * descriptors of desc_bits / 8 bytes each (uint32_t, or uint64_t for a 64-bit
 * plan).  tile_num / lane_num (host, optional) receive the sizes.
 * Synchronous. */
int merbit_plan_export(merbit_plan* plan, int32_t* tile_x, uint32_t* tile_y,
                       void* lane_desc, int64_t* tile_num, int64_t* lane_num);

/* y <- A x (Sec. 4.2, Algorithm "MERBIT SpMV"), overwriting y whatever it
 * held.  x: device [n_cols], y: device [n_rows], both of the plan's dtype, not
 * aliased.  Launches: a scatter that zeroes y at the first row of every commit
 * unit, the hot-value gather (partial hot cache only), then the fused kernel. */
int merbit_spmv(merbit_plan* plan, const void* x, void* y, void* stream);

/* Dual-buffer form (Sec. 4.2, optimisation (3)): the fused launch only (plus
 * the hot-value gather).  Requires y to be zero at the first row of every
 * commit unit (every tile for WAVE, every b/64 tiles for BLOCK) on entry: true
 * for a buffer last used as `z` here, or after merbit_zero_boundary; computes
 * y <- A x and zeroes z at the same rows, so z can be the next call's y.  y and
 * z: device [n_rows], distinct, not aliased with x. */
int merbit_spmv_dual(merbit_plan* plan, const void* x, void* y, void* z, void* stream);
/* (A striped plan keeps its own dual buffers of A' x: there y is written
 * whole, z is not touched and merbit_zero_boundary does nothing.) */

/* Zero v (device [n_rows]) at the first row of every commit unit. */
int merbit_zero_boundary(merbit_plan* plan, void* v, void* stream);

/* PageRank by the power method (Sec. 5.5.1) on the plan's matrix, which must
 * be square and column stochastic with rows = destinations (P[v][u] =
 * 1/outdeg(u) for an edge u -> v).  Columns without nonzeros are dangling; their
 * mass is spread uniformly:
 *     x_{t+1} = alpha P x_t + (alpha sum_{u dangling} x_t[u] + 1 - alpha) / n.
 *   alpha      damping in [0, 1]
 *   tol        stop when ||x_{t+1} - x_t||_1 < tol; tested every check_every
 *              iterations (one host synchronisation each); tol <= 0 runs exactly
 *              max_iter iterations with a single synchronisation at the end
 *   max_iter   iteration cap (>= 0)
 *   x_inout    device [n] of the plan's dtype: x_0 on entry, the ranks on exit
 *   iters_out  host, optional: iterations performed
 *   resid_out  host, optional: ||x_iters - x_{iters-1}||_1 of the last iteration
 * Returns MERBIT_OK, or MERBIT_NOT_CONVERGED when tol > 0 was not reached.
 * Synchronises `stream` before returning. */
int merbit_pagerank(merbit_plan* plan, double alpha, double tol, int max_iter,
                    int check_every, void* x_inout, int* iters_out, double* resid_out,
                    void* stream);

/* Bytes of device work space merbit_pagerank_noalloc may use on each GPU. */
#define MERBIT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* merbit_pagerank for callers that cannot allocate device memory (tight
 * serving loops, code that must not call hipMalloc, harnesses that forbid it):
 * the same iteration, kernels, arguments and return codes, but no allocation
 * of any kind -- no hipMalloc / hipFree, no HIP graphs, no timing events.  The
 * work buffers (the SpMV's two output buffers, the second iterate, the
 * per-block reduction pairs, and the dangling mask while the plan has none
 * from an earlier merbit_pagerank) live in a library-owned device array of
 * MERBIT_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, held until the process ends.
 * A call needs 3 n sizeof(value) bytes plus 32 KiB, and n + n / 8 bytes more
 * when it builds the mask: n up to about 5.1M (FP32) or 2.6M (FP64); larger
 * plans return MERBIT_EINVAL with the needed size in the message.  The
 * plan itself (created earlier by merbit_plan_create) is the caller's, as are
 * x_inout and the stream.  The plan's device must be current.  Every call on
 * a GPU uses that GPU's one array: calls that overlap on one GPU (two host
 * threads, or two streams) race and give undefined results; calls in
 * sequence on one stream are safe (each call sets up what must start at zero).
 * Convergence checks copy a few KB to host memory and synchronise `stream`,
 * as merbit_pagerank does. */
int merbit_pagerank_noalloc(merbit_plan* plan, double alpha, double tol, int max_iter,
                            int check_every, void* x_inout, int* iters_out,
                            double* resid_out, void* stream);

/* ------------------------------------------------------ batched forms -- */

/* Y <- A X for k right-hand sides on the same plan (each column is the SpMV
 * of Sec. 4.2).  X: device [n_cols][ldx] row-major (first k columns used),
 * Y: device [n_rows][ldy] row-major, overwritten whatever it held; plan dtype;
 * k >= 1, ldx >= k, ldy >= k; X and Y not aliased.  One wavefront walks one
 * tile of the merge path and its lanes carry the columns of a slab, so every
 * X access is one coalesced read of a row's slab; the columns run in slabs of
 * 32, one launch each (faster than one 64-column launch, FP32 and FP64).
 * Launches: a scatter that zeroes Y at every tile's first row, then the SpMM
 * kernel once per slab. */
int merbit_spmm(merbit_plan* plan, const void* X, int64_t ldx, void* Y, int64_t ldy, int k,
                void* stream);

/* Dual-buffer SpMM: Y must be zero at every tile's first row (columns 0..k-1)
 * on entry; Z (same shape rules) is zeroed at those rows for the next call. */
int merbit_spmm_dual(merbit_plan* plan, const void* X, int64_t ldx, void* Y, int64_t ldy,
                     void* Z, int64_t ldz, int k, void* stream);

/* Zero columns 0..k-1 of Y at every tile's first row. */
int merbit_spmm_zero_boundary(merbit_plan* plan, void* Y, int64_t ldy, int k, void* stream);

/* Personalised PageRank for k sources at once (1 <= k <= 64), on the plan's
 * column-stochastic matrix (rows = destinations).  Column j is the power
 * method of Sec. 5.5.1 with teleport vector e_{sources[j]}; the dangling mass
 * follows the teleport vector:
 *     X'[:, j] = alpha P X[:, j] + (alpha sum_{u dangling} X[u, j] + 1 - alpha) e_{s_j}.
 *   sources    host int32[k], each in [0, n)
 *   X_inout    device [n][k] row-major, plan dtype: initial vectors in (for
 *              example e_{s_j}), ranks out
 *   tol        stop when every column's ||X' - X||_1 < tol, tested every
 *              check_every iterations; tol <= 0 runs exactly max_iter
 *   iters_out  host, optional; resid_out host double[k], optional: last l1
 *              change per column
 * A step is the SpMM (slabs of 32 columns) with the update of every row
 * strictly inside a tile done in its commit, then one kernel for the tiles'
 * first rows.  For k > 32 the iterates are held as compact 32-column slabs
 * (X_inout is converted on entry and back on return).  The plan keeps two
 * (k <= 32) or three (k > 32) n x k work buffers of its dtype after the
 * first call (freed by merbit_plan_destroy).
 * Returns MERBIT_OK or MERBIT_NOT_CONVERGED; synchronises `stream`. */
int merbit_pagerank_personalized(merbit_plan* plan, double alpha, double tol, int max_iter,
                                 int check_every, const int32_t* sources, int k, void* X_inout,
                                 int* iters_out, double* resid_out, void* stream);

/* PageRank of many graphs stored on the diagonal of one matrix, all solved by
 * one plan: graph g owns rows and columns [graph_ptr[g], graph_ptr[g+1]) of
 * the plan's column-stochastic matrix (rows = destinations), and each step is
 * the power method of Sec. 5.5.1 on every graph at once, with the graph's own
 * size n_g, dangling mass and uniform teleport:
 *     x'[r] = alpha (P x)[r] + (alpha sum_{u in g dangling} x[u] + 1 - alpha) / n_g.
 * One fused SpMV covers all graphs (the merge path balances work across them);
 * the per-graph sums are deterministic segment reductions.
 *   graph_ptr  host int64[n_graphs + 1]: 0 = graph_ptr[0] < ... <
 *              graph_ptr[n_graphs] = n (no empty graph).  Nonzeros outside
 *              their row's graph are not checked for; they couple graphs.
 *   x_inout    device [n], plan dtype: x_0 in (e.g. 1/n_g on graph g), ranks out
 *   tol        stop when every graph's ||x' - x||_1 (over its rows) < tol,
 *              tested every check_every iterations; tol <= 0 runs max_iter
 *   resid_out  host double[n_graphs], optional: last l1 change per graph
 * Returns MERBIT_OK or MERBIT_NOT_CONVERGED; synchronises `stream`. */
int merbit_pagerank_multi(merbit_plan* plan, const int64_t* graph_ptr, int n_graphs,
                          double alpha, double tol, int max_iter, int check_every, void* x_inout,
                          int* iters_out, double* resid_out, void* stream);

/* ------------------------------------------- adjoint (differentiation) -- */
/* Pieces for differentiating PageRank (Sec. 5.5.1) with respect to the
 * matrix values.  With x* the fixed point of G(x) = alpha P x +
 * (alpha d^T x + 1 - alpha)/n 1 (d = dangling indicator) and a loss L(x*)
 * with gradient g = dL/dx*, the adjoint vector solves
 *     lambda = g + alpha P^T lambda + (alpha / n) (1^T lambda) d
 * and dL/dP[e] = alpha lambda[row(e)] x*[col(e)] for every nonzero e. */

/* CSR of the transpose of the plan's matrix, for a second plan that runs
 * P^T lambda with the same merge-path kernels.  Outputs (device, caller
 * owned): rowT_ptr int32[n_cols + 1], colT int32[nnz], perm int32[nnz], where
 * row c of A^T lists the nonzeros of column c of A in increasing row order
 * and perm[i] is the index in A of the i-th nonzero of A^T (so A^T's values
 * are values[perm[i]], see merbit_gather_values).  Rows of the nonzeros come
 * from the plan's descriptors; the order is a stable radix sort by column,
 * so the result is deterministic.  Allocates and frees temporary device
 * memory (about 12 bytes per nonzero plus the sort's workspace); synchronises
 * `stream`. */
int merbit_transpose(merbit_plan* plan, int32_t* rowT_ptr, int32_t* colT, int32_t* perm,
                     void* stream);

/* Per-nonzero product on the plan's pattern: out[e] = scale g[row(e)]
 * x[col(e)] (device, plan dtype: g[n_rows], x[n_cols], out[nnz], in the plan's
 * nonzero order).  With g = lambda, x = x*, scale = alpha this is dL/dP. */
int merbit_sddmm(merbit_plan* plan, const void* g, const void* x, double scale, void* out,
                 void* stream);

/* dst[i] = src[perm[i]] (times src2[perm[i]] when src2 is not NULL); device
 * arrays of nnz values of `dtype` (merbit_dtype).  dst must not alias src or
 * src2. */
int merbit_gather_values(int dtype, int64_t nnz, const int32_t* perm, const void* src,
                         const void* src2, void* dst, void* stream);

/* out[e] = (a[e] - t[col[e]]) / s[col[e]] (t may be NULL: out = a / s[col]);
 * device arrays, `dtype` values.  With a = w and s = column sums of w this is
 * the column normalisation P = w / colsum(w); with a = dL/dP and t[c] = sum
 * over column c of dL/dP[e] P[e] it is the derivative dL/dw. */
int merbit_column_scale(int dtype, int64_t nnz, const int32_t* col, const void* a, const void* t,
                        const void* s, void* out, void* stream);

/* Adjoint fixed point: lambda <- g + alpha P^T lambda + (alpha/n) (1^T lambda) d,
 * iterated from lambda_in (e.g. a copy of g).  `plan` is P's plan (square;
 * its dangling mask gives d), `plan_t` the plan of P^T built from
 * merbit_transpose's output with values[perm] (same dtype; its SpMV does
 * P^T lambda).  g, lambda_inout: device [n], plan dtype, not aliased.
 * Stops when ||lambda' - lambda||_1 < tol (tested every check_every
 * iterations) or after max_iter; tol <= 0 runs exactly max_iter.  Uses
 * plan_t's iteration buffers (not concurrently with PageRank on plan_t).
 * Returns MERBIT_OK or MERBIT_NOT_CONVERGED; synchronises `stream`. */
int merbit_pagerank_adjoint(merbit_plan* plan, merbit_plan* plan_t, double alpha, double tol,
                            int max_iter, int check_every, const void* g, void* lambda_inout,
                            int* iters_out, double* resid_out, void* stream);

/* ------------------------------------------------------------- BiCGSTAB -- */

/* Solve A x = b with unpreconditioned BiCGSTAB (van der Vorst 1992), the
 * second iterative workload of Sec. 5.5.2, on the plan's square matrix.  Two
 * fused SpMVs per iteration (dual output buffers, no resets) and five vector
 * kernels whose dot products are reduced deterministically in double.
 *   b          device [n], plan dtype
 *   x_inout    device [n], plan dtype: x_0 in, solution out (not aliased with b)
 *   tol        stop when ||r||_2 / ||b||_2 < tol, r the updated residual
 *              (= b - A x in exact arithmetic), tested before the first
 *              iteration and then every check_every iterations; tol <= 0
 *              runs exactly max_iter iterations
 *   iters_out  host, optional: iterations run
 *   resid_out  host, optional: ||r|| / ||b|| at the last test
 * Returns MERBIT_OK (converged), MERBIT_NOT_CONVERGED (max_iter reached) or
 * MERBIT_BREAKDOWN (rho = 0 or a non-finite residual at a test; x then holds
 * the last iterate).  Iteration chunks are recorded in HIP graphs as for
 * PageRank.  Synchronises `stream`. */
int merbit_bicgstab(merbit_plan* plan, const void* b, void* x_inout, double tol, int max_iter,
                    int check_every, int* iters_out, double* resid_out, void* stream);

/* ------------------------------------------------------------ autotuner -- */

/* Choose sigma (steps per lane) and block_lanes for one matrix by measurement,
 * the sweep of Sec. 4.3 / Sec. 5.3 (the paper tunes sigma per precision).  For
 * every candidate pair a plan is built from the given CSR (device pointers as
 * in merbit_plan_create; validation off), the dual-buffer SpMV is launched
 * 2 + reps times on `stream` with a constant nonzero x, and the mean time of
 * the last reps launches is taken.  With opts_inout->tune_rhs = k > 0 the
 * timed call is merbit_spmm over k right-hand sides (X constant, row-major
 * n_cols x k; the SpMM kernel's block size is fixed, so block_lanes only
 * repeats the measurement).
 *   sigmas, n_sigmas      host int32 candidates; NULL or n <= 0 = 7..12 (F32),
 *                         4..10 (F64)
 *   block_lanes, n_blocks host int32 candidates; NULL or n <= 0 = 256, 512, 1024
 *   opts_inout            host: base options in (commit, hot_columns, ...);
 *                         the best sigma and block_lanes out
 *   us_out                host float[n_sigmas * n_blocks], optional: mean
 *                         microseconds per launch, row-major by sigma; -1 for a
 *                         candidate the kernels do not build
 * Allocates and frees its own buffers; synchronises `stream`.  Returns
 * MERBIT_EUNSUPPORTED if no candidate is built. */
int merbit_tune(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t* row_ptr,
                const int32_t* col_ind, const void* values, int dtype, const int32_t* sigmas,
                int n_sigmas, const int32_t* block_lanes, int n_blocks, int reps,
                merbit_opts_t* opts_inout, float* us_out, void* stream);

/* Kernel timing for the SpMV launches of this plan.  While enabled, every
 * fused SpMV launch (from merbit_spmv, merbit_spmv_dual and the iterative
 * drivers) and every SpMM slab launch is bracketed by HIP events on its
 * stream, and the drivers launch their kernels directly instead of replaying
 * HIP graphs.  merbit_profile_read (synchronous) returns the number of timed
 * launches and their summed duration in ms, then clears the record.  Host
 * pointers. */
int merbit_profile_enable(merbit_plan* plan, int enable);
int merbit_profile_read(merbit_plan* plan, int64_t* launches, double* total_ms);

/* Release the plan and everything it owns (waits for its pending work). */
void merbit_plan_destroy(merbit_plan* plan);

/* Message of the last failed call on this thread ("" if none). */
const char* merbit_last_error(void);

/* Library version string. */
const char* merbit_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MERBIT_H */
