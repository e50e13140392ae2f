/*
 * CPU oracle for the MERBIT hot path.  TEST INFRASTRUCTURE ONLY: only the
 * test-suite, the package smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code with the HIP library.
 *
 * Plain, sequential and slow on purpose.  Every function names the part of
 * the paper ("MERBIT: A GPU-Based SpMV Method for Iterative Workloads") it
 * writes out.
 *
 *   or_spmv          y = A x, the definition of Sec. 3.1, summed in long double
 *   or_abs_spmv      (|A| |x|)[r], the scale used by the parity tolerance
 *   or_path_coords   the merge path of Sec. 3.3 walked step by step
 *   or_merge_search  the diagonal binary search of Algorithm 1 (merge_search)
 *   or_plan          the TILE arrays of Sec. 4.1.1 / 4.1.2 from one sequential walk
 *   or_plan_replay   decode TILE (Sec. 4.1.1 coordinate formula) and redo y = A x
 *   or_plan64 / or_plan_replay64   the same with 64-bit lane descriptors
 *   or_pagerank      power method of Sec. 5.5.1, damping alpha, dangling mass
 *                    spread uniformly
 *   or_spmm          Sec. 3.1 applied to every column of a multi-vector
 *   or_pagerank_teleport  the power method with a general teleport vector
 *   or_transpose     CSR of A^T with the permutation of the nonzeros
 *   or_pagerank_adjoint   the adjoint fixed point of the PageRank step
 *                    (derivative of Sec. 5.5.1's iteration map)
 *   or_bicgstab      BiCGSTAB (Sec. 5.5.2, van der Vorst 1992)
 *
 * Conventions.  CSR: row_ptr has n_rows + 1 entries (Sec. 3.1 says "length n";
 * the algorithms read offset[y + 1], so the array has n + 1 entries), col and
 * values have m = row_ptr[n_rows] entries.  Merge-path coordinates are
 * (x, y) = (nonzeros consumed, rows finished).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ---------------------------------------------------------------- SpMV -- */

/* Sec. 3.1: y[r] = sum over k in [row_ptr[r], row_ptr[r+1]) of
 * values[k] * x[col[k]].  Products and sums in long double (64-bit
 * significand); an empty row gives exactly 0. */
void or_spmv(int64_t n_rows, const int32_t* row_ptr, const int32_t* col,
             const double* values, const double* x, double* y) {
    for (int64_t r = 0; r < n_rows; ++r) {
        long double s = 0.0L;
        for (int64_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k)
            s += (long double)values[k] * (long double)x[col[k]];
        y[r] = (double)s;
    }
}

/* (|A| |x|)[r] = sum |values[k]| |x[col[k]]|, the per-row scale of the
 * parity tolerance (a rounding-error bound for any summation order is a
 * multiple of it). */
void or_abs_spmv(int64_t n_rows, const int32_t* row_ptr, const int32_t* col,
                 const double* values, const double* x, double* y) {
    for (int64_t r = 0; r < n_rows; ++r) {
        long double s = 0.0L;
        for (int64_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k)
            s += fabsl((long double)values[k]) * fabsl((long double)x[col[k]]);
        y[r] = (double)s;
    }
}

/* ----------------------------------------------------------- merge path -- */

/* Sec. 3.3: the merge path runs from (0, 0) to (m, n).  From (x, y) it steps
 * right (consume nonzero x of row y) while x < row_ptr[y + 1], otherwise down
 * (row y is complete).  Writes the coordinate after each of the first d
 * steps, d = 0 .. m + n, into xs[d], ys[d]. */
void or_path_coords(int64_t n_rows, const int32_t* row_ptr, int32_t* xs, int32_t* ys) {
    const int64_t m = row_ptr[n_rows];
    const int64_t L = m + n_rows;
    int64_t x = 0, y = 0;
    xs[0] = 0;
    ys[0] = 0;
    for (int64_t d = 0; d < L; ++d) {
        if (x < row_ptr[y + 1]) ++x; else ++y;
        xs[d + 1] = (int32_t)x;
        ys[d + 1] = (int32_t)y;
    }
}

/* Algorithm 1 (merge_search): binary search along the diagonal x + y = diag
 * for the point where it crosses the merge path.  y ends as the number of
 * rows r whose end offset satisfies row_ptr[r + 1] <= diag - r - 1. */
void or_merge_search(int64_t n_rows, const int32_t* row_ptr, int64_t diag,
                     int64_t* x_out, int64_t* y_out) {
    const int64_t m = row_ptr[n_rows];
    int64_t lo = diag - m > 0 ? diag - m : 0;
    int64_t hi = diag < n_rows ? diag : n_rows;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((int64_t)row_ptr[mid + 1] <= diag - mid - 1) lo = mid + 1;
        else hi = mid;
    }
    *x_out = diag - lo;
    *y_out = lo < n_rows ? lo : n_rows;
}

/* b = ceil(log2(omega * sigma)): the width of each offset field (Sec. 4.1.1). */
int or_offset_bits(int omega, int sigma) {
    int64_t v = (int64_t)omega * sigma;
    int b = 0;
    while (((int64_t)1 << b) < v) ++b;
    return b;
}

/* Sec. 4.1.1 / 4.1.2: the TILE format.
 *   tile_num = ceil((m + n) / (omega sigma)), lane_num = ceil((m + n) / sigma)
 *   tile_x, tile_y [tile_num + 1]: start of tile i = the path coordinate after
 *       i * omega * sigma steps; last entry (m, n).  Bit 31 of tile_y[i] is set
 *       when no step of tile i goes down (the whole tile lies in one row).
 *   lane_desc [lane_num]: lane j covers steps [j sigma, min((j+1) sigma, m+n));
 *       its start minus its tile's start gives (x_off, y_off); bit k of the
 *       flag word is 1 when step k of the lane goes down.  Packed as
 *       flags << 2b | y_off << b | x_off.
 * Built here from a single sequential walk of the path (no search).
 * Returns 0, or -1 when 2b + sigma > 32 (the descriptor does not fit). */
int or_plan(int64_t n_rows, const int32_t* row_ptr, int omega, int sigma,
            int32_t* tile_x, uint32_t* tile_y, uint32_t* lane_desc) {
    const int64_t m = row_ptr[n_rows];
    const int64_t L = m + n_rows;
    const int64_t ws = (int64_t)omega * sigma;
    const int64_t tile_num = (L + ws - 1) / ws;
    const int64_t lane_num = (L + sigma - 1) / sigma;
    const int b = or_offset_bits(omega, sigma);
    if (2 * b + sigma > 32) return -1;

    int64_t x = 0, y = 0;            /* current path coordinate */
    int64_t tx = 0, ty = 0;          /* start of the current tile */
    int tile_has_down = 0;
    uint32_t flags = 0;
    uint32_t lane_x_off = 0, lane_y_off = 0;
    for (int64_t d = 0; d < L; ++d) {
        if (d % ws == 0) {           /* a tile starts here */
            tx = x;
            ty = y;
            tile_has_down = 0;
        }
        if (d % sigma == 0) {        /* a lane starts here */
            lane_x_off = (uint32_t)(x - tx);
            lane_y_off = (uint32_t)(y - ty);
            flags = 0;
        }
        const int k = (int)(d % sigma);
        if (x < row_ptr[y + 1]) {
            ++x;
        } else {
            ++y;
            flags |= 1u << k;
            tile_has_down = 1;
        }
        if (k == sigma - 1 || d == L - 1) {   /* lane ends after this step */
            const int64_t j = d / sigma;
            lane_desc[j] = (flags << (2 * b)) | (lane_y_off << b) | lane_x_off;
        }
        if ((d + 1) % ws == 0 || d == L - 1) { /* tile ends after this step */
            const int64_t i = d / ws;
            tile_x[i] = (int32_t)tx;
            tile_y[i] = (uint32_t)ty | (tile_has_down ? 0u : 0x80000000u);
        }
    }
    (void)lane_num;
    tile_x[tile_num] = (int32_t)m;
    tile_y[tile_num] = (uint32_t)n_rows;
    return 0;
}

/* The same TILE with 64-bit lane descriptors: identical walk and field
 * layout (flags << 2b | y_off << b | x_off), fit condition 2b + sigma <= 64,
 * which admits sigma up to 40 at omega = 64.  For sigma <= 12 every
 * descriptor has the value or_plan gives.  Returns 0 or -1 (does not fit). */
int or_plan64(int64_t n_rows, const int32_t* row_ptr, int omega, int sigma,
              int32_t* tile_x, uint32_t* tile_y, uint64_t* lane_desc) {
    const int64_t m = row_ptr[n_rows];
    const int64_t L = m + n_rows;
    const int64_t ws = (int64_t)omega * sigma;
    const int64_t tile_num = (L + ws - 1) / ws;
    const int b = or_offset_bits(omega, sigma);
    if (2 * b + sigma > 64) return -1;

    int64_t x = 0, y = 0, tx = 0, ty = 0;
    int tile_has_down = 0;
    uint64_t flags = 0, lane_x_off = 0, lane_y_off = 0;
    for (int64_t d = 0; d < L; ++d) {
        if (d % ws == 0) {
            tx = x;
            ty = y;
            tile_has_down = 0;
        }
        if (d % sigma == 0) {
            lane_x_off = (uint64_t)(x - tx);
            lane_y_off = (uint64_t)(y - ty);
            flags = 0;
        }
        const int k = (int)(d % sigma);
        if (x < row_ptr[y + 1]) {
            ++x;
        } else {
            ++y;
            flags |= (uint64_t)1 << k;
            tile_has_down = 1;
        }
        if (k == sigma - 1 || d == L - 1)
            lane_desc[d / sigma] = (flags << (2 * b)) | (lane_y_off << b) | lane_x_off;
        if ((d + 1) % ws == 0 || d == L - 1) {
            const int64_t i = d / ws;
            tile_x[i] = (int32_t)tx;
            tile_y[i] = (uint32_t)ty | (tile_has_down ? 0u : 0x80000000u);
        }
    }
    tile_x[tile_num] = (int32_t)m;
    tile_y[tile_num] = (uint32_t)n_rows;
    return 0;
}

/* or_plan_replay for 64-bit descriptors (same decode, wider words). */
int or_plan_replay64(int64_t n_rows, int64_t m, int omega, int sigma,
                     const int32_t* tile_x, const uint32_t* tile_y, const uint64_t* lane_desc,
                     const int32_t* col, const double* values, const double* xv, double* y) {
    const int64_t L = m + n_rows;
    const int64_t lane_num = (L + sigma - 1) / sigma;
    const int b = or_offset_bits(omega, sigma);
    const uint64_t fmask = ((uint64_t)1 << b) - 1u;
    long double* acc = (long double*)calloc((size_t)(n_rows > 0 ? n_rows : 1), sizeof(long double));
    if (!acc) return -2;
    for (int64_t j = 0; j < lane_num; ++j) {
        const int64_t i = j / omega;
        const uint64_t desc = lane_desc[j];
        int64_t x = (int64_t)tile_x[i] + (int64_t)(desc & fmask);
        int64_t yy = (int64_t)(tile_y[i] & 0x7FFFFFFFu) + (int64_t)((desc >> b) & fmask);
        const uint64_t flags = desc >> (2 * b);
        const int64_t steps = (L - j * sigma) < sigma ? (L - j * sigma) : sigma;
        for (int64_t k = 0; k < steps; ++k) {
            if ((flags >> k) & 1u) {
                if (yy >= n_rows) { free(acc); return -3; }
                ++yy;
            } else {
                if (x >= m || yy >= n_rows) { free(acc); return -4; }
                acc[yy] += (long double)values[x] * (long double)xv[col[x]];
                ++x;
            }
        }
    }
    for (int64_t r = 0; r < n_rows; ++r) y[r] = (double)acc[r];
    free(acc);
    return 0;
}

/* Sec. 4.1.1: the coordinate of step k of lane j in tile i is
 *   (tile_x[i] + x_off + k_x, ROW(tile_y[i]) + y_off + k_y)
 * with k_x, k_y the right and down steps among the first k flag bits.
 * Decodes every lane and replays it: a right step adds values[x] * x[col[x]]
 * to the running sum of the current row, a down step stores it.  Sums are kept
 * per row in path order, so for a correct TILE the result equals or_spmv bit
 * for bit.  nnz_row (optional) receives the row of every nonzero.
 * Returns 0, or a negative code when the descriptors are inconsistent
 * (a step leaves the matrix). */
int or_plan_replay(int64_t n_rows, int64_t m, int omega, int sigma,
                   const int32_t* tile_x, const uint32_t* tile_y, const uint32_t* lane_desc,
                   const int32_t* col, const double* values, const double* xv,
                   double* y, int32_t* nnz_row) {
    const int64_t L = m + n_rows;
    const int64_t lane_num = (L + sigma - 1) / sigma;
    const int b = or_offset_bits(omega, sigma);
    const uint32_t fmask = (b > 0) ? ((1u << b) - 1u) : 0u;
    long double* acc = (long double*)calloc((size_t)(n_rows > 0 ? n_rows : 1), sizeof(long double));
    if (!acc) return -2;
    for (int64_t j = 0; j < lane_num; ++j) {
        const int64_t i = j / omega;
        const uint32_t desc = lane_desc[j];
        int64_t x = (int64_t)tile_x[i] + (desc & fmask);
        int64_t yy = (int64_t)(tile_y[i] & 0x7FFFFFFFu) + ((desc >> b) & fmask);
        const uint32_t flags = desc >> (2 * b);
        const int64_t steps = (L - j * sigma) < sigma ? (L - j * sigma) : sigma;
        for (int64_t k = 0; k < steps; ++k) {
            if ((flags >> k) & 1u) {
                if (yy >= n_rows) { free(acc); return -3; }
                ++yy;                      /* row yy is complete */
            } else {
                if (x >= m || yy >= n_rows) { free(acc); return -4; }
                acc[yy] += (long double)values[x] * (long double)xv[col[x]];
                if (nnz_row) nnz_row[x] = (int32_t)yy;
                ++x;
            }
        }
    }
    for (int64_t r = 0; r < n_rows; ++r) y[r] = (double)acc[r];
    free(acc);
    return 0;
}

/* ------------------------------------------------------------ PageRank -- */

/* Sec. 5.5.1: PageRank by the power method with damping alpha.  The matrix is
 * the column-stochastic transition matrix P stored with rows = destinations
 * (P[v][u] = 1 / outdeg(u) for an edge u -> v).  A column without nonzeros is
 * a dangling vertex; its mass is spread uniformly:
 *     x_{t+1} = alpha P x_t + (alpha * sum_{u dangling} x_t[u] + 1 - alpha) / n.
 * Iterates are kept in long double; x_out gets the last one.  hist (optional,
 * iters * n) receives every iterate, resid (optional, iters) the l1 change
 * ||x_{t+1} - x_t||_1 of every step. */
int or_pagerank(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* values,
                double alpha, int iters, const double* x0, double* x_out,
                double* hist, double* resid) {
    const int64_t m = row_ptr[n];
    unsigned char* has_out = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
    long double* x = (long double*)malloc(sizeof(long double) * (size_t)(n > 0 ? n : 1));
    long double* xn = (long double*)malloc(sizeof(long double) * (size_t)(n > 0 ? n : 1));
    if (!has_out || !x || !xn) { free(has_out); free(x); free(xn); return -2; }
    for (int64_t k = 0; k < m; ++k) has_out[col[k]] = 1;
    for (int64_t i = 0; i < n; ++i) x[i] = x0[i];
    const long double a = alpha;
    for (int t = 0; t < iters; ++t) {
        long double dangling = 0.0L;
        for (int64_t u = 0; u < n; ++u)
            if (!has_out[u]) dangling += x[u];
        const long double teleport = (a * dangling + 1.0L - a) / (long double)n;
        long double change = 0.0L;
        for (int64_t r = 0; r < n; ++r) {
            long double s = 0.0L;
            for (int64_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k)
                s += (long double)values[k] * x[col[k]];
            xn[r] = a * s + teleport;
            change += fabsl(xn[r] - x[r]);
        }
        long double* tmp = x; x = xn; xn = tmp;
        if (resid) resid[t] = (double)change;
        if (hist)
            for (int64_t r = 0; r < n; ++r) hist[(int64_t)t * n + r] = (double)x[r];
    }
    for (int64_t r = 0; r < n; ++r) x_out[r] = (double)x[r];
    free(has_out);
    free(x);
    free(xn);
    return 0;
}

/* -------------------------------------------------------- batched forms -- */

/* Y = A X for k right-hand sides (Sec. 3.1 applied to every column of X):
 * X is n_cols x k and Y is n_rows x k, both row-major.  Long-double sums. */
void or_spmm(int64_t n_rows, const int32_t* row_ptr, const int32_t* col, const double* values,
             int k, const double* X, double* Y) {
    for (int64_t r = 0; r < n_rows; ++r) {
        for (int j = 0; j < k; ++j) {
            long double s = 0.0L;
            for (int64_t p = row_ptr[r]; p < row_ptr[r + 1]; ++p)
                s += (long double)values[p] * (long double)X[(int64_t)col[p] * k + j];
            Y[r * k + j] = (double)s;
        }
    }
}

/* Power method with a general teleport (personalisation) vector v, sum v = 1:
 *     x_{t+1} = alpha P x_t + (alpha sum_{u dangling} x_t[u] + 1 - alpha) v.
 * The dangling mass follows the teleport vector.  v = 1/n gives the PageRank
 * of Sec. 5.5.1 (or_pagerank); v = e_s gives personalised PageRank for source s.
 * resid (optional, iters): ||x_{t+1} - x_t||_1 per step. */
int or_pagerank_teleport(int64_t n, const int32_t* row_ptr, const int32_t* col,
                         const double* values, double alpha, int iters, const double* v,
                         const double* x0, double* x_out, double* resid) {
    const int64_t m = row_ptr[n];
    unsigned char* has_out = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
    long double* x = (long double*)malloc(sizeof(long double) * (size_t)(n > 0 ? n : 1));
    long double* xn = (long double*)malloc(sizeof(long double) * (size_t)(n > 0 ? n : 1));
    if (!has_out || !x || !xn) { free(has_out); free(x); free(xn); return -2; }
    for (int64_t k = 0; k < m; ++k) has_out[col[k]] = 1;
    for (int64_t i = 0; i < n; ++i) x[i] = x0[i];
    const long double a = alpha;
    for (int t = 0; t < iters; ++t) {
        long double dangling = 0.0L;
        for (int64_t u = 0; u < n; ++u)
            if (!has_out[u]) dangling += x[u];
        const long double scale = a * dangling + 1.0L - a;
        long double change = 0.0L;
        for (int64_t r = 0; r < n; ++r) {
            long double s = 0.0L;
            for (int64_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k)
                s += (long double)values[k] * x[col[k]];
            xn[r] = a * s + scale * (long double)v[r];
            change += fabsl(xn[r] - x[r]);
        }
        long double* tmp = x; x = xn; xn = tmp;
        if (resid) resid[t] = (double)change;
    }
    for (int64_t r = 0; r < n; ++r) x_out[r] = (double)x[r];
    free(has_out);
    free(x);
    free(xn);
    return 0;
}

/* ---------------------------------------------- adjoint of PageRank ---- */

/* CSR of the transpose A^T (n_cols rows): the nonzeros of column c of A, in
 * increasing row order, become row c of A^T.  perm[i] is the index in A of
 * the i-th nonzero of A^T.  One counting pass, then one placement pass in
 * A's storage order (so the order within each row of A^T is stable). */
int or_transpose(int64_t n_rows, int64_t n_cols, const int32_t* row_ptr, const int32_t* col,
                 int32_t* rowT_ptr, int32_t* colT, int32_t* perm) {
    const int64_t m = row_ptr[n_rows];
    int64_t* next = (int64_t*)calloc((size_t)(n_cols + 1), sizeof(int64_t));
    if (!next) return -2;
    for (int64_t c = 0; c <= n_cols; ++c) rowT_ptr[c] = 0;
    for (int64_t k = 0; k < m; ++k) rowT_ptr[col[k] + 1] += 1;
    for (int64_t c = 0; c < n_cols; ++c) rowT_ptr[c + 1] += rowT_ptr[c];
    for (int64_t c = 0; c < n_cols; ++c) next[c] = rowT_ptr[c];
    for (int64_t r = 0; r < n_rows; ++r)
        for (int64_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
            const int64_t pos = next[col[k]]++;
            colT[pos] = (int32_t)r;
            perm[pos] = (int32_t)k;
        }
    free(next);
    return 0;
}

/* Adjoint of the PageRank fixed point of Sec. 5.5.1.  The step is
 *     G(x) = alpha P x + (alpha d^T x + 1 - alpha) / n * 1,
 * d = indicator of the dangling vertices (columns of P without nonzeros), so
 * its Jacobian is M = alpha P + (alpha / n) 1 d^T and the adjoint vector of a
 * loss gradient g solves lambda = g + M^T lambda, i.e.
 *     lambda_{t+1} = g + alpha P^T lambda_t + (alpha / n) (1^T lambda_t) d.
 * P^T lambda is formed straight from P's CSR ((P^T l)[u] = sum over the
 * nonzeros (v, u) of P[v][u] l[v]).  Starts from lambda_0 = g; runs `iters`
 * steps (a contraction with factor alpha in the 1-norm).  Long double. */
int or_pagerank_adjoint(int64_t n, const int32_t* row_ptr, const int32_t* col,
                        const double* values, double alpha, int iters, const double* g,
                        double* lam_out) {
    const int64_t m = row_ptr[n];
    unsigned char* has_out = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
    long double* l = (long double*)malloc(sizeof(long double) * (size_t)(n > 0 ? n : 1));
    long double* pt = (long double*)malloc(sizeof(long double) * (size_t)(n > 0 ? n : 1));
    if (!has_out || !l || !pt) { free(has_out); free(l); free(pt); return -2; }
    for (int64_t k = 0; k < m; ++k) has_out[col[k]] = 1;
    for (int64_t i = 0; i < n; ++i) l[i] = g[i];
    const long double a = alpha;
    for (int t = 0; t < iters; ++t) {
        long double total = 0.0L;
        for (int64_t i = 0; i < n; ++i) {
            total += l[i];
            pt[i] = 0.0L;
        }
        for (int64_t v = 0; v < n; ++v)
            for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k)
                pt[col[k]] += (long double)values[k] * l[v];
        const long double dang = a * total / (long double)n;
        for (int64_t u = 0; u < n; ++u)
            l[u] = (long double)g[u] + a * pt[u] + (has_out[u] ? 0.0L : dang);
    }
    for (int64_t i = 0; i < n; ++i) lam_out[i] = (double)l[i];
    free(has_out);
    free(l);
    free(pt);
    return 0;
}

/* ------------------------------------------------------------ BiCGSTAB -- */

/* Unpreconditioned BiCGSTAB (van der Vorst, 1992), the second iterative
 * workload of Sec. 5.5.2: solve A x = b from x0, shadow residual r^ = r_0.
 * Each iteration:
 *     rho = (r^, r);  beta = (rho / rho_prev) (alpha / omega)
 *     p = r + beta (p - omega v);  v = A p;  alpha = rho / (r^, v)
 *     s = r - alpha v;  t = A s;  omega = (t, s) / (t, t)
 *     x = x + alpha p + omega s;  r = s - omega t
 * and stops when ||r||_2 / ||b||_2 < tol (r is the updated residual, equal to
 * b - A x in exact arithmetic) or after max_iter iterations.  Breakdown
 * (rho, (r^, v) or (t, t) equal to 0) stops early.  Dots and vectors in long
 * double.  resid_hist (optional, max_iter entries): ||r|| / ||b|| per
 * iteration.  Returns the iteration count, or -2 on allocation failure;
 * *status = 0 converged, 1 iteration cap, 2 breakdown. */
int or_bicgstab(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* values,
                const double* b, const double* x0, double tol, int max_iter, double* x_out,
                double* resid_hist, int* status) {
    long double *x = 0, *r = 0, *rh = 0, *p = 0, *v = 0, *s = 0, *t = 0;
    const size_t sz = sizeof(long double) * (size_t)(n > 0 ? n : 1);
    x = malloc(sz); r = malloc(sz); rh = malloc(sz); p = malloc(sz); v = malloc(sz);
    s = malloc(sz); t = malloc(sz);
    if (!x || !r || !rh || !p || !v || !s || !t) {
        free(x); free(r); free(rh); free(p); free(v); free(s); free(t);
        return -2;
    }
    long double bnorm = 0.0L;
    for (int64_t i = 0; i < n; ++i) {
        x[i] = x0[i];
        bnorm += (long double)b[i] * b[i];
    }
    bnorm = sqrtl(bnorm);
    for (int64_t i = 0; i < n; ++i) {  /* r = b - A x0 */
        long double ax = 0.0L;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) ax += (long double)values[k] * x[col[k]];
        r[i] = (long double)b[i] - ax;
        rh[i] = r[i];
        p[i] = v[i] = 0.0L;
    }
    long double rho_prev = 1.0L, alpha = 1.0L, omega = 1.0L;
    int it = 0;
    *status = 1;
    if (bnorm == 0.0L) bnorm = 1.0L;
    {
        long double rr = 0.0L;
        for (int64_t i = 0; i < n; ++i) rr += r[i] * r[i];
        if (sqrtl(rr) / bnorm < tol) { *status = 0; max_iter = 0; }
    }
    while (it < max_iter) {
        long double rho = 0.0L;
        for (int64_t i = 0; i < n; ++i) rho += rh[i] * r[i];
        if (rho == 0.0L) { *status = 2; break; }
        const long double beta = (rho / rho_prev) * (alpha / omega);
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        long double rhv = 0.0L;
        for (int64_t i = 0; i < n; ++i) {
            long double a = 0.0L;
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) a += (long double)values[k] * p[col[k]];
            v[i] = a;
            rhv += rh[i] * a;
        }
        if (rhv == 0.0L) { *status = 2; break; }
        alpha = rho / rhv;
        for (int64_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        long double ts = 0.0L, tt = 0.0L;
        for (int64_t i = 0; i < n; ++i) {
            long double a = 0.0L;
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) a += (long double)values[k] * s[col[k]];
            t[i] = a;
            ts += a * s[i];
            tt += a * a;
        }
        if (tt == 0.0L) {  /* s = 0 exactly: x + alpha p solves the system */
            for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] = s[i]; }
            ++it;
            if (resid_hist) resid_hist[it - 1] = 0.0;
            *status = 0;
            break;
        }
        omega = ts / tt;
        long double rr = 0.0L;
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i] + omega * s[i];
            r[i] = s[i] - omega * t[i];
            rr += r[i] * r[i];
        }
        ++it;
        const long double rel = sqrtl(rr) / bnorm;
        if (resid_hist) resid_hist[it - 1] = (double)rel;
        rho_prev = rho;
        if (rel < tol) { *status = 0; break; }
        if (omega == 0.0L) { *status = 2; break; }
    }
    for (int64_t i = 0; i < n; ++i) x_out[i] = (double)x[i];
    free(x); free(r); free(rh); free(p); free(v); free(s); free(t);
    return it;
}
