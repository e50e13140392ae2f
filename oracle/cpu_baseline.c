/* Timed CPU baseline of the PageRank workload -- BENCHMARK INFRASTRUCTURE ONLY.
 *
 * Only the benchmark's CPU-baseline leg calls this file; the product path
 * never does, and the parity tests use the checker functions of
 * merbit_oracle.c instead (long-double sums, sequential).  This is the
 * timed variant: the same power method (Sec. 5.5.1) as the oracle's
 * or_pagerank, on the same CSR (rows = destinations, columns without
 * nonzeros dangling, their mass spread uniformly), with plain double
 * accumulation, row-parallel with OpenMP when threads > 1.  It shares no
 * code with the HIP library.
 *
 *     x_{t+1}[r] = alpha sum_k values[k] x_t[col[k]] + (alpha sum_{u dangling} x_t[u] + 1 - alpha) / n
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>

/* iters power-method steps from x (n doubles, overwritten with x_iters).
 * threads <= 0: OpenMP's default team size.  Returns the number of threads
 * the row loop ran with, or -1 if memory ran out. */
int cb_pagerank(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* values,
                double alpha, int iters, double* x, int threads) {
    const int64_t m = row_ptr[n];
    unsigned char* has_out = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
    double* buf = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!has_out || !buf) {
        free(has_out);
        free(buf);
        return -1;
    }
    if (threads <= 0) threads = omp_get_max_threads();
    for (int64_t k = 0; k < m; ++k) has_out[col[k]] = 1;
    double* cur = x;
    double* nxt = buf;
    int used = 1;
    for (int t = 0; t < iters; ++t) {
        double dangling = 0.0;
#pragma omp parallel for num_threads(threads) reduction(+ : dangling) schedule(static)
        for (int64_t u = 0; u < n; ++u)
            if (!has_out[u]) dangling += cur[u];
        const double teleport = (alpha * dangling + 1.0 - alpha) / (double)n;
#pragma omp parallel num_threads(threads)
        {
#pragma omp single
            used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 4096)
            for (int64_t r = 0; r < n; ++r) {
                double s = 0.0;
                for (int32_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) s += values[k] * cur[col[k]];
                nxt[r] = alpha * s + teleport;
            }
        }
        double* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    if (cur != x)
        for (int64_t r = 0; r < n; ++r) x[r] = cur[r];
    free(has_out);
    free(buf);
    return used;
}
