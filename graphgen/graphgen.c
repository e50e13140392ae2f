/*
 * Seeded synthetic sparse-matrix generators (host only).
 *
 * These build the inputs that both the CPU oracle and the HIP library are
 * checked on.  They hold none of the SpMV or merge-path arithmetic: they only
 * draw graphs, turn them into CSR with merged duplicates, and draw the value
 * and vector streams.
 *
 * Random numbers.  Every draw is counter based, so any entry can be produced
 * independently of all others and the generators parallelise without changing
 * their output.  A draw is identified by (seed, stream, index):
 *     key   = mix64(seed + stream * G)
 *     bits  = mix64(key + (index + 1) * G)            G = 0x9E3779B97F4A7C15
 *     u01   = (bits >> 11) * 2^-53                     in [0, 1)
 * where mix64 is the output function of Vigna's SplitMix64 generator
 * (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014; constants as published by Vigna at prng.di.unimi.it).
 *
 * Orientation.  A drawn edge u -> v becomes the nonzero (row v, column u):
 * rows are destinations, as in the column-stochastic PageRank matrix.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define GG_GOLDEN 0x9E3779B97F4A7C15ULL

enum {
    GG_STREAM_RMAT = 1,
    GG_STREAM_EMPTY = 2,
    GG_STREAM_HUB_ROW = 3,
    GG_STREAM_CL_SRC = 10,
    GG_STREAM_CL_DST = 11,
    GG_STREAM_CL_EMPTY = 12,
    GG_STREAM_HUB_COL = 100 /* + hub number */
};

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t gg_key(uint64_t seed, uint64_t stream) {
    return mix64(seed + stream * GG_GOLDEN);
}

static inline double gg_u01_k(uint64_t key, uint64_t index) {
    uint64_t bits = mix64(key + (index + 1) * GG_GOLDEN);
    return (double)(bits >> 11) * (1.0 / 9007199254740992.0);
}

/* Public: uniform doubles in [lo, hi) (closed_high = 0) or (lo, hi]
 * (closed_high = 1, drawn as hi - (hi - lo) * u). */
void gg_uniform(uint64_t seed, uint64_t stream, int64_t count, double lo, double hi,
                int closed_high, double* out) {
    const uint64_t key = gg_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        double u = gg_u01_k(key, (uint64_t)i);
        out[i] = closed_high ? hi - (hi - lo) * u : lo + (hi - lo) * u;
    }
}

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* Sort every row's column list and drop repeated columns.
 * raw_ptr/raw_col hold the unsorted buckets; the merged CSR goes to
 * row_ptr/col_out.  Returns the merged nonzero count. */
static int64_t sort_merge_rows(int64_t n, const int64_t* raw_ptr, int32_t* raw_col,
                               int32_t* row_ptr, int32_t* col_out) {
    int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!cnt) return -1;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t r = 0; r < n; ++r) {
        int64_t b = raw_ptr[r], e = raw_ptr[r + 1];
        if (e - b > 1) qsort(raw_col + b, (size_t)(e - b), sizeof(int32_t), cmp_i32);
        int64_t u = 0;
        for (int64_t k = b; k < e; ++k)
            if (k == b || raw_col[k] != raw_col[k - 1]) ++u;
        cnt[r] = u;
    }
    int64_t acc = 0;
    for (int64_t r = 0; r < n; ++r) {
        row_ptr[r] = (int32_t)acc;
        acc += cnt[r];
    }
    row_ptr[n] = (int32_t)acc;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t r = 0; r < n; ++r) {
        int64_t b = raw_ptr[r], e = raw_ptr[r + 1], o = row_ptr[r];
        for (int64_t k = b; k < e; ++k)
            if (k == b || raw_col[k] != raw_col[k - 1]) col_out[o++] = raw_col[k];
    }
    free(cnt);
    return acc;
}

/* One R-MAT edge: at each of `scale` levels pick a quadrant with
 * probabilities (a, b, c, 1-a-b-c) for (src bit, dst bit) =
 * (0,0), (0,1), (1,0), (1,1); bits are filled from the most significant. */
static inline void rmat_edge(uint64_t key, int scale, int64_t e, double a, double ab,
                             double abc, int32_t* src, int32_t* dst) {
    uint32_t s = 0, d = 0;
    for (int l = 0; l < scale; ++l) {
        double u = gg_u01_k(key, (uint64_t)e * (uint64_t)scale + (uint64_t)l);
        uint32_t sb, db;
        if (u < a) { sb = 0; db = 0; }
        else if (u < ab) { sb = 0; db = 1; }
        else if (u < abc) { sb = 1; db = 0; }
        else { sb = 1; db = 1; }
        s = (s << 1) | sb;
        d = (d << 1) | db;
    }
    *src = (int32_t)s;
    *dst = (int32_t)d;
}

/* R-MAT graph with 2^scale vertices and `nedges` draws, duplicates merged,
 * no noise and no vertex relabelling.  Output: CSR with rows = destinations
 * (row_ptr has 2^scale + 1 entries; col_out needs room for nedges entries).
 * Returns the merged nonzero count, or -1 on allocation failure. */
int64_t gg_rmat(int scale, int64_t nedges, double a, double b, double c, uint64_t seed,
                int32_t* row_ptr, int32_t* col_out) {
    const int64_t n = (int64_t)1 << scale;
    const uint64_t key = gg_key(seed, GG_STREAM_RMAT);
    const double ab = a + b, abc = a + b + c;
    int64_t* raw_ptr = (int64_t*)calloc((size_t)(n + 1), sizeof(int64_t));
    int32_t* raw_col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nedges > 0 ? nedges : 1));
    if (!raw_ptr || !raw_col) { free(raw_ptr); free(raw_col); return -1; }
    /* pass 1: count edges per destination row */
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nedges; ++e) {
        int32_t s, d;
        rmat_edge(key, scale, e, a, ab, abc, &s, &d);
        __atomic_fetch_add(&raw_ptr[d + 1], 1, __ATOMIC_RELAXED);
    }
    for (int64_t r = 0; r < n; ++r) raw_ptr[r + 1] += raw_ptr[r];
    int64_t* cursor = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!cursor) { free(raw_ptr); free(raw_col); return -1; }
    memcpy(cursor, raw_ptr, sizeof(int64_t) * (size_t)n);
    /* pass 2: redraw each edge and drop its source into the row bucket */
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nedges; ++e) {
        int32_t s, d;
        rmat_edge(key, scale, e, a, ab, abc, &s, &d);
        int64_t pos = __atomic_fetch_add(&cursor[d], 1, __ATOMIC_RELAXED);
        raw_col[pos] = s;
    }
    free(cursor);
    int64_t nnz = sort_merge_rows(n, raw_ptr, raw_col, row_ptr, col_out);
    free(raw_ptr);
    free(raw_col);
    return nnz;
}

/* Stress modification of a CSR pattern (n rows, n_cols columns):
 *  1. every row r with u(EMPTY, r) < empty_frac is cleared;
 *  2. n_hubs distinct rows that were not cleared are drawn (u(HUB_ROW, i)*n,
 *     i = 0, 1, ... skipping cleared or already chosen rows) and each is
 *     replaced by hub_nnz distinct uniformly chosen columns, sorted
 *     (Knuth's selection sampling, Algorithm S, over the n_cols columns).
 * hub_rows_out receives the chosen rows.  col_out needs room for
 * nnz_in + n_hubs * hub_nnz entries.  Returns the new nonzero count. */
int64_t gg_stress(int64_t n, int64_t n_cols, const int32_t* row_ptr_in, const int32_t* col_in,
                  uint64_t seed, double empty_frac, int n_hubs, int64_t hub_nnz,
                  int32_t* row_ptr, int32_t* col_out, int32_t* hub_rows_out) {
    const uint64_t kempty = gg_key(seed, GG_STREAM_EMPTY);
    const uint64_t khub = gg_key(seed, GG_STREAM_HUB_ROW);
    unsigned char* kind = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1); /* 0 keep, 1 empty, 2 hub */
    if (!kind) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r)
        if (gg_u01_k(kempty, (uint64_t)r) < empty_frac) kind[r] = 1;
    int chosen = 0;
    const uint64_t max_draws = 64u * (uint64_t)n + 1024u; /* ends even if too few rows remain */
    for (uint64_t i = 0; chosen < n_hubs && n > 0 && i < max_draws; ++i) {
        int64_t r = (int64_t)(gg_u01_k(khub, i) * (double)n);
        if (r >= n) r = n - 1;
        if (kind[r] != 0) continue;
        kind[r] = 2;
        hub_rows_out[chosen++] = (int32_t)r;
    }
    /* new row lengths */
    int64_t acc = 0;
    for (int64_t r = 0; r < n; ++r) {
        row_ptr[r] = (int32_t)acc;
        int64_t len = kind[r] == 0 ? (int64_t)(row_ptr_in[r + 1] - row_ptr_in[r])
                      : kind[r] == 2 ? hub_nnz : 0;
        acc += len;
    }
    row_ptr[n] = (int32_t)acc;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t r = 0; r < n; ++r) {
        int64_t o = row_ptr[r];
        if (kind[r] == 0) {
            for (int64_t k = row_ptr_in[r]; k < row_ptr_in[r + 1]; ++k) col_out[o++] = col_in[k];
        }
    }
    /* hub rows: selection sampling keeps exactly hub_nnz sorted columns */
    for (int h = 0; h < chosen; ++h) {
        int64_t r = hub_rows_out[h];
        const uint64_t kc = gg_key(seed, GG_STREAM_HUB_COL + (uint64_t)h);
        int64_t o = row_ptr[r], need = hub_nnz;
        for (int64_t cidx = 0; cidx < n_cols && need > 0; ++cidx) {
            double u = gg_u01_k(kc, (uint64_t)cidx);
            if ((double)(n_cols - cidx) * u < (double)need) {
                col_out[o++] = (int32_t)cidx;
                --need;
            }
        }
    }
    free(kind);
    return acc;
}

/* Directed Chung-Lu graph on n vertices from `nedges` independent draws.
 * Source weights follow a power law, w_out(i) = (i + 1)^(-1/(gamma - 1));
 * target weights are 1, except for vertices with u(CL_EMPTY, i) < empty_frac,
 * which get weight 0 (so their rows stay empty).  Draw e picks a source in
 * proportion to w_out (inverse CDF by binary search) and a target uniformly
 * among the vertices of weight 1.  Duplicates are merged.
 * col_out needs room for nedges entries.  Returns the nonzero count. */
int64_t gg_chung_lu(int64_t n, int64_t nedges, double gamma_out, double empty_frac,
                    uint64_t seed, int32_t* row_ptr, int32_t* col_out) {
    const uint64_t ksrc = gg_key(seed, GG_STREAM_CL_SRC);
    const uint64_t kdst = gg_key(seed, GG_STREAM_CL_DST);
    const uint64_t kemp = gg_key(seed, GG_STREAM_CL_EMPTY);
    double* cdf = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int32_t* targets = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t* raw_ptr = (int64_t*)calloc((size_t)(n + 1), sizeof(int64_t));
    int32_t* raw_col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nedges > 0 ? nedges : 1));
    int32_t* esrc = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nedges > 0 ? nedges : 1));
    int32_t* edst = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nedges > 0 ? nedges : 1));
    if (!cdf || !targets || !raw_ptr || !raw_col || !esrc || !edst) {
        free(cdf); free(targets); free(raw_ptr); free(raw_col); free(esrc); free(edst);
        return -1;
    }
    const double expo = -1.0 / (gamma_out - 1.0);
    double total = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        total += pow((double)(i + 1), expo);
        cdf[i] = total;
    }
    int64_t nt = 0;
    for (int64_t i = 0; i < n; ++i)
        if (!(gg_u01_k(kemp, (uint64_t)i) < empty_frac)) targets[nt++] = (int32_t)i;
    if (nt == 0) nedges = 0;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nedges; ++e) {
        double us = gg_u01_k(ksrc, (uint64_t)e) * total;
        int64_t lo = 0, hi = n - 1; /* first i with cdf[i] > us */
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (cdf[mid] > us) hi = mid; else lo = mid + 1;
        }
        int64_t ti = (int64_t)(gg_u01_k(kdst, (uint64_t)e) * (double)nt);
        if (ti >= nt) ti = nt - 1;
        esrc[e] = (int32_t)lo;
        edst[e] = targets[ti];
    }
    for (int64_t e = 0; e < nedges; ++e) raw_ptr[edst[e] + 1]++;
    for (int64_t r = 0; r < n; ++r) raw_ptr[r + 1] += raw_ptr[r];
    {
        int64_t* cursor = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        if (!cursor) { nedges = -1; }
        else {
            memcpy(cursor, raw_ptr, sizeof(int64_t) * (size_t)n);
            for (int64_t e = 0; e < nedges; ++e) raw_col[cursor[edst[e]]++] = esrc[e];
            free(cursor);
        }
    }
    int64_t nnz = nedges < 0 ? -1 : sort_merge_rows(n, raw_ptr, raw_col, row_ptr, col_out);
    free(cdf); free(targets); free(raw_ptr); free(raw_col); free(esrc); free(edst);
    return nnz;
}

int gg_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
