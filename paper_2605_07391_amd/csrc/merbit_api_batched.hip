// C ABI of libmerbit, batched forms: SpMM over up to 64 right-hand sides per
// launch and personalised PageRank for many sources at once.
#include <math.h>
#include <string.h>

#include "merbit_host.hpp"

using namespace merbit;

extern "C" {

static SpmmArgs spmm_args(const merbit_plan* p, const void* X, int64_t ldx, void* Y,
                          int64_t ldy, void* Z, int64_t ldz, int k) {
  SpmmArgs a;
  a.tile_x = p->tile_x;
  a.tile_y = p->tile_y;
  a.lane_desc = p->lane_desc;
  a.col = p->col;
  a.val = p->values;
  a.X = X;
  a.Y = Y;
  a.Z = Z;
  a.ldx = ldx;
  a.ldy = ldy;
  a.ldz = ldz;
  a.x_rows = p->n_cols;
  a.k = k;
  a.tile_num = (int32_t)p->tile_num;
  a.lane_num = (int32_t)p->lane_num;
  a.path_len = (int32_t)(p->nnz + p->n_rows);
  a.n_rows = (int32_t)p->n_rows;
  a.Xn = nullptr;  // plain Y = A X
  a.src = nullptr;
  a.sums_in = nullptr;
  a.dmask = nullptr;
  a.part = nullptr;
  a.alpha = 0.0;
  a.col0 = 0;
  a.dmask_words = 0;
  return a;
}

// One SpMM launch per slab of at most kSlab columns, the slabs one after
// another; the whole call is bracketed by one pair of events when profiling
// is on.  64 columns of R-MAT 22 took, as 1 / 2 / 4 launches: FP32 2.89 /
// 2.53 / 13.7 ms (as many L2 misses and bytes read in the 2 launches as in
// the 1: the misses are served faster), FP64 6.2 / 5.4 / 9.1 ms.

static int run_spmm(merbit_plan* p, const void* X, int64_t ldx, void* Y, int64_t ldy, void* Z,
                    int64_t ldz, int k, hipStream_t st) {
  const size_t vs = vsize(p->dtype);
  const int slab = kSlab;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (p->profiling) {
    if (p->events_used == p->events.size()) {
      hipEvent_t a, b;
      HIP_TRY(hipEventCreate(&a));
      HIP_TRY(hipEventCreate(&b));
      p->events.emplace_back(a, b);
    }
    e0 = p->events[p->events_used].first;
    e1 = p->events[p->events_used].second;
    ++p->events_used;
    HIP_TRY(hipEventRecord(e0, st));
  }
  for (int c0 = 0; c0 < k; c0 += slab) {
    const int kk = k - c0 < slab ? k - c0 : slab;
    HIP_TRY(launch_spmm(p->dtype, p->sigma,
                        spmm_args(p, static_cast<const char*>(X) + vs * c0, ldx,
                                  static_cast<char*>(Y) + vs * c0, ldy,
                                  Z ? static_cast<char*>(Z) + vs * c0 : nullptr, ldz, kk),
                        st));
  }
  if (p->profiling) HIP_TRY(hipEventRecord(e1, st));
  p->last_stream = st;
  return MERBIT_OK;
}

int merbit_spmm(merbit_plan* p, const void* X, int64_t ldx, void* Y, int64_t ldy, int k,
                void* stream) try {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->stripes > 1) return fail(MERBIT_EUNSUPPORTED, "not available on a striped plan");
  if (p->desc_bits != 32)
    return fail(MERBIT_EUNSUPPORTED, "this call needs a plan with 32-bit descriptors");
  if (k < 1) return fail(MERBIT_EINVAL, "k < 1");
  if (ldx < k || ldy < k) return fail(MERBIT_EINVAL, "leading dimension < k");
  if (p->n_rows == 0) return MERBIT_OK;
  if (!Y || (p->nnz > 0 && !X)) return fail(MERBIT_EINVAL, "X or Y is NULL");
  if (X == Y) return fail(MERBIT_EINVAL, "X and Y alias");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t vs = vsize(p->dtype);
  for (int c0 = 0; c0 < k; c0 += 64) {
    const int kk = k - c0 < 64 ? k - c0 : 64;
    HIP_TRY(launch_spmm_zero(p->dtype, p->tile_y, (int32_t)p->tile_num,
                             static_cast<char*>(Y) + vs * c0, ldy, kk, st));
  }
  return run_spmm(p, X, ldx, Y, ldy, nullptr, 0, k, st);
} catch (...) {
  return merbit::host_exception();
}

int merbit_spmm_dual(merbit_plan* p, const void* X, int64_t ldx, void* Y, int64_t ldy, void* Z,
                     int64_t ldz, int k, void* stream) try {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->stripes > 1) return fail(MERBIT_EUNSUPPORTED, "not available on a striped plan");
  if (p->desc_bits != 32)
    return fail(MERBIT_EUNSUPPORTED, "this call needs a plan with 32-bit descriptors");
  if (k < 1) return fail(MERBIT_EINVAL, "k < 1");
  if (ldx < k || ldy < k || ldz < k) return fail(MERBIT_EINVAL, "leading dimension < k");
  if (p->n_rows == 0) return MERBIT_OK;
  if (!Y || !Z || (p->nnz > 0 && !X)) return fail(MERBIT_EINVAL, "X, Y or Z is NULL");
  if (X == Y || Y == Z || X == Z) return fail(MERBIT_EINVAL, "X, Y, Z must be distinct");
  return run_spmm(p, X, ldx, Y, ldy, Z, ldz, k, static_cast<hipStream_t>(stream));
} catch (...) {
  return merbit::host_exception();
}

int merbit_spmm_zero_boundary(merbit_plan* p, void* Y, int64_t ldy, int k, void* stream) try {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->stripes > 1) return fail(MERBIT_EUNSUPPORTED, "not available on a striped plan");
  if (k < 1 || ldy < k) return fail(MERBIT_EINVAL, "bad k / leading dimension");
  if (p->tile_num == 0) return MERBIT_OK;
  if (!Y) return fail(MERBIT_EINVAL, "Y is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t vs = vsize(p->dtype);
  for (int c0 = 0; c0 < k; c0 += 64) {
    const int kk = k - c0 < 64 ? k - c0 : 64;
    HIP_TRY(launch_spmm_zero(p->dtype, p->tile_y, (int32_t)p->tile_num,
                             static_cast<char*>(Y) + vs * c0, ldy, kk, st));
  }
  p->last_stream = st;
  return MERBIT_OK;
} catch (...) {
  return merbit::host_exception();
}

// Buffers of the personalised PageRank, all in the slab layout of its
// kernels (merbit_batched.hip): pbuf[0] holds A X at the tiles' first rows
// (zero there between steps), pbuf[1] (k > kSlab only: the caller's
// row-major array is then converted) and pbuf[2] the iterates; ppart the
// per-block parts of one step (the SpMM's blocks, then the first-row
// fix-up's, then the l1 change's, then the first level of their sum).
static int ensure_ppr_state(merbit_plan* p, int k, hipStream_t st) {
  int rc = ensure_dmask(p, st);
  if (rc != MERBIT_OK) return rc;
  if (p->ppr_k != k) {
    invalidate_graphs(p);
    for (int b = 0; b < 3; ++b) {
      if (p->pbuf[b]) (void)hipFree(p->pbuf[b]);
      p->pbuf[b] = nullptr;
    }
    const size_t bytes = vsize(p->dtype) * (size_t)p->n_rows * (size_t)k;
    HIP_TRY(hipMalloc(&p->pbuf[0], bytes));
    if (k > kSlab) HIP_TRY(hipMalloc(&p->pbuf[1], bytes));
    HIP_TRY(hipMalloc(&p->pbuf[2], bytes));
    p->ppr_k = k;
    p->ppr_zeroed = -1;
  }
  if (!p->ppart) {
    p->ppr_grid_n = ppr_grid(p->n_rows);
    // the step's parts, then the first level of their sum
    const size_t rows = (size_t)spmm_blocks(p->tile_num) + (size_t)ppr_fixup_grid(p->tile_num) +
                        (size_t)p->ppr_grid_n + (size_t)ppr_sum_scratch_rows();
    HIP_TRY(hipMalloc(&p->ppart, sizeof(double) * 2 * 64 * rows));
    HIP_TRY(hipMalloc(&p->psums[0], sizeof(double) * 2 * 64));
    HIP_TRY(hipMalloc(&p->psums[1], sizeof(double) * 2 * 64));
    HIP_TRY(hipMalloc(&p->psrc, sizeof(int32_t) * 64));
  }
  return MERBIT_OK;
}

// One personalised-PageRank step X -> Xn (kernels in merbit_batched.hip):
// the SpMM slabs with the rows inside tiles finished in their commit, the
// tiles' first rows, on request the l1 change, and the per-column sums of
// the parts into sums_out.  The SpMM launches are bracketed by one pair of
// events when profiling is on.
static int ppr_step(merbit_plan* p, const void* X, void* Xn, int k, double alpha,
                    const double* sums_in, double* sums_out, bool resid, hipStream_t st) {
  const size_t vs = vsize(p->dtype);
  const int64_t n = p->n_rows;
  const int sb = spmm_blocks(p->tile_num), fb = ppr_fixup_grid(p->tile_num);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (p->profiling) {
    if (p->events_used == p->events.size()) {
      hipEvent_t a, b;
      HIP_TRY(hipEventCreate(&a));
      HIP_TRY(hipEventCreate(&b));
      p->events.emplace_back(a, b);
    }
    e0 = p->events[p->events_used].first;
    e1 = p->events[p->events_used].second;
    ++p->events_used;
    HIP_TRY(hipEventRecord(e0, st));
  }
  for (int c0 = 0; c0 < k; c0 += kSlab) {
    const int kk = k - c0 < kSlab ? k - c0 : kSlab;
    const size_t off = vs * (size_t)c0 * (size_t)n;  // the slab's n x kk block
    SpmmArgs a = spmm_args(p, static_cast<const char*>(X) + off, kk,
                           static_cast<char*>(p->pbuf[0]) + off, kk, nullptr, 0, kk);
    a.Xn = static_cast<char*>(Xn) + off;
    a.src = p->psrc + c0;
    a.sums_in = sums_in + 2 * c0;
    a.dmask = p->dmask;
    a.part = p->ppart;
    a.alpha = alpha;
    a.col0 = c0;
    a.dmask_words = (int32_t)((n + 31) / 32);
    HIP_TRY(launch_spmm(p->dtype, p->sigma, a, st));
  }
  if (p->profiling) HIP_TRY(hipEventRecord(e1, st));
  HIP_TRY(launch_ppr_fixup(p->dtype, p->tile_y, (int32_t)p->tile_num, p->pbuf[0], Xn, n, k,
                           alpha, p->psrc, sums_in, p->dmask, p->ppart + (size_t)sb * 128, fb,
                           st));
  int nb = sb + fb;
  if (resid) {
    HIP_TRY(launch_ppr_resid(p->dtype, Xn, X, n, k, p->ppart + (size_t)nb * 128, p->ppr_grid_n,
                             st));
    nb += p->ppr_grid_n;
  }
  HIP_TRY(launch_ppr_sum(p->ppart, nb, k, sums_out,
                         p->ppart + (size_t)(sb + fb + p->ppr_grid_n) * 128, st));
  p->last_stream = st;
  return MERBIT_OK;
}

int merbit_pagerank_personalized(merbit_plan* p, double alpha, double tol, int max_iter,
                                 int check_every, const int32_t* sources, int k, void* X_inout,
                                 int* iters_out, double* resid_out, void* stream) try {
  if (iters_out) *iters_out = 0;
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->stripes > 1) return fail(MERBIT_EUNSUPPORTED, "not available on a striped plan");
  if (p->desc_bits != 32)
    return fail(MERBIT_EUNSUPPORTED, "this call needs a plan with 32-bit descriptors");
  if (p->n_rows != p->n_cols) return fail(MERBIT_EINVAL, "PageRank needs a square matrix");
  if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(MERBIT_EINVAL, "alpha must be in [0, 1]");
  if (k < 1 || k > 64) return fail(MERBIT_EINVAL, "k must be in 1..64");
  if (max_iter < 0) return fail(MERBIT_EINVAL, "max_iter < 0");
  if (!sources) return fail(MERBIT_EINVAL, "sources is NULL");
  for (int j = 0; j < k; ++j)
    if (sources[j] < 0 || sources[j] >= p->n_rows)
      return fail(MERBIT_EINVAL, "source out of range");
  if (resid_out)
    for (int j = 0; j < k; ++j) resid_out[j] = 0.0;
  if (p->n_rows == 0 || max_iter == 0) return MERBIT_OK;
  if (!X_inout) return fail(MERBIT_EINVAL, "X is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = ensure_ppr_state(p, k, st);
  if (rc != MERBIT_OK) return rc;
  if (check_every <= 0) check_every = 10;
  const int64_t n = p->n_rows;
  const size_t bytes = vsize(p->dtype) * (size_t)n * (size_t)k;
  HIP_TRY(hipMemcpyAsync(p->psrc, sources, sizeof(int32_t) * (size_t)k, hipMemcpyHostToDevice,
                         st));
  // k <= kSlab: the slab layout is the caller's, and X_inout is the first
  // iterate buffer itself
  const bool convert = k > kSlab;
  void* xs[2] = {convert ? p->pbuf[1] : X_inout, p->pbuf[2]};
  if (convert)
    HIP_TRY(launch_ppr_to_slabs(p->dtype, X_inout, xs[0], p->dmask, n, k, p->ppart,
                                p->psums[0], p->ppr_grid_n, st));
  else
    HIP_TRY(launch_ppr_dangling(p->dtype, xs[0], p->dmask, n, k, p->ppart, p->psums[0],
                                p->ppr_grid_n, st));
  if (p->ppr_zeroed < 0) {  // A X's buffer: zero at the tiles' first rows
    for (int c0 = 0; c0 < k; c0 += kSlab) {
      const int kk = k - c0 < kSlab ? k - c0 : kSlab;
      HIP_TRY(launch_spmm_zero(p->dtype, p->tile_y, (int32_t)p->tile_num,
                               static_cast<char*>(p->pbuf[0]) + vsize(p->dtype) * c0 * n, kk,
                               kk, st));
    }
    p->ppr_zeroed = 0;
  }
  double host_sums[128];
  int t = 0;
  bool converged = false;
  while (t < max_iter) {
    int len = check_every - t % check_every;
    if (len > max_iter - t) len = max_iter - t;
    const int t0 = t;
    // the l1 change is computed on the chunk's last step only (the host
    // reads it after the chunk)
    auto enqueue = [&](hipStream_t s) -> int {
      for (int i = 0; i < len; ++i) {
        const int cur = (t0 + i) & 1;
        const int r = ppr_step(p, xs[cur], xs[cur ^ 1], k, alpha, p->psums[cur],
                               p->psums[cur ^ 1], i == len - 1, s);
        if (r != MERBIT_OK) return r;
      }
      return MERBIT_OK;
    };
    rc = len == check_every
             ? run_chunk(p, kLoopPersonalized, t0 & 1, 0, len, k, X_inout, alpha, enqueue, st)
             : enqueue(st);
    if (rc != MERBIT_OK) return rc;
    t += len;
    if (tol > 0.0 || t == max_iter) {
      HIP_TRY(hipMemcpyAsync(host_sums, p->psums[t & 1], sizeof host_sums,
                             hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      double worst = 0.0;
      for (int j = 0; j < k; ++j) {
        if (resid_out) resid_out[j] = host_sums[2 * j + 1];
        if (host_sums[2 * j + 1] > worst) worst = host_sums[2 * j + 1];
      }
      if (tol > 0.0 && worst < tol) {
        converged = true;
        break;
      }
    }
  }
  p->last_stream = st;
  if (convert)
    HIP_TRY(launch_ppr_from_slabs(p->dtype, xs[t & 1], X_inout, n, k, st));
  else if (t & 1)
    HIP_TRY(hipMemcpyAsync(X_inout, p->pbuf[2], bytes, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (iters_out) *iters_out = t;
  return (tol > 0.0 && !converged) ? MERBIT_NOT_CONVERGED : MERBIT_OK;
} catch (...) {
  return merbit::host_exception();
}

// Row-chunk tables for the graphs of graph_ptr (rebuilt when it changes).

}  // extern "C"
