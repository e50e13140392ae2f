// C ABI of libmerbit, iterative drivers: PageRank (Sec. 5.5.1), PageRank of
// many graphs on one diagonal, the PageRank adjoint fixed point and BiCGSTAB
// (Sec. 5.5.2), each looping over the plan's fused SpMV with iteration chunks
// recorded into HIP graphs.
#include <math.h>
#include <algorithm>
#include <string.h>

#include "merbit_host.hpp"

using namespace merbit;

namespace merbit {

int pagerank_loop(merbit_plan* p, PageRankWork& w, double alpha, double tol, int max_iter,
                  int check_every, void* x_inout, int* iters_out, double* resid_out,
                  hipStream_t st) {
  if (check_every <= 0) check_every = 10;
  const int64_t n = p->n_rows;
  const size_t vb = vsize(p->dtype) * (size_t)n;
  int rc;

  // delta_0: per-block dangling mass of x_0 into partials[0]
  HIP_TRY(launch_dangling_sum(p->dtype, x_inout, w.dmask, n, w.partials[0], w.reduce_grid, st));
  int yb = w.zeroed_buf;
  if (yb < 0) {
    yb = 0;
    rc = zero_boundary(p, w.ybuf[0], st);
    if (rc != MERBIT_OK) return rc;
  }
  void* xs[2] = {x_inout, w.xwork};
  int t = 0;
  double resid = 0.0;
  bool converged = false;
  while (t < max_iter) {
    // iterations up to the next check (or max_iter), as one chunk
    int len = check_every - t % check_every;
    if (len > max_iter - t) len = max_iter - t;
    const int t0 = t, yb0 = yb;
    // with a partial hot-column cache the update also writes the next
    // iterate's hot values, so only the call's first SpMV gathers them
    const bool fuse_hot = p->hot_n > 0 && !p->hot_all;
    auto enqueue = [&](hipStream_t s) -> int {
      for (int i = 0; i < len; ++i) {
        const int cur = (t0 + i) & 1, b = yb0 ^ (i & 1);
        const int r = run_fused(p, xs[cur], w.ybuf[b], w.ybuf[b ^ 1], s,
                                fuse_hot && t0 + i > 0, w.timed);
        if (r != MERBIT_OK) return r;
        // the l1 change only on the chunk's last step (the host reads it
        // after the chunk)
        HIP_TRY(launch_pr_update(p->dtype, w.ybuf[b], xs[cur], xs[cur ^ 1], w.dmask, n, alpha,
                                 w.partials[cur], w.reduce_grid, w.partials[cur ^ 1],
                                 w.reduce_grid, s, fuse_hot ? p->hot_cols : nullptr,
                                 fuse_hot ? p->hot_n : 0, fuse_hot ? p->x_hot : nullptr,
                                 i == len - 1));
      }
      return MERBIT_OK;
    };
    // the call's first chunk gathers the hot values, later ones do not: a
    // different graph (key k = 1 for the first chunk)
    rc = w.graphs && len == check_every
             ? run_chunk(p, kLoopPageRank, t0 & 1, yb0, len, t0 == 0 ? 1 : 0, x_inout, alpha,
                         enqueue, st)
             : enqueue(st);
    if (rc != MERBIT_OK) return rc;
    t += len;
    yb ^= len & 1;
    if (tol > 0.0 || t == max_iter) {
      // l1 change of this iteration: sum of the blocks' second components
      HIP_TRY(hipMemcpyAsync(w.host_pairs, w.partials[t & 1],
                             sizeof(double) * 2 * (size_t)w.reduce_grid, hipMemcpyDeviceToHost,
                             st));
      HIP_TRY(hipStreamSynchronize(st));
      resid = 0.0;
      for (int b = 0; b < w.reduce_grid; ++b) resid += w.host_pairs[2 * (size_t)b + 1];
      if (tol > 0.0 && resid < tol) {
        converged = true;
        break;
      }
    }
  }
  w.zeroed_buf = yb;
  p->last_stream = st;
  if (t & 1) HIP_TRY(hipMemcpyAsync(x_inout, w.xwork, vb, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (iters_out) *iters_out = t;
  if (resid_out) *resid_out = resid;
  return (tol > 0.0 && !converged) ? MERBIT_NOT_CONVERGED : MERBIT_OK;
}

}  // namespace merbit

extern "C" {

int merbit_pagerank(merbit_plan* p, double alpha, double tol, int max_iter, int check_every,
                    void* x_inout, int* iters_out, double* resid_out, void* stream) try {
  if (iters_out) *iters_out = 0;
  if (resid_out) *resid_out = 0.0;
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->n_rows != p->n_cols) return fail(MERBIT_EINVAL, "PageRank needs a square matrix");
  if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(MERBIT_EINVAL, "alpha must be in [0, 1]");
  if (max_iter < 0) return fail(MERBIT_EINVAL, "max_iter < 0");
  if (p->n_rows == 0 || max_iter == 0) return MERBIT_OK;
  if (!x_inout) return fail(MERBIT_EINVAL, "x is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = ensure_pagerank_state(p, st);
  if (rc != MERBIT_OK) return rc;
  std::vector<double> host_pairs(2 * (size_t)p->reduce_grid);
  PageRankWork w;
  w.ybuf[0] = p->ybuf[0];
  w.ybuf[1] = p->ybuf[1];
  w.xwork = p->xwork;
  w.partials[0] = p->partials[0];
  w.partials[1] = p->partials[1];
  w.dmask = p->dmask;
  w.reduce_grid = p->reduce_grid;
  w.zeroed_buf = p->zeroed_buf;
  w.graphs = true;
  w.timed = true;
  w.host_pairs = host_pairs.data();
  rc = pagerank_loop(p, w, alpha, tol, max_iter, check_every, x_inout, iters_out, resid_out, st);
  p->zeroed_buf = w.zeroed_buf;
  return rc;
} catch (...) {
  return merbit::host_exception();
}

static int ensure_multi_tables(merbit_plan* p, const int64_t* graph_ptr, int n_graphs,
                               hipStream_t st) {
  std::vector<int64_t> gp(graph_ptr, graph_ptr + n_graphs + 1);
  if (gp == p->multi_gp && p->multi_part) return MERBIT_OK;
  const int64_t R = multi_chunk_rows();
  std::vector<int32_t> chunk_row, chunk_graph, chunk_ptr(1, 0);
  std::vector<double> gsize(n_graphs);
  for (int g = 0; g < n_graphs; ++g) {
    for (int64_t r = gp[g]; r < gp[g + 1]; r += R) {
      chunk_row.push_back((int32_t)r);
      chunk_graph.push_back(g);
    }
    chunk_ptr.push_back((int32_t)chunk_row.size());
    gsize[g] = (double)(gp[g + 1] - gp[g]);
  }
  chunk_row.push_back((int32_t)gp[n_graphs]);
  // the graph of each hot column slot, for the update's copy of the hot
  // values (a partial cache only)
  std::vector<int32_t> hot_graph;
  if (p->hot_n > 0 && !p->hot_all) {
    hot_graph.resize((size_t)p->hot_n);
    HIP_TRY(hipMemcpy(hot_graph.data(), p->hot_cols, sizeof(int32_t) * (size_t)p->hot_n,
                      hipMemcpyDeviceToHost));
    for (int32_t& h : hot_graph) {
      const int64_t c = h;
      if (c < 0 || c >= gp[n_graphs]) return fail(MERBIT_EINVAL, "hot column out of range");
      h = (int32_t)(std::upper_bound(gp.begin(), gp.end(), c) - gp.begin() - 1);
    }
  }
  void* old[] = {p->multi_chunk_row, p->multi_chunk_graph, p->multi_chunk_ptr, p->multi_gsize,
                 p->multi_part, p->multi_gsum[0], p->multi_gsum[1], p->multi_hot_graph};
  HIP_TRY(hipStreamSynchronize(st));  // earlier calls may still read the old tables
  invalidate_graphs(p);
  for (void* b : old)
    if (b) (void)hipFree(b);
  p->multi_chunk_row = p->multi_chunk_graph = p->multi_chunk_ptr = nullptr;
  p->multi_gsize = p->multi_part = p->multi_gsum[0] = p->multi_gsum[1] = nullptr;
  p->multi_hot_graph = nullptr;
  p->multi_gp.clear();
  const size_t C = chunk_graph.size();
  HIP_TRY(hipMalloc(&p->multi_chunk_row, sizeof(int32_t) * (C + 1)));
  HIP_TRY(hipMalloc(&p->multi_chunk_graph, sizeof(int32_t) * C));
  HIP_TRY(hipMalloc(&p->multi_chunk_ptr, sizeof(int32_t) * (size_t)(n_graphs + 1)));
  HIP_TRY(hipMalloc(&p->multi_gsize, sizeof(double) * (size_t)n_graphs));
  HIP_TRY(hipMalloc(&p->multi_part, sizeof(double) * 2 * C));
  HIP_TRY(hipMalloc(&p->multi_gsum[0], sizeof(double) * 2 * (size_t)n_graphs));
  HIP_TRY(hipMalloc(&p->multi_gsum[1], sizeof(double) * 2 * (size_t)n_graphs));
  HIP_TRY(hipMemcpy(p->multi_chunk_row, chunk_row.data(), sizeof(int32_t) * (C + 1),
                    hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->multi_chunk_graph, chunk_graph.data(), sizeof(int32_t) * C,
                    hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->multi_chunk_ptr, chunk_ptr.data(), sizeof(int32_t) * (n_graphs + 1),
                    hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->multi_gsize, gsize.data(), sizeof(double) * n_graphs,
                    hipMemcpyHostToDevice));
  if (!hot_graph.empty()) {
    HIP_TRY(hipMalloc(&p->multi_hot_graph, sizeof(int32_t) * hot_graph.size()));
    HIP_TRY(hipMemcpy(p->multi_hot_graph, hot_graph.data(), sizeof(int32_t) * hot_graph.size(),
                      hipMemcpyHostToDevice));
  }
  p->multi_chunks = (int32_t)C;
  p->multi_gp = gp;
  return MERBIT_OK;
}

int merbit_pagerank_multi(merbit_plan* p, const int64_t* graph_ptr, int n_graphs, double alpha,
                          double tol, int max_iter, int check_every, void* x_inout,
                          int* iters_out, double* resid_out, void* stream) try {
  if (iters_out) *iters_out = 0;
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->n_rows != p->n_cols) return fail(MERBIT_EINVAL, "PageRank needs a square matrix");
  if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(MERBIT_EINVAL, "alpha must be in [0, 1]");
  if (max_iter < 0) return fail(MERBIT_EINVAL, "max_iter < 0");
  if (!graph_ptr || n_graphs < 1) return fail(MERBIT_EINVAL, "graph_ptr is NULL or n_graphs < 1");
  if (graph_ptr[0] != 0 || graph_ptr[n_graphs] != p->n_rows)
    return fail(MERBIT_EINVAL, "graph_ptr must run from 0 to n");
  for (int g = 0; g < n_graphs; ++g)
    if (graph_ptr[g + 1] <= graph_ptr[g])
      return fail(MERBIT_EINVAL, "graph_ptr must be strictly increasing (no empty graph)");
  if (resid_out)
    for (int g = 0; g < n_graphs; ++g) resid_out[g] = 0.0;
  if (max_iter == 0) return MERBIT_OK;
  if (!x_inout) return fail(MERBIT_EINVAL, "x is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = ensure_pagerank_state(p, st);
  if (rc != MERBIT_OK) return rc;
  rc = ensure_multi_tables(p, graph_ptr, n_graphs, st);
  if (rc != MERBIT_OK) return rc;
  if (check_every <= 0) check_every = 10;
  MultiTables mt;
  mt.chunk_row = p->multi_chunk_row;
  mt.chunk_graph = p->multi_chunk_graph;
  mt.chunk_ptr = p->multi_chunk_ptr;
  mt.gsize = p->multi_gsize;
  mt.part = p->multi_part;
  mt.hot_graph = p->multi_hot_graph;
  mt.n_chunks = p->multi_chunks;
  mt.n_graphs = n_graphs;
  const size_t vb = vsize(p->dtype) * (size_t)p->n_rows;

  HIP_TRY(launch_multi_dangling(p->dtype, x_inout, p->dmask, mt, p->multi_gsum[0], st));
  int yb = p->zeroed_buf;
  if (yb < 0) {
    yb = 0;
    rc = zero_boundary(p, p->ybuf[0], st);
    if (rc != MERBIT_OK) return rc;
  }
  void* xs[2] = {x_inout, p->xwork};
  std::vector<double> host_sums(2 * (size_t)n_graphs);
  int t = 0;
  bool converged = false;
  while (t < max_iter) {
    int len = check_every - t % check_every;
    if (len > max_iter - t) len = max_iter - t;
    const int t0 = t, yb0 = yb;
    // with a partial hot-column cache the update also writes the next
    // iterate's hot values, so only the call's first SpMV gathers them
    const bool fuse_hot = p->hot_n > 0 && !p->hot_all;
    auto enqueue = [&](hipStream_t s) -> int {
      for (int i = 0; i < len; ++i) {
        const int cur = (t0 + i) & 1, b = yb0 ^ (i & 1);
        const int r = run_fused(p, xs[cur], p->ybuf[b], p->ybuf[b ^ 1], s,
                                fuse_hot && t0 + i > 0);
        if (r != MERBIT_OK) return r;
        HIP_TRY(launch_multi_update(p->dtype, p->ybuf[b], xs[cur], xs[cur ^ 1], p->dmask, mt,
                                    alpha, p->multi_gsum[cur], p->multi_gsum[cur ^ 1], s,
                                    fuse_hot ? p->hot_cols : nullptr, fuse_hot ? p->hot_n : 0,
                                    fuse_hot ? p->x_hot : nullptr, i == len - 1));
      }
      return MERBIT_OK;
    };
    // the call's first chunk gathers the hot values, later ones do not: a
    // different graph (the key's count is negated for the first chunk)
    rc = len == check_every
             ? run_chunk(p, kLoopMulti, t0 & 1, yb0, len, t0 == 0 ? -n_graphs : n_graphs,
                         x_inout, alpha, enqueue, st)
             : enqueue(st);
    if (rc != MERBIT_OK) return rc;
    t += len;
    yb ^= len & 1;
    if (tol > 0.0 || t == max_iter) {
      HIP_TRY(hipMemcpyAsync(host_sums.data(), p->multi_gsum[t & 1],
                             sizeof(double) * host_sums.size(), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      double worst = 0.0;
      for (int g = 0; g < n_graphs; ++g) {
        const double r = host_sums[2 * (size_t)g + 1];
        if (resid_out) resid_out[g] = r;
        if (r > worst) worst = r;
      }
      if (tol > 0.0 && worst < tol) {
        converged = true;
        break;
      }
    }
  }
  p->zeroed_buf = yb;
  p->last_stream = st;
  if (t & 1) HIP_TRY(hipMemcpyAsync(x_inout, p->xwork, vb, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (iters_out) *iters_out = t;
  return (tol > 0.0 && !converged) ? MERBIT_NOT_CONVERGED : MERBIT_OK;
} catch (...) {
  return merbit::host_exception();
}

int merbit_pagerank_adjoint(merbit_plan* p, merbit_plan* pt, double alpha, double tol,
                            int max_iter, int check_every, const void* g, void* lam_inout,
                            int* iters_out, double* resid_out, void* stream) try {
  if (iters_out) *iters_out = 0;
  if (resid_out) *resid_out = 0.0;
  if (!p || !pt) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->n_rows != p->n_cols) return fail(MERBIT_EINVAL, "PageRank needs a square matrix");
  if (pt->n_rows != p->n_cols || pt->n_cols != p->n_rows || pt->nnz != p->nnz ||
      pt->dtype != p->dtype)
    return fail(MERBIT_EINVAL, "second plan is not of the transpose's shape and dtype");
  if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(MERBIT_EINVAL, "alpha must be in [0, 1]");
  if (max_iter < 0) return fail(MERBIT_EINVAL, "max_iter < 0");
  if (p->n_rows == 0 || max_iter == 0) return MERBIT_OK;
  if (!g || !lam_inout) return fail(MERBIT_EINVAL, "g or lambda is NULL");
  if (g == lam_inout) return fail(MERBIT_EINVAL, "g and lambda alias");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = ensure_dmask(p, st);  // dangling = columns of P without nonzeros
  if (rc != MERBIT_OK) return rc;
  rc = ensure_pagerank_state(pt, st);
  if (rc != MERBIT_OK) return rc;
  if (check_every <= 0) check_every = 10;
  const int64_t n = p->n_rows;
  const size_t vb = vsize(p->dtype) * (size_t)n;
  HIP_TRY(launch_adj_sum(p->dtype, lam_inout, n, pt->partials[0], pt->reduce_grid, st));
  int yb = pt->zeroed_buf;
  if (yb < 0) {
    yb = 0;
    const int rz = zero_boundary(pt, pt->ybuf[0], st);
    if (rz != MERBIT_OK) return rz;
  }
  void* ls[2] = {lam_inout, pt->xwork};
  std::vector<double> host_pairs(2 * (size_t)pt->reduce_grid);
  int t = 0;
  double resid = 0.0;
  bool converged = false;
  while (t < max_iter) {
    int len = check_every - t % check_every;
    if (len > max_iter - t) len = max_iter - t;
    const int t0 = t, yb0 = yb;
    // as in PageRank: the update writes the next SpMV's hot values
    const bool fuse_hot = pt->hot_n > 0 && !pt->hot_all;
    auto enqueue = [&](hipStream_t s) -> int {
      for (int i = 0; i < len; ++i) {
        const int cur = (t0 + i) & 1, b = yb0 ^ (i & 1);
        const int r = run_fused(pt, ls[cur], pt->ybuf[b], pt->ybuf[b ^ 1], s,
                                fuse_hot && t0 + i > 0);
        if (r != MERBIT_OK) return r;
        HIP_TRY(launch_adj_update(p->dtype, pt->ybuf[b], ls[cur], ls[cur ^ 1], g, p->dmask, n,
                                  alpha, pt->partials[cur], pt->reduce_grid,
                                  pt->partials[cur ^ 1], pt->reduce_grid, s,
                                  fuse_hot ? pt->hot_cols : nullptr, fuse_hot ? pt->hot_n : 0,
                                  fuse_hot ? pt->x_hot : nullptr));
      }
      return MERBIT_OK;
    };
    // the call's first chunk gathers the hot values, later ones do not: a
    // different graph (key k = 1 for the first chunk)
    rc = len == check_every ? run_chunk(pt, kLoopAdjoint, t0 & 1, yb0, len, t0 == 0 ? 1 : 0,
                                        lam_inout, alpha, enqueue, st, g)
                            : enqueue(st);
    if (rc != MERBIT_OK) return rc;
    t += len;
    yb ^= len & 1;
    if (tol > 0.0 || t == max_iter) {
      HIP_TRY(hipMemcpyAsync(host_pairs.data(), pt->partials[t & 1],
                             sizeof(double) * host_pairs.size(), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      resid = 0.0;
      for (int b = 0; b < pt->reduce_grid; ++b) resid += host_pairs[2 * (size_t)b + 1];
      if (tol > 0.0 && resid < tol) {
        converged = true;
        break;
      }
    }
  }
  pt->zeroed_buf = yb;
  pt->last_stream = st;
  p->last_stream = st;
  if (t & 1) HIP_TRY(hipMemcpyAsync(lam_inout, pt->xwork, vb, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (iters_out) *iters_out = t;
  if (resid_out) *resid_out = resid;
  return (tol > 0.0 && !converged) ? MERBIT_NOT_CONVERGED : MERBIT_OK;
} catch (...) {
  return merbit::host_exception();
}

// ------------------------------------------------------------ BiCGSTAB --

int merbit_bicgstab(merbit_plan* p, const void* b, void* x_inout, double tol, int max_iter,
                    int check_every, int* iters_out, double* resid_out, void* stream) try {
  if (iters_out) *iters_out = 0;
  if (resid_out) *resid_out = 0.0;
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->n_rows != p->n_cols) return fail(MERBIT_EINVAL, "BiCGSTAB needs a square matrix");
  if (max_iter < 0) return fail(MERBIT_EINVAL, "max_iter < 0");
  if (p->n_rows == 0) return MERBIT_OK;
  if (!b || !x_inout) return fail(MERBIT_EINVAL, "b or x is NULL");
  if (b == x_inout) return fail(MERBIT_EINVAL, "b and x alias");
  if (check_every <= 0) check_every = 10;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t n = p->n_rows;
  if (!p->bvec[0]) {
    for (int k = 0; k < 7; ++k) HIP_TRY(hipMalloc(&p->bvec[k], vsize(p->dtype) * (size_t)n));
    p->bicg_G = bicg_grid(n);
    for (int k = 0; k < 7; ++k)
      HIP_TRY(hipMalloc(&p->bpart[k], sizeof(double) * 2 * (size_t)p->bicg_G));
  }
  // bvec: 0 r, 1 r^, 2 p, 3 v (even iterations), 4 v (odd), 5 s, 6 t
  // bpart: 0/1 (r^.r, r.r) by parity, 2/3 (r^.v, 0), 4/5 ((t,s), (t,t)), 6 (b.b, 0)
  BicgArgs a;
  memset(&a, 0, sizeof a);
  a.n = n;
  a.G = p->bicg_G;
  a.b = b;
  a.x = x_inout;
  a.r = p->bvec[0];
  a.rh = p->bvec[1];
  a.p = p->bvec[2];
  a.s = p->bvec[5];
  a.t = p->bvec[6];
  // r_0 = b - A x_0 (t holds A x_0; the launch leaves v_even zero at the
  // boundary rows for iteration 0)
  int rc = zero_boundary(p, a.t, st);
  if (rc != MERBIT_OK) return rc;
  rc = run_fused(p, x_inout, a.t, p->bvec[3], st);
  if (rc != MERBIT_OK) return rc;
  a.pa_next = p->bpart[0];
  a.pb_norm = p->bpart[6];
  HIP_TRY(launch_bicg(p->dtype, a, kBicgInit, st));
  std::vector<double> host(4 * (size_t)p->bicg_G);
  HIP_TRY(hipMemcpyAsync(host.data(), p->bpart[6], sizeof(double) * 2 * p->bicg_G,
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(host.data() + 2 * p->bicg_G, p->bpart[0],
                         sizeof(double) * 2 * p->bicg_G, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double bb = 0.0, rr = 0.0;
  for (int k = 0; k < p->bicg_G; ++k) {
    bb += host[2 * (size_t)k];
    rr += host[2 * ((size_t)p->bicg_G + k) + 1];
  }
  const double bnorm = bb > 0.0 ? std::sqrt(bb) : 1.0;
  double rel = std::sqrt(rr) / bnorm;
  if (resid_out) *resid_out = rel;
  p->last_stream = st;
  if (tol > 0.0 && rel < tol) return MERBIT_OK;
  int t = 0;
  int status = MERBIT_NOT_CONVERGED;
  while (t < max_iter) {
    int len = check_every - t % check_every;
    if (len > max_iter - t) len = max_iter - t;
    const int t0 = t;
    auto enqueue = [&](hipStream_t s) -> int {
      for (int i = 0; i < len; ++i) {
        const int it = t0 + i, c = it & 1;
        BicgArgs q = a;
        q.first = it == 0;
        q.pa_cur = p->bpart[c];
        q.pa_prev = p->bpart[c ^ 1];
        q.pb_prev = p->bpart[2 + (c ^ 1)];
        q.pc_prev = p->bpart[4 + (c ^ 1)];
        q.pb_cur = p->bpart[2 + c];
        q.pc_cur = p->bpart[4 + c];
        q.pa_next = p->bpart[c ^ 1];
        void* v_cur = p->bvec[3 + c];
        void* v_prev = p->bvec[3 + (c ^ 1)];
        q.v = v_prev;
        HIP_TRY(launch_bicg(p->dtype, q, kBicgUpdateP, s));
        int r = run_fused(p, q.p, v_cur, q.t, s);  // v = A p; clears t's boundary rows
        if (r != MERBIT_OK) return r;
        q.v = v_cur;
        HIP_TRY(launch_bicg(p->dtype, q, kBicgDot1, s));
        HIP_TRY(launch_bicg(p->dtype, q, kBicgUpdateS, s));
        r = run_fused(p, q.s, q.t, v_prev, s);  // t = A s; clears v_prev for it + 1
        if (r != MERBIT_OK) return r;
        HIP_TRY(launch_bicg(p->dtype, q, kBicgDot2, s));
        HIP_TRY(launch_bicg(p->dtype, q, kBicgUpdateXR, s));
      }
      return MERBIT_OK;
    };
    rc = len == check_every ? run_chunk(p, kLoopBicgstab, t0 & 1, t0 == 0, len, 0, x_inout, 0.0,
                                        enqueue, st, b)
                            : enqueue(st);
    if (rc != MERBIT_OK) return rc;
    t += len;
    if (tol > 0.0 || t == max_iter) {
      HIP_TRY(hipMemcpyAsync(host.data(), p->bpart[t & 1], sizeof(double) * 2 * p->bicg_G,
                             hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      double rho = 0.0;
      rr = 0.0;
      for (int k = 0; k < p->bicg_G; ++k) {
        rho += host[2 * (size_t)k];
        rr += host[2 * (size_t)k + 1];
      }
      rel = std::sqrt(rr) / bnorm;
      if (resid_out) *resid_out = rel;
      if (tol > 0.0 && rel < tol) {
        status = MERBIT_OK;
        break;
      }
      if (!std::isfinite(rel) || (tol > 0.0 && rho == 0.0)) {
        status = MERBIT_BREAKDOWN;
        break;
      }
    }
  }
  HIP_TRY(hipStreamSynchronize(st));
  p->last_stream = st;
  if (iters_out) *iters_out = t;
  if (tol <= 0.0 && status == MERBIT_NOT_CONVERGED) status = MERBIT_OK;
  return status;
} catch (...) {
  return merbit::host_exception();
}

}  // extern "C"
