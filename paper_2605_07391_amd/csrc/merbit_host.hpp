// Host-side state of a plan and the helpers the C-ABI entry points share
// (internal to libmerbit; the public interface is include/merbit.h).
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/merbit.h"

#include "merbit_internal.hpp"

struct merbit_plan {
  int64_t n_rows = 0, n_cols = 0, nnz = 0;
  int dtype = 0, sigma = 0, block_lanes = 0, waves = 0, bits = 0;
  int device = 0;
  int commit = MERBIT_COMMIT_WAVE;  // kernel family
  int blocks_per_cu_req = 0;
  int64_t tile_num = 0, lane_num = 0;
  int64_t chunk_num = 0;  // commit units
  int unit_tiles = 1;     // tiles per commit unit: 1 (wave) or waves (block)
  int grid = 0, chunks_per_block = 1;
  int32_t* tile_x = nullptr;
  uint32_t* tile_y = nullptr;
  uint32_t* lane_desc = nullptr;
  uint64_t* lane_desc64 = nullptr;  // set instead of lane_desc for 64-bit descriptors
  int desc_bits = 32;
  const int32_t* col = nullptr;
  const void* values = nullptr;
  hipStream_t last_stream = nullptr;
  // small device scratch: [0] validation flags / fast-tile count
  unsigned long long* scratch = nullptr;
  // hot-column x cache (hot_n > 0: the fused kernel reads col from colx)
  int32_t hot_n = 0;
  bool hot_all = false;        // every column is hot: slot = column, x itself is copied
  int32_t* hot_cols = nullptr; // [hot_n] column of each slot (partial mode)
  int32_t* colx = nullptr;     // [nnz] recoded column stream
  void* x_hot = nullptr;       // [hot_n] gathered hot x values (partial mode)
  size_t hot_lds_bytes = 0;
  double hot_coverage = 0.0;   // fraction of nonzeros whose column is hot
  // column stripes (stripes > 1): TILE is the plan of the stacked matrix A'
  // (rows = non-empty (stripe, row) pairs, plan_rows of them), whose column
  // stream and values the plan keeps in stacked order; the fused kernel writes
  // A' x into yv[yv_cur] (dual buffers) and a second launch sums each row's
  // pairs into y.  ranges > 1: the fused launch's tiles are split into
  // contiguous ranges (range_tile), each with its own hot set (hot_off).
  int stripes = 1;
  int64_t plan_rows = 0;
  int64_t words = 0;                 // 64-row words per stripe
  int stripe_shift = 0;              // stripe of column c = c >> stripe_shift
  int32_t* sperm = nullptr;          // [nnz] stacked position -> matrix position
  int32_t* scol = nullptr;           // [nnz] stacked column stream
  void* svals = nullptr;             // [nnz] stacked values
  merbit::StripeWord* swords = nullptr;  // [words][stripes] combine table
  void* yv[2] = {nullptr, nullptr};  // [plan_rows] A' x, dual buffers
  int yv_cur = 0;
  int ranges = 1;
  int32_t* range_tile = nullptr;     // [ranges + 1]
  int32_t* hot_off = nullptr;        // [ranges + 1]
  unsigned long long* queue = nullptr;  // wave kernel tile queues: [ranges][kQueueStride]
  // PageRank state
  uint32_t* dmask = nullptr;
  void* ybuf[2] = {nullptr, nullptr};
  void* xwork = nullptr;
  // per-block (dangling mass, l1 change) pairs of the last two reductions
  double* partials[2] = {nullptr, nullptr};
  int reduce_grid = 0;
  int zeroed_buf = -1;  // which ybuf is zero at the boundary rows, -1 if none
  // personalised PageRank state (k columns)
  int ppr_k = 0;
  void* pbuf[3] = {nullptr, nullptr, nullptr};  // A X at the tiles' first rows, -, one iterate
  double* ppart = nullptr;                      // per-block, per-column pairs
  double* psums[2] = {nullptr, nullptr};        // per-column (dangling mass, l1 change)
  int32_t* psrc = nullptr;
  int ppr_grid_n = 0;
  int ppr_zeroed = -1;  // 0 once pbuf[0] is zero at the tiles' first rows
  // PageRank of the graphs on the diagonal (tables for the last graph_ptr)
  std::vector<int64_t> multi_gp;
  int32_t* multi_chunk_row = nullptr;
  int32_t* multi_chunk_graph = nullptr;
  int32_t* multi_chunk_ptr = nullptr;
  double* multi_gsize = nullptr;
  double* multi_part = nullptr;
  double* multi_gsum[2] = {nullptr, nullptr};
  int32_t* multi_hot_graph = nullptr;  // graph of each hot column slot
  int32_t multi_chunks = 0;
  // BiCGSTAB state: r, r^, p, v (two), s, t; pair arrays of the dot products
  void* bvec[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  double* bpart[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  int bicg_G = 0;
  // HIP graphs of iteration chunks (the PageRank drivers); a graph holds the
  // pointers and scalars it was captured with, so any change of a captured
  // buffer bumps `generation` and drops the graphs
  bool eager_loops = false;
  hipStream_t cap_stream = nullptr;
  uint64_t generation = 0;
  struct LoopGraph {
    int kind, parity, ybuf, len, k;
    int sp_in, sp_out;  // stacked-buffer parity (yv_cur) before / after the chunk
    const void* x;
    const void* aux;  // a second captured operand (adjoint: g)
    double alpha;
    uint64_t gen;
    hipGraphExec_t exec;
  };
  std::vector<LoopGraph> loop_graphs;
  int64_t graph_captures = 0, graph_replays = 0;
  // kernel timing
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t events_used = 0;
};

namespace merbit {

// Set the calling thread's error message; returns code.
int fail(int code, const std::string& msg);
// MERBIT_ENOMEM or MERBIT_EHIP with the HIP error string.
int fail_hip(const char* what, hipError_t e);
// Called from a catch (...) handler of a C-ABI entry point: no C++ exception
// leaves the library; a failed host allocation (std::bad_alloc) becomes
// MERBIT_ENOMEM, anything else MERBIT_EHIP, with the message set.
int host_exception() noexcept;

#define HIP_TRY(expr)                                  \
  do {                                                 \
    hipError_t _e = (expr);                            \
    if (_e != hipSuccess) return merbit::fail_hip(#expr, _e);  \
  } while (0)

inline size_t vsize(int dtype) { return dtype == MERBIT_F64 ? sizeof(double) : sizeof(float); }

void plan_free_all(merbit_plan* p);
// The fused SpMV y = A x (z: the other dual buffer, cleared at boundary rows,
// or nullptr).  hot_ready: the plan's hot-column copy already holds x's hot
// values (written by the PageRank update), so the gather launch is skipped.
// timed: bracket the launches with the plan's timing events when timing is
// on (creating events as needed); false never creates any.
int run_fused(merbit_plan* p, const void* x, void* y, void* z, hipStream_t st,
              bool hot_ready = false, bool timed = true);
// A buffer or value array that captured graphs use has changed: drop them.
void invalidate_graphs(merbit_plan* p);
// Zero v at the first row of every commit unit (nothing for a striped plan,
// whose fused kernel writes only its own buffers).
int zero_boundary(merbit_plan* p, void* v, hipStream_t st);
// Striped plans: the stacked matrix, its plan, and the per-range hot sets.
int build_striped(merbit_plan* p, const int32_t* row_ptr, int hot_columns, hipStream_t st);
// copy values into the stacked order
int stripes_copy_values(merbit_plan* p, const void* values, hipStream_t st);
// allocate TILE for plan_rows rows and build it from row_ptr
int build_tile(merbit_plan* p, const int32_t* row_ptr, hipStream_t st);
// largest number of hot values that fit next to the kernel's static LDS
int64_t hot_cap_lds(const merbit_plan* p);
int size_grid(merbit_plan* p);
// Dangling mask and the PageRank iteration buffers (allocated on first use).
int ensure_dmask(merbit_plan* p, hipStream_t st);
int ensure_pagerank_state(merbit_plan* p, hipStream_t st);

// Work buffers of one PageRank call: the SpMV's two output buffers (dual
// buffers), the second iterate, the per-block (dangling mass, l1 change)
// pairs of the last two reductions (reduce_grid pairs each), the dangling
// mask, and a host array of 2 reduce_grid doubles for the residual.
struct PageRankWork {
  void* ybuf[2] = {nullptr, nullptr};
  void* xwork = nullptr;
  double* partials[2] = {nullptr, nullptr};
  const uint32_t* dmask = nullptr;
  int reduce_grid = 0;
  int zeroed_buf = -1;  // in: which ybuf is zero at the boundary rows (-1: none); out: same
  bool graphs = true;   // record full chunks into HIP graphs (plan-owned buffers only)
  bool timed = true;    // kernel timing events allowed
  double* host_pairs = nullptr;
};
// The power method of Sec. 5.5.1 on work buffers w (merbit_pagerank's loop);
// argument meaning and return codes as merbit_pagerank.
int pagerank_loop(merbit_plan* p, PageRankWork& w, double alpha, double tol, int max_iter,
                  int check_every, void* x_inout, int* iters_out, double* resid_out,
                  hipStream_t st);

enum { kLoopPageRank = 1, kLoopPersonalized = 2, kLoopMulti = 3, kLoopAdjoint = 4,
       kLoopBicgstab = 5 };

// Enqueue one chunk of iterations on `st`.  The first time a chunk with this
// key is seen, `enqueue` is recorded on the plan's capture stream into a HIP
// graph, which is instantiated and kept; later chunks with the same key launch
// the graph (one launch instead of two or three per iteration).  Without
// graphs (eager_loops, or while kernel timing is on) `enqueue` runs on `st`.
template <typename F>
int run_chunk(merbit_plan* p, int kind, int parity, int ybuf, int len, int k,
                     const void* x, double alpha, F&& enqueue, hipStream_t st,
                     const void* aux = nullptr) {
  if (p->eager_loops || p->profiling) return enqueue(st);
  for (auto& g : p->loop_graphs)
    if (g.kind == kind && g.parity == parity && g.ybuf == ybuf && g.len == len && g.k == k &&
        g.x == x && g.aux == aux && g.alpha == alpha && g.gen == p->generation &&
        g.sp_in == p->yv_cur) {
      HIP_TRY(hipGraphLaunch(g.exec, st));
      p->yv_cur = g.sp_out;  // the replay used the buffers the capture did
      ++p->graph_replays;
      return MERBIT_OK;
    }
  const int sp_in = p->yv_cur;
  if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed));
  const int rc = enqueue(p->cap_stream);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
  if (rc != MERBIT_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return fail_hip("hipStreamEndCapture", e);
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) return fail_hip("hipGraphInstantiate", e2);
  if (p->loop_graphs.size() >= 8) {  // keep a few; the oldest goes first
    HIP_TRY(hipStreamSynchronize(st));
    (void)hipGraphExecDestroy(p->loop_graphs.front().exec);
    p->loop_graphs.erase(p->loop_graphs.begin());
  }
  p->loop_graphs.push_back(
      {kind, parity, ybuf, len, k, sp_in, p->yv_cur, x, aux, alpha, p->generation, exec});
  ++p->graph_captures;
  HIP_TRY(hipGraphLaunch(exec, st));
  return MERBIT_OK;
}

}  // namespace merbit
