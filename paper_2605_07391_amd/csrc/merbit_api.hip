// C ABI of libmerbit (declared in include/merbit.h): plan object, argument
// checks, dispatch to the kernels, PageRank driver loop, error reporting.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/merbit.h"

#include "merbit_internal.hpp"

using namespace merbit;

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
  void* pbuf[3] = {nullptr, nullptr, nullptr};  // two SpMM outputs, one iterate
  double* ppart = nullptr;                      // per-block, per-column pairs
  double* psums[2] = {nullptr, nullptr};        // per-column (dangling mass, l1 change)
  int32_t* psrc = nullptr;
  int ppr_grid_n = 0;
  int ppr_zeroed = -1;
  // PageRank of the graphs on the diagonal (tables for the last graph_ptr)
  std::vector<int64_t> multi_gp;
  int32_t* multi_chunk_row = nullptr;
  int32_t* multi_chunk_graph = nullptr;
  int32_t* multi_chunk_ptr = nullptr;
  double* multi_gsize = nullptr;
  double* multi_part = nullptr;
  double* multi_gsum[2] = {nullptr, nullptr};
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
    const void* x;
    const void* aux;  // a second captured operand (adjoint: g)
    double alpha;
    uint64_t gen;
    hipGraphExec_t exec;
  };
  std::vector<LoopGraph> loop_graphs;
  // kernel timing
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t events_used = 0;
};

static thread_local std::string g_last_error;

static int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

static int fail_hip(const char* what, hipError_t e) {
  return fail(e == hipErrorOutOfMemory ? MERBIT_ENOMEM : MERBIT_EHIP,
              std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                  \
  do {                                                 \
    hipError_t _e = (expr);                            \
    if (_e != hipSuccess) return fail_hip(#expr, _e);  \
  } while (0)

static size_t vsize(int dtype) { return dtype == MERBIT_F64 ? sizeof(double) : sizeof(float); }

static void drop_graphs(merbit_plan* p) {
  for (auto& g : p->loop_graphs) (void)hipGraphExecDestroy(g.exec);
  p->loop_graphs.clear();
}

static void plan_free_all(merbit_plan* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  drop_graphs(p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  void* bufs[] = {p->tile_x, p->tile_y, p->lane_desc, p->lane_desc64, p->scratch, p->dmask, p->ybuf[0],
                  p->ybuf[1], p->xwork, p->partials[0], p->partials[1], p->hot_cols,
                  p->colx, p->x_hot, p->pbuf[0], p->pbuf[1], p->pbuf[2], p->ppart,
                  p->psums[0], p->psums[1], p->psrc, p->multi_chunk_row,
                  p->multi_chunk_graph, p->multi_chunk_ptr, p->multi_gsize, p->multi_part,
                  p->multi_gsum[0], p->multi_gsum[1], p->bvec[0], p->bvec[1], p->bvec[2],
                  p->bvec[3], p->bvec[4], p->bvec[5], p->bvec[6], p->bpart[0], p->bpart[1],
                  p->bpart[2], p->bpart[3], p->bpart[4], p->bpart[5], p->bpart[6]};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  for (auto& ev : p->events) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  delete p;
}

static SpmvArgs spmv_args(const merbit_plan* p, const void* x, void* y, void* z) {
  SpmvArgs a;
  a.tile_x = p->tile_x;
  a.tile_y = p->tile_y;
  a.lane_desc = p->lane_desc;
  a.lane_desc64 = p->lane_desc64;
  a.col = p->hot_n > 0 ? p->colx : p->col;
  a.val = p->values;
  a.x = x;
  a.x_hot = p->hot_n > 0 ? (p->hot_all ? x : p->x_hot) : nullptr;
  a.y = y;
  a.z = z;
  a.tile_num = (int32_t)p->tile_num;
  a.lane_num = (int32_t)p->lane_num;
  a.path_len = (int32_t)(p->nnz + p->n_rows);
  a.n_rows = (int32_t)p->n_rows;
  a.chunk_num = (int32_t)p->chunk_num;  // commit units of the block kernel
  a.chunks_per_block = p->chunks_per_block;
  a.grid = p->grid;
  a.hot_n = p->hot_n;
  return a;
}

// Launch the fused kernel (after the hot gather), bracketed by events when
// profiling is on.
static int run_fused(merbit_plan* p, const void* x, void* y, void* z, hipStream_t st) {
  if (p->chunk_num == 0) return MERBIT_OK;
  if (p->hot_n > 0 && !p->hot_all)
    HIP_TRY(launch_hot_gather(p->dtype, x, p->hot_cols, p->hot_n, p->x_hot, st));
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
  if (p->commit == MERBIT_COMMIT_WAVE)
    HIP_TRY(launch_spmv_wave(p->dtype, p->sigma, p->waves, p->hot_n > 0, p->hot_lds_bytes,
                             spmv_args(p, x, y, z), st, p->desc_bits == 64));
  else
    HIP_TRY(launch_spmv(p->dtype, p->sigma, p->waves, p->hot_n > 0, p->hot_lds_bytes,
                        spmv_args(p, x, y, z), st));
  if (p->profiling) HIP_TRY(hipEventRecord(e1, st));
  p->last_stream = st;
  return MERBIT_OK;
}

enum { kLoopPageRank = 1, kLoopPersonalized = 2, kLoopMulti = 3, kLoopAdjoint = 4,
       kLoopBicgstab = 5 };

// Enqueue one chunk of iterations on `st`.  The first time a chunk with this
// key is seen, `enqueue` is recorded on the plan's capture stream into a HIP
// graph, which is instantiated and kept; later chunks with the same key launch
// the graph (one launch instead of two or three per iteration).  Without
// graphs (eager_loops, or while kernel timing is on) `enqueue` runs on `st`.
template <typename F>
static int run_chunk(merbit_plan* p, int kind, int parity, int ybuf, int len, int k,
                     const void* x, double alpha, F&& enqueue, hipStream_t st,
                     const void* aux = nullptr) {
  if (p->eager_loops || p->profiling) return enqueue(st);
  for (auto& g : p->loop_graphs)
    if (g.kind == kind && g.parity == parity && g.ybuf == ybuf && g.len == len && g.k == k &&
        g.x == x && g.aux == aux && g.alpha == alpha && g.gen == p->generation) {
      HIP_TRY(hipGraphLaunch(g.exec, st));
      return MERBIT_OK;
    }
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
  p->loop_graphs.push_back({kind, parity, ybuf, len, k, x, aux, alpha, p->generation, exec});
  HIP_TRY(hipGraphLaunch(exec, st));
  return MERBIT_OK;
}

// A buffer or value array that graphs captured has changed.
static void invalidate_graphs(merbit_plan* p) {
  ++p->generation;
  if (!p->loop_graphs.empty()) {
    (void)hipDeviceSynchronize();
    drop_graphs(p);
  }
}

extern "C" {

const char* merbit_last_error(void) { return g_last_error.c_str(); }

const char* merbit_version(void) { return "merbit-mi355x 0.1 (gfx950, wave64)"; }

// Static LDS of the fused kernel: block kernel = products + row slots of b
// lanes plus head/tail partials; wave kernel = 64 sigma values per wavefront.
static size_t static_lds_bytes(const merbit_plan* p) {
  const size_t vs = vsize(p->dtype);
  if (p->commit == MERBIT_COMMIT_WAVE) return (size_t)p->waves * kOmega * p->sigma * vs + 64;
  return ((size_t)p->waves * kOmega * p->sigma + 1 + 2 * (size_t)p->waves) * vs + 64;
}

static bool kernel_supported(const merbit_plan* p, bool hot) {
  return p->commit == MERBIT_COMMIT_WAVE
             ? spmv_wave_supported(p->dtype, p->sigma, p->waves, hot, p->desc_bits == 64)
                                         : spmv_supported(p->dtype, p->sigma, p->waves, hot);
}

// Choose the grid.  Block kernel: one commit unit (b lanes) per block, or with
// the hot cache as many blocks as fit at once, each taking a run of units.
// Wave kernel: as many resident blocks as LDS and wavefront slots allow (or
// blocks_per_cu), every wavefront striding over the tiles.
static int size_grid(merbit_plan* p) {
  p->unit_tiles = p->commit == MERBIT_COMMIT_WAVE ? 1 : p->waves;
  p->chunk_num = (p->tile_num + p->unit_tiles - 1) / p->unit_tiles;
  p->chunks_per_block = 1;
  p->grid = (int)((p->tile_num + p->waves - 1) / p->waves);
  if (p->tile_num == 0) return MERBIT_OK;
  if (p->commit != MERBIT_COMMIT_WAVE && p->hot_n == 0) return MERBIT_OK;
  int cus = 0, lds_cu = 0;
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device));
  HIP_TRY(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                p->device));
  const size_t per_block = static_lds_bytes(p) + p->hot_lds_bytes;
  int64_t blocks_per_cu = (int64_t)lds_cu / (int64_t)per_block;
  const int64_t wave_cap = 32 / p->waves;  // 8 wavefronts per SIMD, 4 SIMDs per CU
  if (blocks_per_cu > wave_cap) blocks_per_cu = wave_cap;
  if (p->blocks_per_cu_req > 0 && p->blocks_per_cu_req < blocks_per_cu)
    blocks_per_cu = p->blocks_per_cu_req;
  if (blocks_per_cu < 1) blocks_per_cu = 1;
  int64_t grid = (int64_t)cus * blocks_per_cu;
  if (p->commit == MERBIT_COMMIT_WAVE) {
    const int64_t need = (p->tile_num + p->waves - 1) / p->waves;  // one tile per wavefront
    p->grid = (int)(grid < need ? grid : need);
    return MERBIT_OK;
  }
  if (grid > p->chunk_num) grid = p->chunk_num;
  p->chunks_per_block = (int)((p->chunk_num + grid - 1) / grid);
  p->grid = (int)((p->chunk_num + p->chunks_per_block - 1) / p->chunks_per_block);
  return MERBIT_OK;
}

// Hot-column cache: pick at most `cap` most frequent columns (or every column
// when they all fit) and recode the column stream.  `cap` < 0 picks the
// largest cap that leaves one block per CU room for its LDS, and keeps the
// cache only if the hot columns hold at least 20 % of the nonzeros.
static int build_hot_cache(merbit_plan* p, int cap_req, hipStream_t st) {
  p->hot_n = 0;
  if (cap_req == 0 || p->nnz == 0 || p->n_cols == 0) return MERBIT_OK;
  // Automatic sizing enables the cache for the wave kernel only: with the
  // block kernel the LDS fill leaves one block per CU and its barriers make
  // every wavefront of a block wait for the slowest, which measured slower
  // than no cache at every size (R-MAT 22).  An explicit size is honoured.
  if (cap_req < 0 && p->commit != MERBIT_COMMIT_WAVE) return MERBIT_OK;
  if (!kernel_supported(p, true))
    return cap_req > 0 ? fail(MERBIT_EUNSUPPORTED, "hot cache not built for this block size")
                       : MERBIT_OK;
  int lds_block = 0;
  HIP_TRY(hipDeviceGetAttribute(&lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                p->device));
  const size_t vs = vsize(p->dtype);
  int64_t cap_lds = ((int64_t)lds_block - (int64_t)static_lds_bytes(p)) / (int64_t)vs;
  cap_lds = (cap_lds / 256) * 256;
  int64_t cap = cap_req > 0 ? cap_req : cap_lds;
  if (cap > cap_lds) return fail(MERBIT_EUNSUPPORTED, "hot_columns exceeds the LDS budget");
  if (cap <= 0) return MERBIT_OK;

  const int64_t nc = p->n_cols;
  if (nc <= cap) {
    // every column fits: the slot of column c is c and x is copied as is
    p->hot_all = true;
    p->hot_n = (int32_t)nc;
    p->hot_coverage = 1.0;
  } else {
    int32_t* counts = nullptr;
    int32_t* hist = nullptr;
    HIP_TRY(hipMalloc(&counts, sizeof(int32_t) * (size_t)nc));
    HIP_TRY(hipMalloc(&hist, sizeof(int32_t) * kHotHistBins));
    std::vector<int32_t> h(kHotHistBins);
    // sampled counts: one nonzero in `sample`, about two samples per column
    int64_t sample = p->nnz / (2 * nc);
    sample = sample < 1 ? 1 : (sample > 8 ? 8 : sample);
    hipError_t e = hot_count_columns(p->col, p->nnz, nc, (int)sample, counts, hist, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h.data(), hist, sizeof(int32_t) * kHotHistBins, hipMemcpyDeviceToHost,
                         st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      (void)hipFree(counts);
      (void)hipFree(hist);
      return fail_hip("hot column counts", e);
    }
    // smallest threshold t >= 1 with at most cap columns of (sampled) count >= t
    int64_t taken = 0;
    double covered = 0.0;
    int32_t t = kHotHistBins;
    for (int b = kHotHistBins - 1; b >= 1; --b) {
      if (taken + h[b] > cap) break;
      taken += h[b];
      covered += (double)b * h[b];
      t = b;
    }
    p->hot_coverage = covered * (double)sample / (double)p->nnz;  // estimate when sampled
    if (p->hot_coverage > 1.0) p->hot_coverage = 1.0;
    const bool keep = taken > 0 && (cap_req > 0 || p->hot_coverage >= 0.2);
    if (keep) {
      const int nb = hot_select_blocks(nc);
      int32_t* blk = nullptr;
      int32_t* slot_of = nullptr;
      std::vector<int32_t> hb(nb);
      e = hipMalloc(&blk, sizeof(int32_t) * (size_t)nb);
      if (e == hipSuccess) e = hipMalloc(&slot_of, sizeof(int32_t) * (size_t)nc);
      if (e == hipSuccess) e = hipMalloc(&p->hot_cols, sizeof(int32_t) * (size_t)taken);
      if (e == hipSuccess) e = hot_select_count(counts, nc, t, blk, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(hb.data(), blk, sizeof(int32_t) * (size_t)nb, hipMemcpyDeviceToHost,
                           st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e == hipSuccess) {
        int32_t acc = 0;
        for (int b = 0; b < nb; ++b) {
          const int32_t c = hb[b];
          hb[b] = acc;
          acc += c;
        }
        e = hipMemcpyAsync(blk, hb.data(), sizeof(int32_t) * (size_t)nb, hipMemcpyHostToDevice,
                           st);
      }
      if (e == hipSuccess) e = hot_select_assign(counts, nc, t, blk, slot_of, p->hot_cols, st);
      if (e == hipSuccess) e = hipMalloc(&p->colx, sizeof(int32_t) * (size_t)p->nnz);
      if (e == hipSuccess) e = hot_recode(p->col, p->nnz, slot_of, p->colx, st);
      if (e == hipSuccess) e = hipMalloc(&p->x_hot, vs * (size_t)taken);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      (void)hipFree(blk);
      (void)hipFree(slot_of);
      if (e != hipSuccess) {
        (void)hipFree(counts);
        (void)hipFree(hist);
        return fail_hip("hot column selection", e);
      }
      p->hot_n = (int32_t)taken;
    }
    (void)hipFree(counts);
    (void)hipFree(hist);
  }
  if (p->hot_n > 0) {
    if (p->hot_all) {
      // slot = column: the recoded stream is -1 - col
      HIP_TRY(hipMalloc(&p->colx, sizeof(int32_t) * (size_t)p->nnz));
      HIP_TRY(hot_recode(p->col, p->nnz, nullptr, p->colx, st));
    }
    p->hot_lds_bytes = vs * (size_t)p->hot_n;
    if (p->commit == MERBIT_COMMIT_WAVE)
      HIP_TRY(spmv_wave_set_hot_lds(p->dtype, p->sigma, p->waves, p->hot_lds_bytes,
                                    p->desc_bits == 64));
    else
      HIP_TRY(spmv_set_hot_lds(p->dtype, p->sigma, p->waves, p->hot_lds_bytes));
  }
  return MERBIT_OK;
}

void merbit_opts_init(merbit_opts_t* o) {
  if (!o) return;
  memset(o, 0, sizeof *o);
  o->hot_columns = -1;
  o->validate = 1;
}

int merbit_plan_create(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t* row_ptr,
                       const int32_t* col_ind, const void* values, int dtype,
                       const merbit_opts_t* opts_in, void* stream, merbit_plan** out) {
  g_last_error.clear();
  merbit_opts_t opts;
  if (opts_in) opts = *opts_in;
  else merbit_opts_init(&opts);
  int sigma = opts.sigma, block_lanes = opts.block_lanes;
  const int hot_columns = opts.hot_columns, validate = opts.validate;
  int commit = opts.commit == MERBIT_COMMIT_AUTO ? MERBIT_COMMIT_WAVE : opts.commit;
  if (commit != MERBIT_COMMIT_WAVE && commit != MERBIT_COMMIT_BLOCK)
    return fail(MERBIT_EINVAL, "commit must be MERBIT_COMMIT_AUTO, _BLOCK or _WAVE");
  if (!out) return fail(MERBIT_EINVAL, "out is NULL");
  *out = nullptr;
  if (dtype != MERBIT_F32 && dtype != MERBIT_F64) return fail(MERBIT_EUNSUPPORTED, "dtype");
  if (n_rows < 0 || n_cols < 0 || nnz < 0) return fail(MERBIT_EINVAL, "negative size");
  if (n_rows + nnz >= ((int64_t)1 << 31))
    return fail(MERBIT_EINVAL, "n_rows + nnz must be < 2^31");
  if (n_cols >= ((int64_t)1 << 31)) return fail(MERBIT_EINVAL, "n_cols must be < 2^31");
  if (n_rows > 0 && !row_ptr) return fail(MERBIT_EINVAL, "row_ptr is NULL");
  if (nnz > 0 && (!col_ind || !values)) return fail(MERBIT_EINVAL, "col_ind/values NULL");
  if (nnz > 0 && n_rows == 0) return fail(MERBIT_EINVAL, "nonzeros without rows");
  if (sigma == 0) sigma = dtype == MERBIT_F32 ? 12 : 7;
  if (block_lanes == 0) block_lanes = commit == MERBIT_COMMIT_WAVE ? 512 : 256;
  const int desc_bits = opts.desc_bits == 0 ? 32 : opts.desc_bits;
  if (desc_bits != 32 && desc_bits != 64) return fail(MERBIT_EINVAL, "desc_bits must be 32 or 64");
  if (desc_bits == 64 && commit != MERBIT_COMMIT_WAVE)
    return fail(MERBIT_EUNSUPPORTED, "64-bit descriptors need the wave commit kernel");
  if (sigma < 1 || sigma > (desc_bits == 64 ? kMaxSigma64 : kMaxSigma))
    return fail(MERBIT_EUNSUPPORTED,
                desc_bits == 64 ? "sigma must be in 1..40" : "sigma must be in 1..12");
  const int bits = ceil_log2(kOmega * sigma);
  if (2 * bits + sigma > desc_bits)
    return fail(MERBIT_EUNSUPPORTED, "descriptor exceeds its width");
  if (block_lanes % kOmega != 0) return fail(MERBIT_EINVAL, "block_lanes % 64 != 0");
  const int waves = block_lanes / kOmega;
  if (commit == MERBIT_COMMIT_WAVE ? !spmv_wave_supported(dtype, sigma, waves, false,
                                                          desc_bits == 64)
                                   : !spmv_supported(dtype, sigma, waves, false))
    return fail(MERBIT_EUNSUPPORTED,
                desc_bits == 64 ? (dtype == MERBIT_F32
                                       ? "64-bit descriptors: sigma 16, 20 or 24, 256 or 512 lanes"
                                       : "64-bit descriptors: sigma 14 or 16, 256 or 512 lanes")
                : commit == MERBIT_COMMIT_WAVE ? "block_lanes must be 256, 512 or 1024"
                                               : "block_lanes must be 128, 256, 512 or 1024");
  if (opts.blocks_per_cu < 0) return fail(MERBIT_EINVAL, "blocks_per_cu < 0");

  hipStream_t st = static_cast<hipStream_t>(stream);
  merbit_plan* p = new merbit_plan();
  p->n_rows = n_rows;
  p->n_cols = n_cols;
  p->nnz = nnz;
  p->dtype = dtype;
  p->sigma = sigma;
  p->block_lanes = block_lanes;
  p->waves = waves;
  p->bits = bits;
  p->commit = commit;
  p->blocks_per_cu_req = opts.blocks_per_cu;
  p->eager_loops = opts.eager_loops != 0;
  p->desc_bits = desc_bits;
  p->col = col_ind;
  p->values = values;
  p->last_stream = st;
  (void)hipGetDevice(&p->device);
  const int64_t L = nnz + n_rows;
  p->tile_num = (L + (int64_t)kOmega * sigma - 1) / ((int64_t)kOmega * sigma);
  p->lane_num = (L + sigma - 1) / sigma;

  hipError_t e;
#define CREATE_TRY(expr)                       \
  do {                                         \
    e = (expr);                                \
    if (e != hipSuccess) {                     \
      int rc = fail_hip(#expr, e);             \
      plan_free_all(p);                        \
      return rc;                               \
    }                                          \
  } while (0)

  CREATE_TRY(hipMalloc(&p->scratch, 64));
  CREATE_TRY(hipMalloc(&p->tile_x, sizeof(int32_t) * (size_t)(p->tile_num + 1)));
  CREATE_TRY(hipMalloc(&p->tile_y, sizeof(uint32_t) * (size_t)(p->tile_num + 1)));
  if (desc_bits == 64)
    CREATE_TRY(hipMalloc(&p->lane_desc64,
                         sizeof(uint64_t) * (size_t)(p->lane_num > 0 ? p->lane_num : 1)));
  else
    CREATE_TRY(hipMalloc(&p->lane_desc,
                         sizeof(uint32_t) * (size_t)(p->lane_num > 0 ? p->lane_num : 1)));

  if (validate && (n_rows > 0 || nnz > 0)) {
    CREATE_TRY(hipMemsetAsync(p->scratch, 0, 64, st));
    CREATE_TRY(launch_validate(row_ptr, col_ind, n_rows, n_cols, nnz,
                               reinterpret_cast<unsigned*>(p->scratch), st));
    unsigned flags = 0;
    CREATE_TRY(hipMemcpyAsync(&flags, p->scratch, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    CREATE_TRY(hipStreamSynchronize(st));
    if (flags) {
      char buf[160];
      snprintf(buf, sizeof buf, "CSR validation failed:%s%s%s%s",
               (flags & 1) ? " row_ptr[0]!=0" : "", (flags & 2) ? " row_ptr[n]!=nnz" : "",
               (flags & 4) ? " row_ptr decreasing" : "", (flags & 8) ? " column out of range" : "");
      plan_free_all(p);
      return fail(MERBIT_EINVAL, buf);
    }
  }
  if (n_rows == 0) {
    // empty path: TILE = {[0], [0]}
    CREATE_TRY(hipMemsetAsync(p->tile_x, 0, sizeof(int32_t), st));
    CREATE_TRY(hipMemsetAsync(p->tile_y, 0, sizeof(uint32_t), st));
  } else {
    PlanArgs pa;
    pa.row_ptr = row_ptr;
    pa.n_rows = (int32_t)n_rows;
    pa.nnz = (int32_t)nnz;
    pa.sigma = sigma;
    pa.bits = bits;
    pa.lane_num = p->lane_num;
    pa.tile_num = p->tile_num;
    pa.tile_x = p->tile_x;
    pa.tile_y = p->tile_y;
    pa.lane_desc = p->lane_desc;
    pa.lane_desc64 = p->lane_desc64;
    CREATE_TRY(launch_plan(pa, st));
  }
#undef CREATE_TRY
  int rc = build_hot_cache(p, hot_columns, st);
  if (rc == MERBIT_OK) rc = size_grid(p);
  if (rc != MERBIT_OK) {
    std::string msg = g_last_error;
    plan_free_all(p);
    return fail(rc, msg);
  }
  *out = p;
  return MERBIT_OK;
}

int merbit_plan_set_values(merbit_plan* p, const void* values) {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->nnz > 0 && !values) return fail(MERBIT_EINVAL, "values is NULL");
  if (values != p->values) invalidate_graphs(p);
  p->values = values;
  return MERBIT_OK;
}

int merbit_plan_info(merbit_plan* p, merbit_plan_info_t* info) {
  if (!p || !info) return fail(MERBIT_EINVAL, "NULL argument");
  memset(info, 0, sizeof *info);
  info->n_rows = p->n_rows;
  info->n_cols = p->n_cols;
  info->nnz = p->nnz;
  info->tile_num = p->tile_num;
  info->lane_num = p->lane_num;
  info->chunk_num = p->chunk_num;
  info->commit = p->commit;
  info->grid = p->grid;
  info->chunks_per_block = p->chunks_per_block;
  info->hot_columns = p->hot_n;
  info->hot_coverage = p->hot_coverage;
  info->omega = kOmega;
  info->sigma = p->sigma;
  info->block_lanes = p->block_lanes;
  info->offset_bits = p->bits;
  info->dtype = p->dtype;
  info->lds_bytes = (int32_t)(static_lds_bytes(p) + p->hot_lds_bytes);
  info->desc_bits = p->desc_bits;
  if (p->tile_num > 0) {
    hipStream_t st = p->last_stream;
    unsigned long long cnt = 0;
    HIP_TRY(hipMemsetAsync(p->scratch, 0, sizeof(unsigned long long), st));
    HIP_TRY(launch_count_fast(p->tile_y, p->tile_num, p->scratch, st));
    HIP_TRY(hipMemcpyAsync(&cnt, p->scratch, sizeof cnt, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    info->fast_tiles = (int64_t)cnt;
  }
  return MERBIT_OK;
}

int merbit_plan_export(merbit_plan* p, int32_t* tile_x, uint32_t* tile_y, void* lane_desc,
                       int64_t* tile_num, int64_t* lane_num) {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (tile_num) *tile_num = p->tile_num;
  if (lane_num) *lane_num = p->lane_num;
  hipStream_t st = p->last_stream;
  HIP_TRY(hipStreamSynchronize(st));
  if (tile_x)
    HIP_TRY(hipMemcpy(tile_x, p->tile_x, sizeof(int32_t) * (size_t)(p->tile_num + 1),
                      hipMemcpyDeviceToHost));
  if (tile_y)
    HIP_TRY(hipMemcpy(tile_y, p->tile_y, sizeof(uint32_t) * (size_t)(p->tile_num + 1),
                      hipMemcpyDeviceToHost));
  if (lane_desc && p->lane_num > 0)
    HIP_TRY(hipMemcpy(lane_desc,
                      p->desc_bits == 64 ? (const void*)p->lane_desc64 : (const void*)p->lane_desc,
                      (size_t)(p->desc_bits / 8) * (size_t)p->lane_num,
                      hipMemcpyDeviceToHost));
  return MERBIT_OK;
}

int merbit_zero_boundary(merbit_plan* p, void* v, void* stream) {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->chunk_num == 0) return MERBIT_OK;
  if (!v) return fail(MERBIT_EINVAL, "vector is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(launch_zero_boundary(p->dtype, p->tile_y, (int32_t)p->chunk_num, p->unit_tiles, v, st));
  p->last_stream = st;
  return MERBIT_OK;
}

int merbit_spmv(merbit_plan* p, const void* x, void* y, void* stream) {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->n_rows == 0) return MERBIT_OK;
  if (!y || (p->nnz > 0 && !x)) return fail(MERBIT_EINVAL, "x or y is NULL");
  if (x == y) return fail(MERBIT_EINVAL, "x and y alias");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(launch_zero_boundary(p->dtype, p->tile_y, (int32_t)p->chunk_num, p->unit_tiles, y, st));
  return run_fused(p, x, y, nullptr, st);
}

int merbit_spmv_dual(merbit_plan* p, const void* x, void* y, void* z, void* stream) {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->n_rows == 0) return MERBIT_OK;
  if (!y || !z || (p->nnz > 0 && !x)) return fail(MERBIT_EINVAL, "x, y or z is NULL");
  if (x == y || y == z || x == z) return fail(MERBIT_EINVAL, "x, y, z must be distinct");
  return run_fused(p, x, y, z, static_cast<hipStream_t>(stream));
}

// Bit u of the dangling mask is set when column u holds no nonzero (vertex u
// has no out-edge); built once per plan, shared by both PageRank drivers.
static int ensure_dmask(merbit_plan* p, hipStream_t st) {
  if (p->dmask) return MERBIT_OK;
  unsigned char* bytes = nullptr;
  HIP_TRY(hipMalloc(&p->dmask, sizeof(uint32_t) * (size_t)((p->n_cols + 31) / 32 + 1)));
  HIP_TRY(hipMalloc(&bytes, (size_t)(p->n_cols > 0 ? p->n_cols : 1)));
  hipError_t e = launch_dangling_mask(p->col, p->nnz, p->n_cols, bytes, p->dmask, st);
  hipError_t e2 = hipStreamSynchronize(st);
  (void)hipFree(bytes);
  if (e != hipSuccess) return fail_hip("dangling mask", e);
  if (e2 != hipSuccess) return fail_hip("dangling mask sync", e2);
  return MERBIT_OK;
}

static int ensure_pagerank_state(merbit_plan* p, hipStream_t st) {
  const size_t vb = vsize(p->dtype) * (size_t)p->n_rows;
  int rc = ensure_dmask(p, st);
  if (rc != MERBIT_OK) return rc;
  if (!p->ybuf[0]) {
    HIP_TRY(hipMalloc(&p->ybuf[0], vb));
    HIP_TRY(hipMalloc(&p->ybuf[1], vb));
    HIP_TRY(hipMalloc(&p->xwork, vb));
    p->zeroed_buf = -1;
  }
  if (!p->partials[0]) {
    p->reduce_grid = pr_reduce_grid(p->n_rows);
    HIP_TRY(hipMalloc(&p->partials[0], 2 * sizeof(double) * (size_t)p->reduce_grid));
    HIP_TRY(hipMalloc(&p->partials[1], 2 * sizeof(double) * (size_t)p->reduce_grid));
  }
  return MERBIT_OK;
}

int merbit_pagerank(merbit_plan* p, double alpha, double tol, int max_iter, int check_every,
                    void* x_inout, int* iters_out, double* resid_out, void* stream) {
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
  if (check_every <= 0) check_every = 10;
  const int64_t n = p->n_rows;
  const size_t vb = vsize(p->dtype) * (size_t)n;

  // delta_0: per-block dangling mass of x_0 into partials[0]
  HIP_TRY(launch_dangling_sum(p->dtype, x_inout, p->dmask, n, p->partials[0], p->reduce_grid,
                              st));
  int yb = p->zeroed_buf;
  if (yb < 0) {
    yb = 0;
    HIP_TRY(launch_zero_boundary(p->dtype, p->tile_y, (int32_t)p->chunk_num, p->unit_tiles,
                                 p->ybuf[0], st));
  }
  void* xs[2] = {x_inout, p->xwork};
  std::vector<double> host_pairs(2 * (size_t)p->reduce_grid);
  int t = 0;
  double resid = 0.0;
  bool converged = false;
  while (t < max_iter) {
    // iterations up to the next check (or max_iter), as one chunk
    int len = check_every - t % check_every;
    if (len > max_iter - t) len = max_iter - t;
    const int t0 = t, yb0 = yb;
    auto enqueue = [&](hipStream_t s) -> int {
      for (int i = 0; i < len; ++i) {
        const int cur = (t0 + i) & 1, b = yb0 ^ (i & 1);
        const int r = run_fused(p, xs[cur], p->ybuf[b], p->ybuf[b ^ 1], s);
        if (r != MERBIT_OK) return r;
        HIP_TRY(launch_pr_update(p->dtype, p->ybuf[b], xs[cur], xs[cur ^ 1], p->dmask, n, alpha,
                                 p->partials[cur], p->reduce_grid, p->partials[cur ^ 1],
                                 p->reduce_grid, s));
      }
      return MERBIT_OK;
    };
    rc = len == check_every
             ? run_chunk(p, kLoopPageRank, t0 & 1, yb0, len, 0, x_inout, alpha, enqueue, st)
             : enqueue(st);
    if (rc != MERBIT_OK) return rc;
    t += len;
    yb ^= len & 1;
    if (tol > 0.0 || t == max_iter) {
      // l1 change of this iteration: sum of the blocks' second components
      HIP_TRY(hipMemcpyAsync(host_pairs.data(), p->partials[t & 1],
                             sizeof(double) * host_pairs.size(), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      resid = 0.0;
      for (int b = 0; b < p->reduce_grid; ++b) resid += host_pairs[2 * (size_t)b + 1];
      if (tol > 0.0 && resid < tol) {
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
  if (resid_out) *resid_out = resid;
  return (tol > 0.0 && !converged) ? MERBIT_NOT_CONVERGED : MERBIT_OK;
}

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
  a.k = k;
  a.tile_num = (int32_t)p->tile_num;
  a.lane_num = (int32_t)p->lane_num;
  a.path_len = (int32_t)(p->nnz + p->n_rows);
  a.n_rows = (int32_t)p->n_rows;
  return a;
}

// One SpMM launch per slab of at most 64 columns, bracketed by events when
// profiling is on.
static int run_spmm(merbit_plan* p, const void* X, int64_t ldx, void* Y, int64_t ldy, void* Z,
                    int64_t ldz, int k, hipStream_t st) {
  const size_t vs = vsize(p->dtype);
  for (int c0 = 0; c0 < k; c0 += 64) {
    const int kk = k - c0 < 64 ? k - c0 : 64;
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
    HIP_TRY(launch_spmm(p->dtype, p->sigma,
                        spmm_args(p, static_cast<const char*>(X) + vs * c0, ldx,
                                  static_cast<char*>(Y) + vs * c0, ldy,
                                  Z ? static_cast<char*>(Z) + vs * c0 : nullptr, ldz, kk),
                        st));
    if (p->profiling) HIP_TRY(hipEventRecord(e1, st));
  }
  p->last_stream = st;
  return MERBIT_OK;
}

int merbit_spmm(merbit_plan* p, const void* X, int64_t ldx, void* Y, int64_t ldy, int k,
                void* stream) {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
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
}

int merbit_spmm_dual(merbit_plan* p, const void* X, int64_t ldx, void* Y, int64_t ldy, void* Z,
                     int64_t ldz, int k, void* stream) {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->desc_bits != 32)
    return fail(MERBIT_EUNSUPPORTED, "this call needs a plan with 32-bit descriptors");
  if (k < 1) return fail(MERBIT_EINVAL, "k < 1");
  if (ldx < k || ldy < k || ldz < k) return fail(MERBIT_EINVAL, "leading dimension < k");
  if (p->n_rows == 0) return MERBIT_OK;
  if (!Y || !Z || (p->nnz > 0 && !X)) return fail(MERBIT_EINVAL, "X, Y or Z is NULL");
  if (X == Y || Y == Z || X == Z) return fail(MERBIT_EINVAL, "X, Y, Z must be distinct");
  return run_spmm(p, X, ldx, Y, ldy, Z, ldz, k, static_cast<hipStream_t>(stream));
}

int merbit_spmm_zero_boundary(merbit_plan* p, void* Y, int64_t ldy, int k, void* stream) {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
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
}

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
    for (int b = 0; b < 3; ++b) HIP_TRY(hipMalloc(&p->pbuf[b], bytes));
    p->ppr_k = k;
    p->ppr_zeroed = -1;
  }
  if (!p->ppart) {
    p->ppr_grid_n = ppr_grid(p->n_rows);
    HIP_TRY(hipMalloc(&p->ppart, sizeof(double) * 2 * 64 * (size_t)p->ppr_grid_n));
    HIP_TRY(hipMalloc(&p->psums[0], sizeof(double) * 2 * 64));
    HIP_TRY(hipMalloc(&p->psums[1], sizeof(double) * 2 * 64));
    HIP_TRY(hipMalloc(&p->psrc, sizeof(int32_t) * 64));
  }
  return MERBIT_OK;
}

int merbit_pagerank_personalized(merbit_plan* p, double alpha, double tol, int max_iter,
                                 int check_every, const int32_t* sources, int k, void* X_inout,
                                 int* iters_out, double* resid_out, void* stream) {
  if (iters_out) *iters_out = 0;
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
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
  HIP_TRY(launch_ppr_dangling(p->dtype, X_inout, p->dmask, n, k, p->ppart, p->psums[0],
                              p->ppr_grid_n, st));
  int yb = p->ppr_zeroed;
  if (yb < 0) {
    yb = 0;
    HIP_TRY(launch_spmm_zero(p->dtype, p->tile_y, (int32_t)p->tile_num, p->pbuf[0], k, k, st));
  }
  void* xs[2] = {X_inout, p->pbuf[2]};
  double host_sums[128];
  int t = 0;
  bool converged = false;
  while (t < max_iter) {
    int len = check_every - t % check_every;
    if (len > max_iter - t) len = max_iter - t;
    const int t0 = t, yb0 = yb;
    auto enqueue = [&](hipStream_t s) -> int {
      for (int i = 0; i < len; ++i) {
        const int cur = (t0 + i) & 1, b = yb0 ^ (i & 1);
        const int r = run_spmm(p, xs[cur], k, p->pbuf[b], k, p->pbuf[b ^ 1], k, k, s);
        if (r != MERBIT_OK) return r;
        HIP_TRY(launch_ppr_update(p->dtype, p->pbuf[b], xs[cur], xs[cur ^ 1], p->dmask, n, k,
                                  alpha, p->psrc, p->psums[cur], p->ppart, p->psums[cur ^ 1],
                                  p->ppr_grid_n, s));
      }
      return MERBIT_OK;
    };
    rc = len == check_every
             ? run_chunk(p, kLoopPersonalized, t0 & 1, yb0, len, k, X_inout, alpha, enqueue, st)
             : enqueue(st);
    if (rc != MERBIT_OK) return rc;
    t += len;
    yb ^= len & 1;
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
  p->ppr_zeroed = yb;
  p->last_stream = st;
  if (t & 1) HIP_TRY(hipMemcpyAsync(X_inout, p->pbuf[2], bytes, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (iters_out) *iters_out = t;
  return (tol > 0.0 && !converged) ? MERBIT_NOT_CONVERGED : MERBIT_OK;
}

// Row-chunk tables for the graphs of graph_ptr (rebuilt when it changes).
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
  void* old[] = {p->multi_chunk_row, p->multi_chunk_graph, p->multi_chunk_ptr, p->multi_gsize,
                 p->multi_part, p->multi_gsum[0], p->multi_gsum[1]};
  HIP_TRY(hipStreamSynchronize(st));  // earlier calls may still read the old tables
  invalidate_graphs(p);
  for (void* b : old)
    if (b) (void)hipFree(b);
  p->multi_chunk_row = p->multi_chunk_graph = p->multi_chunk_ptr = nullptr;
  p->multi_gsize = p->multi_part = p->multi_gsum[0] = p->multi_gsum[1] = nullptr;
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
  p->multi_chunks = (int32_t)C;
  p->multi_gp = gp;
  return MERBIT_OK;
}

int merbit_pagerank_multi(merbit_plan* p, const int64_t* graph_ptr, int n_graphs, double alpha,
                          double tol, int max_iter, int check_every, void* x_inout,
                          int* iters_out, double* resid_out, void* stream) {
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
  mt.n_chunks = p->multi_chunks;
  mt.n_graphs = n_graphs;
  const size_t vb = vsize(p->dtype) * (size_t)p->n_rows;

  HIP_TRY(launch_multi_dangling(p->dtype, x_inout, p->dmask, mt, p->multi_gsum[0], st));
  int yb = p->zeroed_buf;
  if (yb < 0) {
    yb = 0;
    HIP_TRY(launch_zero_boundary(p->dtype, p->tile_y, (int32_t)p->chunk_num, p->unit_tiles,
                                 p->ybuf[0], st));
  }
  void* xs[2] = {x_inout, p->xwork};
  std::vector<double> host_sums(2 * (size_t)n_graphs);
  int t = 0;
  bool converged = false;
  while (t < max_iter) {
    int len = check_every - t % check_every;
    if (len > max_iter - t) len = max_iter - t;
    const int t0 = t, yb0 = yb;
    auto enqueue = [&](hipStream_t s) -> int {
      for (int i = 0; i < len; ++i) {
        const int cur = (t0 + i) & 1, b = yb0 ^ (i & 1);
        const int r = run_fused(p, xs[cur], p->ybuf[b], p->ybuf[b ^ 1], s);
        if (r != MERBIT_OK) return r;
        HIP_TRY(launch_multi_update(p->dtype, p->ybuf[b], xs[cur], xs[cur ^ 1], p->dmask, mt,
                                    alpha, p->multi_gsum[cur], p->multi_gsum[cur ^ 1], s));
      }
      return MERBIT_OK;
    };
    rc = len == check_every
             ? run_chunk(p, kLoopMulti, t0 & 1, yb0, len, n_graphs, x_inout, alpha, enqueue, st)
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
}

// Autotuner: one plan per (sigma, block size) candidate, each timed over
// `reps` dual-buffer SpMV launches (the PageRank regime) after two warm-up
// launches; x is a constant nonzero vector.  Candidates the kernels do not
// build are reported as -1 and skipped.
int merbit_tune(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t* row_ptr,
                const int32_t* col_ind, const void* values, int dtype, const int32_t* sigmas,
                int n_sigmas, const int32_t* block_lanes, int n_blocks, int reps,
                merbit_opts_t* opts_inout, float* us_out, void* stream) {
  if (!opts_inout) return fail(MERBIT_EINVAL, "opts is NULL");
  if (dtype != MERBIT_F32 && dtype != MERBIT_F64) return fail(MERBIT_EUNSUPPORTED, "dtype");
  if (reps < 1) return fail(MERBIT_EINVAL, "reps < 1");
  static const int32_t def_sigma_f32[] = {7, 8, 9, 10, 11, 12};
  static const int32_t def_sigma_f64[] = {4, 5, 6, 7, 8, 9, 10};
  static const int32_t def_blocks[] = {256, 512, 1024};
  if (!sigmas || n_sigmas <= 0) {
    sigmas = dtype == MERBIT_F32 ? def_sigma_f32 : def_sigma_f64;
    n_sigmas = dtype == MERBIT_F32 ? 6 : 7;
  }
  if (!block_lanes || n_blocks <= 0) {
    block_lanes = def_blocks;
    n_blocks = 3;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t vs = vsize(dtype);
  void *x = nullptr, *y0 = nullptr, *y1 = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (x) (void)hipFree(x);
    if (y0) (void)hipFree(y0);
    if (y1) (void)hipFree(y1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
#define TUNE_TRY(expr)                          \
  do {                                          \
    hipError_t _e = (expr);                     \
    if (_e != hipSuccess) {                     \
      cleanup();                                \
      return fail_hip(#expr, _e);               \
    }                                           \
  } while (0)
  TUNE_TRY(hipMalloc(&x, vs * (size_t)(n_cols > 0 ? n_cols : 1)));
  TUNE_TRY(hipMalloc(&y0, vs * (size_t)(n_rows > 0 ? n_rows : 1)));
  TUNE_TRY(hipMalloc(&y1, vs * (size_t)(n_rows > 0 ? n_rows : 1)));
  // x = 1.0f (F32) or the double with two 1.0f words (about 1.0000002, F64)
  TUNE_TRY(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(x), 0x3f800000u,
                             (vs / 4) * (size_t)(n_cols > 0 ? n_cols : 1), st));
  TUNE_TRY(hipEventCreate(&e0));
  TUNE_TRY(hipEventCreate(&e1));
  float best = -1.0f;
  int best_sigma = 0, best_b = 0;
  for (int i = 0; i < n_sigmas; ++i) {
    for (int j = 0; j < n_blocks; ++j) {
      if (us_out) us_out[i * n_blocks + j] = -1.0f;
      merbit_opts_t o = *opts_inout;
      o.sigma = sigmas[i];
      o.block_lanes = block_lanes[j];
      o.validate = 0;
      merbit_plan* p = nullptr;
      const int rc = merbit_plan_create(n_rows, n_cols, nnz, row_ptr, col_ind, values, dtype, &o,
                                        stream, &p);
      if (rc == MERBIT_EUNSUPPORTED) continue;
      if (rc != MERBIT_OK) {
        cleanup();
        return rc;
      }
      int r2 = merbit_zero_boundary(p, y0, stream);
      void* ys[2] = {y0, y1};
      for (int k = 0; r2 == MERBIT_OK && k < 2 + reps; ++k) {
        if (k == 2) {
          hipError_t e = hipEventRecord(e0, st);
          if (e != hipSuccess) r2 = fail_hip("hipEventRecord", e);
        }
        if (r2 == MERBIT_OK) r2 = run_fused(p, x, ys[k & 1], ys[(k + 1) & 1], st);
      }
      float ms = 0.0f;
      if (r2 == MERBIT_OK) {
        hipError_t e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) r2 = fail_hip("tune timing", e);
      }
      plan_free_all(p);
      if (r2 != MERBIT_OK) {
        cleanup();
        return r2;
      }
      const float us = ms * 1000.0f / (float)reps;
      if (us_out) us_out[i * n_blocks + j] = us;
      if (best < 0.0f || us < best) {
        best = us;
        best_sigma = sigmas[i];
        best_b = block_lanes[j];
      }
    }
  }
#undef TUNE_TRY
  cleanup();
  if (best < 0.0f) return fail(MERBIT_EUNSUPPORTED, "no candidate is built");
  opts_inout->sigma = best_sigma;
  opts_inout->block_lanes = best_b;
  return MERBIT_OK;
}

// ------------------------------------------------------------- adjoint --

static TileRowsArgs tile_rows_args(const merbit_plan* p) {
  TileRowsArgs a;
  memset(&a, 0, sizeof a);
  a.tile_x = p->tile_x;
  a.tile_y = p->tile_y;
  a.lane_desc = p->lane_desc;
  a.tile_num = (int32_t)p->tile_num;
  a.lane_num = (int32_t)p->lane_num;
  a.path_len = (int32_t)(p->nnz + p->n_rows);
  a.col = p->col;
  return a;
}

int merbit_transpose(merbit_plan* p, int32_t* rowT_ptr, int32_t* colT, int32_t* perm,
                     void* stream) {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->desc_bits != 32)
    return fail(MERBIT_EUNSUPPORTED, "this call needs a plan with 32-bit descriptors");
  if (!rowT_ptr || (p->nnz > 0 && (!colT || !perm)))
    return fail(MERBIT_EINVAL, "output array is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t m = p->nnz;
  int end_bit = 1;
  while (end_bit < 31 && ((int64_t)1 << end_bit) < p->n_cols) ++end_bit;
  size_t sort_bytes = 0;
  if (m > 0) HIP_TRY(transpose_sort_bytes(m, end_bit, &sort_bytes));
  int32_t *rows = nullptr, *iota = nullptr;
  uint32_t* keys = nullptr;
  void* tmp = nullptr;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    if (rows) (void)hipFree(rows);
    if (iota) (void)hipFree(iota);
    if (keys) (void)hipFree(keys);
    if (tmp) (void)hipFree(tmp);
  };
  hipError_t e = hipSuccess;
  const size_t mm = (size_t)(m > 0 ? m : 1);
  if (e == hipSuccess) e = hipMalloc(&rows, sizeof(int32_t) * mm);
  if (e == hipSuccess) e = hipMalloc(&iota, sizeof(int32_t) * mm);
  if (e == hipSuccess) e = hipMalloc(&keys, sizeof(uint32_t) * mm);
  if (e == hipSuccess) e = hipMalloc(&tmp, sort_bytes > 0 ? sort_bytes : 16);
  if (e == hipSuccess && m > 0) {
    TileRowsArgs a = tile_rows_args(p);
    a.rows = rows;
    e = launch_tile_rows(p->dtype, p->sigma, false, a, st);
  }
  if (e == hipSuccess)
    e = launch_transpose(p->col, rows, m, p->n_cols, end_bit, tmp, sort_bytes, keys, iota,
                         rowT_ptr, colT, perm, st);
  cleanup();
  if (e != hipSuccess) return fail_hip("transpose", e);
  p->last_stream = st;
  return MERBIT_OK;
}

int merbit_sddmm(merbit_plan* p, const void* g, const void* x, double scale, void* out,
                 void* stream) {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->desc_bits != 32)
    return fail(MERBIT_EUNSUPPORTED, "this call needs a plan with 32-bit descriptors");
  if (p->nnz == 0) return MERBIT_OK;
  if (!g || !x || !out) return fail(MERBIT_EINVAL, "g, x or out is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  TileRowsArgs a = tile_rows_args(p);
  a.g = g;
  a.x = x;
  a.scale = scale;
  a.out = out;
  HIP_TRY(launch_tile_rows(p->dtype, p->sigma, true, a, st));
  p->last_stream = st;
  return MERBIT_OK;
}

int merbit_gather_values(int dtype, int64_t nnz, const int32_t* perm, const void* src,
                         const void* src2, void* dst, void* stream) {
  if (dtype != MERBIT_F32 && dtype != MERBIT_F64) return fail(MERBIT_EUNSUPPORTED, "dtype");
  if (nnz < 0) return fail(MERBIT_EINVAL, "nnz < 0");
  if (nnz == 0) return MERBIT_OK;
  if (!perm || !src || !dst) return fail(MERBIT_EINVAL, "perm, src or dst is NULL");
  if (dst == src || (src2 && dst == src2)) return fail(MERBIT_EINVAL, "dst aliases an input");
  HIP_TRY(launch_gather_values(dtype, perm, src, src2, dst, nnz, static_cast<hipStream_t>(stream)));
  return MERBIT_OK;
}

int merbit_column_scale(int dtype, int64_t nnz, const int32_t* col, const void* a, const void* t,
                        const void* s, void* out, void* stream) {
  if (dtype != MERBIT_F32 && dtype != MERBIT_F64) return fail(MERBIT_EUNSUPPORTED, "dtype");
  if (nnz < 0) return fail(MERBIT_EINVAL, "nnz < 0");
  if (nnz == 0) return MERBIT_OK;
  if (!col || !a || !s || !out) return fail(MERBIT_EINVAL, "col, a, s or out is NULL");
  HIP_TRY(launch_column_scale(dtype, col, a, t, s, out, nnz, static_cast<hipStream_t>(stream)));
  return MERBIT_OK;
}

int merbit_pagerank_adjoint(merbit_plan* p, merbit_plan* pt, double alpha, double tol,
                            int max_iter, int check_every, const void* g, void* lam_inout,
                            int* iters_out, double* resid_out, void* stream) {
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
    HIP_TRY(launch_zero_boundary(pt->dtype, pt->tile_y, (int32_t)pt->chunk_num, pt->unit_tiles,
                                 pt->ybuf[0], st));
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
    auto enqueue = [&](hipStream_t s) -> int {
      for (int i = 0; i < len; ++i) {
        const int cur = (t0 + i) & 1, b = yb0 ^ (i & 1);
        const int r = run_fused(pt, ls[cur], pt->ybuf[b], pt->ybuf[b ^ 1], s);
        if (r != MERBIT_OK) return r;
        HIP_TRY(launch_adj_update(p->dtype, pt->ybuf[b], ls[cur], ls[cur ^ 1], g, p->dmask, n,
                                  alpha, pt->partials[cur], pt->reduce_grid,
                                  pt->partials[cur ^ 1], pt->reduce_grid, s));
      }
      return MERBIT_OK;
    };
    rc = len == check_every ? run_chunk(pt, kLoopAdjoint, t0 & 1, yb0, len, 0, lam_inout, alpha,
                                        enqueue, st, g)
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
}

// ------------------------------------------------------------ BiCGSTAB --

int merbit_bicgstab(merbit_plan* p, const void* b, void* x_inout, double tol, int max_iter,
                    int check_every, int* iters_out, double* resid_out, void* stream) {
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
  HIP_TRY(launch_zero_boundary(p->dtype, p->tile_y, (int32_t)p->chunk_num, p->unit_tiles, a.t,
                               st));
  int rc = run_fused(p, x_inout, a.t, p->bvec[3], st);
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
}

int merbit_profile_enable(merbit_plan* p, int enable) {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  p->profiling = enable != 0;
  return MERBIT_OK;
}

int merbit_profile_read(merbit_plan* p, int64_t* launches, double* total_ms) {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  double total = 0.0;
  for (size_t k = 0; k < p->events_used; ++k) {
    HIP_TRY(hipEventSynchronize(p->events[k].second));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, p->events[k].first, p->events[k].second));
    total += ms;
  }
  if (launches) *launches = (int64_t)p->events_used;
  if (total_ms) *total_ms = total;
  p->events_used = 0;
  return MERBIT_OK;
}

void merbit_plan_destroy(merbit_plan* p) { plan_free_all(p); }

}  // extern "C"
