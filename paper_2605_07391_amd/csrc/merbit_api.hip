// C ABI of libmerbit (declared in include/merbit.h), plan side: the plan
// object's life cycle, options and hot-column cache, the SpMV entry points,
// kernel timing and the helpers the iterative drivers share.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <exception>
#include <new>

#include "merbit_host.hpp"

namespace merbit {

static thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int host_exception() noexcept {
  int code = MERBIT_EHIP;
  const char* msg = "unexpected C++ exception on the host";
  try {
    throw;
  } catch (const std::bad_alloc&) {
    code = MERBIT_ENOMEM;
    msg = "host memory exhausted";
  } catch (...) {
  }
  try {
    g_last_error = msg;
  } catch (...) {
  }
  return code;
}

int fail_hip(const char* what, hipError_t e) {
  return fail(e == hipErrorOutOfMemory ? MERBIT_ENOMEM : MERBIT_EHIP,
              std::string(what) + ": " + hipGetErrorString(e));
}

static void drop_graphs(merbit_plan* p) {
  for (auto& g : p->loop_graphs) (void)hipGraphExecDestroy(g.exec);
  p->loop_graphs.clear();
}

void plan_free_all(merbit_plan* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  drop_graphs(p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  void* bufs[] = {p->tile_x, p->tile_y, p->lane_desc, p->lane_desc64, p->scratch, p->dmask,
                  p->ybuf[0], p->ybuf[1], p->xwork, p->partials[0], p->partials[1], p->hot_cols,
                  p->colx, p->x_hot, p->pbuf[0], p->pbuf[1], p->pbuf[2], p->ppart, p->psums[0],
                  p->psums[1], p->psrc, p->multi_chunk_row, p->multi_chunk_graph,
                  p->multi_chunk_ptr, p->multi_gsize, p->multi_part, p->multi_gsum[0],
                  p->multi_gsum[1], p->multi_hot_graph, p->bvec[0], p->bvec[1], p->bvec[2], p->bvec[3], p->bvec[4],
                  p->bvec[5], p->bvec[6], p->bpart[0], p->bpart[1], p->bpart[2], p->bpart[3],
                  p->bpart[4], p->bpart[5], p->bpart[6], p->sperm, p->scol, p->svals, p->swords,
                  p->yv[0], p->yv[1], p->range_tile, p->hot_off, p->queue};
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
  a.col = p->hot_n > 0 ? p->colx : (p->stripes > 1 ? p->scol : p->col);
  a.val = p->stripes > 1 ? p->svals : p->values;
  a.x = x;
  a.x_hot = p->hot_n > 0 ? (p->hot_all ? x : p->x_hot) : nullptr;
  a.y = y;
  a.z = z;
  a.tile_num = (int32_t)p->tile_num;
  a.lane_num = (int32_t)p->lane_num;
  a.path_len = (int32_t)(p->nnz + p->plan_rows);
  a.n_rows = (int32_t)p->plan_rows;
  a.chunk_num = (int32_t)p->chunk_num;  // commit units of the block kernel
  a.chunks_per_block = p->chunks_per_block;
  a.grid = p->grid;
  a.hot_n = p->hot_n;
  a.ranges = p->ranges;
  a.range_tile = p->range_tile;
  a.hot_off = p->hot_off;
  a.queue = p->queue;
  return a;
}

int zero_boundary(merbit_plan* p, void* v, hipStream_t st) {
  if (p->stripes > 1 || p->chunk_num == 0) return MERBIT_OK;
  HIP_TRY(launch_zero_boundary(p->dtype, p->tile_y, (int32_t)p->chunk_num, p->unit_tiles, v, st));
  return MERBIT_OK;
}

// Launch the fused kernel (after the hot gather), bracketed by events when
// profiling is on.  A striped plan runs the kernel on its own dual buffers of
// A' x and then sums each row's stripes into y (inside the same events).
int run_fused(merbit_plan* p, const void* x, void* y, void* z, hipStream_t st, bool hot_ready,
              bool timed) {
  if (p->chunk_num == 0) {
    // no tiles: the planned matrix has no rows (a striped plan always has
    // nonzeros, so it never gets here)
    return MERBIT_OK;
  }
  if (p->hot_n > 0 && !p->hot_all && !hot_ready)
    HIP_TRY(launch_hot_gather(p->dtype, x, p->hot_cols, p->hot_n, p->x_hot, st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool events = p->profiling && timed;
  if (events) {
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
  if (p->stripes > 1) {
    const int c = p->yv_cur;
    HIP_TRY(launch_spmv_wave(p->dtype, p->sigma, p->waves, p->hot_n > 0, p->hot_lds_bytes,
                             spmv_args(p, x, p->yv[c], p->yv[c ^ 1]), st, p->desc_bits == 64));
    HIP_TRY(launch_stripe_combine(p->dtype, p->stripes, p->yv[c], p->plan_rows, p->swords,
                                  p->words, p->n_rows, y, st));
    p->yv_cur = c ^ 1;
  } else if (p->commit == MERBIT_COMMIT_WAVE)
    HIP_TRY(launch_spmv_wave(p->dtype, p->sigma, p->waves, p->hot_n > 0, p->hot_lds_bytes,
                             spmv_args(p, x, y, z), st, p->desc_bits == 64));
  else
    HIP_TRY(launch_spmv(p->dtype, p->sigma, p->waves, p->hot_n > 0, p->hot_lds_bytes,
                        spmv_args(p, x, y, z), st));
  if (events) HIP_TRY(hipEventRecord(e1, st));
  p->last_stream = st;
  return MERBIT_OK;
}

// A buffer or value array that graphs captured has changed.
void invalidate_graphs(merbit_plan* p) {
  ++p->generation;
  if (!p->loop_graphs.empty()) {
    (void)hipDeviceSynchronize();
    drop_graphs(p);
  }
}

// Bit u of the dangling mask is set when column u holds no nonzero (vertex u
// has no out-edge); built once per plan, shared by both PageRank drivers.
int ensure_dmask(merbit_plan* p, hipStream_t st) {
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

int ensure_pagerank_state(merbit_plan* p, hipStream_t st) {
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
// blocks_per_cu), every wavefront striding over the tiles; a striped plan
// rounds the grid down to a multiple of the XCD count and gives each XCD's
// blocks (block b runs on XCD b mod 8) one contiguous range of tiles.
int size_grid(merbit_plan* p) {
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
    if (p->stripes > 1 && p->grid >= kXcds) {
      p->grid -= p->grid % kXcds;
      p->ranges = kXcds;
    } else {
      p->ranges = 1;
    }
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
int64_t hot_cap_lds(const merbit_plan* p) {
  int lds_block = 0;
  if (hipDeviceGetAttribute(&lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) !=
      hipSuccess)
    return 0;
  int64_t cap = ((int64_t)lds_block - (int64_t)static_lds_bytes(p)) / (int64_t)vsize(p->dtype);
  return (cap / 256) * 256;
}

constexpr int64_t kHotMinTilesPerWave = 4;

static int build_hot_cache(merbit_plan* p, int cap_req, hipStream_t st) {
  p->hot_n = 0;
  if (cap_req == 0 || p->nnz == 0 || p->n_cols == 0) return MERBIT_OK;
  // Automatic sizing enables the cache for the wave kernel only: with the
  // block kernel the LDS fill leaves one block per CU and its barriers make
  // every wavefront of a block wait for the slowest, which measured slower
  // than no cache at every size (R-MAT 22).  An explicit size is honoured.
  if (cap_req < 0 && p->commit != MERBIT_COMMIT_WAVE) return MERBIT_OK;
  // Nor for a plan too small to amortise the fill: with fewer than
  // kHotMinTilesPerWave tiles per wavefront of one block per CU, each block
  // copies x into LDS for about one tile of work (the 10,000-vertex
  // Chung-Lu matrix: 7.3 instead of 8.9 us per SpMV without the cache).
  if (cap_req < 0) {
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device));
    if (p->tile_num < (int64_t)kHotMinTilesPerWave * cus * p->waves) return MERBIT_OK;
  }
  if (!kernel_supported(p, true))
    return cap_req > 0 ? fail(MERBIT_EUNSUPPORTED, "hot cache not built for this block size")
                       : MERBIT_OK;
  const size_t vs = vsize(p->dtype);
  const int64_t cap_lds = hot_cap_lds(p);
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
    // sampled counts: one nonzero in `sample`, about two samples per column;
    // the cache takes the columns of count >= t for the smallest t that keeps
    // them within cap (a tie at the cut is left out whole)
    int64_t sample = p->nnz / (2 * nc);
    sample = sample < 1 ? 1 : (sample > 8 ? 8 : sample);
    HotSeg seg{};
    seg.lo = 0;
    seg.len = p->nnz;
    seg.span = nc;
    seg.c_lo = 0;
    seg.sample = (int32_t)sample;
    // one temporary allocation: the selection's work space, then its result
    const size_t wb = (hot_select_layout(&seg, 1) + 255) & ~(size_t)255;
    unsigned char* tmp = nullptr;
    auto release = [&]() {
      (void)hipStreamSynchronize(st);
      if (tmp) (void)hipFree(tmp);
    };
    hipError_t e = hipMalloc(&tmp, wb + sizeof(HotSel));
    HotSel* sel_dev = reinterpret_cast<HotSel*>(tmp + wb);
    if (e == hipSuccess) e = hipMalloc(&p->hot_cols, sizeof(int32_t) * (size_t)cap);
    if (e == hipSuccess)
      e = hot_select_ranges(p->col, &seg, 1, cap, true, tmp, p->hot_cols, sel_dev, st);
    HotSel sel{};
    if (e == hipSuccess)
      e = hipMemcpyAsync(&sel, sel_dev, sizeof sel, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      release();
      return fail_hip("hot column selection", e);
    }
    const int64_t taken = sel.taken;
    const double covered = sel.covered;
    p->hot_coverage = covered * (double)sample / (double)p->nnz;  // estimate when sampled
    if (p->hot_coverage > 1.0) p->hot_coverage = 1.0;
    const bool keep = taken > 0 && (cap_req > 0 || p->hot_coverage >= 0.2);
    if (keep) {
      e = hipMalloc(&p->colx, sizeof(int32_t) * (size_t)p->nnz);
      if (e == hipSuccess) e = hot_recode_ranges(p->col, &seg, 1, tmp, p->colx, st);
      if (e == hipSuccess) e = hipMalloc(&p->x_hot, vs * (size_t)taken);
      if (e == hipSuccess) p->hot_n = (int32_t)taken;
    } else {
      (void)hipStreamSynchronize(st);
      (void)hipFree(p->hot_cols);
      p->hot_cols = nullptr;
    }
    release();
    if (e != hipSuccess) return fail_hip("hot column recode", e);
  }
  if (p->hot_n > 0) {
    if (p->hot_all) {
      // slot = column: the recoded stream is -1 - col
      HIP_TRY(hipMalloc(&p->colx, sizeof(int32_t) * (size_t)p->nnz));
      HIP_TRY(hot_recode_all(p->col, p->nnz, p->colx, st));
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

int build_tile(merbit_plan* p, const int32_t* row_ptr, hipStream_t st) {
  const int64_t L = p->nnz + p->plan_rows;
  const int sigma = p->sigma;
  p->tile_num = (L + (int64_t)kOmega * sigma - 1) / ((int64_t)kOmega * sigma);
  p->lane_num = (L + sigma - 1) / sigma;
  HIP_TRY(hipMalloc(&p->tile_x, sizeof(int32_t) * (size_t)(p->tile_num + 1)));
  HIP_TRY(hipMalloc(&p->tile_y, sizeof(uint32_t) * (size_t)(p->tile_num + 1)));
  const size_t lanes = (size_t)(p->lane_num > 0 ? p->lane_num : 1);
  if (p->desc_bits == 64) HIP_TRY(hipMalloc(&p->lane_desc64, sizeof(uint64_t) * lanes));
  else HIP_TRY(hipMalloc(&p->lane_desc, sizeof(uint32_t) * lanes));
  if (p->plan_rows == 0) {
    // empty path: TILE = {[0], [0]}
    HIP_TRY(hipMemsetAsync(p->tile_x, 0, sizeof(int32_t), st));
    HIP_TRY(hipMemsetAsync(p->tile_y, 0, sizeof(uint32_t), st));
    return MERBIT_OK;
  }
  PlanArgs pa;
  pa.row_ptr = row_ptr;
  pa.n_rows = (int32_t)p->plan_rows;
  pa.nnz = (int32_t)p->nnz;
  pa.sigma = sigma;
  pa.bits = p->bits;
  pa.lane_num = p->lane_num;
  pa.tile_num = p->tile_num;
  pa.tile_x = p->tile_x;
  pa.tile_y = p->tile_y;
  pa.lane_desc = p->lane_desc;
  pa.lane_desc64 = p->lane_desc64;
  HIP_TRY(launch_plan(pa, st));
  return MERBIT_OK;
}

}  // namespace merbit

using namespace merbit;

extern "C" {

const char* merbit_last_error(void) { return g_last_error.c_str(); }

const char* merbit_version(void) { return "merbit-mi355x 0.1 (gfx950, wave64)"; }

void merbit_opts_init(merbit_opts_t* o) {
  if (!o) return;
  memset(o, 0, sizeof *o);
  o->hot_columns = -1;
  o->validate = 1;
}

int merbit_plan_create(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t* row_ptr,
                       const int32_t* col_ind, const void* values, int dtype,
                       const merbit_opts_t* opts_in, void* stream, merbit_plan** out) try {
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
  // defaults: the best block size measured for each family (R-MAT 22)
  if (block_lanes == 0)
    block_lanes = commit != MERBIT_COMMIT_WAVE                   ? 256
                  : (dtype == MERBIT_F32 && opts.desc_bits != 64) ? 1024
                                                                  : 512;
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
                                       ? "64-bit descriptors: sigma 16, 20, 24, 28 or 32, 256 or 512 lanes"
                                       : "64-bit descriptors: sigma 14, 16, 20 or 24, 256 or 512 lanes")
                : commit == MERBIT_COMMIT_WAVE ? "block_lanes must be 256, 512 or 1024"
                                               : "block_lanes must be 128, 256, 512 or 1024");
  if (opts.blocks_per_cu < 0) return fail(MERBIT_EINVAL, "blocks_per_cu < 0");
  const int stripes = opts.stripes <= 1 ? 1 : opts.stripes;
  if (opts.stripes < 0 || (stripes & (stripes - 1)) != 0 || stripes > 32)
    return fail(MERBIT_EINVAL, "stripes must be 0, 1, 2, 4, 8, 16 or 32");
  if (stripes > 1 && commit != MERBIT_COMMIT_WAVE)
    return fail(MERBIT_EUNSUPPORTED, "column stripes need the wave commit kernel");
  if (stripes > 1 && nnz >= ((int64_t)1 << 30))
    return fail(MERBIT_EUNSUPPORTED, "column stripes need nnz < 2^30");

  hipStream_t st = static_cast<hipStream_t>(stream);
  merbit_plan* p = new merbit_plan();
  // a host exception during the build (the error returns free the plan
  // themselves) frees it on the way out
  struct FreeOnThrow {
    merbit_plan* p;
    ~FreeOnThrow() {
      if (std::uncaught_exceptions() > 0) plan_free_all(p);
    }
  } free_on_throw{p};
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
#undef CREATE_TRY
  int rc;
  if (stripes > 1 && nnz > 0) {
    p->stripes = stripes;
    rc = build_striped(p, row_ptr, hot_columns, st);
  } else {
    p->plan_rows = n_rows;
    rc = build_tile(p, row_ptr, st);
    if (rc == MERBIT_OK) rc = build_hot_cache(p, hot_columns, st);
    if (rc == MERBIT_OK) rc = size_grid(p);
  }
  if (rc == MERBIT_OK && p->commit == MERBIT_COMMIT_WAVE && p->tile_num > 0 && p->ranges > 1 &&
      p->tile_num >= (int64_t)kQueueMinTilesPerWave * p->grid * p->waves) {
    // tile queues of the wave kernel, zero before the first launch.  Only with
    // ranges: one counter for a whole grid (4,096 wavefronts on R-MAT 22) is
    // served one atomic at a time and made a plain plan's SpMV 4x slower; and
    // only with several tiles per wavefront: on R-MAT 20 (about 6) the
    // atomics cost more than the balance gains (78 against 71 us).
    const size_t qb = sizeof(unsigned long long) * kQueueStride * (size_t)p->ranges;
    hipError_t qe = hipMalloc(&p->queue, qb);
    if (qe == hipSuccess) qe = hipMemsetAsync(p->queue, 0, qb, st);
    if (qe != hipSuccess) rc = fail_hip("tile queue", qe);
  }
  if (rc != MERBIT_OK) {
    std::string msg = g_last_error;
    plan_free_all(p);
    return fail(rc, msg);
  }
  *out = p;
  return MERBIT_OK;
} catch (...) {
  return merbit::host_exception();
}

int merbit_plan_set_values(merbit_plan* p, const void* values) try {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->nnz > 0 && !values) return fail(MERBIT_EINVAL, "values is NULL");
  if (p->stripes > 1) {
    // the stacked copy is rewritten in place: graphs keep valid pointers
    p->values = values;
    return stripes_copy_values(p, values, p->last_stream);
  }
  if (values != p->values) invalidate_graphs(p);
  p->values = values;
  return MERBIT_OK;
} catch (...) {
  return merbit::host_exception();
}

int merbit_plan_info(merbit_plan* p, merbit_plan_info_t* info) try {
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
  info->stripes = p->stripes;
  info->ranges = p->ranges;
  info->plan_rows = p->plan_rows;
  info->graph_captures = p->graph_captures;
  info->graph_replays = p->graph_replays;
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
} catch (...) {
  return merbit::host_exception();
}

int merbit_plan_export(merbit_plan* p, int32_t* tile_x, uint32_t* tile_y, void* lane_desc,
                       int64_t* tile_num, int64_t* lane_num) try {
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
} catch (...) {
  return merbit::host_exception();
}

int merbit_zero_boundary(merbit_plan* p, void* v, void* stream) try {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->chunk_num == 0) return MERBIT_OK;
  if (!v) return fail(MERBIT_EINVAL, "vector is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int rc = zero_boundary(p, v, st);
  if (rc != MERBIT_OK) return rc;
  p->last_stream = st;
  return MERBIT_OK;
} catch (...) {
  return merbit::host_exception();
}

int merbit_spmv(merbit_plan* p, const void* x, void* y, void* stream) try {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->n_rows == 0) return MERBIT_OK;
  if (!y || (p->nnz > 0 && !x)) return fail(MERBIT_EINVAL, "x or y is NULL");
  if (x == y) return fail(MERBIT_EINVAL, "x and y alias");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int rc = zero_boundary(p, y, st);
  if (rc != MERBIT_OK) return rc;
  return run_fused(p, x, y, nullptr, st);
} catch (...) {
  return merbit::host_exception();
}

int merbit_spmv_dual(merbit_plan* p, const void* x, void* y, void* z, void* stream) try {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->n_rows == 0) return MERBIT_OK;
  if (!y || !z || (p->nnz > 0 && !x)) return fail(MERBIT_EINVAL, "x, y or z is NULL");
  if (x == y || y == z || x == z) return fail(MERBIT_EINVAL, "x, y, z must be distinct");
  return run_fused(p, x, y, z, static_cast<hipStream_t>(stream));
} catch (...) {
  return merbit::host_exception();
}

int merbit_profile_enable(merbit_plan* p, int enable) try {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  p->profiling = enable != 0;
  return MERBIT_OK;
} catch (...) {
  return merbit::host_exception();
}

int merbit_profile_read(merbit_plan* p, int64_t* launches, double* total_ms) try {
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
} catch (...) {
  return merbit::host_exception();
}

void merbit_plan_destroy(merbit_plan* p) { plan_free_all(p); }

}  // extern "C"
