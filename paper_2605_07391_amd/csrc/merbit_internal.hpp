// Internal declarations of libmerbit: wavefront helpers and the kernel
// launchers that the C-ABI layer (merbit_api.hip) dispatches to.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

namespace merbit {

constexpr int kOmega = 64;                 // lanes per tile = CDNA wavefront size
constexpr int kSlab = 32;                  // right-hand-side columns per SpMM launch
constexpr uint32_t kRowMask = 0x7FFFFFFFu; // tile_y: row index
constexpr uint32_t kFastBit = 0x80000000u; // tile_y: long-row (single-row) tile mark
constexpr int kMaxSigma = 12;              // 2 ceil(log2(64 sigma)) + sigma <= 32
constexpr int kMaxSigma64 = 40;            // 2 ceil(log2(64 sigma)) + sigma <= 64
constexpr int kHotHistBins = 65536;        // column-count histogram of the hot cache
constexpr int kXcds = 8;                   // MI355X: accelerator dies, one L2 each

// ceil(log2(v)) for v >= 1: width of the x_offset / y_offset fields.
__host__ __device__ constexpr int ceil_log2(int v) {
  int b = 0;
  while ((1 << b) < v) ++b;
  return b;
}

// ------------------------------------------------------------ device side --
#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)

// Make this wavefront's LDS writes visible to its other lanes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Device-scope float add on global memory (native global_atomic_add_f32/f64).
template <typename V>
__device__ __forceinline__ void global_add(V* p, V v) {
  unsafeAtomicAdd(p, v);
}

template <typename V>
__device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// DPP move of a 32-bit value (lanes without a source lane receive 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xF, false);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(float, dpp_i<CTRL, ROW_MASK>(__builtin_bit_cast(int, v)));
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = dpp_i<CTRL, ROW_MASK>((int)(b & 0xFFFFFFFFll));
  const int hi = dpp_i<CTRL, ROW_MASK>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// DPP controls (GFX9): row shift right by n within rows of 16 lanes,
// broadcast of lane 15 / 31 of a row into the next row(s), whole-wave shift.
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143, kWaveShr1 = 0x138;

// Inclusive segmented scan across the wavefront.  seg = index of the last
// segment head at or before this lane (lane 0 is always a head).  Each step
// adds the value from `dist` lanes below only if no head lies in between.
template <typename V>
__device__ __forceinline__ V wave_segmented_scan(V v, int lid, int seg) {
  V t;
  t = dpp_move<kRowShr1, 0xF>(v);
  if (seg <= lid - 1) v += t;
  t = dpp_move<kRowShr2, 0xF>(v);
  if (seg <= lid - 2) v += t;
  t = dpp_move<kRowShr4, 0xF>(v);
  if (seg <= lid - 4) v += t;
  t = dpp_move<kRowShr8, 0xF>(v);
  if (seg <= lid - 8) v += t;
  // rows 1 and 3 take the end of rows 0 and 2
  t = dpp_move<kRowBcast15, 0xA>(v);
  if ((lid & 16) && seg < (lid & ~15)) v += t;
  // rows 2 and 3 take lane 31
  t = dpp_move<kRowBcast31, 0xC>(v);
  if (lid >= 32 && seg < 32) v += t;
  return v;
}

template <typename V>
__device__ __forceinline__ V wave_total(V v) {
  // the segmented scan with a single head at lane 0 is a plain inclusive scan
  v = wave_segmented_scan(v, (int)__lane_id(), 0);
  return __shfl(v, kOmega - 1, kOmega);
}

#endif

// -------------------------------------------------------------- launchers --
// Row of each nonzero of tile t, relative to the tile's first row, into
// wrow[0 .. x_se) (LDS of one wavefront).  Lane j replays its descriptor
// (Sec. 4.1.1): its k-th right step is nonzero x_off + (right steps before it)
// of the tile and lies in row y_off + (down steps before it).  A long-row tile
// has one row.  The caller synchronises the wavefront before reading wrow.
template <int SIGMA>
__device__ __forceinline__ void tile_nz_rows(const uint32_t* __restrict__ lane_desc,
                                             int lane_num, int path_len, int t, uint32_t tyw,
                                             int x_se, int lid, int32_t* wrow) {
  constexpr int BITS = ceil_log2(kOmega * SIGMA);
  constexpr uint32_t FMASK = (1u << BITS) - 1u;
  if (x_se <= 0) return;
  if (tyw & kFastBit) {
    for (int q = lid; q < x_se; q += kOmega) wrow[q] = 0;
    return;
  }
  const int j = t * kOmega + lid;
  if (j >= lane_num) return;
  const uint32_t d = lane_desc[j];
  int xo = (int)(d & FMASK);
  int yo = (int)((d >> BITS) & FMASK);
  const uint32_t flags = d >> (2 * BITS);
  const int steps = min(SIGMA, path_len - j * SIGMA);
  for (int k = 0; k < steps; ++k) {
    if ((flags >> k) & 1u) {
      ++yo;
    } else {
      wrow[xo] = yo;
      ++xo;
    }
  }
}

// Threads per block of the reduction kernels.
constexpr int kReduceThreads = 256;

// Sum (a, b) over the block in a fixed order; thread 0 gets the totals.
__device__ __forceinline__ void block_sum2(double& a, double& b) {
  __shared__ double sa[kReduceThreads / kOmega], sb[kReduceThreads / kOmega];
  const int tid = threadIdx.x, lid = tid & (kOmega - 1), wid = tid / kOmega;
  a = wave_sum(a);
  b = wave_sum(b);
  __syncthreads();  // sa/sb may still be read from a previous call
  if (lid == 0) {
    sa[wid] = a;
    sb[wid] = b;
  }
  __syncthreads();
  if (tid == 0) {
    double ta = 0.0, tb = 0.0;
    for (int w = 0; w < kReduceThreads / kOmega; ++w) {
      ta += sa[w];
      tb += sb[w];
    }
    a = ta;
    b = tb;
  }
}

struct PlanArgs {
  const int32_t* row_ptr;
  int32_t n_rows;
  int32_t nnz;
  int32_t sigma;
  int32_t bits;
  int64_t lane_num;
  int64_t tile_num;
  int32_t* tile_x;
  uint32_t* tile_y;
  uint32_t* lane_desc;      // 32-bit descriptors, or
  uint64_t* lane_desc64;    // 64-bit descriptors (exactly one is set)
};

struct SpmvArgs {
  const int32_t* tile_x;
  const uint32_t* tile_y;
  const uint32_t* lane_desc;
  const uint64_t* lane_desc64;  // 64-bit descriptor plans (wave kernel only)
  const int32_t* col;   // column stream: col_ind, or the recoded one with hot slots < 0
  const void* val;
  const void* x;
  const void* x_hot;    // hot x values (hot variant), hot_n of them
  void* y;
  void* z;              // dual buffer to clear at boundary rows, or nullptr
  int32_t tile_num;
  int32_t lane_num;
  int32_t path_len;     // nnz + n_rows
  int32_t n_rows;
  int32_t chunk_num;    // chunks of WAVES tiles (the commit unit)
  int32_t chunks_per_block;
  int32_t grid;
  int32_t hot_n;
  // wave kernel: tiles split into `ranges` contiguous parts (1: one part);
  // block b works on part b % ranges, whose tiles are
  // [range_tile[k], range_tile[k + 1]) and whose hot x values are
  // x_hot[hot_off[k] .. hot_off[k + 1]).  grid is a multiple of ranges.
  int32_t ranges;
  const int32_t* range_tile;
  const int32_t* hot_off;
  // wave kernel: per range, two counters kQueueStride words apart from the
  // next range's: [0] tiles taken beyond the first one of each wavefront, [1]
  // wavefronts finished.  Zero before a launch; the launch's last wavefront of
  // the range sets them back to zero.  nullptr (plans without ranges, or with
  // fewer than kQueueMinTilesPerWave tiles per wavefront): every wavefront
  // takes a fixed arithmetic sequence of tiles.
  unsigned long long* queue;
};

// words between two ranges' tile-queue counters (one 256-byte line each)
constexpr int kQueueStride = 32;
// tiles per wavefront below which a striped plan keeps the fixed tile sequence
constexpr int kQueueMinTilesPerWave = 12;

struct SpmmArgs {
  const int32_t* tile_x;
  const uint32_t* tile_y;
  const uint32_t* lane_desc;
  const int32_t* col;
  const void* val;
  const void* X;   // first column of the slab; row stride ldx
  void* Y;         // row stride ldy
  void* Z;         // dual buffer (row stride ldz) cleared at tile starts, or nullptr
  int64_t ldx, ldy, ldz;
  int64_t x_rows;  // rows of X (the matrix's column count)
  int32_t k;       // columns in this slab, 1..64
  int32_t tile_num;
  int32_t lane_num;
  int32_t path_len;
  int32_t n_rows;
  // A personalised-PageRank step finished in the commit (Xn == nullptr: plain
  // Y = A X).  Rows strictly inside a tile become Xn = alpha (A X) plus the
  // teleport at their column's source and add their dangling mass to the
  // block's part; a tile's first and last rows still go to Y, which
  // ppr_fixup finishes (and clears) after the launch.
  void* Xn;                // next iterate: the slab's first column, row stride ldx
  const int32_t* src;      // per column of the slab: its source row
  const double* sums_in;   // per column of the slab: (dangling mass, l1 change) of X
  const uint32_t* dmask;   // dangling rows, one bit each
  double* part;            // [blocks][64][2]: the block's (dangling mass, 0) per column
  double alpha;
  int32_t col0;            // the slab's first column (its place among part's 64)
  int32_t dmask_words;     // ceil(n_rows / 32)
};

// CSR checks; *flags gets bit 0: row_ptr[0] != 0, bit 1: row_ptr[n] != nnz,
// bit 2: row_ptr decreasing, bit 3: column out of range.
hipError_t launch_validate(const int32_t* row_ptr, const int32_t* col, int64_t n_rows,
                           int64_t n_cols, int64_t nnz, unsigned* flags, hipStream_t st);
hipError_t launch_plan(const PlanArgs& a, hipStream_t st);
hipError_t launch_count_fast(const uint32_t* tile_y, int64_t tile_num,
                             unsigned long long* count, hipStream_t st);

bool spmv_supported(int dtype, int sigma, int waves, bool hot);
// dynamic LDS bytes of the hot variant go in hot_lds_bytes (0 for the plain one)
hipError_t launch_spmv(int dtype, int sigma, int waves, bool hot, size_t hot_lds_bytes,
                       const SpmvArgs& a, hipStream_t st);
// allow the hot variant to use `bytes` of dynamic LDS
hipError_t spmv_set_hot_lds(int dtype, int sigma, int waves, size_t bytes);
// wave-granular persistent kernel (commit unit = one tile)
bool spmv_wave_supported(int dtype, int sigma, int waves, bool hot, bool desc64 = false);
hipError_t launch_spmv_wave(int dtype, int sigma, int waves, bool hot, size_t hot_lds_bytes,
                            const SpmvArgs& a, hipStream_t st, bool desc64 = false);
hipError_t spmv_wave_set_hot_lds(int dtype, int sigma, int waves, size_t bytes,
                                 bool desc64 = false);

constexpr int kMaxLdsDevices = 64;
// Dynamic-LDS opt-in of one kernel instance.  The attribute belongs to the
// instance (per device), not to a plan, so it only ever grows: a plan built
// later with a smaller hot set must not shrink what an earlier plan of the
// same instance launches with.
inline hipError_t raise_dynamic_lds(const void* fn, size_t bytes, std::mutex& mu,
                                    size_t* granted) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxLdsDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (bytes <= granted[dev]) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) granted[dev] = bytes;
  return e;
}

// Hot-column cache.
// The hot columns of R column streams are chosen at once (one stream per
// tile range of a column-stripe plan, R = 1 for a plain plan).  Range k
// counts col[lo .. lo + len) on every sample-th nonzero over its column span
// c_lo .. c_lo + span - 1 and takes the at most `cap` columns of largest
// count, ties by increasing column (whole_ties: a tie at the cut is taken
// whole or not at all), in slots 0 .. taken - 1 of increasing column.
struct HotSeg {
  int64_t lo, len;  // the range's nonzeros in the column stream
  int64_t span;     // its columns: c_lo .. c_lo + span - 1
  int64_t coff;     // its counts and slot map in the work space (hot_select_layout)
  int64_t boff;     // its selection blocks in the work space (hot_select_layout)
  int32_t c_lo;
  int32_t sample;   // >= 1
};
struct HotSel {
  int32_t t;       // cut count: columns above it are taken
  int32_t extra;   // columns at the cut count taken (the first in column order)
  int64_t taken;
  double covered;  // sum of the taken columns' (sampled) counts
};
// Sets every range's coff and boff; returns the bytes of the work space that
// hot_select_ranges and hot_recode_ranges take for these ranges.
size_t hot_select_layout(HotSeg* segs, int R);
// Range k's hot columns (full column indices) go to hot_cols[k * cap ..] and
// its HotSel to sel[k] (both device); the work space keeps each range's slot
// map for hot_recode_ranges.  Asynchronous on st; segs (host) must stay
// alive until the stream has passed this call.
hipError_t hot_select_ranges(const int32_t* col, const HotSeg* segs, int R, int64_t cap,
                             bool whole_ties, void* work, int32_t* hot_cols, HotSel* sel,
                             hipStream_t st);
// colx[lo + i] = -1 - slot for a column that hot_select_ranges took, the
// column otherwise, over every range
hipError_t hot_recode_ranges(const int32_t* col, const HotSeg* segs, int R, const void* work,
                             int32_t* colx, hipStream_t st);
// colx[k] = -1 - col[k]: a cache of every column (slot = column)
hipError_t hot_recode_all(const int32_t* col, int64_t nnz, int32_t* colx, hipStream_t st);
// packed = range 0's taken columns, then range 1's, ...: the parts
// stage[k * cap ..] of sel[k].taken columns each (sel on the device)
hipError_t hot_pack_ranges(const int32_t* stage, int64_t cap, const HotSel* sel, int R,
                           int32_t* packed, hipStream_t st);
// out[i] = src[idx[i]] for i < n <= kMaxPeek: a few scattered values of a
// device array gathered for one copy to the host (idx on the host)
constexpr int kMaxPeek = 64;
hipError_t launch_peek(const int32_t* src, const int64_t* idx, int n, int32_t* out,
                       hipStream_t st);
hipError_t launch_hot_gather(int dtype, const void* x, const int32_t* hot_cols, int32_t hot_n,
                             void* x_hot, hipStream_t st);
// zero v at tile_y[k * unit] for k < units (the first row of every commit unit)
hipError_t launch_zero_boundary(int dtype, const uint32_t* tile_y, int32_t units, int32_t unit,
                                void* v, hipStream_t st);

// PageRank pieces.
hipError_t launch_dangling_mask(const int32_t* col, int64_t nnz, int64_t n,
                                unsigned char* scratch_bytes, uint32_t* dmask, hipStream_t st);
hipError_t launch_dangling_sum(int dtype, const void* x, const uint32_t* dmask, int64_t n,
                               double* partials_out, int grid, hipStream_t st);
// resid: also the l1 change (second components of partials_out; else 0)
hipError_t launch_pr_update(int dtype, const void* y, const void* x_old, void* x_new,
                            const uint32_t* dmask, int64_t n, double alpha,
                            const double* partials_in, int n_in, double* partials_out, int grid,
                            hipStream_t st, const int32_t* hot_cols = nullptr,
                            int32_t hot_n = 0, void* x_hot = nullptr, bool resid = true);
int pr_reduce_grid(int64_t n);

// Adjoint pieces.
struct TileRowsArgs {
  const int32_t* tile_x;
  const uint32_t* tile_y;
  const uint32_t* lane_desc;
  int32_t tile_num, lane_num, path_len;
  const int32_t* col;
  const void* g;    // SDDMM: per-row factor
  const void* x;    // SDDMM: per-column factor
  double scale;
  void* out;        // SDDMM: per-nonzero output
  int32_t* rows;    // row of every nonzero (row decode)
};
hipError_t launch_tile_rows(int dtype, int sigma, bool sddmm, const TileRowsArgs& a,
                            hipStream_t st);
// CSR of A^T from the rows and columns of A's nonzeros (stable by row):
// rowT [n_cols + 1], colT [m], perm [m] (A position of each A^T nonzero).
// temp: transpose_temp_bytes(m, end_bit) bytes; columns are < 2^end_bit.
size_t transpose_temp_bytes(int64_t m, int end_bit);
hipError_t launch_transpose(const int32_t* col, const int32_t* rows, int64_t m, int64_t n_cols,
                            int end_bit, void* temp, int32_t* rowT, int32_t* colT,
                            int32_t* perm, hipStream_t st);
hipError_t launch_gather_values(int dtype, const int32_t* perm, const void* src, const void* src2,
                                void* dst, int64_t m, hipStream_t st);
hipError_t launch_column_scale(int dtype, const int32_t* col, const void* a, const void* t,
                               const void* s, void* out, int64_t m, hipStream_t st);
hipError_t launch_adj_sum(int dtype, const void* v, int64_t n, double* part_out, int grid,
                          hipStream_t st);
// hot_n > 0: also the next SpMV's hot-column copy of lam_new into x_hot
hipError_t launch_adj_update(int dtype, const void* y, const void* lam_old, void* lam_new,
                             const void* g, const uint32_t* dmask, int64_t n, double alpha,
                             const double* part_in, int n_in, double* part_out, int grid,
                             hipStream_t st, const int32_t* hot_cols = nullptr,
                             int32_t hot_n = 0, void* x_hot = nullptr);

// BiCGSTAB.
enum { kBicgInit = 0, kBicgUpdateP, kBicgDot1, kBicgUpdateS, kBicgDot2, kBicgUpdateXR };
struct BicgArgs {
  int64_t n;
  int G;       // blocks of every vector kernel = pairs per reduction
  int first;   // iteration 0: p = r
  const void* b;
  void *x, *r, *rh, *p, *v, *s, *t;
  const double *pa_cur, *pa_prev, *pb_prev, *pc_prev;
  double *pb_cur, *pc_cur, *pa_next, *pb_norm;
};
int bicg_grid(int64_t n);
hipError_t launch_bicg(int dtype, const BicgArgs& a, int stage, hipStream_t st);

// Scans of int32 arrays (in == out allowed) and one stable radix-sort pass
// of (key, value) pairs by the digit (key >> shift) & (2^bits - 1), bits in
// 1..8 (val_in == nullptr: the values are the positions 0 .. n - 1).  temp:
// scan_temp_bytes(n) / radix_temp_bytes(n, bits) bytes of device memory.
enum ScanKind { kScanExclusiveSum = 0, kScanInclusiveSum = 1, kScanInclusiveMax = 2 };
size_t scan_temp_bytes(int64_t n);
hipError_t launch_scan_i32(const int32_t* in, int32_t* out, int64_t n, ScanKind kind,
                           void* temp, hipStream_t st);
size_t radix_temp_bytes(int64_t n, int bits);
hipError_t launch_radix_pass(const uint32_t* key_in, const int32_t* val_in, uint32_t* key_out,
                             int32_t* val_out, int64_t n, int shift, int bits, void* temp,
                             hipStream_t st);

// Column stripes (a matrix stacked by column stripe, rows = the non-empty
// (stripe, row) pairs) and the per-row sum of the stripes' results.
// Entry [w][s] of the combine table: which of rows 64 w .. 64 w + 63 have
// nonzeros in stripe s, and the stacked row of the first of them.
struct alignas(16) StripeWord {
  unsigned long long bits;
  int32_t rank;
  int32_t pad;
};
struct StripeSplitArgs {
  const int32_t* row_ptr;  // [n_rows + 1] of the matrix
  const int32_t* col;      // [m]
  int64_t n_rows, m;
  int shift;               // stripe of column c = c >> shift
  int key_bits;            // bits of the stripe index (one radix pass)
  int64_t stripes, words;  // words = ceil(n_rows / 64) per stripe
  void* temp;              // stripe_temp_bytes()
  int32_t* rows;           // [m] row of each nonzero
  int32_t* perm;           // [m] position in the matrix of the i-th stacked nonzero
  int32_t* col_s;          // [m] stacked column stream
  int32_t* row_s;          // [m] row of each stacked nonzero
  int32_t* flag;           // [m] 1 where a (stripe, row) pair begins
  int32_t* vidx;           // [m] exclusive scan of flag
  int32_t* vrow_ptr;       // [V + 1] row pointer of the stacked matrix
  int32_t* vrow_row;       // [V] row of each stacked row
  uint32_t* vrow_stripe;   // [V] stripe of each stacked row
  StripeWord* sw;          // [words][stripes] combine table
  int32_t* wcnt;           // [stripes * words] popcounts, stripe-major
  int32_t* rank;           // [stripes * words] their exclusive scan
};
size_t stripe_temp_bytes(int64_t m, int64_t n_words, int key_bits);
// rows, the stable sort by stripe, the stacked column stream and pair flags
hipError_t launch_stripe_split(const StripeSplitArgs& a, hipStream_t st);
// with V = number of pairs known: vrow_* , the bitmap and the ranks
hipError_t launch_stripe_rows(const StripeSplitArgs& a, int64_t nv, hipStream_t st);
hipError_t launch_stripe_combine(int dtype, int stripes, const void* yv, int64_t nv,
                                 const StripeWord* sw, int64_t words, int64_t n_rows, void* y,
                                 hipStream_t st);

// Batched forms.
struct MultiTables {  // device row-chunk tables of a block-diagonal matrix
  const int32_t* chunk_row;    // [n_chunks + 1]
  const int32_t* chunk_graph;  // [n_chunks]
  const int32_t* chunk_ptr;    // [n_graphs + 1]
  const double* gsize;         // [n_graphs] vertex count of each graph
  double* part;                // [2 n_chunks] per-chunk pairs
  const int32_t* hot_graph;    // [hot_n] graph of each hot column slot (or null)
  int32_t n_chunks;
  int32_t n_graphs;
};
int multi_chunk_rows();
hipError_t launch_multi_dangling(int dtype, const void* x, const uint32_t* dmask,
                                 const MultiTables& mt, double* gsum_out, hipStream_t st);
// hot_n > 0 (needs mt.hot_graph): also the next SpMV's hot-column copy of x'
// resid: also the per-graph l1 change (second components of gsum_out; else 0)
hipError_t launch_multi_update(int dtype, const void* y, const void* x_old, void* x_new,
                               const uint32_t* dmask, const MultiTables& mt, double alpha,
                               const double* gsum_in, double* gsum_out, hipStream_t st,
                               const int32_t* hot_cols = nullptr, int32_t hot_n = 0,
                               void* x_hot = nullptr, bool resid = true);
hipError_t launch_spmm(int dtype, int sigma, const SpmmArgs& a, hipStream_t st);
hipError_t launch_spmm_zero(int dtype, const uint32_t* tile_y, int32_t tile_num, void* Y,
                            int64_t ld, int k, hipStream_t st);
int ppr_grid(int64_t n);
// blocks of one SpMM launch over tile_num tiles (the fused step's part rows)
int spmm_blocks(int64_t tile_num);
// blocks of ppr_fixup over tile_num tiles
int ppr_fixup_grid(int64_t tile_num);
hipError_t launch_ppr_dangling(int dtype, const void* X, const uint32_t* dmask, int64_t n, int k,
                               double* part, double* sums, int grid, hipStream_t st);
// The tiles' first rows (each once) of a fused personalised-PageRank step:
// Xn = alpha Y + teleport at the source, Y cleared there for the next step,
// the dangling mass into part ([grid][64][2]).  All k columns (ld = k).
hipError_t launch_ppr_fixup(int dtype, const uint32_t* tile_y, int32_t tile_num, void* Y,
                            void* Xn, int64_t n, int k, double alpha, const int32_t* src,
                            const double* sums_in, const uint32_t* dmask, double* part, int grid,
                            hipStream_t st);
// part ([grid][64][2]) = per block and column (0, sum over rows of |Xn - Xo|)
hipError_t launch_ppr_resid(int dtype, const void* Xn, const void* Xo, int64_t n, int k,
                            double* part, int grid, hipStream_t st);
// sums[2j], sums[2j + 1] = column j's totals over nblocks part rows, j < k
// per-column totals of per-block part rows (64 columns x 2 doubles each);
// scratch (ppr_sum_scratch_rows() rows) lets a long list be summed in two
// levels, in a fixed order either way
hipError_t launch_ppr_sum(const double* part, int nblocks, int k, double* sums, double* scratch,
                          hipStream_t st);
int ppr_sum_scratch_rows();
// personalised PageRank iterate: the caller's row-major n x k into 32-column
// slabs (with its per-column dangling mass into sums, like
// launch_ppr_dangling), and back
hipError_t launch_ppr_to_slabs(int dtype, const void* X, void* Xs, const uint32_t* dmask,
                               int64_t n, int k, double* part, double* sums, int grid,
                               hipStream_t st);
hipError_t launch_ppr_from_slabs(int dtype, const void* Xs, void* X, int64_t n, int k,
                                 hipStream_t st);

}  // namespace merbit
