// Internal declarations of libmerbit: wavefront helpers and the kernel
// launchers that the C-ABI layer (merbit_api.hip) dispatches to.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace merbit {

constexpr int kOmega = 64;                 // lanes per tile = CDNA wavefront size
constexpr uint32_t kRowMask = 0x7FFFFFFFu; // tile_y: row index
constexpr uint32_t kFastBit = 0x80000000u; // tile_y: long-row (single-row) tile mark
constexpr int kMaxSigma = 12;              // 2 ceil(log2(64 sigma)) + sigma <= 32
constexpr int kHotHistBins = 65536;        // column-count histogram of the hot cache

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
  uint32_t* lane_desc;
};

struct SpmvArgs {
  const int32_t* tile_x;
  const uint32_t* tile_y;
  const uint32_t* lane_desc;
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
bool spmv_wave_supported(int dtype, int sigma, int waves, bool hot);
hipError_t launch_spmv_wave(int dtype, int sigma, int waves, bool hot, size_t hot_lds_bytes,
                            const SpmvArgs& a, hipStream_t st);
hipError_t spmv_wave_set_hot_lds(int dtype, int sigma, int waves, size_t bytes);

// Hot-column cache.
hipError_t hot_count_columns(const int32_t* col, int64_t nnz, int64_t n_cols, int32_t* counts,
                             int32_t* hist, hipStream_t st);
int hot_select_blocks(int64_t n_cols);
hipError_t hot_select_count(const int32_t* counts, int64_t n_cols, int32_t threshold,
                            int32_t* block_counts, hipStream_t st);
hipError_t hot_select_assign(const int32_t* counts, int64_t n_cols, int32_t threshold,
                             const int32_t* block_offsets, int32_t* slot_of, int32_t* hot_cols,
                             hipStream_t st);
hipError_t hot_recode(const int32_t* col, int64_t nnz, const int32_t* slot_of, int32_t* colx,
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
hipError_t launch_pr_update(int dtype, const void* y, const void* x_old, void* x_new,
                            const uint32_t* dmask, int64_t n, double alpha,
                            const double* partials_in, int n_in, double* partials_out, int grid,
                            hipStream_t st);
int pr_reduce_grid(int64_t n);

}  // namespace merbit
