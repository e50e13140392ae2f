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

template <typename V>
__device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
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
  const int32_t* col;
  const void* val;
  const void* x;
  void* y;
  void* z;            // dual buffer to clear at boundary rows, or nullptr
  int32_t tile_num;
  int32_t lane_num;
  int32_t path_len;   // nnz + n_rows
  int32_t n_rows;
  int32_t block_num;
};

// CSR checks; *flags gets bit 0: row_ptr[0] != 0, bit 1: row_ptr[n] != nnz,
// bit 2: row_ptr decreasing, bit 3: column out of range.
hipError_t launch_validate(const int32_t* row_ptr, const int32_t* col, int64_t n_rows,
                           int64_t n_cols, int64_t nnz, unsigned* flags, hipStream_t st);
hipError_t launch_plan(const PlanArgs& a, hipStream_t st);
hipError_t launch_count_fast(const uint32_t* tile_y, int64_t tile_num,
                             unsigned long long* count, hipStream_t st);

bool spmv_supported(int dtype, int sigma, int waves);
hipError_t launch_spmv(int dtype, int sigma, int waves, const SpmvArgs& a, hipStream_t st);
hipError_t launch_zero_boundary(int dtype, const uint32_t* tile_y, int32_t block_num,
                                int32_t waves, void* v, hipStream_t st);

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
