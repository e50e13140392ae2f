// One-time preprocessing: CSR validation and TILE generation
// (Sec. 4.1.1 format, Sec. 4.1.2 preprocessing; the lane start search is
// Algorithm 1).
//
// One thread per lane, one 64-lane wavefront per tile (omega = 64).  The
// merge path (Sec. 3.3) leaves row r by its down step at path position
// p(r) = row_ptr[r + 1] + r, and p increases strictly with r.  Lane j covers
// positions [d, d + s) with d = j sigma, s = min(sigma, m + n - d):
//   - its start row y0 is the number of rows with p(r) < d (a binary search
//     over r, Algorithm 1) and its start column is d - y0;
//   - its down steps are those of rows y0, y0 + 1, ... while p(r) < d + s,
//     and the step at offset k is a down step exactly when p(r) = d + k for
//     one of them, so the flag word is the OR of 1 << (p(r) - d) over those
//     rows (one iteration per down step, not per step);
//   - the tile starts at its lane 0, and a tile is a single-row ("fast")
//     tile when none of its lanes has a down step.
// Cost O(lane_num log n + n + m / sigma).
#include "merbit_internal.hpp"

namespace merbit {

__global__ void validate_kernel(const int32_t* __restrict__ row_ptr,
                                const int32_t* __restrict__ col, int64_t n_rows, int64_t n_cols,
                                int64_t nnz, unsigned* __restrict__ flags) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned f = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n_rows; i += stride) {
    const int32_t v = row_ptr[i];
    if (i == 0 && v != 0) f |= 1u;
    if (i == n_rows && (int64_t)v != nnz) f |= 2u;
    if (i < n_rows && v > row_ptr[i + 1]) f |= 4u;
  }
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += stride) {
    const int32_t c = col[k];
    if (c < 0 || (int64_t)c >= n_cols) f |= 8u;
  }
  if (f) atomicOr(flags, f);
}

hipError_t launch_validate(const int32_t* row_ptr, const int32_t* col, int64_t n_rows,
                           int64_t n_cols, int64_t nnz, unsigned* flags, hipStream_t st) {
  const int64_t work = (n_rows + 1 > nnz ? n_rows + 1 : nnz);
  int64_t grid = (work + 255) / 256;
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(validate_kernel, dim3((unsigned)grid), dim3(256), 0, st, row_ptr, col,
                     n_rows, n_cols, nnz, flags);
  return hipGetLastError();
}

// Algorithm 1: number of rows finished before path position `diag`, i.e.
// of rows r with p(r) = row_ptr[r + 1] + r < diag (p increases with r).
__device__ __forceinline__ int32_t merge_search_rows(const int32_t* __restrict__ row_ptr,
                                                     int32_t n_rows, int32_t nnz, int32_t diag) {
  int32_t lo = diag - nnz > 0 ? diag - nnz : 0;
  int32_t hi = diag < n_rows ? diag : n_rows;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (row_ptr[mid + 1] + mid < diag) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// D = uint32_t or uint64_t: the descriptor word (flags << 2b | y_off << b | x_off)
template <typename D>
__global__ __launch_bounds__(256) void plan_kernel(PlanArgs a, D* __restrict__ lane_desc) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lid = threadIdx.x & (kOmega - 1);
  const int32_t L = a.nnz + a.n_rows;
  if (j < a.lane_num) {
    const int32_t d = (int32_t)j * a.sigma;
    const int32_t end = L - d < a.sigma ? L : d + a.sigma;
    const int32_t y0 = merge_search_rows(a.row_ptr, a.n_rows, a.nnz, d);
    D flags = 0;
    for (int32_t r = y0; r < a.n_rows; ++r) {
      const int32_t pos = a.row_ptr[r + 1] + r;
      // pos < d only for a row_ptr that is not monotone (never validated)
      if (pos >= end || pos < d) break;
      flags |= (D)1 << (pos - d);
    }
    // the tile's start: lane 0 of the wavefront, active whenever any lane is
    const int32_t ty = __builtin_amdgcn_readfirstlane(y0);
    const int32_t tx = __builtin_amdgcn_readfirstlane(d - y0);
    const D x_off = (D)(d - y0 - tx);
    const D y_off = (D)(y0 - ty);
    lane_desc[j] = (flags << (2 * a.bits)) | (y_off << a.bits) | x_off;
    const bool single_row = __ballot(flags != 0) == 0ull;
    if (lid == 0) {
      const int64_t i = j / kOmega;
      a.tile_x[i] = tx;
      a.tile_y[i] = (uint32_t)ty | (single_row ? kFastBit : 0u);
    }
  } else if (j == a.lane_num) {
    a.tile_x[a.tile_num] = a.nnz;
    a.tile_y[a.tile_num] = (uint32_t)a.n_rows;
  }
}

hipError_t launch_plan(const PlanArgs& a, hipStream_t st) {
  const int64_t threads = a.lane_num + 1;
  const int64_t grid = (threads + 255) / 256;
  if (a.lane_desc64)
    hipLaunchKernelGGL(plan_kernel<uint64_t>, dim3((unsigned)grid), dim3(256), 0, st, a,
                       a.lane_desc64);
  else
    hipLaunchKernelGGL(plan_kernel<uint32_t>, dim3((unsigned)grid), dim3(256), 0, st, a,
                       a.lane_desc);
  return hipGetLastError();
}

__global__ void count_fast_kernel(const uint32_t* __restrict__ tile_y, int64_t tile_num,
                                  unsigned long long* __restrict__ count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tile_num; i += stride)
    c += (tile_y[i] >> 31) & 1u;
  c = wave_sum(c);
  if ((threadIdx.x & (kOmega - 1)) == 0 && c) atomicAdd(count, c);
}

hipError_t launch_count_fast(const uint32_t* tile_y, int64_t tile_num, unsigned long long* count,
                             hipStream_t st) {
  int64_t grid = (tile_num + 255) / 256;
  if (grid > 2048) grid = 2048;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(count_fast_kernel, dim3((unsigned)grid), dim3(256), 0, st, tile_y,
                     tile_num, count);
  return hipGetLastError();
}

}  // namespace merbit
