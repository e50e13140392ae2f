// Hot-column x cache (plan side and per-call gather).
//
// The x gathers of the fused SpMV are limited on gfx950 by the rate at which
// scattered L1 misses are served by L2.  Power-law matrices concentrate their
// nonzeros on few columns (R-MAT scale 22: the 32K most frequent columns hold
// 53 % of all nonzeros), so the plan picks the H most frequent columns and
// rewrites the column stream: a hot column c becomes -1 - slot(c).  Per call,
// the H hot x values are gathered once into a contiguous array, every block
// of the fused kernel copies them into LDS, and a hot nonzero reads its x
// value from LDS instead of issuing a global gather.  Sums and their order
// are unchanged: only where the x value is read from differs.
#include "merbit_internal.hpp"

namespace merbit {

// counts[c] = number of sampled nonzeros in column c: every `sample`-th
// nonzero of the stream (1 = exact counts).  The selection only needs the
// order of the large counts, which a 1-in-8 sample keeps (R-MAT scale 22:
// 52.9 % coverage of the top 32K columns either way) at an eighth of the
// global atomics.
__global__ void col_count_kernel(const int32_t* __restrict__ col, int64_t nnz, int sample,
                                 int32_t* __restrict__ counts) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t ns = (nnz + sample - 1) / sample;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += stride)
    atomicAdd(&counts[col[i * sample]], 1);
}

// hist[min(count, kHotHistBins - 1)] += 1 over the columns.  Most columns
// have small counts, so the low bins are counted per block in LDS and added
// to the global histogram once per block; only large counts go straight to
// global atomics.
constexpr int kHistLdsBins = 2048;

__global__ __launch_bounds__(256) void count_hist_kernel(const int32_t* __restrict__ counts,
                                                         int64_t n_cols,
                                                         int32_t* __restrict__ hist) {
  __shared__ int32_t s_hist[kHistLdsBins];
  for (int b = threadIdx.x; b < kHistLdsBins; b += blockDim.x) s_hist[b] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cols; c += stride) {
    const int32_t v = counts[c];
    const int32_t bin = v < kHotHistBins - 1 ? v : kHotHistBins - 1;
    if (bin < kHistLdsBins) atomicAdd(&s_hist[bin], 1);
    else atomicAdd(&hist[bin], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kHistLdsBins; b += blockDim.x)
    if (s_hist[b]) atomicAdd(&hist[b], s_hist[b]);
}

// Selection in column order: block b owns columns [b * kSelSpan, (b+1) * kSelSpan).
// Pass 1 counts the selected columns per block; pass 2 (after an exclusive
// scan of those counts) gives them consecutive slots, so slots are
// deterministic and follow column order.
constexpr int kSelThreads = 256;
constexpr int kSelPerThread = 16;
constexpr int kSelSpan = kSelThreads * kSelPerThread;

__global__ __launch_bounds__(kSelThreads) void select_count_kernel(
    const int32_t* __restrict__ counts, int64_t n_cols, int32_t threshold,
    int32_t* __restrict__ block_counts) {
  __shared__ int32_t s_cnt[kSelThreads / kOmega];
  const int64_t base = (int64_t)blockIdx.x * kSelSpan;
  int c = 0;
  for (int k = 0; k < kSelPerThread; ++k) {
    const int64_t col = base + (int64_t)k * kSelThreads + threadIdx.x;
    if (col < n_cols && counts[col] >= threshold) ++c;
  }
  c = wave_sum(c);
  if ((threadIdx.x & (kOmega - 1)) == 0) s_cnt[threadIdx.x / kOmega] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kSelThreads / kOmega; ++w) t += s_cnt[w];
    block_counts[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kSelThreads) void select_assign_kernel(
    const int32_t* __restrict__ counts, int64_t n_cols, int32_t threshold,
    const int32_t* __restrict__ block_offsets, int32_t* __restrict__ slot_of,
    int32_t* __restrict__ hot_cols) {
  __shared__ int32_t s_wave[kSelThreads / kOmega];
  __shared__ int32_t s_base;
  const int64_t base = (int64_t)blockIdx.x * kSelSpan;
  const int lid = threadIdx.x & (kOmega - 1), wid = threadIdx.x / kOmega;
  if (threadIdx.x == 0) s_base = block_offsets[blockIdx.x];
  __syncthreads();
  for (int k = 0; k < kSelPerThread; ++k) {
    const int64_t col = base + (int64_t)k * kSelThreads + threadIdx.x;
    const bool sel = col < n_cols && counts[col] >= threshold;
    const unsigned long long mask = __ballot(sel);
    const int below = __popcll(mask & ((1ull << lid) - 1ull));
    if (lid == 0) s_wave[wid] = __popcll(mask);
    __syncthreads();
    int wave_off = 0;
    for (int w = 0; w < wid; ++w) wave_off += s_wave[w];
    int total = 0;
    for (int w = 0; w < kSelThreads / kOmega; ++w) total += s_wave[w];
    if (col < n_cols) {
      if (sel) {
        const int slot = s_base + wave_off + below;
        slot_of[col] = slot;
        hot_cols[slot] = (int32_t)col;
      } else {
        slot_of[col] = -1;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) s_base += total;
    __syncthreads();
  }
}

// colx[k] = -1 - slot(col[k]) for a hot column, col[k] otherwise
__global__ void recode_kernel(const int32_t* __restrict__ col, int64_t nnz,
                              const int32_t* __restrict__ slot_of, int32_t* __restrict__ colx) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += stride) {
    const int32_t c = col[k];
    const int32_t s = slot_of ? slot_of[c] : c;  // no map: every column is hot, slot = column
    colx[k] = s >= 0 ? -1 - s : c;
  }
}

static unsigned grid_for(int64_t n, int64_t cap) {
  int64_t g = (n + 255) / 256;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

hipError_t hot_count_columns(const int32_t* col, int64_t nnz, int64_t n_cols, int sample,
                             int32_t* counts, int32_t* hist, hipStream_t st) {
  hipError_t e = hipMemsetAsync(counts, 0, sizeof(int32_t) * (size_t)n_cols, st);
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(hist, 0, sizeof(int32_t) * kHotHistBins, st);
  if (e != hipSuccess) return e;
  if (nnz > 0) {
    hipLaunchKernelGGL(col_count_kernel, dim3(grid_for(nnz / sample + 1, 8192)), dim3(256), 0,
                       st, col, nnz, sample, counts);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(count_hist_kernel, dim3(grid_for(n_cols, 512)), dim3(256), 0, st, counts,
                     n_cols, hist);
  return hipGetLastError();
}

int hot_select_blocks(int64_t n_cols) { return (int)((n_cols + kSelSpan - 1) / kSelSpan); }

hipError_t hot_select_count(const int32_t* counts, int64_t n_cols, int32_t threshold,
                            int32_t* block_counts, hipStream_t st) {
  hipLaunchKernelGGL(select_count_kernel, dim3(hot_select_blocks(n_cols)), dim3(kSelThreads), 0,
                     st, counts, n_cols, threshold, block_counts);
  return hipGetLastError();
}

hipError_t hot_select_assign(const int32_t* counts, int64_t n_cols, int32_t threshold,
                             const int32_t* block_offsets, int32_t* slot_of, int32_t* hot_cols,
                             hipStream_t st) {
  hipLaunchKernelGGL(select_assign_kernel, dim3(hot_select_blocks(n_cols)), dim3(kSelThreads), 0,
                     st, counts, n_cols, threshold, block_offsets, slot_of, hot_cols);
  return hipGetLastError();
}

hipError_t hot_recode(const int32_t* col, int64_t nnz, const int32_t* slot_of, int32_t* colx,
                      hipStream_t st) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(recode_kernel, dim3(grid_for(nnz, 8192)), dim3(256), 0, st, col, nnz,
                     slot_of, colx);
  return hipGetLastError();
}

// x_hot[s] = x[hot_cols[s]]
template <typename V>
__global__ void hot_gather_kernel(const V* __restrict__ x, const int32_t* __restrict__ hot_cols,
                                  int32_t hot_n, V* __restrict__ x_hot) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < hot_n) x_hot[s] = x[hot_cols[s]];
}

hipError_t launch_hot_gather(int dtype, const void* x, const int32_t* hot_cols, int32_t hot_n,
                             void* x_hot, hipStream_t st) {
  if (hot_n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((hot_n + 255) / 256);
  if (dtype == 0)
    hipLaunchKernelGGL(hot_gather_kernel<float>, dim3(grid), dim3(256), 0, st,
                       static_cast<const float*>(x), hot_cols, hot_n, static_cast<float*>(x_hot));
  else
    hipLaunchKernelGGL(hot_gather_kernel<double>, dim3(grid), dim3(256), 0, st,
                       static_cast<const double*>(x), hot_cols, hot_n,
                       static_cast<double*>(x_hot));
  return hipGetLastError();
}

}  // namespace merbit
