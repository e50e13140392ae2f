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
#include <vector>

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
// A column is taken when its count is above the threshold t, or equal to t
// and among the first tie_take[b] such columns of its block (ties go to the
// smaller columns).  Pass 1 counts, per block, the columns above t and those
// at t; the host turns them into per-block tie budgets and slot offsets; pass
// 2 gives the taken columns consecutive slots in column order, so slots are
// deterministic.
constexpr int kSelThreads = 256;
constexpr int kSelPerThread = 16;
constexpr int kSelSpan = kSelThreads * kSelPerThread;

__global__ __launch_bounds__(kSelThreads) void select_count_kernel(
    const int32_t* __restrict__ counts, int64_t n_cols, int32_t threshold,
    int32_t* __restrict__ block_counts) {
  __shared__ int32_t s_cnt[2][kSelThreads / kOmega];
  const int64_t base = (int64_t)blockIdx.x * kSelSpan;
  int above = 0, at = 0;
  for (int k = 0; k < kSelPerThread; ++k) {
    const int64_t col = base + (int64_t)k * kSelThreads + threadIdx.x;
    if (col < n_cols) {
      const int32_t c = min(counts[col], kHotHistBins - 1);  // as the histogram bins it
      above += c > threshold;
      at += c == threshold;
    }
  }
  above = wave_sum(above);
  at = wave_sum(at);
  if ((threadIdx.x & (kOmega - 1)) == 0) {
    s_cnt[0][threadIdx.x / kOmega] = above;
    s_cnt[1][threadIdx.x / kOmega] = at;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int ta = 0, tt = 0;
    for (int w = 0; w < kSelThreads / kOmega; ++w) {
      ta += s_cnt[0][w];
      tt += s_cnt[1][w];
    }
    block_counts[2 * blockIdx.x] = ta;
    block_counts[2 * blockIdx.x + 1] = tt;
  }
}

// block_plan[2b] = first slot of block b, block_plan[2b + 1] = its tie budget
__global__ __launch_bounds__(kSelThreads) void select_assign_kernel(
    const int32_t* __restrict__ counts, int64_t n_cols, int32_t threshold,
    const int32_t* __restrict__ block_plan, int32_t* __restrict__ slot_of,
    int32_t* __restrict__ hot_cols) {
  __shared__ int32_t s_sel[kSelThreads / kOmega], s_tie[kSelThreads / kOmega];
  const int64_t base = (int64_t)blockIdx.x * kSelSpan;
  const int lid = threadIdx.x & (kOmega - 1), wid = threadIdx.x / kOmega;
  const unsigned long long below = (1ull << lid) - 1ull;
  int32_t slot_base = block_plan[2 * blockIdx.x];
  int32_t ties_left = block_plan[2 * blockIdx.x + 1];
  for (int k = 0; k < kSelPerThread; ++k) {
    const int64_t col = base + (int64_t)k * kSelThreads + threadIdx.x;
    const int32_t c = col < n_cols ? min(counts[col], kHotHistBins - 1) : -1;
    // rank of this tie among this step's ties (wavefronts in order)
    const bool tie = col < n_cols && c == threshold;
    const unsigned long long tmask = __ballot(tie);
    if (lid == 0) s_tie[wid] = __popcll(tmask);
    __syncthreads();
    int tie_rank = __popcll(tmask & below), ties_step = 0;
    for (int w = 0; w < kSelThreads / kOmega; ++w) {
      if (w < wid) tie_rank += s_tie[w];
      ties_step += s_tie[w];
    }
    const bool sel = (col < n_cols && c > threshold) || (tie && tie_rank < ties_left);
    const unsigned long long smask = __ballot(sel);
    if (lid == 0) s_sel[wid] = __popcll(smask);
    __syncthreads();
    int wave_off = 0, total = 0;
    for (int w = 0; w < kSelThreads / kOmega; ++w) {
      if (w < wid) wave_off += s_sel[w];
      total += s_sel[w];
    }
    if (col < n_cols) {
      if (sel) {
        const int slot = slot_base + wave_off + __popcll(smask & below);
        slot_of[col] = slot;
        hot_cols[slot] = (int32_t)col;
      } else {
        slot_of[col] = -1;
      }
    }
    slot_base += total;
    ties_left -= ties_step < ties_left ? ties_step : ties_left;
    __syncthreads();  // s_sel / s_tie are rewritten by the next step
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

static int64_t select_blocks(int64_t n_cols) { return (n_cols + kSelSpan - 1) / kSelSpan; }

size_t hot_select_temp_bytes(int64_t n_cols) {
  return sizeof(int32_t) * 2 * (size_t)(select_blocks(n_cols) > 0 ? select_blocks(n_cols) : 1);
}

hipError_t hot_select_top(const int32_t* counts, const int32_t* hist, int64_t n_cols, int64_t cap,
                          bool whole_ties, void* temp, int32_t* slot_of, int32_t* hot_cols,
                          int64_t* taken_out, double* covered_out, hipStream_t st) {
  *taken_out = 0;
  *covered_out = 0.0;
  std::vector<int32_t> h(kHotHistBins);
  hipError_t e = hipMemcpyAsync(h.data(), hist, sizeof(int32_t) * kHotHistBins,
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  // walk the counts down from the largest: every column above t is taken,
  // and `extra` of the columns at t
  int64_t taken = 0, extra = 0;
  double covered = 0.0;
  int32_t t = kHotHistBins;  // nothing taken yet
  for (int b = kHotHistBins - 1; b >= 1; --b) {
    if (h[b] == 0) continue;
    if (taken + h[b] <= cap) {
      taken += h[b];
      covered += (double)b * h[b];
      t = b;
      extra = h[b];
      continue;
    }
    if (!whole_ties) {
      extra = cap - taken;
      taken = cap;
      covered += (double)b * extra;
      t = b;
    }
    break;
  }
  if (taken == 0) return hipSuccess;
  // columns above t (all taken) and at t (the first `extra` in column order)
  const int64_t nb = select_blocks(n_cols);
  int32_t* plan = static_cast<int32_t*>(temp);
  hipLaunchKernelGGL(select_count_kernel, dim3((unsigned)nb), dim3(kSelThreads), 0, st, counts,
                     n_cols, t, plan);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  std::vector<int32_t> hb(2 * (size_t)nb);
  e = hipMemcpyAsync(hb.data(), plan, sizeof(int32_t) * hb.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  int64_t slot = 0, ties = extra;
  for (int64_t b = 0; b < nb; ++b) {
    const int32_t above = hb[2 * b], at = hb[2 * b + 1];
    const int64_t take = at < ties ? at : ties;
    hb[2 * b] = (int32_t)slot;
    hb[2 * b + 1] = (int32_t)take;
    slot += above + take;
    ties -= take;
  }
  if (slot != taken) return hipErrorUnknown;  // counts changed under the histogram
  e = hipMemcpyAsync(plan, hb.data(), sizeof(int32_t) * hb.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(select_assign_kernel, dim3((unsigned)nb), dim3(kSelThreads), 0, st, counts,
                     n_cols, t, plan, slot_of, hot_cols);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = hipStreamSynchronize(st);  // hb is read by the copy above
  if (e != hipSuccess) return e;
  *taken_out = taken;
  *covered_out = covered;
  return hipSuccess;
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
