// PageRank power-method pieces around the fused SpMV (Sec. 5.5.1 of the
// MERBIT paper: damping alpha, dangling mass spread uniformly).
//
// Per iteration t the host enqueues
//   spmv_dual(x_t -> y)            y = P x_t
//   pr_update(y, x_t -> x_{t+1})   x_{t+1} = alpha y + (alpha delta_t + 1 - alpha) / n
// and the update also produces delta_{t+1} = sum of x_{t+1} over dangling
// vertices and r_{t+1} = ||x_{t+1} - x_t||_1 for the next step.  Both sums
// are reduced in double: per block in the update kernel, then over the blocks
// by the next update kernel (delta) or by the host (r), always in the same
// order, so they are deterministic.
#include "merbit_internal.hpp"

namespace merbit {

// ------------------------------------------------------- dangling mask ----

__global__ void mark_out_kernel(const int32_t* __restrict__ col, int64_t nnz,
                                unsigned char* __restrict__ has_out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += stride)
    has_out[col[k]] = 1;
}

// dmask bit u = 1 when column u has no nonzero (vertex u is dangling)
__global__ void pack_dangling_kernel(const unsigned char* __restrict__ has_out, int64_t n,
                                     uint32_t* __restrict__ dmask) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t words = (n + 31) / 32;
  if (w >= words) return;
  uint32_t bits = 0;
  for (int b = 0; b < 32; ++b) {
    const int64_t u = w * 32 + b;
    if (u < n && !has_out[u]) bits |= 1u << b;
  }
  dmask[w] = bits;
}

__global__ void zero_bytes_kernel(unsigned char* __restrict__ p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

hipError_t launch_dangling_mask(const int32_t* col, int64_t nnz, int64_t n,
                                unsigned char* scratch_bytes, uint32_t* dmask, hipStream_t st) {
  // cleared by a kernel, not a memset node: callers may record this into a graph
  hipError_t e;
  if (n > 0) {
    int64_t zgrid = (n + 255) / 256;
    if (zgrid > 4096) zgrid = 4096;
    hipLaunchKernelGGL(zero_bytes_kernel, dim3((unsigned)zgrid), dim3(256), 0, st,
                       scratch_bytes, n);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (nnz > 0) {
    int64_t grid = (nnz + 255) / 256;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(mark_out_kernel, dim3((unsigned)grid), dim3(256), 0, st, col, nnz,
                       scratch_bytes);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t words = (n + 31) / 32;
  if (words > 0) {
    hipLaunchKernelGGL(pack_dangling_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0,
                       st, scratch_bytes, n, dmask);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------ two-value reduction ----
//
// Each block of a reduction kernel writes its pair of sums to partials[2b],
// partials[2b+1] with plain stores; the kernel that consumes the total (the
// next update, or the host) sums the pairs in block order.  Kernel boundaries
// order the writes before the reads, so no device-scope fence is needed, and
// every consumer block computes the same bits.

// Total of the first components of n_in pairs, identical in every block.
__device__ __forceinline__ double sum_partials_first(const double* __restrict__ p, int n_in) {
  __shared__ double total;
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < n_in; k += kReduceThreads) a += p[2 * k];
  block_sum2(a, b);
  if (threadIdx.x == 0) total = a;
  __syncthreads();
  return total;
}

// Four passes of the update's loop per thread (16 elements), up to 1,024
// blocks; a small vector (up to 64 blocks) is spread further, one pass per
// thread, so that no thread waits for more than one round of loads (the
// 10,000-vertex Chung-Lu update: 3 blocks of 4 passes took 5.5 us a launch).
int pr_reduce_grid(int64_t n) {
  int64_t g = (n + kReduceThreads * 16 - 1) / (kReduceThreads * 16);
  int64_t g1 = (n + kReduceThreads * 4 - 1) / (kReduceThreads * 4);
  if (g1 > 64) g1 = 64;
  if (g < g1) g = g1;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  return (int)g;
}

template <typename V>
__global__ __launch_bounds__(kReduceThreads) void dangling_sum_kernel(
    const V* __restrict__ x, const uint32_t* __restrict__ dmask, int64_t n,
    double* __restrict__ partials_out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double d = 0.0, z = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    if ((dmask[i >> 5] >> (i & 31)) & 1u) d += (double)x[i];
  block_sum2(d, z);
  if (threadIdx.x == 0) {
    partials_out[2 * blockIdx.x] = d;
    partials_out[2 * blockIdx.x + 1] = 0.0;
  }
}

hipError_t launch_dangling_sum(int dtype, const void* x, const uint32_t* dmask, int64_t n,
                               double* partials_out, int grid, hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL(dangling_sum_kernel<float>, dim3(grid), dim3(kReduceThreads), 0, st,
                       static_cast<const float*>(x), dmask, n, partials_out);
  else
    hipLaunchKernelGGL(dangling_sum_kernel<double>, dim3(grid), dim3(kReduceThreads), 0, st,
                       static_cast<const double*>(x), dmask, n, partials_out);
  return hipGetLastError();
}

// x_new = alpha y + (alpha delta + 1 - alpha) / n, with delta the dangling
// mass of x_old (summed from the previous kernel's partials).  Writes this
// block's dangling mass of x_new and, with RESID, ||x_new - x_old||_1 to
// partials_out (without RESID x_old is not read and the second component is
// 0: the l1 change is needed only where the host reads it).
// With hot_n > 0 it also writes the hot-column copy of x_new that the next
// SpMV's LDS cache reads (x_hot[s] = x_new[hot_cols[s]], the same fused
// multiply-add on the same operands), so that SpMV needs no gather launch.
template <typename V, bool RESID>
__global__ __launch_bounds__(kReduceThreads) void pr_update_kernel(
    const V* __restrict__ y, const V* __restrict__ x_old, V* __restrict__ x_new,
    const uint32_t* __restrict__ dmask, int64_t n, double alpha,
    const double* __restrict__ partials_in, int n_in, double* __restrict__ partials_out,
    const int32_t* __restrict__ hot_cols, int32_t hot_n, V* __restrict__ x_hot) {
  constexpr int ILP = 4;
  const V a = (V)alpha;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * ILP;
  const int64_t hstride = (int64_t)gridDim.x * blockDim.x;
  const int64_t h0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // one pass of ILP elements per thread; the next pass's loads go out before
  // the current one is used, and the first pass's (with the first hot
  // column) before the previous step's partials are summed
  auto load = [&](int64_t b, V (&yv)[ILP], V (&xo)[ILP], uint32_t (&mw)[ILP]) {
#pragma unroll
    for (int u = 0; u < ILP; ++u) {
      const int64_t i = min(b + (int64_t)u * kReduceThreads, n - 1);
      yv[u] = y[i];
      if constexpr (RESID) xo[u] = x_old[i];
      mw[u] = dmask[i >> 5];
    }
  };
  int64_t base = (int64_t)blockIdx.x * blockDim.x * ILP + threadIdx.x;
  V yv[ILP], xo[ILP];
  uint32_t mw[ILP];
  if (base < n) load(base, yv, xo, mw);
  const int32_t hc0 = h0 < hot_n ? hot_cols[h0] : 0;
  const double delta = sum_partials_first(partials_in, n_in);
  const V teleport = (V)((alpha * delta + 1.0 - alpha) / (double)n);
  double dsum = 0.0, rsum = 0.0;
  while (base < n) {
    const int64_t next = base + stride;
    V yn[ILP], xn[ILP];
    uint32_t mn[ILP];
    if (next < n) load(next, yn, xn, mn);
#pragma unroll
    for (int u = 0; u < ILP; ++u) {
      const int64_t i = base + (int64_t)u * kReduceThreads;
      if (i < n) {
        const V v = fma(a, yv[u], teleport);
        x_new[i] = v;
        if constexpr (RESID) rsum += fabs((double)v - (double)xo[u]);
        if ((mw[u] >> (i & 31)) & 1u) dsum += (double)v;
      }
    }
    base = next;
    if (base < n) {
#pragma unroll
      for (int u = 0; u < ILP; ++u) {
        yv[u] = yn[u];
        if constexpr (RESID) xo[u] = xn[u];
        mw[u] = mn[u];
      }
    }
  }
  for (int64_t h = h0; h < hot_n; h += hstride)
    x_hot[h] = fma(a, y[h == h0 ? hc0 : hot_cols[h]], teleport);
  block_sum2(dsum, rsum);
  if (threadIdx.x == 0) {
    partials_out[2 * blockIdx.x] = dsum;
    partials_out[2 * blockIdx.x + 1] = rsum;
  }
}

template <typename V>
static void pr_update_launch(bool resid, const void* y, const void* x_old, void* x_new,
                             const uint32_t* dmask, int64_t n, double alpha,
                             const double* partials_in, int n_in, double* partials_out, int grid,
                             hipStream_t st, const int32_t* hot_cols, int32_t hot_n,
                             void* x_hot) {
  const V* yv = static_cast<const V*>(y);
  const V* xo = static_cast<const V*>(x_old);
  V* xn = static_cast<V*>(x_new);
  V* xh = static_cast<V*>(x_hot);
  if (resid)
    hipLaunchKernelGGL((pr_update_kernel<V, true>), dim3(grid), dim3(kReduceThreads), 0, st, yv,
                       xo, xn, dmask, n, alpha, partials_in, n_in, partials_out, hot_cols, hot_n,
                       xh);
  else
    hipLaunchKernelGGL((pr_update_kernel<V, false>), dim3(grid), dim3(kReduceThreads), 0, st,
                       yv, xo, xn, dmask, n, alpha, partials_in, n_in, partials_out, hot_cols,
                       hot_n, xh);
}

hipError_t launch_pr_update(int dtype, const void* y, const void* x_old, void* x_new,
                            const uint32_t* dmask, int64_t n, double alpha,
                            const double* partials_in, int n_in, double* partials_out, int grid,
                            hipStream_t st, const int32_t* hot_cols, int32_t hot_n,
                            void* x_hot, bool resid) {
  if (dtype == 0)
    pr_update_launch<float>(resid, y, x_old, x_new, dmask, n, alpha, partials_in, n_in,
                            partials_out, grid, st, hot_cols, hot_n, x_hot);
  else
    pr_update_launch<double>(resid, y, x_old, x_new, dmask, n, alpha, partials_in, n_in,
                             partials_out, grid, st, hot_cols, hot_n, x_hot);
  return hipGetLastError();
}

}  // namespace merbit
