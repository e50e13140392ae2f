// PageRank power-method pieces around the fused SpMV (Sec. 5.5.1 of the
// MERBIT paper: damping alpha, dangling mass spread uniformly).
//
// Per iteration t the host enqueues
//   spmv_dual(x_t -> y)            y = P x_t
//   pr_update(y, x_t -> x_{t+1})   x_{t+1} = alpha y + (alpha delta_t + 1 - alpha) / n
// and the update also produces delta_{t+1} = sum of x_{t+1} over dangling
// vertices and r_{t+1} = ||x_{t+1} - x_t||_1 for the next step.  Both sums
// are reduced in double, per block and then by the last block to finish, in
// a fixed order (so they are deterministic); the last block also resets the
// arrival counter, so no memset is needed between launches.
#include "merbit_internal.hpp"

namespace merbit {

constexpr int kReduceThreads = 256;

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

hipError_t launch_dangling_mask(const int32_t* col, int64_t nnz, int64_t n,
                                unsigned char* scratch_bytes, uint32_t* dmask, hipStream_t st) {
  hipError_t e = hipMemsetAsync(scratch_bytes, 0, (size_t)(n > 0 ? n : 1), st);
  if (e != hipSuccess) return e;
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
  }
  return e;
}

// ------------------------------------------------ two-value reduction ----

// Reduce (a, b) over the grid.  Every block writes its pair to partials; the
// last block to arrive sums all pairs in block order and writes out[0..1].
__device__ void grid_reduce2(double a, double b, double* __restrict__ partials,
                             unsigned* __restrict__ counter, double* __restrict__ out) {
  __shared__ double sa[kReduceThreads / kOmega], sb[kReduceThreads / kOmega];
  __shared__ int is_last;
  const int tid = threadIdx.x, lid = tid & (kOmega - 1), wid = tid / kOmega;
  a = wave_sum(a);
  b = wave_sum(b);
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
    __hip_atomic_store(&partials[2 * blockIdx.x], ta, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&partials[2 * blockIdx.x + 1], tb, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    const unsigned prev =
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    is_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __atomic_thread_fence(__ATOMIC_ACQUIRE);
  double pa = 0.0, pb = 0.0;
  for (unsigned k = tid; k < gridDim.x; k += kReduceThreads) {
    pa += __hip_atomic_load(&partials[2 * k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    pb += __hip_atomic_load(&partials[2 * k + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  pa = wave_sum(pa);
  pb = wave_sum(pb);
  __syncthreads();
  if (lid == 0) {
    sa[wid] = pa;
    sb[wid] = pb;
  }
  __syncthreads();
  if (tid == 0) {
    double ta = 0.0, tb = 0.0;
    for (int w = 0; w < kReduceThreads / kOmega; ++w) {
      ta += sa[w];
      tb += sb[w];
    }
    out[0] = ta;
    out[1] = tb;
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

int pr_reduce_grid(int64_t n) {
  int64_t g = (n + kReduceThreads * 8 - 1) / (kReduceThreads * 8);
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  return (int)g;
}

template <typename V>
__global__ __launch_bounds__(kReduceThreads) void dangling_sum_kernel(
    const V* __restrict__ x, const uint32_t* __restrict__ dmask, int64_t n,
    double* __restrict__ partials, unsigned* __restrict__ counter, double* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double d = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    if ((dmask[i >> 5] >> (i & 31)) & 1u) d += (double)x[i];
  grid_reduce2(d, 0.0, partials, counter, out);
}

hipError_t launch_dangling_sum(int dtype, const void* x, const uint32_t* dmask, int64_t n,
                               double* partials, unsigned* counter, double* out, int grid,
                               hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL(dangling_sum_kernel<float>, dim3(grid), dim3(kReduceThreads), 0, st,
                       static_cast<const float*>(x), dmask, n, partials, counter, out);
  else
    hipLaunchKernelGGL(dangling_sum_kernel<double>, dim3(grid), dim3(kReduceThreads), 0, st,
                       static_cast<const double*>(x), dmask, n, partials, counter, out);
  return hipGetLastError();
}

// x_new = alpha y + (alpha delta + 1 - alpha) / n; accumulates the dangling
// mass of x_new and ||x_new - x_old||_1 into acc_out[0], acc_out[1].
template <typename V>
__global__ __launch_bounds__(kReduceThreads) void pr_update_kernel(
    const V* __restrict__ y, const V* __restrict__ x_old, V* __restrict__ x_new,
    const uint32_t* __restrict__ dmask, int64_t n, double alpha,
    const double* __restrict__ acc_in, double* __restrict__ partials,
    unsigned* __restrict__ counter, double* __restrict__ acc_out) {
  const double delta = acc_in[0];
  const V teleport = (V)((alpha * delta + 1.0 - alpha) / (double)n);
  const V a = (V)alpha;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double dsum = 0.0, rsum = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const V xn = a * y[i] + teleport;
    x_new[i] = xn;
    rsum += fabs((double)xn - (double)x_old[i]);
    if ((dmask[i >> 5] >> (i & 31)) & 1u) dsum += (double)xn;
  }
  grid_reduce2(dsum, rsum, partials, counter, acc_out);
}

hipError_t launch_pr_update(int dtype, const void* y, const void* x_old, void* x_new,
                            const uint32_t* dmask, int64_t n, double alpha, const double* acc_in,
                            double* partials, unsigned* counter, double* acc_out, int grid,
                            hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL(pr_update_kernel<float>, dim3(grid), dim3(kReduceThreads), 0, st,
                       static_cast<const float*>(y), static_cast<const float*>(x_old),
                       static_cast<float*>(x_new), dmask, n, alpha, acc_in, partials, counter,
                       acc_out);
  else
    hipLaunchKernelGGL(pr_update_kernel<double>, dim3(grid), dim3(kReduceThreads), 0, st,
                       static_cast<const double*>(y), static_cast<const double*>(x_old),
                       static_cast<double*>(x_new), dmask, n, alpha, acc_in, partials, counter,
                       acc_out);
  return hipGetLastError();
}

}  // namespace merbit
