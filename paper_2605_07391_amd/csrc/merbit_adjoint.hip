// Pieces of the PageRank adjoint (the derivative of the fixed point of
// Sec. 5.5.1 with respect to the matrix values), all on the merge-path plan:
//   - the row of every nonzero, decoded from the plan's descriptors;
//   - the transpose A^T in CSR plus the permutation of the nonzeros (a stable
//     sort of the nonzeros by column), from which a second plan is built;
//   - the per-nonzero product out[e] = scale g[row(e)] x[col(e)] (the value
//     gradient alpha lambda[row] x*[col]);
//   - gathers through the permutation and column scaling (the column
//     normalisation of edge weights and its derivative);
//   - the adjoint fixed-point update
//       lambda' = g + alpha P^T lambda + (alpha / n) (1^T lambda) d,
//     d the dangling indicator, with deterministic two-level sums.
#include "merbit_internal.hpp"

namespace merbit {

constexpr int kDecodeWaves = 4;

// One wavefront per tile: rows of the tile's nonzeros into LDS, then either
// rows[e] = row(e) (SDDMM = false) or out[e] = scale g[row(e)] x[col(e)].
template <typename V, int SIGMA, bool SDDMM>
__global__ __launch_bounds__(kDecodeWaves * 64) void tile_rows_kernel(
    const int32_t* __restrict__ tile_x, const uint32_t* __restrict__ tile_y,
    const uint32_t* __restrict__ lane_desc, int32_t tile_num, int32_t lane_num, int32_t path_len,
    const int32_t* __restrict__ col, const V* __restrict__ g, const V* __restrict__ x, V scale,
    V* __restrict__ out, int32_t* __restrict__ rows) {
  constexpr int WLDS = kOmega * SIGMA;
  __shared__ int32_t s_row[kDecodeWaves * WLDS];
  const int lid = threadIdx.x & (kOmega - 1);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kOmega);
  const int t = blockIdx.x * kDecodeWaves + wid;
  if (t >= tile_num) return;  // no block-wide synchronisation in this kernel
  int32_t* wrow = s_row + wid * WLDS;
  const int x_ws = tile_x[t];
  const int x_se = tile_x[t + 1] - x_ws;
  if (x_se == 0) return;
  const uint32_t tyw = tile_y[t];
  const int y_ws = (int)(tyw & kRowMask);
  tile_nz_rows<SIGMA>(lane_desc, lane_num, path_len, t, tyw, x_se, lid, wrow);
  wave_lds_sync();
  for (int q = lid; q < x_se; q += kOmega) {
    const int r = y_ws + wrow[q];
    if (SDDMM) out[x_ws + q] = scale * g[r] * x[col[x_ws + q]];
    else rows[x_ws + q] = r;
  }
}

template <typename V, bool SDDMM>
static hipError_t tile_rows_pick(int sigma, const TileRowsArgs& a, hipStream_t st) {
  const unsigned grid = (unsigned)((a.tile_num + kDecodeWaves - 1) / kDecodeWaves);
  const V* g = static_cast<const V*>(a.g);
  const V* x = static_cast<const V*>(a.x);
  V* out = static_cast<V*>(a.out);
  const V scale = (V)a.scale;
  switch (sigma) {
#define MERBIT_RCASE(S)                                                                    \
  case S:                                                                                  \
    hipLaunchKernelGGL((tile_rows_kernel<V, S, SDDMM>), dim3(grid), dim3(kDecodeWaves * 64), \
                       0, st, a.tile_x, a.tile_y, a.lane_desc, a.tile_num, a.lane_num,     \
                       a.path_len, a.col, g, x, scale, out, a.rows);                       \
    return hipGetLastError();
    MERBIT_RCASE(1) MERBIT_RCASE(2) MERBIT_RCASE(3) MERBIT_RCASE(4) MERBIT_RCASE(5)
    MERBIT_RCASE(6) MERBIT_RCASE(7) MERBIT_RCASE(8) MERBIT_RCASE(9) MERBIT_RCASE(10)
    MERBIT_RCASE(11) MERBIT_RCASE(12)
#undef MERBIT_RCASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tile_rows(int dtype, int sigma, bool sddmm, const TileRowsArgs& a,
                            hipStream_t st) {
  if (a.tile_num == 0) return hipSuccess;
  if (dtype == 0)
    return sddmm ? tile_rows_pick<float, true>(sigma, a, st)
                 : tile_rows_pick<float, false>(sigma, a, st);
  return sddmm ? tile_rows_pick<double, true>(sigma, a, st)
               : tile_rows_pick<double, false>(sigma, a, st);
}

// ------------------------------------------------------------ transpose --

// rowT[c] = first position of key c in the sorted keys (m if none follows),
// for c = 0 .. n_cols: every c is written by exactly one thread.
__global__ void row_starts_kernel(const uint32_t* __restrict__ keys, int64_t m, int64_t n_cols,
                                  int32_t* __restrict__ rowT) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > m) return;
  const int64_t lo = i == 0 ? 0 : (int64_t)keys[i - 1] + 1;
  const int64_t hi = i == m ? n_cols : (int64_t)keys[i];
  for (int64_t c = lo; c <= hi; ++c) rowT[c] = (int32_t)i;
}

__global__ void gather_i32_kernel(const int32_t* __restrict__ src, const int32_t* __restrict__ idx,
                                  int32_t* __restrict__ dst, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) dst[i] = src[idx[i]];
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

static int radix_passes(int end_bit) { return (end_bit + 7) / 8; }

size_t transpose_temp_bytes(int64_t m, int end_bit) {
  // two key buffers and one spare position buffer, then the pass's own temp
  const size_t arrays = 3 * (((size_t)(m > 0 ? m : 1) * sizeof(int32_t) + 255) & ~(size_t)255);
  return arrays + radix_temp_bytes(m, end_bit < 8 ? end_bit : 8);
}

hipError_t launch_transpose(const int32_t* col, const int32_t* rows, int64_t m, int64_t n_cols,
                            int end_bit, void* temp, int32_t* rowT, int32_t* colT,
                            int32_t* perm, hipStream_t st) {
  const size_t arr = ((size_t)(m > 0 ? m : 1) * sizeof(int32_t) + 255) & ~(size_t)255;
  unsigned char* t = static_cast<unsigned char*>(temp);
  uint32_t* keys[2] = {reinterpret_cast<uint32_t*>(t), reinterpret_cast<uint32_t*>(t + arr)};
  int32_t* spare = reinterpret_cast<int32_t*>(t + 2 * arr);
  void* pass_tmp = t + 3 * arr;
  if (m > 0) {
    // stable LSD radix sort of (column, position) pairs, 8 bits a pass: within
    // a column the positions stay increasing, i.e. the rows of A in order.
    // Pass p writes buffer (P - 1 - p) & 1, so the last one lands in perm.
    const int P = radix_passes(end_bit);
    int32_t* vals[2] = {perm, spare};
    for (int p = 0; p < P; ++p) {
      const int shift = 8 * p;
      const int bits = end_bit - shift < 8 ? end_bit - shift : 8;
      const int out = (P - 1 - p) & 1, in = out ^ 1;
      const uint32_t* kin = p == 0 ? reinterpret_cast<const uint32_t*>(col) : keys[in];
      const int32_t* vin = p == 0 ? nullptr : vals[in];
      hipError_t e = launch_radix_pass(kin, vin, keys[out], vals[out], m, shift, bits, pass_tmp,
                                       st);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(gather_i32_kernel, dim3(blocks_for(m)), dim3(256), 0, st, rows, perm,
                       colT, m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(row_starts_kernel, dim3(blocks_for(m + 1)), dim3(256), 0, st, keys[0], m,
                     n_cols, rowT);
  return hipGetLastError();
}

// ------------------------------------------------ gathers and scaling --

template <typename V>
__global__ void gather_values_kernel(const int32_t* __restrict__ perm, const V* __restrict__ src,
                                     const V* __restrict__ src2, V* __restrict__ dst, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t k = perm[i];
  dst[i] = src2 ? src[k] * src2[k] : src[k];
}

hipError_t launch_gather_values(int dtype, const int32_t* perm, const void* src, const void* src2,
                                void* dst, int64_t m, hipStream_t st) {
  if (m == 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(gather_values_kernel<float>, dim3(blocks_for(m)), dim3(256), 0, st, perm,
                       static_cast<const float*>(src), static_cast<const float*>(src2),
                       static_cast<float*>(dst), m);
  else
    hipLaunchKernelGGL(gather_values_kernel<double>, dim3(blocks_for(m)), dim3(256), 0, st, perm,
                       static_cast<const double*>(src), static_cast<const double*>(src2),
                       static_cast<double*>(dst), m);
  return hipGetLastError();
}

template <typename V>
__global__ void column_scale_kernel(const int32_t* __restrict__ col, const V* __restrict__ a,
                                    const V* __restrict__ t, const V* __restrict__ s,
                                    V* __restrict__ out, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t c = col[i];
  out[i] = (t ? a[i] - t[c] : a[i]) / s[c];
}

hipError_t launch_column_scale(int dtype, const int32_t* col, const void* a, const void* t,
                               const void* s, void* out, int64_t m, hipStream_t st) {
  if (m == 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(column_scale_kernel<float>, dim3(blocks_for(m)), dim3(256), 0, st, col,
                       static_cast<const float*>(a), static_cast<const float*>(t),
                       static_cast<const float*>(s), static_cast<float*>(out), m);
  else
    hipLaunchKernelGGL(column_scale_kernel<double>, dim3(blocks_for(m)), dim3(256), 0, st, col,
                       static_cast<const double*>(a), static_cast<const double*>(t),
                       static_cast<const double*>(s), static_cast<double*>(out), m);
  return hipGetLastError();
}

// ------------------------------------------------------ adjoint update --

// (sum of v, 0) per block
template <typename V>
__global__ __launch_bounds__(kReduceThreads) void adj_sum_kernel(const V* __restrict__ v,
                                                                int64_t n,
                                                                double* __restrict__ part_out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double a = 0.0, z = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    a += (double)v[i];
  block_sum2(a, z);
  if (threadIdx.x == 0) {
    part_out[2 * blockIdx.x] = a;
    part_out[2 * blockIdx.x + 1] = 0.0;
  }
}

// lam_new = g + alpha y + (alpha / n) S d, S = sum of lam_old (first
// components of part_in); writes this block's (sum lam_new, l1 change).
// With hot_n > 0 it also writes the hot-column copy of lam_new that the next
// SpMV's LDS cache reads (x_hot[s] = lam_new[hot_cols[s]], the same
// operations on the same operands), so that SpMV needs no gather launch.
template <typename V>
__global__ __launch_bounds__(kReduceThreads) void adj_update_kernel(
    const V* __restrict__ y, const V* __restrict__ lam_old, V* __restrict__ lam_new,
    const V* __restrict__ g, const uint32_t* __restrict__ dmask, int64_t n, double alpha,
    const double* __restrict__ part_in, int n_in, double* __restrict__ part_out,
    const int32_t* __restrict__ hot_cols, int32_t hot_n, V* __restrict__ x_hot) {
  __shared__ double total;
  {
    double a = 0.0, z = 0.0;
    for (int k = threadIdx.x; k < n_in; k += kReduceThreads) a += part_in[2 * k];
    block_sum2(a, z);
    if (threadIdx.x == 0) total = a;
    __syncthreads();
  }
  const V dang = (V)(alpha * total / (double)n);
  const V al = (V)alpha;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double ssum = 0.0, rsum = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    V v = fma(al, y[i], g[i]);
    if ((dmask[i >> 5] >> (i & 31)) & 1u) v += dang;
    lam_new[i] = v;
    ssum += (double)v;
    rsum += fabs((double)v - (double)lam_old[i]);
  }
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < hot_n; h += stride) {
    const int64_t c = hot_cols[h];
    V v = fma(al, y[c], g[c]);
    if ((dmask[c >> 5] >> (c & 31)) & 1u) v += dang;
    x_hot[h] = v;
  }
  block_sum2(ssum, rsum);
  if (threadIdx.x == 0) {
    part_out[2 * blockIdx.x] = ssum;
    part_out[2 * blockIdx.x + 1] = rsum;
  }
}

hipError_t launch_adj_sum(int dtype, const void* v, int64_t n, double* part_out, int grid,
                          hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL(adj_sum_kernel<float>, dim3(grid), dim3(kReduceThreads), 0, st,
                       static_cast<const float*>(v), n, part_out);
  else
    hipLaunchKernelGGL(adj_sum_kernel<double>, dim3(grid), dim3(kReduceThreads), 0, st,
                       static_cast<const double*>(v), n, part_out);
  return hipGetLastError();
}

hipError_t launch_adj_update(int dtype, const void* y, const void* lam_old, void* lam_new,
                             const void* g, const uint32_t* dmask, int64_t n, double alpha,
                             const double* part_in, int n_in, double* part_out, int grid,
                             hipStream_t st, const int32_t* hot_cols, int32_t hot_n,
                             void* x_hot) {
  if (dtype == 0)
    hipLaunchKernelGGL(adj_update_kernel<float>, dim3(grid), dim3(kReduceThreads), 0, st,
                       static_cast<const float*>(y), static_cast<const float*>(lam_old),
                       static_cast<float*>(lam_new), static_cast<const float*>(g), dmask, n,
                       alpha, part_in, n_in, part_out, hot_cols, hot_n,
                       static_cast<float*>(x_hot));
  else
    hipLaunchKernelGGL(adj_update_kernel<double>, dim3(grid), dim3(kReduceThreads), 0, st,
                       static_cast<const double*>(y), static_cast<const double*>(lam_old),
                       static_cast<double*>(lam_new), static_cast<const double*>(g), dmask, n,
                       alpha, part_in, n_in, part_out, hot_cols, hot_n,
                       static_cast<double*>(x_hot));
  return hipGetLastError();
}

}  // namespace merbit
