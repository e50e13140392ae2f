// Column-stripe split of a CSR matrix, and the sum of the stripes' row
// results (a gfx950 layout around the MERBIT plan; the plan, descriptors and
// fused kernel are unchanged).
//
// The x gathers of the fused SpMV run at the rate L1 misses are served, and a
// miss served by the XCD's own L2 (4 MB) costs less than one served further
// out.  A matrix whose x does not fit in L2 is cut into S column stripes of
// equal width: A = sum_s A_s, with A_s holding the nonzeros of columns in
// stripe s.  The stripes are stacked into one CSR matrix A' whose rows are
// the non-empty (stripe, row) pairs in stripe-major order (within a stripe
// in row order), so y' = A' x is a plain SpMV that MERBIT plans as usual.
// The plan's tiles are then split into one contiguous range per XCD, so an
// XCD gathers from about one stripe of x at a time (and its blocks can keep
// the most frequent columns of their own range in LDS); a second kernel adds
// each row's stripe results:
//   y[r] = sum over stripes s holding a nonzero of row r of y'[v(s, r)],
// with v(s, r) found from a bitmap of the rows present in each stripe and
// the rank of each 64-row word.
#include "merbit_internal.hpp"

namespace merbit {

static unsigned blocks_of(int64_t n) { return (unsigned)((n + 255) / 256); }

// rows[row_ptr[r]] = r for every non-empty row r: each position is the start
// of at most one non-empty row, so it is written at most once.
__global__ void row_heads_kernel(const int32_t* __restrict__ row_ptr, int64_t n_rows,
                                 int32_t* __restrict__ rows) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n_rows && row_ptr[r + 1] > row_ptr[r]) rows[row_ptr[r]] = (int32_t)r;
}

// After the stable sort by stripe (col_s = the stacked column stream, perm =
// matrix position of each stacked nonzero): row_s[i] = rows[perm[i]], and
// flag[i] = 1 where a new (stripe, row) pair begins.
__global__ void stripe_gather_kernel(const int32_t* __restrict__ perm,
                                     const int32_t* __restrict__ rows,
                                     const int32_t* __restrict__ col_s, int shift, int64_t m,
                                     int32_t* __restrict__ row_s, int32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t r = rows[perm[i]];
  row_s[i] = r;
  flag[i] = (i == 0 || ((uint32_t)col_s[i] >> shift) != ((uint32_t)col_s[i - 1] >> shift) ||
             rows[perm[i - 1]] != r)
                ? 1
                : 0;
}

// For each pair start i (flag set): v = vidx[i], vrow_ptr[v] = i, and the
// pair's row and stripe.  vrow_ptr[V] = m is set by the host.
__global__ void vrow_emit_kernel(const int32_t* __restrict__ flag,
                                 const int32_t* __restrict__ vidx,
                                 const int32_t* __restrict__ row_s,
                                 const int32_t* __restrict__ col_s, int shift, int64_t m,
                                 int32_t* __restrict__ vrow_ptr, int32_t* __restrict__ vrow_row,
                                 uint32_t* __restrict__ vrow_stripe) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m || !flag[i]) return;
  const int32_t v = vidx[i];
  vrow_ptr[v] = (int32_t)i;
  vrow_row[v] = row_s[i];
  vrow_stripe[v] = (uint32_t)col_s[i] >> shift;
}

__global__ void store_i32_kernel(int32_t* __restrict__ p, int32_t v) {
  if (threadIdx.x == 0) p[0] = v;
}

// bit (r mod 64) of entry [r / 64][s] is set for each pair (s, r)
__global__ void stripe_bitmap_kernel(const int32_t* __restrict__ vrow_row,
                                     const uint32_t* __restrict__ vrow_stripe, int64_t nv,
                                     int64_t stripes, StripeWord* __restrict__ sw) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const int32_t r = vrow_row[v];
  atomicOr(&sw[(int64_t)(r >> 6) * stripes + vrow_stripe[v]].bits, 1ull << (r & 63));
}

// cnt[s * words + w] = popcount of entry [w][s] (stripe-major, the order of
// the stacked rows)
__global__ void popcount_kernel(const StripeWord* __restrict__ sw, int64_t stripes,
                                int64_t words, int32_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= stripes * words) return;
  const int64_t s = i / words, w = i - s * words;
  cnt[i] = __popcll(sw[w * stripes + s].bits);
}

__global__ void rank_store_kernel(const int32_t* __restrict__ rank, int64_t stripes,
                                  int64_t words, StripeWord* __restrict__ sw) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= stripes * words) return;
  const int64_t s = i / words, w = i - s * words;
  sw[w * stripes + s].rank = rank[i];
}

// One wavefront per 64-row word: lane b sums row 64 w + b over the stripes.
// The S table entries of the word are read by every lane (the same address
// across the wavefront: one request each), all before any is used, and every
// lane loads every stripe's value (a lane whose row is absent from a stripe
// reads a valid entry nearby and drops it), so the S loads go out together
// instead of one branch at a time; the stripes are added in stripe order (a
// fixed order).
template <typename V, int S>
__global__ __launch_bounds__(256) void stripe_combine_kernel(const V* __restrict__ yv,
                                                             int64_t nv,
                                                             const StripeWord* __restrict__ sw,
                                                             int64_t words, int64_t n_rows,
                                                             V* __restrict__ y) {
  const int lid = threadIdx.x & (kOmega - 1);
  const int64_t w = (int64_t)blockIdx.x * (blockDim.x / kOmega) +
                    __builtin_amdgcn_readfirstlane(threadIdx.x / kOmega);
  if (w >= words) return;
  const unsigned long long below = (1ull << lid) - 1ull;
  // the entries as 16-byte vector loads (bits low / high, rank, pad)
  typedef int32_t i4v __attribute__((ext_vector_type(4)));
  const i4v* __restrict__ e = reinterpret_cast<const i4v*>(sw + w * S) + (lid & 0);
  i4v ent[S];
#pragma unroll
  for (int s = 0; s < S; ++s) ent[s] = e[s];
  unsigned long long word[S];
  int32_t base[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    word[s] = ((unsigned long long)(uint32_t)ent[s].y << 32) | (uint32_t)ent[s].x;
    base[s] = ent[s].z;
  }
  V part[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int64_t k = (int64_t)base[s] + __popcll(word[s] & below);
    part[s] = yv[k < nv ? k : nv - 1];
  }
#pragma unroll
  for (int s = 0; s < S; ++s)
    if (!((word[s] >> lid) & 1ull)) part[s] = V(0);
  V sum = V(0);
#pragma unroll
  for (int s = 0; s < S; ++s) sum += part[s];
  const int64_t r = w * kOmega + lid;
  if (r < n_rows) y[r] = sum;
}

// ------------------------------------------------------------ launchers --

size_t stripe_temp_bytes(int64_t m, int64_t n_words, int key_bits) {
  const size_t a = scan_temp_bytes(m > n_words ? m : n_words);
  const size_t b = radix_temp_bytes(m, key_bits);
  return a > b ? a : b;
}

hipError_t launch_stripe_split(const StripeSplitArgs& a, hipStream_t st) {
  const int64_t m = a.m;
  hipError_t e;
  // row of every nonzero: the row's index at its first nonzero, 0 elsewhere,
  // then a running maximum
  e = hipMemsetAsync(a.rows, 0, sizeof(int32_t) * (size_t)m, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(row_heads_kernel, dim3(blocks_of(a.n_rows)), dim3(256), 0, st, a.row_ptr,
                     a.n_rows, a.rows);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = launch_scan_i32(a.rows, a.rows, m, kScanInclusiveMax, a.temp, st);
  if (e != hipSuccess) return e;
  // stable sort of the nonzeros by stripe: one pass over the stripe digit of
  // the column (the columns come out in stacked order, with their positions)
  e = launch_radix_pass(reinterpret_cast<const uint32_t*>(a.col), nullptr,
                        reinterpret_cast<uint32_t*>(a.col_s), a.perm, m, a.shift, a.key_bits,
                        a.temp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(stripe_gather_kernel, dim3(blocks_of(m)), dim3(256), 0, st, a.perm, a.rows,
                     a.col_s, a.shift, m, a.row_s, a.flag);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return launch_scan_i32(a.flag, a.vidx, m, kScanExclusiveSum, a.temp, st);
}

hipError_t launch_stripe_rows(const StripeSplitArgs& a, int64_t nv, hipStream_t st) {
  hipError_t e;
  hipLaunchKernelGGL(vrow_emit_kernel, dim3(blocks_of(a.m)), dim3(256), 0, st, a.flag, a.vidx,
                     a.row_s, a.col_s, a.shift, a.m, a.vrow_ptr, a.vrow_row, a.vrow_stripe);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(store_i32_kernel, dim3(1), dim3(64), 0, st, a.vrow_ptr + nv, (int32_t)a.m);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // the rows present in each stripe and the stacked row of each entry's first
  const int64_t nw = a.stripes * a.words;
  e = hipMemsetAsync(a.sw, 0, sizeof(StripeWord) * (size_t)nw, st);
  if (e != hipSuccess) return e;
  if (nv > 0) {
    hipLaunchKernelGGL(stripe_bitmap_kernel, dim3(blocks_of(nv)), dim3(256), 0, st, a.vrow_row,
                       a.vrow_stripe, nv, a.stripes, a.sw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(popcount_kernel, dim3(blocks_of(nw)), dim3(256), 0, st, a.sw, a.stripes,
                     a.words, a.wcnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = launch_scan_i32(a.wcnt, a.rank, nw, kScanExclusiveSum, a.temp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rank_store_kernel, dim3(blocks_of(nw)), dim3(256), 0, st, a.rank, a.stripes,
                     a.words, a.sw);
  return hipGetLastError();
}

template <typename V, int S>
static void combine_t(const void* yv, int64_t nv, const StripeWord* sw, int64_t words,
                      int64_t n_rows, void* y, hipStream_t st) {
  const unsigned grid = (unsigned)((words + 3) / 4);
  hipLaunchKernelGGL((stripe_combine_kernel<V, S>), dim3(grid), dim3(256), 0, st,
                     static_cast<const V*>(yv), nv, sw, words, n_rows, static_cast<V*>(y));
}

template <typename V>
static hipError_t combine_pick(int stripes, const void* yv, int64_t nv, const StripeWord* sw,
                               int64_t words, int64_t n_rows, void* y, hipStream_t st) {
  switch (stripes) {
    case 2: combine_t<V, 2>(yv, nv, sw, words, n_rows, y, st); break;
    case 4: combine_t<V, 4>(yv, nv, sw, words, n_rows, y, st); break;
    case 8: combine_t<V, 8>(yv, nv, sw, words, n_rows, y, st); break;
    case 16: combine_t<V, 16>(yv, nv, sw, words, n_rows, y, st); break;
    case 32: combine_t<V, 32>(yv, nv, sw, words, n_rows, y, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_stripe_combine(int dtype, int stripes, const void* yv, int64_t nv,
                                 const StripeWord* sw, int64_t words, int64_t n_rows, void* y,
                                 hipStream_t st) {
  if (words == 0 || nv <= 0) return hipSuccess;
  return dtype == 0 ? combine_pick<float>(stripes, yv, nv, sw, words, n_rows, y, st)
                    : combine_pick<double>(stripes, yv, nv, sw, words, n_rows, y, st);
}

}  // namespace merbit
