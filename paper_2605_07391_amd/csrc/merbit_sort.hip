// Scans and a stable radix-sort pass for the one-time plan work (column
// stripes, hot-column selection, the transpose of the adjoint).
//
// Scan: three launches over chunks of kScanChunk values -- each block reduces
// its chunk, one block scans the chunk totals, each block scans its chunk
// from its total's prefix.  Sum and max, inclusive or exclusive, int32.
//
// Radix pass: a stable counting sort of (key, value) pairs by the digit
// (key >> shift) & (2^bits - 1), bits <= 8.  Each wavefront owns a segment of
// kSortSeg consecutive pairs.  A first launch counts the digits of every
// segment (the lanes that hold equal digits find each other with one ballot
// per digit bit, and the highest of them adds their number to the
// wavefront's LDS counter); the counts, stored digit-major, are scanned; a
// second launch walks the segment again in the same order and writes each
// pair at its digit's running position.  Digit-major order of the counts
// keeps equal digits in segment order, and the walk keeps them in order
// inside a segment, so the pass is stable.  LSD passes over successive digit
// fields sort by the whole key.
#include <limits.h>

#include "merbit_internal.hpp"

namespace merbit {

// ------------------------------------------------------------------ scan --

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanChunk = kScanThreads * kScanItems;
constexpr int kPartThreads = 1024;

struct ScanSum {
  static __device__ __forceinline__ int32_t id() { return 0; }
  static __device__ __forceinline__ int32_t op(int32_t a, int32_t b) { return a + b; }
};
struct ScanMax {
  static __device__ __forceinline__ int32_t id() { return INT_MIN; }
  static __device__ __forceinline__ int32_t op(int32_t a, int32_t b) { return a > b ? a : b; }
};

// Inclusive scan over the block's threads (blockDim.x = THREADS, a multiple
// of 64); every thread gets its own inclusive value, *total the block's.
template <class Op, int THREADS>
__device__ __forceinline__ int32_t block_inclusive_scan(int32_t v, int32_t* s_wave,
                                                        int32_t* total) {
  const int lid = threadIdx.x & (kOmega - 1), wid = threadIdx.x / kOmega;
#pragma unroll
  for (int d = 1; d < kOmega; d <<= 1) {
    const int32_t t = __shfl_up(v, d, kOmega);
    if (lid >= d) v = Op::op(t, v);
  }
  if (lid == kOmega - 1) s_wave[wid] = v;
  __syncthreads();
  int32_t before = Op::id();
  int32_t all = Op::id();
  for (int w = 0; w < THREADS / kOmega; ++w) {
    if (w < wid) before = Op::op(before, s_wave[w]);
    all = Op::op(all, s_wave[w]);
  }
  __syncthreads();  // s_wave may be reused by the caller
  *total = all;
  return Op::op(before, v);
}

template <class Op>
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const int32_t* __restrict__ in,
                                                                   int64_t n,
                                                                   int32_t* __restrict__ part) {
  __shared__ int32_t s_wave[kScanThreads / kOmega];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  int32_t acc = Op::id();
#pragma unroll
  for (int it = 0; it < kScanItems; ++it) {
    const int64_t i = base + it * kScanThreads + threadIdx.x;
    if (i < n) acc = Op::op(acc, in[i]);
  }
  int32_t total;
  (void)block_inclusive_scan<Op, kScanThreads>(acc, s_wave, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// part[0 .. nb) <- its exclusive scan (one block)
template <class Op>
__global__ __launch_bounds__(kPartThreads) void scan_parts_kernel(int32_t* __restrict__ part,
                                                                  int64_t nb) {
  __shared__ int32_t s_wave[kPartThreads / kOmega];
  __shared__ int32_t s_incl[kPartThreads];
  int32_t carry = Op::id();
  for (int64_t b0 = 0; b0 < nb; b0 += kPartThreads) {
    const int64_t b = b0 + threadIdx.x;
    const int32_t v = b < nb ? part[b] : Op::id();
    int32_t total;
    const int32_t incl = block_inclusive_scan<Op, kPartThreads>(v, s_wave, &total);
    s_incl[threadIdx.x] = incl;
    __syncthreads();
    const int32_t excl = threadIdx.x == 0 ? carry : Op::op(carry, s_incl[threadIdx.x - 1]);
    if (b < nb) part[b] = excl;
    carry = Op::op(carry, total);
    __syncthreads();
  }
}

// LDS index of chunk element i: one pad word per 16 keeps a thread's run of
// kScanItems consecutive elements on distinct banks across the wavefront
__device__ __forceinline__ int scan_lds(int i) { return i + (i >> 4); }

template <class Op, bool EXCLUSIVE>
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(
    const int32_t* in, int32_t* out, int64_t n, const int32_t* __restrict__ part) {
  // in == out is allowed: the block reads its whole chunk before writing it
  __shared__ int32_t s[kScanChunk + kScanChunk / 16];
  __shared__ int32_t s_wave[kScanThreads / kOmega];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
#pragma unroll
  for (int it = 0; it < kScanItems; ++it) {
    const int k = it * kScanThreads + threadIdx.x;
    s[scan_lds(k)] = base + k < n ? in[base + k] : Op::id();
  }
  __syncthreads();
  const int first = threadIdx.x * kScanItems;
  int32_t run = Op::id();
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) run = Op::op(run, s[scan_lds(first + k)]);
  int32_t total;
  const int32_t incl = block_inclusive_scan<Op, kScanThreads>(run, s_wave, &total);
  // everything before this thread's run: the chunk's prefix and the previous
  // thread's inclusive value (max has no inverse, so no subtraction)
  __shared__ int32_t s_prev[kScanThreads];
  s_prev[threadIdx.x] = incl;
  __syncthreads();
  int32_t acc =
      threadIdx.x == 0 ? part[blockIdx.x] : Op::op(part[blockIdx.x], s_prev[threadIdx.x - 1]);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int li = scan_lds(first + k);
    const int32_t v = s[li];
    if (EXCLUSIVE) {
      s[li] = acc;
      acc = Op::op(acc, v);
    } else {
      acc = Op::op(acc, v);
      s[li] = acc;
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kScanItems; ++it) {
    const int k = it * kScanThreads + threadIdx.x;
    if (base + k < n) out[base + k] = s[scan_lds(k)];
  }
}

int64_t scan_blocks(int64_t n) { return (n + kScanChunk - 1) / kScanChunk; }

size_t scan_temp_bytes(int64_t n) {
  return sizeof(int32_t) * (size_t)(scan_blocks(n) > 0 ? scan_blocks(n) : 1);
}

template <class Op, bool EXCLUSIVE>
static hipError_t scan_t(const int32_t* in, int32_t* out, int64_t n, int32_t* part,
                         hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = scan_blocks(n);
  hipLaunchKernelGGL((scan_reduce_kernel<Op>), dim3((unsigned)nb), dim3(kScanThreads), 0, st, in,
                     n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((scan_parts_kernel<Op>), dim3(1), dim3(kPartThreads), 0, st, part, nb);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((scan_apply_kernel<Op, EXCLUSIVE>), dim3((unsigned)nb), dim3(kScanThreads),
                     0, st, in, out, n, part);
  return hipGetLastError();
}

hipError_t launch_scan_i32(const int32_t* in, int32_t* out, int64_t n, ScanKind kind,
                           void* temp, hipStream_t st) {
  int32_t* part = static_cast<int32_t*>(temp);
  switch (kind) {
    case kScanExclusiveSum: return scan_t<ScanSum, true>(in, out, n, part, st);
    case kScanInclusiveSum: return scan_t<ScanSum, false>(in, out, n, part, st);
    case kScanInclusiveMax: return scan_t<ScanMax, false>(in, out, n, part, st);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------ radix pass --

constexpr int kSortWaves = 4;
constexpr int kSortItems = 32;
constexpr int kSortSeg = kOmega * kSortItems;
constexpr int kSortMaxDigits = 256;

// Lanes of the wavefront whose `valid` digit equals this lane's.
__device__ __forceinline__ unsigned long long digit_peers(uint32_t d, bool valid, int bits) {
  unsigned long long m = __ballot(valid);
  for (int b = 0; b < bits; ++b) {
    const bool on = (d >> b) & 1u;
    const unsigned long long bal = __ballot(valid && on);
    m &= on ? bal : ~bal;
  }
  return m;
}

__global__ __launch_bounds__(kSortWaves * kOmega) void radix_count_kernel(
    const uint32_t* __restrict__ key, int64_t n, int shift, int bits, int64_t nseg,
    int32_t* __restrict__ counts) {
  __shared__ int32_t s_cnt[kSortWaves][kSortMaxDigits];
  const int lid = threadIdx.x & (kOmega - 1);
  const int wid = threadIdx.x / kOmega;
  const int64_t seg = (int64_t)blockIdx.x * kSortWaves + wid;
  if (seg >= nseg) return;  // no block-wide barrier below
  const int nd = 1 << bits;
  const uint32_t dmask = (uint32_t)nd - 1u;
  int32_t* cnt = s_cnt[wid];
  for (int d = lid; d < nd; d += kOmega) cnt[d] = 0;
  wave_lds_sync();
  const int64_t base = seg * kSortSeg;
  for (int it = 0; it < kSortItems; ++it) {
    const int64_t i = base + (int64_t)it * kOmega + lid;
    const bool valid = i < n;
    const uint32_t d = valid ? (key[i] >> shift) & dmask : 0u;
    const unsigned long long peers = digit_peers(d, valid, bits);
    // the highest lane of each group of equal digits adds the group's size
    if (valid && 63 - __builtin_clzll(peers) == lid) cnt[d] += __popcll(peers);
    wave_lds_sync();
  }
  for (int d = lid; d < nd; d += kOmega) counts[(int64_t)d * nseg + seg] = cnt[d];
}

__global__ __launch_bounds__(kSortWaves * kOmega) void radix_scatter_kernel(
    const uint32_t* __restrict__ key_in, const int32_t* __restrict__ val_in,
    uint32_t* __restrict__ key_out, int32_t* __restrict__ val_out, int64_t n, int shift,
    int bits, int64_t nseg, const int32_t* __restrict__ offsets) {
  __shared__ int32_t s_pos[kSortWaves][kSortMaxDigits];
  const int lid = threadIdx.x & (kOmega - 1);
  const int wid = threadIdx.x / kOmega;
  const int64_t seg = (int64_t)blockIdx.x * kSortWaves + wid;
  if (seg >= nseg) return;
  const int nd = 1 << bits;
  const uint32_t dmask = (uint32_t)nd - 1u;
  int32_t* pos = s_pos[wid];
  for (int d = lid; d < nd; d += kOmega) pos[d] = offsets[(int64_t)d * nseg + seg];
  wave_lds_sync();
  const unsigned long long below = (1ull << lid) - 1ull;
  const int64_t base = seg * kSortSeg;
  for (int it = 0; it < kSortItems; ++it) {
    const int64_t i = base + (int64_t)it * kOmega + lid;
    const bool valid = i < n;
    const uint32_t k = valid ? key_in[i] : 0u;
    const uint32_t d = (k >> shift) & dmask;
    const unsigned long long peers = digit_peers(d, valid, bits);
    const int32_t at = valid ? pos[d] + __popcll(peers & below) : 0;
    wave_lds_sync();  // every lane has read its digit's position
    if (valid) {
      key_out[at] = k;
      val_out[at] = val_in ? val_in[i] : (int32_t)i;
      if (63 - __builtin_clzll(peers) == lid) pos[d] = at + 1;
    }
    wave_lds_sync();
  }
}

static int64_t sort_segments(int64_t n) { return (n + kSortSeg - 1) / kSortSeg; }

size_t radix_temp_bytes(int64_t n, int bits) {
  const int64_t counts = sort_segments(n) * ((int64_t)1 << bits);
  return sizeof(int32_t) * (size_t)(counts > 0 ? counts : 1) + scan_temp_bytes(counts) + 256;
}

hipError_t launch_radix_pass(const uint32_t* key_in, const int32_t* val_in, uint32_t* key_out,
                             int32_t* val_out, int64_t n, int shift, int bits, void* temp,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (bits < 1 || bits > 8) return hipErrorInvalidValue;
  const int64_t nseg = sort_segments(n);
  const int64_t nc = nseg * ((int64_t)1 << bits);
  int32_t* counts = static_cast<int32_t*>(temp);
  int32_t* part = reinterpret_cast<int32_t*>(
      static_cast<unsigned char*>(temp) + ((sizeof(int32_t) * (size_t)nc + 255) & ~(size_t)255));
  const unsigned grid = (unsigned)((nseg + kSortWaves - 1) / kSortWaves);
  hipLaunchKernelGGL(radix_count_kernel, dim3(grid), dim3(kSortWaves * kOmega), 0, st, key_in, n,
                     shift, bits, nseg, counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_scan_i32(counts, counts, nc, kScanExclusiveSum, part, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(radix_scatter_kernel, dim3(grid), dim3(kSortWaves * kOmega), 0, st, key_in,
                     val_in, key_out, val_out, n, shift, bits, nseg, counts);
  return hipGetLastError();
}

}  // namespace merbit
