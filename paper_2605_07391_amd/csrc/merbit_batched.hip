// Batched forms on the same plan: Y = A X for up to 64 right-hand sides at
// once, the per-column PageRank update for personalised PageRank, and the
// per-graph PageRank update for many graphs stored on the diagonal of one
// matrix.
//
// SpMM (one wavefront per tile, lanes = right-hand-side columns of a slab;
// the driver runs one launch per slab of 32 columns).  The
// tile's merge-path segment (Sec. 4.1) fixes its nonzeros [x_ws, x_we) and
// rows [y_ws, y_we]; every nonzero is a 64-wide row operation
// Y[row, :] += v * X[col, :], so each X access is one coalesced row load.
//   1. each lane decodes its descriptor (Sec. 4.1.1) and writes, for each of
//      its right steps, the row (relative to the tile) of that nonzero into
//      LDS: nonzero x_off + r of lane j lies in row y_off + (downs before it);
//   2. the tile's nonzeros are taken 64 at a time, lane l holding nonzero
//      q0 + l (coalesced loads of col_ind / values, its row from LDS, the
//      byte offset of its X row); one ballot marks the nonzeros that start a
//      new row;
//   3. the wavefront then walks those 64 nonzeros in order: each X row load
//      takes its offset from the owning lane (a lane read into a scalar
//      register, used as the buffer load's scalar offset), kSpmmGroup rows
//      are in flight before the first is used, each product is one fused
//      multiply-add with the value read from its lane, and a marked nonzero
//      first finishes the previous row.
// Per nonzero the wavefront spends one load and a few lane reads, not an
// LDS round trip, so the X row loads (the bulk of the traffic) stay
// back to back.  Rows strictly inside the tile are stored; the tile's first
// and last rows (shared with neighbouring tiles) are added atomically to Y,
// which is zero there before the launch.  Empty rows inside the tile are
// written as 0.
#include "merbit_internal.hpp"

namespace merbit {

constexpr int kSpmmWaves = 4;
constexpr int kSpmmGroup = 16;

template <typename V>
__device__ __forceinline__ void spmm_commit(V* Y, int64_t ld, int row_abs, int rel, int last_rel,
                                            int n_rows, V acc, bool lane_on, int lid) {
  if (!lane_on) return;
  V* p = Y + (int64_t)row_abs * ld + lid;
  if (rel == 0 || rel == last_rel) {
    if (row_abs < n_rows) global_add(p, acc);  // shared with a neighbouring tile
  } else {
    __builtin_nontemporal_store(acc, p);  // written once, not read here again
  }
}

// Per-lane state of a fused personalised-PageRank step (SpmmArgs::Xn).
template <typename V>
struct PprRow {
  V* Xn;
  int64_t ld;
  V a;          // alpha
  V tele;       // alpha delta_j + 1 - alpha, added at the column's source row
  int sj;       // the column's source row (-1: lane past the slab)
  int w0;       // dmask word of the tile's first row
  uint32_t dm;  // lane l: dmask word w0 + l (the tile's rows are < 32 words)
  double dsum;  // dangling mass of the rows this lane finished
};

// Row row_abs, strictly inside the tile, is complete: its next iterate
// value, written here instead of Y (called by the whole wavefront).
template <typename V>
__device__ __forceinline__ void ppr_finish_row(PprRow<V>& f, int row_abs, V acc, bool lane_on,
                                               int lid) {
  V xn = f.a * acc;
  if (row_abs == f.sj) xn += f.tele;
  if (lane_on) __builtin_nontemporal_store(xn, f.Xn + (int64_t)row_abs * f.ld + lid);
  const uint32_t word = (uint32_t)__builtin_amdgcn_readlane((int)f.dm, (row_abs >> 5) - f.w0);
  if ((word >> (row_abs & 31)) & 1u) f.dsum += (double)xn;
}

// A finished row of the tile: the first and last rows go to Y (shared with
// neighbouring tiles); the others are stored (plain SpMM) or finished as
// the next iterate (fused step).  Called by the whole wavefront.
template <typename V, bool FUSE>
__device__ __forceinline__ void spmm_row(V* Y, int64_t ld, int row_abs, int rel, int last_rel,
                                         int n_rows, V acc, bool lane_on, int lid,
                                         PprRow<V>& f) {
  if constexpr (FUSE) {
    if (rel == 0 || rel == last_rel) {
      if (lane_on && row_abs < n_rows) global_add(Y + (int64_t)row_abs * ld + lid, acc);
    } else {
      ppr_finish_row(f, row_abs, acc, lane_on, lid);
    }
  } else {
    spmm_commit(Y, ld, row_abs, rel, last_rel, n_rows, acc, lane_on, lid);
  }
}

// An empty row strictly inside the tile.
template <typename V, bool FUSE>
__device__ __forceinline__ void spmm_empty_row(V* Y, int64_t ld, int row_abs, bool lane_on,
                                               int lid, PprRow<V>& f) {
  if constexpr (FUSE) {
    ppr_finish_row(f, row_abs, V(0), lane_on, lid);
  } else {
    if (lane_on) Y[(int64_t)row_abs * ld + lid] = V(0);
  }
}

// value of lane `lane` of v (lane uniform), in scalar registers
__device__ __forceinline__ int lane_value(int v, int lane) {
  return __builtin_amdgcn_readlane(v, lane);
}
__device__ __forceinline__ float lane_value(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
__device__ __forceinline__ double lane_value(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// word 3 of a raw (unformatted, stride 0) buffer resource on gfx950
constexpr int kSpmmBufferWord3 = 0x00020000;

// One X row element per lane for the nonzero held by lane q of this chunk:
// through a buffer resource with the row's byte offset as the scalar offset
// (X no larger than 2 GiB), or through a 64-bit scalar row address.
// Every lane loads (no branch, so the group's loads go out back to back):
// lanes at or past k read the row's element k - 1 again (the same line, so a
// slab narrower than 64 columns fetches no part of X it does not use), and
// their values are never stored.
template <typename V, bool BUF>
__device__ __forceinline__ V load_x_row(__amdgpu_buffer_rsrc_t rx, const V* __restrict__ X,
                                        int64_t ldx, uint32_t off_l, int c_l, int q, int lane) {
  if constexpr (BUF) {
    const int soff = __builtin_amdgcn_readlane((int)off_l, q);
    if constexpr (sizeof(V) == 4)
      return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(rx, lane * 4, soff, 0));
    else
      return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(rx, lane * 8, soff, 0));
  } else {
    const V* __restrict__ xr = X + (int64_t)lane_value(c_l, q) * ldx;
    return xr[lane];
  }
}

template <typename V, int SIGMA, bool BUF, bool FUSE>
__device__ __forceinline__ void spmm_walk(const SpmmArgs& a, const int32_t* __restrict__ wrow,
                                          int x_ws, int x_se, int y_ws, int last_rel, int lid,
                                          bool lane_on, V& acc, int& cur, PprRow<V>& f) {
  const V* __restrict__ X = static_cast<const V*>(a.X);
  V* __restrict__ Y = static_cast<V*>(a.Y);
  const int32_t* __restrict__ col = a.col + x_ws;
  const V* __restrict__ val = static_cast<const V*>(a.val) + x_ws;
  const int64_t ldx = a.ldx, ldy = a.ldy;
  // (unused by the 64-bit path)
  const int bytes = BUF ? (int)((((int64_t)a.x_rows - 1) * ldx + a.k) * (int64_t)sizeof(V)) : 0;
  const __amdgpu_buffer_rsrc_t rx =
      __builtin_amdgcn_make_buffer_rsrc((void*)X, (short)0, bytes, kSpmmBufferWord3);
  const uint32_t row_bytes = (uint32_t)(ldx * (int64_t)sizeof(V));
  // lanes past k stay on the slab's last column
  const int lane = min(lid, a.k - 1);
  for (int q0 = 0; q0 < x_se; q0 += kOmega) {
    const int ql = q0 + lid;
    const bool valid = ql < x_se;
    // the matrix stream is read once: non-temporal, so it does not push the
    // reused X rows out of L2
    const int c_l = valid ? __builtin_nontemporal_load(col + ql) : 0;
    const V v_l = valid ? __builtin_nontemporal_load(val + ql) : V(0);
    const int r_l = valid ? wrow[ql] : 0;
    const uint32_t off_l = (uint32_t)c_l * row_bytes;
    // bit l: nonzero q0 + l lies in another row than the nonzero before it
    // (every lane takes part in the shuffle: a lane outside it gives no value)
    const int up = __shfl_up(r_l, 1, kOmega);
    const int prev = lid == 0 ? cur : up;
    const unsigned long long starts = __ballot(valid && r_l != prev);
    const int cnt = min(kOmega, x_se - q0);
    for (int u0 = 0; u0 < cnt; u0 += kSpmmGroup) {
      V xr[kSpmmGroup];
#pragma unroll
      for (int u = 0; u < kSpmmGroup; ++u) {
        const int q = min(u0 + u, cnt - 1);  // past the end: a repeat, never used
        xr[u] = load_x_row<V, BUF>(rx, X, ldx, off_l, c_l, q, lane);
      }
#pragma unroll
      for (int u = 0; u < kSpmmGroup; ++u) {
        const int q = u0 + u;
        if (q < cnt) {
          if ((starts >> q) & 1ull) {
            const int r = lane_value(r_l, q);
            spmm_row<V, FUSE>(Y, ldy, y_ws + cur, cur, last_rel, a.n_rows, acc, lane_on, lid, f);
            for (int e = cur + 1; e < r; ++e)  // empty rows strictly inside the tile
              spmm_empty_row<V, FUSE>(Y, ldy, y_ws + e, lane_on, lid, f);
            cur = r;
            acc = V(0);
          }
          acc += lane_value(v_l, q) * xr[u];
        }
      }
    }
  }
}

template <typename V, int SIGMA, bool FUSE>
__global__ __launch_bounds__(kSpmmWaves * 64) void spmm_kernel(SpmmArgs a) {
  constexpr int WLDS = kOmega * SIGMA;
  __shared__ int32_t s_row[kSpmmWaves * WLDS];

  const int lid = threadIdx.x & (kOmega - 1);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kOmega);
  const int t = blockIdx.x * kSpmmWaves + wid;
  const bool lane_on = lid < a.k;
  PprRow<V> f{};
  if constexpr (FUSE) {
    f.Xn = static_cast<V*>(a.Xn);
    f.ld = a.ldx;
    f.a = (V)a.alpha;
    f.sj = lane_on ? a.src[lid] : -1;
    f.tele = lane_on ? (V)(a.alpha * a.sums_in[2 * lid] + 1.0 - a.alpha) : V(0);
    f.dsum = 0.0;
  }
  // without the fused step no block-wide synchronisation follows: a
  // wavefront past the last tile may leave at once
  if (t < a.tile_num) {
    int32_t* wrow = s_row + wid * WLDS;
    V* __restrict__ Y = static_cast<V*>(a.Y);
    const int x_ws = a.tile_x[t];
    const int x_se = a.tile_x[t + 1] - x_ws;
    const uint32_t tyw = a.tile_y[t];
    const int y_ws = (int)(tyw & kRowMask);
    const int y_we = (int)(a.tile_y[t + 1] & kRowMask);
    const int last_rel = y_we - y_ws;
    if constexpr (FUSE) {
      // the tile's rows y_ws .. y_we span at most 64 sigma / 32 + 2 words
      f.w0 = y_ws >> 5;
      f.dm = f.w0 + lid < a.dmask_words ? a.dmask[f.w0 + lid] : 0u;
    }

    tile_nz_rows<SIGMA>(a.lane_desc, a.lane_num, a.path_len, t, tyw, x_se, lid, wrow);
    wave_lds_sync();

    V acc = V(0);
    int cur = 0;  // current row, relative to y_ws
    const bool buf = ((int64_t)a.x_rows * a.ldx) * (int64_t)sizeof(V) < ((int64_t)1 << 31);
    if (buf)
      spmm_walk<V, SIGMA, true, FUSE>(a, wrow, x_ws, x_se, y_ws, last_rel, lid, lane_on, acc,
                                      cur, f);
    else
      spmm_walk<V, SIGMA, false, FUSE>(a, wrow, x_ws, x_se, y_ws, last_rel, lid, lane_on, acc,
                                       cur, f);
    const int64_t ldy = a.ldy;
    if (x_se > 0)
      spmm_row<V, FUSE>(Y, ldy, y_ws + cur, cur, last_rel, a.n_rows, acc, lane_on, lid, f);
    // rows after the last nonzero and strictly inside the tile are empty
    for (int e = (x_se > 0 ? cur + 1 : 1); e < last_rel; ++e)
      spmm_empty_row<V, FUSE>(Y, ldy, y_ws + e, lane_on, lid, f);
    if (a.Z != nullptr && lane_on)
      static_cast<V*>(a.Z)[(int64_t)y_ws * a.ldz + lid] = V(0);
  }
  if constexpr (FUSE) {
    // the block's dangling mass per column, its wavefronts added in order
    __shared__ double s_d[kSpmmWaves][kOmega];
    s_d[wid][lid] = f.dsum;
    __syncthreads();
    if (wid == 0 && lane_on) {
      double d = 0.0;
      for (int w = 0; w < kSpmmWaves; ++w) d += s_d[w][lid];
      double* o = a.part + ((int64_t)blockIdx.x * kOmega + a.col0 + lid) * 2;
      o[0] = d;
      o[1] = 0.0;
    }
  }
}

int spmm_blocks(int64_t tile_num) { return (int)((tile_num + kSpmmWaves - 1) / kSpmmWaves); }

template <typename V, int S>
static hipError_t spmm_launch_t(const SpmmArgs& a, hipStream_t st) {
  const unsigned grid = (unsigned)spmm_blocks(a.tile_num);
  if (a.Xn != nullptr)
    hipLaunchKernelGGL((spmm_kernel<V, S, true>), dim3(grid), dim3(kSpmmWaves * 64), 0, st, a);
  else
    hipLaunchKernelGGL((spmm_kernel<V, S, false>), dim3(grid), dim3(kSpmmWaves * 64), 0, st, a);
  return hipGetLastError();
}

typedef hipError_t (*spmm_fn)(const SpmmArgs&, hipStream_t);

template <typename V>
static spmm_fn spmm_pick(int sigma) {
  switch (sigma) {
#define MERBIT_MCASE(S) \
  case S: return spmm_launch_t<V, S>;
    MERBIT_MCASE(1) MERBIT_MCASE(2) MERBIT_MCASE(3) MERBIT_MCASE(4) MERBIT_MCASE(5)
    MERBIT_MCASE(6) MERBIT_MCASE(7) MERBIT_MCASE(8) MERBIT_MCASE(9) MERBIT_MCASE(10)
    MERBIT_MCASE(11) MERBIT_MCASE(12)
#undef MERBIT_MCASE
    default: return nullptr;
  }
}

hipError_t launch_spmm(int dtype, int sigma, const SpmmArgs& a, hipStream_t st) {
  if (a.tile_num == 0) return hipSuccess;
  spmm_fn f = dtype == 0 ? spmm_pick<float>(sigma) : spmm_pick<double>(sigma);
  if (!f) return hipErrorInvalidValue;
  return f(a, st);
}

// Zero Y[tile_y[t], col0 .. col0 + k) for every tile t (the rows the SpMM adds onto).
template <typename V>
__global__ void spmm_zero_kernel(const uint32_t* __restrict__ tile_y, int32_t tile_num, V* Y,
                                 int64_t ld, int k) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t t = e / 64, j = e % 64;
  if (t < tile_num && j < k) Y[(int64_t)(tile_y[t] & kRowMask) * ld + j] = V(0);
}

hipError_t launch_spmm_zero(int dtype, const uint32_t* tile_y, int32_t tile_num, void* Y,
                            int64_t ld, int k, hipStream_t st) {
  if (tile_num == 0) return hipSuccess;
  const unsigned grid = (unsigned)(((int64_t)tile_num * 64 + 255) / 256);
  if (dtype == 0)
    hipLaunchKernelGGL(spmm_zero_kernel<float>, dim3(grid), dim3(256), 0, st, tile_y, tile_num,
                       static_cast<float*>(Y), ld, k);
  else
    hipLaunchKernelGGL(spmm_zero_kernel<double>, dim3(grid), dim3(256), 0, st, tile_y, tile_num,
                       static_cast<double*>(Y), ld, k);
  return hipGetLastError();
}

// ---------------------------------------------- personalised PageRank step --
//
// Column j of X is the rank vector of source src[j]:
//   X'[r, j] = alpha Y[r, j] + (r == src[j]) (alpha delta_j + 1 - alpha),
// with delta_j the dangling mass of column j and Y = A X.  The SpMM finishes
// every row strictly inside a tile as X' itself (SpmmArgs::Xn) and adds its
// dangling mass to a per-block, per-column part; ppr_fixup_kernel finishes
// the tiles' first rows from Y (where neighbouring tiles added into them)
// and clears those slots of Y for the next step; on the last step of a
// chunk ppr_resid_kernel adds the l1 change.  A last kernel (one block per
// column) sums the parts in a fixed order for the next step and the host.
// Thread t of these kernels always handles column t % 64, so each
// wavefront reads and writes whole rows (coalesced).
//
// The iterates (and A X) are held as slabs of kSlab columns one after
// another: slab s is the row-major n x W_s block of columns 32 s .. 32 s +
// W_s - 1 (W_s = min(32, k - 32 s)), so every SpMM launch reads and writes a
// compact array (for k <= 32 this is the row-major n x k layout).  Compact
// slabs took the 64-column SpMM of R-MAT 22 from 2.51 to 2.34 ms (FP32)
// against the two halves of a row-major n x 64 array.

// offset of element (r, j) of an n x k iterate in the slab layout
__device__ __forceinline__ int64_t ppr_at(int64_t r, int j, int64_t n, int k) {
  const int c0 = j & ~(kSlab - 1);
  const int w = min(kSlab, k - c0);
  return (int64_t)c0 * n + r * w + (j - c0);
}

constexpr int kPprThreads = 256;
constexpr int kPprWaves = kPprThreads / 64;
constexpr int kPprRows = 4;

// 64 per-thread (a, b) pairs of the block (thread t: column t % 64) summed
// over its wavefronts in order, written as part_out row blockIdx.x
__device__ __forceinline__ void ppr_block_part(double a, double b, double* __restrict__ part_out) {
  __shared__ double s_a[kPprThreads], s_b[kPprThreads];
  s_a[threadIdx.x] = a;
  s_b[threadIdx.x] = b;
  __syncthreads();
  if (threadIdx.x < 64) {
    double x = 0.0, y = 0.0;
    for (int q = 0; q < kPprWaves; ++q) {
      x += s_a[q * 64 + threadIdx.x];
      y += s_b[q * 64 + threadIdx.x];
    }
    part_out[((int64_t)blockIdx.x * 64 + threadIdx.x) * 2] = x;
    part_out[((int64_t)blockIdx.x * 64 + threadIdx.x) * 2 + 1] = y;
  }
}

int ppr_fixup_grid(int64_t tile_num) {
  int64_t g = (tile_num + kPprWaves * 8 - 1) / (kPprWaves * 8);
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

template <typename V>
__global__ __launch_bounds__(kPprThreads) void ppr_fixup_kernel(
    const uint32_t* __restrict__ tile_y, int32_t tile_num, V* __restrict__ Y,
    V* __restrict__ Xn, int64_t n, int k, double alpha, const int32_t* __restrict__ src,
    const double* __restrict__ sums_in, const uint32_t* __restrict__ dmask,
    double* __restrict__ part_out) {
  const int j = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const bool on = j < k;
  const int sj = on ? src[j] : -1;
  const V a = (V)alpha;
  const V tele = on ? (V)(alpha * sums_in[2 * j] + 1.0 - alpha) : V(0);
  double dsum = 0.0;
  const int64_t step = (int64_t)gridDim.x * kPprWaves;
  for (int64_t t = (int64_t)blockIdx.x * kPprWaves + w; t < tile_num; t += step) {
    const int64_t r = tile_y[t] & kRowMask;
    // each first row once (a long row is the first row of several tiles)
    if (r >= n || (t > 0 && (int64_t)(tile_y[t - 1] & kRowMask) == r)) continue;
    if (on) {
      const int64_t e = ppr_at(r, j, n, k);
      V xn = a * Y[e];
      Y[e] = V(0);
      if (r == sj) xn += tele;
      Xn[e] = xn;
      if ((dmask[r >> 5] >> (r & 31)) & 1u) dsum += (double)xn;
    }
  }
  ppr_block_part(dsum, 0.0, part_out);
}

template <typename V>
__global__ __launch_bounds__(kPprThreads) void ppr_resid_kernel(const V* __restrict__ Xn,
                                                                const V* __restrict__ Xo,
                                                                int64_t n, int k,
                                                                double* __restrict__ part_out) {
  const int j = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  double rsum = 0.0;
  const int64_t step = (int64_t)gridDim.x * kPprWaves * kPprRows;
  for (int64_t r0 = ((int64_t)blockIdx.x * kPprWaves + w) * kPprRows; j < k && r0 < n;
       r0 += step) {
    V xn[kPprRows], xo[kPprRows];
#pragma unroll
    for (int u = 0; u < kPprRows; ++u) {
      const int64_t e = ppr_at(min(r0 + u, n - 1), j, n, k);
      xn[u] = Xn[e];
      xo[u] = Xo[e];
    }
#pragma unroll
    for (int u = 0; u < kPprRows; ++u)
      if (r0 + u < n) rsum += fabs((double)xn[u] - (double)xo[u]);
  }
  ppr_block_part(0.0, rsum, part_out);
}

// dangling mass of X (per column) -> the same per-block part layout
template <typename V>
__global__ __launch_bounds__(kPprThreads) void ppr_dangling_kernel(
    const V* __restrict__ X, const uint32_t* __restrict__ dmask, int64_t n, int k,
    double* __restrict__ part_out) {
  const int j = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  double dsum = 0.0;
  const int64_t step = (int64_t)gridDim.x * kPprWaves * kPprRows;
  for (int64_t r0 = ((int64_t)blockIdx.x * kPprWaves + w) * kPprRows; j < k && r0 < n;
       r0 += step) {
#pragma unroll
    for (int u = 0; u < kPprRows; ++u) {
      const int64_t r = r0 + u;
      if (r < n && ((dmask[r >> 5] >> (r & 31)) & 1u)) dsum += (double)X[ppr_at(r, j, n, k)];
    }
  }
  ppr_block_part(dsum, 0.0, part_out);
}

// the slab layout back into the caller's row-major n x k (ld k), one
// wavefront per row
template <typename V>
__global__ __launch_bounds__(kPprThreads) void ppr_from_slabs_kernel(const V* __restrict__ src,
                                                                     V* __restrict__ dst,
                                                                     int64_t n, int k) {
  const int j = threadIdx.x & 63;
  if (j >= k) return;
  const int64_t step = (int64_t)gridDim.x * kPprWaves;
  for (int64_t r = (int64_t)blockIdx.x * kPprWaves + (threadIdx.x >> 6); r < n; r += step)
    dst[r * k + j] = src[ppr_at(r, j, n, k)];
}

hipError_t launch_ppr_from_slabs(int dtype, const void* Xs, void* X, int64_t n, int k,
                                 hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>((n + kPprWaves - 1) / kPprWaves, 8192);
  if (dtype == 0)
    hipLaunchKernelGGL(ppr_from_slabs_kernel<float>, dim3(grid), dim3(kPprThreads), 0, st,
                       static_cast<const float*>(Xs), static_cast<float*>(X), n, k);
  else
    hipLaunchKernelGGL(ppr_from_slabs_kernel<double>, dim3(grid), dim3(kPprThreads), 0, st,
                       static_cast<const double*>(Xs), static_cast<double*>(X), n, k);
  return hipGetLastError();
}

// the caller's row-major X into the slab layout, with X's dangling mass per
// column (the same parts as ppr_dangling_kernel, from the same pass)
template <typename V>
__global__ __launch_bounds__(kPprThreads) void ppr_to_slabs_kernel(
    const V* __restrict__ src, V* __restrict__ dst, const uint32_t* __restrict__ dmask,
    int64_t n, int k, double* __restrict__ part_out) {
  const int j = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  double dsum = 0.0;
  const int64_t step = (int64_t)gridDim.x * kPprWaves * kPprRows;
  for (int64_t r0 = ((int64_t)blockIdx.x * kPprWaves + w) * kPprRows; j < k && r0 < n;
       r0 += step) {
    V v[kPprRows];
#pragma unroll
    for (int u = 0; u < kPprRows; ++u) v[u] = src[min(r0 + u, n - 1) * k + j];
#pragma unroll
    for (int u = 0; u < kPprRows; ++u) {
      const int64_t r = r0 + u;
      if (r < n) {
        dst[ppr_at(r, j, n, k)] = v[u];
        if ((dmask[r >> 5] >> (r & 31)) & 1u) dsum += (double)v[u];
      }
    }
  }
  ppr_block_part(dsum, 0.0, part_out);
}

// sums[2j], sums[2j+1] = totals over the blocks of column j's parts: block j
// of this kernel; thread t adds parts t, t + 256, ... in order, then a
// fixed-order block reduction
__global__ __launch_bounds__(kReduceThreads) void ppr_sum_parts_kernel(
    const double* __restrict__ part, int nblocks, double* __restrict__ sums) {
  const int j = blockIdx.x;
  double d = 0.0, r = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kReduceThreads) {
    d += part[((int64_t)b * 64 + j) * 2];
    r += part[((int64_t)b * 64 + j) * 2 + 1];
  }
  block_sum2(d, r);
  if (threadIdx.x == 0) {
    sums[2 * j] = d;
    sums[2 * j + 1] = r;
  }
}

int ppr_grid(int64_t n) {
  int64_t g = (n + kPprWaves * kPprRows * 8 - 1) / (kPprWaves * kPprRows * 8);
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

// First level for long part lists (the fused SpMM writes one part row per
// block: 54K at R-MAT 22, sigma 5): block g adds rows g, g + G, g + 2G, ...
// with thread t on entry t of a row (rows are read whole, coalesced), in a
// fixed order (eight running sums, then a fixed tree), into row g of out.
constexpr int kPartLevelRows = 1024;  // G; out holds G rows
constexpr int kPartDirectMax = 4096;  // at most this many rows: no first level

__global__ __launch_bounds__(128) void ppr_part_rows_kernel(const double* __restrict__ part,
                                                            int nblocks,
                                                            double* __restrict__ out) {
  const int t = threadIdx.x;
  const int G = gridDim.x;
  double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int b = blockIdx.x;
  for (; b + 7 * G < nblocks; b += 8 * G) {
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] += part[((int64_t)b + (int64_t)u * G) * 128 + t];
  }
  for (; b < nblocks; b += G) s[0] += part[(int64_t)b * 128 + t];
  out[(int64_t)blockIdx.x * 128 + t] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

int ppr_sum_scratch_rows() { return kPartLevelRows; }

hipError_t launch_ppr_sum(const double* part, int nblocks, int k, double* sums, double* scratch,
                          hipStream_t st) {
  if (nblocks > kPartDirectMax && scratch != nullptr) {
    hipLaunchKernelGGL(ppr_part_rows_kernel, dim3(kPartLevelRows), dim3(128), 0, st, part,
                       nblocks, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    part = scratch;
    nblocks = kPartLevelRows;
  }
  hipLaunchKernelGGL(ppr_sum_parts_kernel, dim3(k), dim3(kReduceThreads), 0, st, part, nblocks,
                     sums);
  return hipGetLastError();
}

hipError_t launch_ppr_dangling(int dtype, const void* X, const uint32_t* dmask, int64_t n, int k,
                               double* part, double* sums, int grid, hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL(ppr_dangling_kernel<float>, dim3(grid), dim3(kPprThreads), 0, st,
                       static_cast<const float*>(X), dmask, n, k, part);
  else
    hipLaunchKernelGGL(ppr_dangling_kernel<double>, dim3(grid), dim3(kPprThreads), 0, st,
                       static_cast<const double*>(X), dmask, n, k, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_ppr_sum(part, grid, k, sums, nullptr, st);
}

hipError_t launch_ppr_to_slabs(int dtype, const void* X, void* Xs, const uint32_t* dmask,
                               int64_t n, int k, double* part, double* sums, int grid,
                               hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL(ppr_to_slabs_kernel<float>, dim3(grid), dim3(kPprThreads), 0, st,
                       static_cast<const float*>(X), static_cast<float*>(Xs), dmask, n, k, part);
  else
    hipLaunchKernelGGL(ppr_to_slabs_kernel<double>, dim3(grid), dim3(kPprThreads), 0, st,
                       static_cast<const double*>(X), static_cast<double*>(Xs), dmask, n, k,
                       part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_ppr_sum(part, grid, k, sums, nullptr, st);
}

hipError_t launch_ppr_fixup(int dtype, const uint32_t* tile_y, int32_t tile_num, void* Y,
                            void* Xn, int64_t n, int k, double alpha, const int32_t* src,
                            const double* sums_in, const uint32_t* dmask, double* part, int grid,
                            hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL(ppr_fixup_kernel<float>, dim3(grid), dim3(kPprThreads), 0, st, tile_y,
                       tile_num, static_cast<float*>(Y), static_cast<float*>(Xn), n, k, alpha,
                       src, sums_in, dmask, part);
  else
    hipLaunchKernelGGL(ppr_fixup_kernel<double>, dim3(grid), dim3(kPprThreads), 0, st, tile_y,
                       tile_num, static_cast<double*>(Y), static_cast<double*>(Xn), n, k, alpha,
                       src, sums_in, dmask, part);
  return hipGetLastError();
}

hipError_t launch_ppr_resid(int dtype, const void* Xn, const void* Xo, int64_t n, int k,
                            double* part, int grid, hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL(ppr_resid_kernel<float>, dim3(grid), dim3(kPprThreads), 0, st,
                       static_cast<const float*>(Xn), static_cast<const float*>(Xo), n, k, part);
  else
    hipLaunchKernelGGL(ppr_resid_kernel<double>, dim3(grid), dim3(kPprThreads), 0, st,
                       static_cast<const double*>(Xn), static_cast<const double*>(Xo), n, k,
                       part);
  return hipGetLastError();
}

// ------------------------------------------------ PageRank of many graphs --
//
// The graphs lie on the diagonal of one matrix: graph g owns rows and columns
// [gp[g], gp[g+1]), and its step is the PageRank step of Sec. 5.5.1 with its
// own size, dangling mass and teleport:
//   x'[r] = alpha y[r] + (alpha delta_g + 1 - alpha) / n_g   for r in graph g.
// Rows are cut into chunks of at most kMultiRows rows that never cross a
// graph; chunk c is rows [chunk_row[c], chunk_row[c+1]) of graph
// chunk_graph[c], and graph g's chunks are chunk_ptr[g] .. chunk_ptr[g+1]-1.
// One block per chunk writes the chunk's (dangling mass, l1 change) pair; a
// second kernel adds each graph's pairs in chunk order (deterministic).

constexpr int kMultiILP = 4;
constexpr int kMultiRows = kReduceThreads * kMultiILP;

int multi_chunk_rows() { return kMultiRows; }

// With hot_n > 0 the kernel also writes the hot-column copy of x' that the
// next SpMV's LDS cache reads: slot s holds column hot_cols[s] of graph
// hot_graph[s], computed with the same operations as that row's x'.
// Without RESID x_old is not read and the l1 parts are 0 (the host reads
// the l1 change only after a chunk's last step).
template <typename V, bool RESID>
__global__ __launch_bounds__(kReduceThreads) void multi_update_kernel(
    const V* __restrict__ y, const V* __restrict__ x_old, V* __restrict__ x_new,
    const uint32_t* __restrict__ dmask, const int32_t* __restrict__ chunk_row,
    const int32_t* __restrict__ chunk_graph, const double* __restrict__ gsum_in,
    const double* __restrict__ gsize, double alpha, double* __restrict__ part_out,
    const int32_t* __restrict__ hot_cols, const int32_t* __restrict__ hot_graph, int32_t hot_n,
    V* __restrict__ x_hot) {
  const int c = blockIdx.x;
  const int64_t r0 = chunk_row[c], r1 = chunk_row[c + 1];
  const int g = chunk_graph[c];
  const V tele = (V)((alpha * gsum_in[2 * g] + 1.0 - alpha) / gsize[g]);
  const V a = (V)alpha;
  V yv[kMultiILP], xo[kMultiILP];
  uint32_t mw[kMultiILP];
#pragma unroll
  for (int u = 0; u < kMultiILP; ++u) {
    const int64_t i = min(r0 + threadIdx.x + (int64_t)u * kReduceThreads, r1 - 1);
    yv[u] = y[i];
    if constexpr (RESID) xo[u] = x_old[i];
    mw[u] = dmask[i >> 5];
  }
  double dsum = 0.0, rsum = 0.0;
#pragma unroll
  for (int u = 0; u < kMultiILP; ++u) {
    const int64_t i = r0 + threadIdx.x + (int64_t)u * kReduceThreads;
    if (i < r1) {
      const V xn = fma(a, yv[u], tele);
      x_new[i] = xn;
      if constexpr (RESID) rsum += fabs((double)xn - (double)xo[u]);
      if ((mw[u] >> (i & 31)) & 1u) dsum += (double)xn;
    }
  }
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < hot_n;
       h += (int64_t)gridDim.x * blockDim.x) {
    const int gh = hot_graph[h];
    const V th = (V)((alpha * gsum_in[2 * gh] + 1.0 - alpha) / gsize[gh]);
    x_hot[h] = fma(a, y[hot_cols[h]], th);
  }
  block_sum2(dsum, rsum);
  if (threadIdx.x == 0) {
    part_out[2 * c] = dsum;
    part_out[2 * c + 1] = rsum;
  }
}

template <typename V>
__global__ __launch_bounds__(kReduceThreads) void multi_dangling_kernel(
    const V* __restrict__ x, const uint32_t* __restrict__ dmask,
    const int32_t* __restrict__ chunk_row, double* __restrict__ part_out) {
  const int c = blockIdx.x;
  const int64_t r0 = chunk_row[c], r1 = chunk_row[c + 1];
  double dsum = 0.0, zero = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += kReduceThreads)
    if ((dmask[i >> 5] >> (i & 31)) & 1u) dsum += (double)x[i];
  block_sum2(dsum, zero);
  if (threadIdx.x == 0) {
    part_out[2 * c] = dsum;
    part_out[2 * c + 1] = 0.0;
  }
}

// One wavefront per graph: lane l adds chunks chunk_ptr[g] + l, + l + 64, ...
// in order, then a fixed-order wavefront reduction.
__global__ __launch_bounds__(256) void multi_sum_kernel(const double* __restrict__ part,
                                                         const int32_t* __restrict__ chunk_ptr,
                                                         int n_graphs,
                                                         double* __restrict__ gsum_out) {
  const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lid = threadIdx.x & 63;
  if (g >= n_graphs) return;
  double d = 0.0, r = 0.0;
  for (int c = chunk_ptr[g] + lid; c < chunk_ptr[g + 1]; c += 64) {
    d += part[2 * c];
    r += part[2 * c + 1];
  }
  d = wave_sum(d);
  r = wave_sum(r);
  if (lid == 0) {
    gsum_out[2 * g] = d;
    gsum_out[2 * g + 1] = r;
  }
}

static hipError_t launch_multi_sum(const double* part, const int32_t* chunk_ptr, int n_graphs,
                                   double* gsum_out, hipStream_t st) {
  hipLaunchKernelGGL(multi_sum_kernel, dim3((unsigned)((n_graphs + 3) / 4)), dim3(256), 0, st,
                     part, chunk_ptr, n_graphs, gsum_out);
  return hipGetLastError();
}

hipError_t launch_multi_dangling(int dtype, const void* x, const uint32_t* dmask,
                                 const MultiTables& mt, double* gsum_out, hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL(multi_dangling_kernel<float>, dim3((unsigned)mt.n_chunks),
                       dim3(kReduceThreads), 0, st, static_cast<const float*>(x), dmask,
                       mt.chunk_row, mt.part);
  else
    hipLaunchKernelGGL(multi_dangling_kernel<double>, dim3((unsigned)mt.n_chunks),
                       dim3(kReduceThreads), 0, st, static_cast<const double*>(x), dmask,
                       mt.chunk_row, mt.part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_multi_sum(mt.part, mt.chunk_ptr, mt.n_graphs, gsum_out, st);
}

template <typename V>
static void multi_update_launch(bool resid, const void* y, const void* x_old, void* x_new,
                                const uint32_t* dmask, const MultiTables& mt, double alpha,
                                const double* gsum_in, hipStream_t st, const int32_t* hot_cols,
                                int32_t hot_n, void* x_hot) {
  const V* yv = static_cast<const V*>(y);
  const V* xo = static_cast<const V*>(x_old);
  V* xn = static_cast<V*>(x_new);
  V* xh = static_cast<V*>(x_hot);
  if (resid)
    hipLaunchKernelGGL((multi_update_kernel<V, true>), dim3((unsigned)mt.n_chunks),
                       dim3(kReduceThreads), 0, st, yv, xo, xn, dmask, mt.chunk_row,
                       mt.chunk_graph, gsum_in, mt.gsize, alpha, mt.part, hot_cols,
                       mt.hot_graph, hot_n, xh);
  else
    hipLaunchKernelGGL((multi_update_kernel<V, false>), dim3((unsigned)mt.n_chunks),
                       dim3(kReduceThreads), 0, st, yv, xo, xn, dmask, mt.chunk_row,
                       mt.chunk_graph, gsum_in, mt.gsize, alpha, mt.part, hot_cols,
                       mt.hot_graph, hot_n, xh);
}

hipError_t launch_multi_update(int dtype, const void* y, const void* x_old, void* x_new,
                               const uint32_t* dmask, const MultiTables& mt, double alpha,
                               const double* gsum_in, double* gsum_out, hipStream_t st,
                               const int32_t* hot_cols, int32_t hot_n, void* x_hot, bool resid) {
  if (hot_n > 0 && mt.hot_graph == nullptr) return hipErrorInvalidValue;
  if (dtype == 0)
    multi_update_launch<float>(resid, y, x_old, x_new, dmask, mt, alpha, gsum_in, st, hot_cols,
                               hot_n, x_hot);
  else
    multi_update_launch<double>(resid, y, x_old, x_new, dmask, mt, alpha, gsum_in, st, hot_cols,
                                hot_n, x_hot);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_multi_sum(mt.part, mt.chunk_ptr, mt.n_graphs, gsum_out, st);
}

}  // namespace merbit
