// Fused MERBIT SpMV for gfx950 (Sec. 4.2 of the MERBIT paper).
//
// Work decomposition: lane = sigma merge-path steps, tile = one 64-lane
// wavefront = 64 sigma steps, block = WAVES consecutive tiles.
//
// Per wavefront, by its tile's start/end on the path (Algorithm "MERBIT SpMV"):
//   - no nonzero in the tile (x_ws == x_we): its inner rows are empty and are
//     written as 0;
//   - single-row tile (tile_y bit 31, Sec. 4.2 opt. (1)): products summed in
//     registers and reduced across the wavefront: one partial for that row;
//   - otherwise the tile's products are staged in LDS (coalesced loads of
//     values / col_ind, then the x gathers), every lane decodes its 32-bit
//     descriptor and walks its sigma steps (right: add the next product, down:
//     finish a row; Algorithm tile_normal_tackle), and a head-flagged
//     segmented scan across the 64 lanes (Algorithm WarpSegmentedSum) carries
//     each lane's trailing sum to the row it belongs to.
// Each wavefront writes every row that starts and ends inside its tile exactly
// once, with a plain LDS store (no atomics, nothing to clear first), and hands
// over two partial sums: for the row the tile starts in and for the row it
// ends in.  After one block barrier, thread 0 chains the WAVES pairs in tile
// order; rows that start and end inside the block are stored, the block's
// first and last rows (shared with the neighbouring blocks) are added
// atomically to y, which is zero there before the launch.  All other rows are
// committed from LDS with coalesced stores.  With a dual buffer z the block
// also zeroes z at its first row, so z is ready to be the next output
// (Sec. 4.2, opt. (3)).
// LDS: m_b products followed by the block's row slots, at most
// WAVES * 64 * sigma + 1 values (Sec. 4.2: a block segment has b sigma steps).
#include "merbit_internal.hpp"

namespace merbit {

template <typename V>
__device__ __forceinline__ void global_add(V* p, V v) {
  unsafeAtomicAdd(p, v);
}

// DPP move of a 32-bit value (lanes without a source lane receive 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xF, false);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(float, dpp_i<CTRL, ROW_MASK>(__builtin_bit_cast(int, v)));
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = dpp_i<CTRL, ROW_MASK>((int)(b & 0xFFFFFFFFll));
  const int hi = dpp_i<CTRL, ROW_MASK>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// DPP controls (GFX9): row shift right by n within rows of 16 lanes,
// broadcast of lane 15 / 31 of a row into the next row(s), whole-wave shift.
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143, kWaveShr1 = 0x138;

// Inclusive segmented scan across the wavefront.  seg = index of the last
// segment head at or before this lane (lane 0 is always a head).  Each step
// adds the value from `dist` lanes below only if no head lies in between.
template <typename V>
__device__ __forceinline__ V wave_segmented_scan(V v, int lid, int seg) {
  V t;
  t = dpp_move<kRowShr1, 0xF>(v);
  if (seg <= lid - 1) v += t;
  t = dpp_move<kRowShr2, 0xF>(v);
  if (seg <= lid - 2) v += t;
  t = dpp_move<kRowShr4, 0xF>(v);
  if (seg <= lid - 4) v += t;
  t = dpp_move<kRowShr8, 0xF>(v);
  if (seg <= lid - 8) v += t;
  // rows 1 and 3 take the end of rows 0 and 2
  t = dpp_move<kRowBcast15, 0xA>(v);
  if ((lid & 16) && seg < (lid & ~15)) v += t;
  // rows 2 and 3 take lane 31
  t = dpp_move<kRowBcast31, 0xC>(v);
  if (lid >= 32 && seg < 32) v += t;
  return v;
}

template <typename V>
__device__ __forceinline__ V wave_total(V v) {
  // the segmented scan with a single head at lane 0 is a plain inclusive scan
  v = wave_segmented_scan(v, (int)__lane_id(), 0);
  return __shfl(v, kOmega - 1, kOmega);
}

template <typename V, int SIGMA, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void spmv_kernel(SpmvArgs a) {
  constexpr int BITS = ceil_log2(kOmega * SIGMA);
  constexpr uint32_t FMASK = (1u << BITS) - 1u;
  constexpr int NT = WAVES * kOmega;
  constexpr int LDS_N = NT * SIGMA + 1;
  __shared__ V s_data[LDS_N];
  __shared__ V s_head[WAVES];
  __shared__ V s_tail[WAVES];

  const int32_t* __restrict__ tile_x = a.tile_x;
  const uint32_t* __restrict__ tile_y = a.tile_y;
  const int32_t* __restrict__ col = a.col;
  const V* __restrict__ val = static_cast<const V*>(a.val);
  const V* __restrict__ x = static_cast<const V*>(a.x);
  V* __restrict__ y = static_cast<V*>(a.y);

  const int tid = threadIdx.x;
  const int lid = tid & (kOmega - 1);
  const int wid = __builtin_amdgcn_readfirstlane(tid / kOmega);
  const int bs = blockIdx.x * WAVES;
  const int be = min(bs + WAVES, a.tile_num);

  // block and tile bounds (prologue of Algorithm "MERBIT SpMV"); a wavefront
  // past the last tile works on a clamped copy and does nothing with it
  const int x_bs = tile_x[bs];
  const int x_be = tile_x[be];
  const int y_bs = (int)(tile_y[bs] & kRowMask);
  const int y_be = (int)(tile_y[be] & kRowMask);
  const int y_se = y_be - y_bs;
  const int i = min(bs + wid, be - 1);
  const bool own_tile = bs + wid < be;
  const int x_ws = tile_x[i];
  const int x_we = tile_x[i + 1];
  const uint32_t tyw = tile_y[i];
  const int y_bw = (int)(tyw & kRowMask) - y_bs;           // tile start row, block-relative
  const int end_slot = (int)(tile_y[i + 1] & kRowMask) - y_bs;  // tile end row
  const int x_se = x_we - x_ws;
  const bool active = own_tile && x_se > 0;
  const bool fast = (tyw & kFastBit) != 0u;
  const int x_bw = x_ws - x_bs;
  V* s_y = s_data + (x_be - x_bs);

  // descriptor of this lane (normal tiles only), issued early
  const int j = i * kOmega + lid;
  uint32_t desc = 0;
  if (active && !fast) desc = a.lane_desc[min(j, a.lane_num - 1)];

  // the tile's nonzeros: coalesced streaming loads, then the x gathers; all
  // loads are unconditional (indices clamped into the tile) so that every one
  // of them is in flight before the first use
  V prod[SIGMA];
  if (active) {
    const int32_t* __restrict__ tc = col + x_ws;
    const V* __restrict__ tv = val + x_ws;
    int cc[SIGMA];
    V vv[SIGMA];
#pragma unroll
    for (int it = 0; it < SIGMA; ++it) {
      const int k = min(lid + it * kOmega, x_se - 1);
      cc[it] = __builtin_nontemporal_load(tc + k);
      vv[it] = __builtin_nontemporal_load(tv + k);
    }
#pragma unroll
    for (int it = 0; it < SIGMA; ++it) prod[it] = vv[it] * x[cc[it]];
  }

  V head_part = V(0), tail_part = V(0);
  if (active) {
    if (fast) {
      V acc = V(0);
#pragma unroll
      for (int it = 0; it < SIGMA; ++it)
        if (lid + it * kOmega < x_se) acc += prod[it];
      head_part = wave_total(acc);
    } else {
      // stage the products (coalesced by lane)
#pragma unroll
      for (int it = 0; it < SIGMA; ++it) {
        const int k = lid + it * kOmega;
        if (k < x_se) s_data[x_bw + k] = prod[it];
      }
      wave_lds_sync();
      // walk this lane's steps: the sum before the first down step belongs to
      // the lane's start row; rows begun and finished inside the lane are
      // stored; the trailing sum goes into the scan
      V sum = V(0), first_sum = V(0);
      bool has_down = false;
      int start_slot = y_bw;
      if (j < a.lane_num) {
        int xo = x_bw + (int)(desc & FMASK);
        int yo = y_bw + (int)((desc >> BITS) & FMASK);
        start_slot = yo;
        const uint32_t flags = desc >> (2 * BITS);
        const int steps = min(SIGMA, a.path_len - j * SIGMA);
#pragma unroll
        for (int k = 0; k < SIGMA; ++k) {
          if (k < steps) {
            if ((flags >> k) & 1u) {
              if (has_down) s_y[yo] = sum;
              else first_sum = sum;
              has_down = true;
              sum = V(0);
              ++yo;
            } else {
              sum += s_data[xo];
              ++xo;
            }
          }
        }
      }
      const unsigned long long heads = __ballot(has_down) | 1ull;
      const unsigned long long upto =
          lid == kOmega - 1 ? ~0ull : ((2ull << lid) - 1ull);
      const int seg = 63 - __builtin_clzll(heads & upto);
      const V scan = wave_segmented_scan(sum, lid, seg);
      const V carry = dpp_move<kWaveShr1, 0xF>(scan);  // scan of lane - 1
      tail_part = __shfl(scan, kOmega - 1, kOmega);
      if (has_down) {
        const V row_val = first_sum + (lid > 0 ? carry : V(0));
        if (start_slot == y_bw) head_part = row_val;  // the tile's first row: a partial
        else s_y[start_slot] = row_val;               // begun inside the tile: complete
      }
      // exactly one lane (the first with a down step) holds the head partial
      head_part = wave_total(head_part);
    }
  } else if (own_tile) {
    // a tile of down steps only: the rows strictly inside it are empty
    for (int r = y_bw + 1 + lid; r < end_slot; r += kOmega) s_y[r] = V(0);
  }
  if (lid == 0) {
    s_head[wid] = head_part;
    s_tail[wid] = tail_part;
  }
  __syncthreads();

  // rows shared between tiles: chain the tiles' partial sums in path order
  if (tid == 0) {
    const int nt = be - bs;
    V running = V(0);
    int row = y_bs;
    for (int w = 0; w < nt; ++w) {
      running += s_head[w];
      const int next_row = (int)(tile_y[bs + w + 1] & kRowMask);
      if (next_row != row) {
        if (row == y_bs) global_add(&y[row], running);  // may continue in the previous block
        else y[row] = running;
        running = s_tail[w];
        row = next_row;
      }
    }
    // the block's last row continues in the next block (when the block lies
    // in a single row this is its first row as well)
    if (y_be < a.n_rows) global_add(&y[y_be], running);
    if (a.z) static_cast<V*>(a.z)[y_bs] = V(0);
  }
  // every other row of the block is complete in LDS: coalesced commit
  for (int r = 1 + tid; r < y_se; r += NT) {
    bool tile_start = false;
#pragma unroll
    for (int w = 1; w < WAVES; ++w)
      tile_start |= (bs + w < be) && (r == (int)(tile_y[bs + w] & kRowMask) - y_bs);
    if (!tile_start) y[y_bs + r] = s_y[r];
  }
}

template <typename V, int S, int W>
static hipError_t launch_t(const SpmvArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((spmv_kernel<V, S, W>), dim3((unsigned)a.block_num), dim3(W * kOmega), 0,
                     st, a);
  return hipGetLastError();
}

typedef hipError_t (*launch_fn)(const SpmvArgs&, hipStream_t);

template <typename V, int W>
static launch_fn pick_sigma(int sigma) {
  switch (sigma) {
    case 1: return launch_t<V, 1, W>;
    case 2: return launch_t<V, 2, W>;
    case 3: return launch_t<V, 3, W>;
    case 4: return launch_t<V, 4, W>;
    case 5: return launch_t<V, 5, W>;
    case 6: return launch_t<V, 6, W>;
    case 7: return launch_t<V, 7, W>;
    case 8: return launch_t<V, 8, W>;
    case 9: return launch_t<V, 9, W>;
    case 10: return launch_t<V, 10, W>;
    case 11: return launch_t<V, 11, W>;
    case 12: return launch_t<V, 12, W>;
    default: return nullptr;
  }
}

template <typename V>
static launch_fn pick(int sigma, int waves) {
  switch (waves) {
    case 2: return pick_sigma<V, 2>(sigma);
    case 4: return pick_sigma<V, 4>(sigma);
    case 8: return pick_sigma<V, 8>(sigma);
    default: return nullptr;
  }
}

static launch_fn pick_any(int dtype, int sigma, int waves) {
  return dtype == 0 ? pick<float>(sigma, waves) : dtype == 1 ? pick<double>(sigma, waves)
                                                             : nullptr;
}

bool spmv_supported(int dtype, int sigma, int waves) {
  return pick_any(dtype, sigma, waves) != nullptr;
}

hipError_t launch_spmv(int dtype, int sigma, int waves, const SpmvArgs& a, hipStream_t st) {
  launch_fn f = pick_any(dtype, sigma, waves);
  if (!f) return hipErrorInvalidValue;
  return f(a, st);
}

// Zero v at every block's first row (the rows the fused kernel adds onto).
template <typename V>
__global__ void zero_boundary_kernel(const uint32_t* __restrict__ tile_y, int32_t block_num,
                                     int32_t waves, V* __restrict__ v) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < block_num) v[tile_y[(int64_t)k * waves] & kRowMask] = V(0);
}

hipError_t launch_zero_boundary(int dtype, const uint32_t* tile_y, int32_t block_num,
                                int32_t waves, void* v, hipStream_t st) {
  const unsigned grid = (unsigned)((block_num + 255) / 256);
  if (grid == 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(zero_boundary_kernel<float>, dim3(grid), dim3(256), 0, st, tile_y,
                       block_num, waves, static_cast<float*>(v));
  else
    hipLaunchKernelGGL(zero_boundary_kernel<double>, dim3(grid), dim3(256), 0, st, tile_y,
                       block_num, waves, static_cast<double*>(v));
  return hipGetLastError();
}

}  // namespace merbit
