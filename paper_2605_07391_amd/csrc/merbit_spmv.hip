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
//
// Hot variant (HOT = true): the column stream is the plan's recoded copy in
// which the most frequent columns are negative LDS slot numbers.  Each block
// first copies the hot x values into LDS and then works through
// chunks_per_block consecutive chunks of WAVES tiles (one commit unit each),
// so the LDS copy is paid once per block; a hot nonzero reads x from LDS.
#include "merbit_internal.hpp"

namespace merbit {

template <typename V, int SIGMA, int WAVES>
constexpr int lds_values() {
  return WAVES * kOmega * SIGMA + 1;
}

// One commit unit: WAVES consecutive tiles starting at tile `chunk * WAVES`.
template <typename V, int SIGMA, int WAVES, bool HOT>
__device__ __forceinline__ void spmv_chunk(const SpmvArgs& a, int chunk, V* s_data, V* s_head,
                                           V* s_tail, const V* s_hot) {
  constexpr int BITS = ceil_log2(kOmega * SIGMA);
  constexpr uint32_t FMASK = (1u << BITS) - 1u;
  constexpr int NT = WAVES * kOmega;

  const int32_t* __restrict__ tile_x = a.tile_x;
  const uint32_t* __restrict__ tile_y = a.tile_y;
  const int32_t* __restrict__ col = a.col;
  const V* __restrict__ val = static_cast<const V*>(a.val);
  const V* __restrict__ x = static_cast<const V*>(a.x);
  V* __restrict__ y = static_cast<V*>(a.y);

  const int tid = threadIdx.x;
  const int lid = tid & (kOmega - 1);
  const int wid = __builtin_amdgcn_readfirstlane(tid / kOmega);
  const int bs = chunk * WAVES;
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
    for (int it = 0; it < SIGMA; ++it) {
      const int c = cc[it];
      if (HOT) {
        V xv;
        if (c >= 0) xv = x[c];
        else xv = s_hot[-1 - c];
        prod[it] = vv[it] * xv;
      } else {
        prod[it] = vv[it] * x[c];
      }
    }
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

template <typename V, int SIGMA, int WAVES, bool HOT>
__global__ __launch_bounds__(WAVES * 64) void spmv_kernel(SpmvArgs a) {
  __shared__ V s_data[lds_values<V, SIGMA, WAVES>()];
  __shared__ V s_head[WAVES];
  __shared__ V s_tail[WAVES];
  if (!HOT) {
    spmv_chunk<V, SIGMA, WAVES, false>(a, blockIdx.x, s_data, s_head, s_tail, nullptr);
    return;
  }
  extern __shared__ __align__(16) unsigned char s_dyn[];
  V* s_hot = reinterpret_cast<V*>(s_dyn);
  const V* __restrict__ xh = static_cast<const V*>(a.x_hot);
  for (int s = threadIdx.x; s < a.hot_n; s += WAVES * kOmega) s_hot[s] = xh[s];
  const int c0 = blockIdx.x * a.chunks_per_block;
  const int c1 = min(c0 + a.chunks_per_block, a.chunk_num);
  for (int chunk = c0; chunk < c1; ++chunk) {
    __syncthreads();  // hot values loaded / the previous chunk is done with LDS
    spmv_chunk<V, SIGMA, WAVES, true>(a, chunk, s_data, s_head, s_tail, s_hot);
  }
}

template <typename V, int S, int W, bool H>
static hipError_t launch_t(const SpmvArgs& a, size_t dyn, hipStream_t st) {
  hipLaunchKernelGGL((spmv_kernel<V, S, W, H>), dim3((unsigned)a.grid), dim3(W * kOmega), dyn, st,
                     a);
  return hipGetLastError();
}

template <typename V, int S, int W, bool H>
static hipError_t set_lds_t(size_t bytes) {
  static std::mutex mu;
  static size_t granted[kMaxLdsDevices] = {};
  return raise_dynamic_lds(reinterpret_cast<const void*>(&spmv_kernel<V, S, W, H>), bytes, mu,
                           granted);
}

struct KernelEntry {
  hipError_t (*launch)(const SpmvArgs&, size_t, hipStream_t);
  hipError_t (*set_lds)(size_t);
};

template <typename V, int W, bool H>
static KernelEntry pick_sigma(int sigma) {
  switch (sigma) {
#define MERBIT_CASE(S) \
  case S: return KernelEntry{launch_t<V, S, W, H>, set_lds_t<V, S, W, H>};
    MERBIT_CASE(1) MERBIT_CASE(2) MERBIT_CASE(3) MERBIT_CASE(4) MERBIT_CASE(5) MERBIT_CASE(6)
    MERBIT_CASE(7) MERBIT_CASE(8) MERBIT_CASE(9) MERBIT_CASE(10) MERBIT_CASE(11) MERBIT_CASE(12)
#undef MERBIT_CASE
    default: return KernelEntry{nullptr, nullptr};
  }
}

template <typename V, bool H>
static KernelEntry pick_waves(int sigma, int waves) {
  switch (waves) {
    case 2: return H ? KernelEntry{nullptr, nullptr} : pick_sigma<V, 2, H>(sigma);
    case 4: return pick_sigma<V, 4, H>(sigma);
    case 8: return pick_sigma<V, 8, H>(sigma);
    case 16: return pick_sigma<V, 16, H>(sigma);
    default: return KernelEntry{nullptr, nullptr};
  }
}

static KernelEntry pick_any(int dtype, int sigma, int waves, bool hot) {
  if (dtype == 0) return hot ? pick_waves<float, true>(sigma, waves)
                             : pick_waves<float, false>(sigma, waves);
  if (dtype == 1) return hot ? pick_waves<double, true>(sigma, waves)
                             : pick_waves<double, false>(sigma, waves);
  return KernelEntry{nullptr, nullptr};
}

bool spmv_supported(int dtype, int sigma, int waves, bool hot) {
  return pick_any(dtype, sigma, waves, hot).launch != nullptr;
}

hipError_t launch_spmv(int dtype, int sigma, int waves, bool hot, size_t hot_lds_bytes,
                       const SpmvArgs& a, hipStream_t st) {
  KernelEntry k = pick_any(dtype, sigma, waves, hot);
  if (!k.launch) return hipErrorInvalidValue;
  return k.launch(a, hot ? hot_lds_bytes : 0, st);
}

hipError_t spmv_set_hot_lds(int dtype, int sigma, int waves, size_t bytes) {
  KernelEntry k = pick_any(dtype, sigma, waves, true);
  if (!k.set_lds) return hipErrorInvalidValue;
  return k.set_lds(bytes);
}

// Zero v at the first row of every commit unit (the rows the fused kernels
// add onto).
template <typename V>
__global__ void zero_boundary_kernel(const uint32_t* __restrict__ tile_y, int32_t units,
                                     int32_t unit, V* __restrict__ v) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < units) v[tile_y[(int64_t)k * unit] & kRowMask] = V(0);
}

hipError_t launch_zero_boundary(int dtype, const uint32_t* tile_y, int32_t units, int32_t unit,
                                void* v, hipStream_t st) {
  const unsigned grid = (unsigned)((units + 255) / 256);
  if (grid == 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(zero_boundary_kernel<float>, dim3(grid), dim3(256), 0, st, tile_y, units,
                       unit, static_cast<float*>(v));
  else
    hipLaunchKernelGGL(zero_boundary_kernel<double>, dim3(grid), dim3(256), 0, st, tile_y, units,
                       unit, static_cast<double*>(v));
  return hipGetLastError();
}

}  // namespace merbit
