// Fused MERBIT SpMV for gfx950 (Sec. 4.2 of the MERBIT paper).
//
// Work decomposition: lane = sigma merge-path steps, tile = one 64-lane
// wavefront = 64 sigma steps, block = WAVES tiles.  Per block:
//   1. zero the block's partial-sum slots in LDS (rows y_bs .. y_be);
//   2. per wavefront, by its tile's start/end on the path:
//      - no nonzero in the tile (x_ws == x_we): nothing to do, its rows stay 0;
//      - single-row tile (tile_y bit 31): coalesced loads, products summed in
//        registers, a wavefront reduction, one LDS add into the row's slot;
//      - otherwise stage the tile's products in LDS with coalesced loads of
//        values / col_ind and gathers of x, then every lane decodes its 32-bit
//        descriptor and walks its sigma steps (right: add the next product,
//        down: finish a row into its slot), and a head-flagged segmented scan
//        across the 64 lanes carries each lane's trailing partial sum to the
//        row it belongs to;
//   3. block barrier, then a coalesced commit: rows strictly inside the
//      block's range are stored; the first and last rows, which neighbouring
//      blocks may share, are added atomically onto zero.  With a dual buffer z
//      the block also zeroes z at its first row, so z is ready to be the next
//      output (Sec. 4.2, optimisation (3)).
// LDS: m_b products followed by the block's row slots, at most
// WAVES * 64 * sigma + 1 values (Sec. 4.2: segment of b sigma steps).
#include "merbit_internal.hpp"

namespace merbit {

template <typename V>
__device__ __forceinline__ void global_add(V* p, V v) {
  unsafeAtomicAdd(p, v);
}

template <typename V, int SIGMA, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void spmv_kernel(SpmvArgs a) {
  constexpr int BITS = ceil_log2(kOmega * SIGMA);
  constexpr uint32_t FMASK = (1u << BITS) - 1u;
  constexpr int NT = WAVES * kOmega;
  constexpr int LDS_N = NT * SIGMA + 1;
  __shared__ V s_data[LDS_N];

  const int32_t* __restrict__ tile_x = a.tile_x;
  const uint32_t* __restrict__ tile_y = a.tile_y;
  const int32_t* __restrict__ col = a.col;
  const V* __restrict__ val = static_cast<const V*>(a.val);
  const V* __restrict__ x = static_cast<const V*>(a.x);
  V* __restrict__ y = static_cast<V*>(a.y);

  const int tid = threadIdx.x;
  const int lid = tid & (kOmega - 1);
  const int wid = tid / kOmega;
  const int bs = blockIdx.x * WAVES;
  const int be = min(bs + WAVES, a.tile_num);

  // block and tile bounds, all read before any wait (Algorithm "MERBIT SpMV",
  // prologue); a wavefront past the last tile works on a clamped copy and
  // does nothing with it
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
  const int end_slot = (int)(tile_y[i + 1] & kRowMask) - y_bs;
  const int x_se = x_we - x_ws;
  const bool active = own_tile && x_se > 0;
  const bool fast = (tyw & kFastBit) != 0u;
  const int y_bw = (int)(tyw & kRowMask) - y_bs;
  const int x_bw = x_ws - x_bs;
  V* s_y = s_data + (x_be - x_bs);

  // descriptor of this lane (normal tiles only), issued early
  const int j = i * kOmega + lid;
  uint32_t desc = 0;
  if (active && !fast) desc = a.lane_desc[min(j, a.lane_num - 1)];

  // the tile's nonzeros: coalesced streaming loads, then the x gathers; all
  // loads are unconditional (indices clamped into the tile) so every one of
  // them is in flight before the first use
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

  for (int r = tid; r <= y_se; r += NT) s_y[r] = V(0);
  __syncthreads();

  if (active) {
    if (fast) {
      // single-row tile (Sec. 4.2 opt. (1)): no descriptor, no staging
      V acc = V(0);
#pragma unroll
      for (int it = 0; it < SIGMA; ++it)
        if (lid + it * kOmega < x_se) acc += prod[it];
      acc = wave_sum(acc);
      if (lid == 0) atomicAdd(&s_y[y_bw], acc);
    } else {
      // stage the products (coalesced by lane)
#pragma unroll
      for (int it = 0; it < SIGMA; ++it) {
        const int k = lid + it * kOmega;
        if (k < x_se) s_data[x_bw + k] = prod[it];
      }
      wave_lds_sync();
      // per-lane walk of its sigma steps (Algorithm tile_normal_tackle)
      V sum = V(0);
      bool head = (lid == 0);
      int start_slot = 0;
      if (j < a.lane_num) {
        int xo = x_bw + (int)(desc & FMASK);
        int yo = y_bw + (int)((desc >> BITS) & FMASK);
        start_slot = yo;
        const uint32_t flags = desc >> (2 * BITS);
        const int steps = min(SIGMA, a.path_len - j * SIGMA);
        bool first = true;
#pragma unroll
        for (int k = 0; k < SIGMA; ++k) {
          if (k < steps) {
            if ((flags >> k) & 1u) {
              if (first) {
                atomicAdd(&s_y[yo], sum);  // row may also get other lanes' sums
                first = false;
              } else {
                s_y[yo] = sum;  // row lies wholly inside this lane
              }
              sum = V(0);
              ++yo;
            } else {
              sum += s_data[xo];
              ++xo;
            }
          }
        }
        head = head || !first;
      }
      // segmented inclusive scan of trailing sums; heads start segments
      const unsigned long long heads = __ballot(head);
      V v = sum;
#pragma unroll
      for (int dist = 1; dist < kOmega; dist <<= 1) {
        const V t = __shfl_up(v, dist, kOmega);
        bool take = lid >= dist;
        if (take) {
          const unsigned long long window = ((1ull << dist) - 1ull) << (lid - dist + 1);
          take = (heads & window) == 0ull;
        }
        if (take) v += t;
      }
      const V carry = __shfl_up(v, 1, kOmega);
      const V tail = __shfl(v, kOmega - 1, kOmega);
      if (lid == 0) {
        // the last segment ends the tile: it belongs to the tile's end row
        atomicAdd(&s_y[end_slot], tail);
      } else if (head) {
        atomicAdd(&s_y[start_slot], carry);
      }
    }
  }
  __syncthreads();

  // commit: interior rows are owned by this block alone
  for (int r = 1 + tid; r < y_se; r += NT) y[y_bs + r] = s_y[r];
  if (tid == 0) {
    global_add(&y[y_bs], s_y[0]);
    if (y_se > 0 && y_be < a.n_rows) global_add(&y[y_be], s_y[y_se]);
    if (a.z) static_cast<V*>(a.z)[y_bs] = V(0);
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
