// MERBIT SpMV with one commit unit per tile (b = 64 lanes = one wavefront),
// persistent and software pipelined, for gfx950.
//
// Same method as the block kernel (Sec. 4.2 of the MERBIT paper): tiles of 64
// lanes x sigma merge-path steps, coalesced loads of values / col_ind, products
// staged in LDS, each lane walking its descriptor, a head-flagged segmented
// scan across the wavefront, long-row fast tiles and empty-tile skips.  The
// paper's block size b is set to one wavefront, so wavefronts never wait for
// each other:
//   - rows that start and end inside a tile are complete after the tile's own
//     scan and are stored with coalesced writes from the wavefront's LDS slots;
//   - the tile's first row and last row may continue in neighbouring tiles and
//     are added atomically to y, which is zero at every tile's first row before
//     the launch (dual buffer: each tile zeroes z at its first row, Sec. 4.2
//     opt. (3)).
// A block of WAVES wavefronts is resident for the whole launch; wavefront g
// of the grid takes tiles g, g + W_total, g + 2 W_total, ...  (with the tiles
// split into ranges, the same within the block's range, over the blocks of
// that range; with a tile queue, only the first tile is fixed and the rest of
// the range is handed out one tile at a time).  The loads of the next tile
// (bounds, descriptor, col_ind, values) are issued before the current tile's
// gathers are consumed, so memory stays busy while a tile is walked and
// committed.
//
// HOT: the block first copies the hot x values into LDS (the plan's recoded
// column stream marks hot columns as -1 - slot) and serves those gathers from
// LDS.
#include "merbit_internal.hpp"

namespace merbit {

// D: the descriptor word, uint32_t (sigma <= 12) or uint64_t (sigma <= 40)
template <typename V, int SIGMA, typename D>
struct WaveTile {
  int x_ws;
  int x_se;
  uint32_t tyw;
  int y_we;
  D desc;
  int cc[SIGMA];
  V vv[SIGMA];
};

template <typename D>
__device__ __forceinline__ D load_desc(const SpmvArgs& a, int j);
template <>
__device__ __forceinline__ uint32_t load_desc<uint32_t>(const SpmvArgs& a, int j) {
  return a.lane_desc[j];
}
template <>
__device__ __forceinline__ uint64_t load_desc<uint64_t>(const SpmvArgs& a, int j) {
  return a.lane_desc64[j];
}

// Buffer-resource loads of the tile stream: faster for FP32 (both descriptor
// widths) and for FP64 with 64-bit descriptors (3.7-5 % per SpMV on R-MAT 22),
// slower by 2 % for FP64 with 32-bit descriptors, which keeps plain loads.
template <typename V, typename D>
constexpr bool kBufferStream = sizeof(V) == 4 || sizeof(D) == 8;
// word 3 of a raw (unformatted, stride 0) buffer resource on gfx950
constexpr int kBufferWord3 = 0x00020000;
// cache policy bits of a gfx950 buffer load: nt (streaming, evicted first)
constexpr int kPolicyStream = 2;
// hot x values loaded per lane before they are stored to LDS (128 bytes:
// 16 -> 32 took FP32 sigma 28 from 226 to 224 us per SpMV; 64 FP64 values
// spill in the 1,024-lane kernels)
template <typename V>
constexpr int kHotBatch = 128 / (int)sizeof(V);

// A load through the constant address space: the tile bounds are never
// written during a launch, and with the tile-queue atomics in the loop the
// compiler could otherwise not prove that, and would load the (uniform) bounds
// with vector loads that wait for every gather in flight.
template <typename T>
__device__ __forceinline__ T const_load(const T* p, int i) {
  typedef const __attribute__((address_space(4))) T ConstT;
  return ((ConstT*)p)[i];
}

template <typename V, int SIGMA, typename D>
__device__ __forceinline__ void wave_load_tile(const SpmvArgs& a, const int32_t* __restrict__ col,
                                               const V* __restrict__ val, int t, int lid,
                                               WaveTile<V, SIGMA, D>& s) {
  s.x_ws = const_load(a.tile_x, t);
  s.x_se = const_load(a.tile_x, t + 1) - s.x_ws;
  s.tyw = const_load(a.tile_y, t);
  s.y_we = (int)(const_load(a.tile_y, t + 1) & kRowMask);
  const bool normal = s.x_se > 0 && !(s.tyw & kFastBit);
  s.desc = 0;
  if (normal) s.desc = load_desc<D>(a, min(t * kOmega + lid, a.lane_num - 1));
  // A tile without nonzeros reads nothing: col / val may be empty (nnz = 0).
  // The branch is uniform across the wavefront.
  if (s.x_se > 0) {
    if constexpr (kBufferStream<V, D>) {
      // buffer loads over the tile's own range (streaming policy): one 32-bit
      // offset per lane instead of a 64-bit address per load, and reads past
      // the tile's end return 0 without a clamp.  A zero column gathers x[0]
      // (x is not empty when the tile has nonzeros) and its product is never
      // staged.
      const int xws = __builtin_amdgcn_readfirstlane(s.x_ws);
      const int xse = __builtin_amdgcn_readfirstlane(s.x_se);
      const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(col + xws), (short)0, xse * 4, kBufferWord3);
      const __amdgpu_buffer_rsrc_t rv = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(val + xws), (short)0, xse * (int)sizeof(V), kBufferWord3);
#pragma unroll
      for (int it = 0; it < SIGMA; ++it) {
        const int k = lid + it * kOmega;
        s.cc[it] = (int)__builtin_amdgcn_raw_buffer_load_b32(rc, k * 4, 0, kPolicyStream);
        if constexpr (sizeof(V) == 4)
          s.vv[it] = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(rv, k * 4, 0,
                                                                                kPolicyStream));
        else
          s.vv[it] = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(rv, k * 8, 0,
                                                                                kPolicyStream));
      }
    } else {
#pragma unroll
      for (int it = 0; it < SIGMA; ++it) {
        const int k = min(lid + it * kOmega, s.x_se - 1);
        s.cc[it] = __builtin_nontemporal_load(col + s.x_ws + k);
        s.vv[it] = __builtin_nontemporal_load(val + s.x_ws + k);
      }
    }
  } else {
#pragma unroll
    for (int it = 0; it < SIGMA; ++it) {
      s.cc[it] = 0;
      s.vv[it] = V(0);
    }
  }
}

template <typename V, int SIGMA, int WAVES, bool HOT, typename D>
__global__ __launch_bounds__(WAVES * 64) void spmv_wave_kernel(SpmvArgs a) {
  constexpr int BITS = ceil_log2(kOmega * SIGMA);
  constexpr uint32_t FMASK = (1u << BITS) - 1u;
  static_assert(2 * BITS + SIGMA <= 8 * (int)sizeof(D), "descriptor does not fit");
  constexpr int WLDS = kOmega * SIGMA;  // per wavefront: products, then inner-row slots
  __shared__ V s_stage[WAVES * WLDS];

  const int32_t* __restrict__ col = a.col;
  const V* __restrict__ val = static_cast<const V*>(a.val);
  const V* __restrict__ x = static_cast<const V*>(a.x);
  V* __restrict__ y = static_cast<V*>(a.y);
  V* __restrict__ z = static_cast<V*>(a.z);

  const int tid = threadIdx.x;
  const int lid = tid & (kOmega - 1);
  const int wid = __builtin_amdgcn_readfirstlane(tid / kOmega);
  V* s_w = s_stage + wid * WLDS;

  // this block's part of the tiles and of the hot values (one part unless
  // the plan splits the tiles into ranges)
  int t_begin = 0, t_end = a.tile_num, slot = blockIdx.x, slots = a.grid;
  int h_begin = 0, h_num = a.hot_n;
  unsigned long long* queue = a.queue;
  if (a.ranges > 1) {
    const int k = blockIdx.x % a.ranges;
    if (queue) queue += kQueueStride * k;
    t_begin = a.range_tile[k];
    t_end = a.range_tile[k + 1];
    slot = blockIdx.x / a.ranges;
    slots = a.grid / a.ranges;
    if (HOT) {
      h_begin = a.hot_off[k];
      h_num = a.hot_off[k + 1] - h_begin;
    }
  }

  extern __shared__ __align__(16) unsigned char s_dyn[];
  const V* s_hot = reinterpret_cast<const V*>(s_dyn);
  if (HOT) {
    // kHotBatch loads per lane in flight before their LDS stores: the copy
    // takes h_num / (kHotBatch * block lanes) memory round trips, not
    // h_num / block lanes (one block per CU waits for it)
    // (buffer loads over the block's hot slice: reads past its end return 0)
    constexpr int NT = WAVES * kOmega;
    V* dst = reinterpret_cast<V*>(s_dyn);
    const __amdgpu_buffer_rsrc_t rh = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(static_cast<const V*>(a.x_hot) + h_begin), (short)0, h_num * (int)sizeof(V),
        kBufferWord3);
    for (int s0 = tid; s0 < h_num; s0 += kHotBatch<V> * NT) {
      V hv[kHotBatch<V>];
#pragma unroll
      for (int u = 0; u < kHotBatch<V>; ++u) {
        const int off = (s0 + u * NT) * (int)sizeof(V);
        if constexpr (sizeof(V) == 4)
          hv[u] = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(rh, off, 0, 0));
        else
          hv[u] = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(rh, off, 0, 0));
      }
#pragma unroll
      for (int u = 0; u < kHotBatch<V>; ++u) {
        const int s = s0 + u * NT;
        if (s < h_num) dst[s] = hv[u];
      }
    }
    __syncthreads();
  }

  // Every wavefront of the range first takes one tile of the range's first
  // slots * WAVES; further tiles come from the range's queue counter, one at a
  // time, so wavefronts that meet cheap tiles take more of them (without a
  // queue: the fixed sequence t + stride, t + 2 stride, ...).  The number of
  // the tile after next is requested while the current tile is worked on and
  // read at the end of it: the atomic's latency hides behind a tile, and
  // waiting for it (memory returns in issue order) never waits for loads the
  // next iteration does not need first anyway.
  const int stride = slots * WAVES;
  auto take = [&]() -> int {
    int q = 0;
    if (lid == 0) q = (int)atomicAdd(queue, 1ull);
    return q;
  };
  auto tile_of = [&](int q) -> int {
    q = __builtin_amdgcn_readfirstlane(q);
    return q < t_end - t_begin - stride ? t_begin + stride + q : t_end;
  };
  int t = t_begin + slot * WAVES + wid;
  int tn = t_end;
  WaveTile<V, SIGMA, D> cur;
  if (t < t_end) {
    wave_load_tile<V, SIGMA, D>(a, col, val, t, lid, cur);
    tn = queue ? tile_of(take()) : t + stride;
  }
  while (t < t_end) {
    // gathers of the current tile (none for a tile without nonzeros: x may be
    // empty then)
    V g[SIGMA];
    if (cur.x_se > 0) {
#pragma unroll
      for (int it = 0; it < SIGMA; ++it) {
        const int c = cur.cc[it];
        if (HOT) {
          if (c >= 0) g[it] = x[c];
          else g[it] = s_hot[-1 - c];
        } else {
          g[it] = x[c];
        }
      }
    }
    // the tile after next, then the loads of the next tile: both go out
    // before the gathers are consumed
    int qn = 0;
    if (queue && tn < t_end) qn = take();
    WaveTile<V, SIGMA, D> nxt;
    if (tn < t_end) wave_load_tile<V, SIGMA, D>(a, col, val, tn, lid, nxt);

    const int x_se = cur.x_se;
    const int y_ws = (int)(cur.tyw & kRowMask);
    const int y_we = cur.y_we;
    if (x_se == 0) {
      // down steps only: the rows strictly inside the tile are empty
      for (int r = y_ws + 1 + lid; r < y_we; r += kOmega) y[r] = V(0);
    } else if (cur.tyw & kFastBit) {
      // single-row tile (Sec. 4.2 opt. (1))
      V acc = V(0);
#pragma unroll
      for (int it = 0; it < SIGMA; ++it)
        if (lid + it * kOmega < x_se) acc += cur.vv[it] * g[it];
      acc = wave_total(acc);
      if (lid == 0) global_add(&y[y_ws], acc);
    } else {
      wave_lds_sync();  // the previous tile's commit has read its slots
#pragma unroll
      for (int it = 0; it < SIGMA; ++it) {
        const int k = lid + it * kOmega;
        if (k < x_se) s_w[k] = cur.vv[it] * g[it];
      }
      wave_lds_sync();
      // walk (Algorithm tile_normal_tackle); inner row r (y_ws < r < y_we)
      // goes to slot x_se + (r - y_ws - 1)
      const int j = t * kOmega + lid;
      V sum = V(0), first_sum = V(0);
      bool has_down = false;
      int start_off = 0;
      if (j < a.lane_num) {
        int xo = (int)(cur.desc & FMASK);
        int yo = (int)((cur.desc >> BITS) & FMASK);
        start_off = yo;
        const D flags = cur.desc >> (2 * BITS);
        const int steps = min(SIGMA, a.path_len - j * SIGMA);
#pragma unroll
        for (int k = 0; k < SIGMA; ++k) {
          if (k < steps) {
            if ((flags >> k) & 1) {
              if (has_down) s_w[x_se + yo - 1] = sum;
              else first_sum = sum;
              has_down = true;
              sum = V(0);
              ++yo;
            } else {
              sum += s_w[xo];
              ++xo;
            }
          }
        }
      }
      const unsigned long long heads = __ballot(has_down) | 1ull;
      const unsigned long long upto = lid == kOmega - 1 ? ~0ull : ((2ull << lid) - 1ull);
      const int seg = 63 - __builtin_clzll(heads & upto);
      const V scan = wave_segmented_scan(sum, lid, seg);
      const V carry = dpp_move<kWaveShr1, 0xF>(scan);
      if (has_down) {
        const V row_val = first_sum + (lid > 0 ? carry : V(0));
        if (start_off == 0) global_add(&y[y_ws], row_val);  // the tile's first row
        else s_w[x_se + start_off - 1] = row_val;           // begun inside the tile
      }
      // the last segment belongs to the row the tile ends in
      if (lid == kOmega - 1 && y_we < a.n_rows && scan != V(0)) global_add(&y[y_we], scan);
      wave_lds_sync();
      for (int r = lid; r < y_we - y_ws - 1; r += kOmega) y[y_ws + 1 + r] = s_w[x_se + r];
    }
    if (z != nullptr && lid == 0) z[y_ws] = V(0);
    if (tn >= t_end) break;
    cur = nxt;
    t = tn;
    tn = queue ? tile_of(qn) : tn + stride;
  }
  // The range's last wavefront to finish sets its counters back to zero for
  // the next launch: every other wavefront of the range has taken its last
  // tile number (and waited for it) before it counts itself finished.
  if (queue && lid == 0) {
    if (atomicAdd(queue + 1, 1ull) == (unsigned long long)(stride - 1)) {
      atomicExch(queue, 0ull);
      atomicExch(queue + 1, 0ull);
    }
  }
}

template <typename V, int S, int W, bool H, typename D>
static hipError_t launch_wave_t(const SpmvArgs& a, size_t dyn, hipStream_t st) {
  hipLaunchKernelGGL((spmv_wave_kernel<V, S, W, H, D>), dim3((unsigned)a.grid), dim3(W * kOmega),
                     dyn, st, a);
  return hipGetLastError();
}

template <typename V, int S, int W, bool H, typename D>
static hipError_t set_wave_lds_t(size_t bytes) {
  static std::mutex mu;
  static size_t granted[kMaxLdsDevices] = {};
  return raise_dynamic_lds(reinterpret_cast<const void*>(&spmv_wave_kernel<V, S, W, H, D>), bytes,
                           mu, granted);
}

struct WaveEntry {
  hipError_t (*launch)(const SpmvArgs&, size_t, hipStream_t);
  hipError_t (*set_lds)(size_t);
};

#define MERBIT_WCASE(S, D) \
  case S: return WaveEntry{launch_wave_t<V, S, W, H, D>, set_wave_lds_t<V, S, W, H, D>};

template <typename V, int W, bool H>
static WaveEntry wave_pick_sigma(int sigma) {
  switch (sigma) {
    MERBIT_WCASE(1, uint32_t) MERBIT_WCASE(2, uint32_t) MERBIT_WCASE(3, uint32_t)
    MERBIT_WCASE(4, uint32_t) MERBIT_WCASE(5, uint32_t) MERBIT_WCASE(6, uint32_t)
    MERBIT_WCASE(7, uint32_t) MERBIT_WCASE(8, uint32_t) MERBIT_WCASE(9, uint32_t)
    MERBIT_WCASE(10, uint32_t) MERBIT_WCASE(11, uint32_t) MERBIT_WCASE(12, uint32_t)
    default: return WaveEntry{nullptr, nullptr};
  }
}

// 64-bit descriptors: longer lanes than 32 bits allow.  FP32: sigma 16, 20,
// 24, 28, 32; FP64 (twice the registers per value): sigma 14, 16, 20, 24.  256 or
// 512 lanes.
template <typename V, int W, bool H>
static WaveEntry wave_pick_sigma64(int sigma) {
  if constexpr (sizeof(V) == 4) {
    switch (sigma) {
      MERBIT_WCASE(16, uint64_t) MERBIT_WCASE(20, uint64_t) MERBIT_WCASE(24, uint64_t)
      MERBIT_WCASE(28, uint64_t) MERBIT_WCASE(32, uint64_t)
      default: return WaveEntry{nullptr, nullptr};
    }
  } else {
    switch (sigma) {
      MERBIT_WCASE(14, uint64_t) MERBIT_WCASE(16, uint64_t) MERBIT_WCASE(20, uint64_t)
      MERBIT_WCASE(24, uint64_t)
      default: return WaveEntry{nullptr, nullptr};
    }
  }
}
#undef MERBIT_WCASE

template <typename V, bool H>
static WaveEntry wave_pick_waves(int sigma, int waves, bool desc64) {
  if (desc64) {
    switch (waves) {
      case 4: return wave_pick_sigma64<V, 4, H>(sigma);
      case 8: return wave_pick_sigma64<V, 8, H>(sigma);
      default: return WaveEntry{nullptr, nullptr};
    }
  }
  switch (waves) {
    case 4: return wave_pick_sigma<V, 4, H>(sigma);
    case 8: return wave_pick_sigma<V, 8, H>(sigma);
    case 16: return wave_pick_sigma<V, 16, H>(sigma);
    default: return WaveEntry{nullptr, nullptr};
  }
}

static WaveEntry wave_pick(int dtype, int sigma, int waves, bool hot, bool desc64) {
  if (dtype == 0) return hot ? wave_pick_waves<float, true>(sigma, waves, desc64)
                             : wave_pick_waves<float, false>(sigma, waves, desc64);
  if (dtype == 1) return hot ? wave_pick_waves<double, true>(sigma, waves, desc64)
                             : wave_pick_waves<double, false>(sigma, waves, desc64);
  return WaveEntry{nullptr, nullptr};
}

bool spmv_wave_supported(int dtype, int sigma, int waves, bool hot, bool desc64) {
  return wave_pick(dtype, sigma, waves, hot, desc64).launch != nullptr;
}

hipError_t launch_spmv_wave(int dtype, int sigma, int waves, bool hot, size_t hot_lds_bytes,
                            const SpmvArgs& a, hipStream_t st, bool desc64) {
  WaveEntry k = wave_pick(dtype, sigma, waves, hot, desc64);
  if (!k.launch) return hipErrorInvalidValue;
  return k.launch(a, hot ? hot_lds_bytes : 0, st);
}

hipError_t spmv_wave_set_hot_lds(int dtype, int sigma, int waves, size_t bytes, bool desc64) {
  WaveEntry k = wave_pick(dtype, sigma, waves, true, desc64);
  if (!k.set_lds) return hipErrorInvalidValue;
  return k.set_lds(bytes);
}

}  // namespace merbit
