// Hot-column x cache (plan side and per-call gather).
//
// The x gathers of the fused SpMV are limited on gfx950 by the rate at which
// scattered L1 misses are served by L2.  Power-law matrices concentrate their
// nonzeros on few columns (R-MAT scale 22: the 32K most frequent columns hold
// 53 % of all nonzeros), so the plan picks the H most frequent columns and
// rewrites the column stream: a hot column c becomes -1 - slot(c).  Per call,
// the H hot x values are gathered once into a contiguous array, every block
// of the fused kernel copies them into LDS, and a hot nonzero reads its x
// value from LDS instead of issuing a global gather.  Sums and their order
// are unchanged: only where the x value is read from differs.
#include <algorithm>

#include "merbit_internal.hpp"

namespace merbit {

// Selection of R ranges at once (one per tile range of a column-stripe plan,
// R = 1 for a plain plan): every step below is one launch whose
// blockIdx.y (or blockIdx.x for the one-block steps) picks the range, so a
// plan's ranges share launches and nothing returns to the host in between.
//
// counts[c] = number of sampled nonzeros in column c of the range: every
// `sample`-th nonzero of its stream (1 = exact counts).  The selection only
// needs the order of the large counts, which a sample keeps (R-MAT scale 22:
// 52.9 % coverage of the top 32K columns at a 1-in-8 sample and exact counts
// alike).  The count is bound by global atomics (device scope: about 8 G
// updates/s measured, against a 42 us pass of plain loads over the same
// samples of R-MAT 22), and a power-law stream repeats its frequent columns,
// so each block first counts in an LDS table (open addressing, a few probes;
// a sample that finds no slot goes straight to the global count) and adds
// every slot to the global counts once at the end: the counts are exact
// either way.  A 1-in-4 sample of the stacked R-MAT 22 stream: 2.0 ms with
// global atomics alone, 1.32 ms with 2048 slots per 8192 samples, 1.06 ms
// with 4096 slots per 16384.  The block's column loads are issued
// kCountUnroll at a time ahead of the table updates.
constexpr int kCountBits = 12;
constexpr int kCountSlots = 1 << kCountBits;
constexpr int kCountProbes = 8;
constexpr int kCountThreads = 256;
constexpr int kCountUnroll = 8;
constexpr int kCountPerBlock = 16384;  // samples per block
static_assert(kCountPerBlock % (kCountThreads * kCountUnroll) == 0, "whole load batches");

__global__ __launch_bounds__(kCountThreads) void col_count_kernel(
    const int32_t* __restrict__ col, const HotSeg* __restrict__ segs,
    int32_t* __restrict__ counts_all) {
  const HotSeg sg = segs[blockIdx.y];
  const int64_t ns = (sg.len + sg.sample - 1) / sg.sample;
  const int64_t b0 = (int64_t)blockIdx.x * kCountPerBlock;
  if (b0 >= ns) return;  // uniform over the block
  const int64_t b1 = b0 + kCountPerBlock < ns ? b0 + kCountPerBlock : ns;
  const int32_t* in = col + sg.lo;
  int32_t* counts = counts_all + sg.coff;
  __shared__ int32_t s_key[kCountSlots];
  __shared__ int32_t s_cnt[kCountSlots];
  for (int i = threadIdx.x; i < kCountSlots; i += kCountThreads) {
    s_key[i] = -1;
    s_cnt[i] = 0;
  }
  __syncthreads();
  for (int64_t i0 = b0; i0 < b1; i0 += kCountThreads * kCountUnroll) {
    int32_t cv[kCountUnroll];
#pragma unroll
    for (int u = 0; u < kCountUnroll; ++u) {
      const int64_t i = i0 + u * kCountThreads + threadIdx.x;
      cv[u] = i < b1 ? in[i * sg.sample] - sg.c_lo : -1;
    }
#pragma unroll
    for (int u = 0; u < kCountUnroll; ++u) {
      const int32_t c = cv[u];
      if (c < 0) continue;
      uint32_t h = ((uint32_t)c * 2654435761u) >> (32 - kCountBits);
      bool done = false;
      for (int p = 0; p < kCountProbes && !done; ++p, h = (h + 1) & (kCountSlots - 1)) {
        int32_t k = s_key[h];
        if (k == -1) k = atomicCAS(&s_key[h], -1, c);  // claim an empty slot
        if (k == -1 || k == c) {
          atomicAdd(&s_cnt[h], 1);
          done = true;
        }
      }
      if (!done) atomicAdd(&counts[c], 1);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kCountSlots; i += kCountThreads)
    if (s_cnt[i] > 0) atomicAdd(&counts[s_key[i]], s_cnt[i]);
}

// hist[min(count, kHotHistBins - 1)] += 1 over the range's columns.  Most
// columns have small counts, so the low bins are counted per block in LDS
// and added to the global histogram once per block; only large counts go
// straight to global atomics.
constexpr int kHistLdsBins = 2048;

__global__ __launch_bounds__(256) void count_hist_kernel(const int32_t* __restrict__ counts_all,
                                                         const HotSeg* __restrict__ segs,
                                                         int32_t* __restrict__ hist_all) {
  const HotSeg sg = segs[blockIdx.y];
  const int32_t* counts = counts_all + sg.coff;
  int32_t* hist = hist_all + (size_t)blockIdx.y * kHotHistBins;
  __shared__ int32_t s_hist[kHistLdsBins];
  for (int b = threadIdx.x; b < kHistLdsBins; b += blockDim.x) s_hist[b] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < sg.span; c += stride) {
    const int32_t v = counts[c];
    const int32_t bin = v < kHotHistBins - 1 ? v : kHotHistBins - 1;
    if (bin < kHistLdsBins) atomicAdd(&s_hist[bin], 1);
    else atomicAdd(&hist[bin], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kHistLdsBins; b += blockDim.x)
    if (s_hist[b]) atomicAdd(&hist[b], s_hist[b]);
}

// Selection in column order: block b of a range owns its columns
// [b * kSelSpan, (b+1) * kSelSpan).  A column is taken when its count is
// above the cut count t, or equal to t and among the first tie_take[b] such
// columns of its block (ties go to the smaller columns):
//   1. select_cut_kernel (a block per range) finds t from the histogram of
//      the counts: the largest count b* whose columns, with all those above
//      it, exceed the cap (t = b*; none: t = 0, every counted column is
//      taken), and how many of the columns at t are taken (none when a tie
//      at the cut is taken whole or not at all);
//   2. select_count_kernel counts, per block, the columns above t and at t;
//   3. select_plan_kernel (a block per range) turns them into each block's
//      first slot and tie budget;
//   4. select_assign_kernel gives the taken columns consecutive slots in
//      column order, so slots are deterministic.
constexpr int kSelThreads = 256;
constexpr int kSelPerThread = 16;
constexpr int kSelSpan = kSelThreads * kSelPerThread;
constexpr int kCutThreads = 1024;
constexpr int kCutGroups = kHotHistBins / kOmega;  // groups of 64 consecutive bins
static_assert(kCutGroups == kCutThreads, "one group of bins per thread");

__host__ __device__ static inline int64_t select_blocks(int64_t span) {
  return (span + kSelSpan - 1) / kSelSpan;
}

// Exclusive sum, in thread order, of one int64 per thread over a block of
// THREADS threads; *total gets the block's sum.  Integer sums: the result
// does not depend on the order of the additions.  Every thread calls it.
template <int THREADS>
__device__ __forceinline__ int64_t block_exscan_i64(int64_t v, int64_t* s_wave, int64_t* total) {
  const int lid = threadIdx.x & (kOmega - 1), wid = threadIdx.x / kOmega;
  int64_t incl = v;
#pragma unroll
  for (int d = 1; d < kOmega; d <<= 1) {
    const int64_t u = __shfl_up(incl, d, kOmega);
    if (lid >= d) incl += u;
  }
  if (lid == kOmega - 1) s_wave[wid] = incl;
  __syncthreads();
  int64_t before = 0, tot = 0;
  for (int w = 0; w < THREADS / kOmega; ++w) {
    const int64_t s = s_wave[w];
    before += w < wid ? s : 0;
    tot += s;
  }
  __syncthreads();  // s_wave is rewritten by the next call
  *total = tot;
  return before + incl - v;
}

// Cut of a range's histogram (bins 1 .. kHotHistBins - 1; bin 0 = uncounted
// columns).  Wavefronts sum the groups of 64 bins with coalesced loads;
// thread i then owns group kCutGroups - 1 - i, so the scan in thread order
// runs from the largest counts down.
__global__ __launch_bounds__(kCutThreads) void select_cut_kernel(
    const int32_t* __restrict__ hist_all, int64_t cap, int whole_ties,
    HotSel* __restrict__ sel_all) {
  constexpr int W = kCutThreads / kOmega;
  __shared__ int64_t s_grp[kCutGroups];
  __shared__ int64_t s_wave[W];
  __shared__ int32_t s_cut;
  __shared__ int64_t s_above;
  const int32_t* hist = hist_all + (size_t)blockIdx.x * kHotHistBins;
  const int lid = threadIdx.x & (kOmega - 1), wid = threadIdx.x / kOmega;
  for (int g = wid; g < kCutGroups; g += W) {
    const int b = g * kOmega + lid;
    const int64_t s = wave_sum((int64_t)(b >= 1 ? hist[b] : 0));
    if (lid == 0) s_grp[g] = s;
  }
  __syncthreads();
  const int g = kCutGroups - 1 - (int)threadIdx.x;
  const int64_t mine = s_grp[g];
  int64_t tot = 0;
  const int64_t before = block_exscan_i64<kCutThreads>(mine, s_wave, &tot);
  if (threadIdx.x == 0) {
    s_cut = 0;  // no cut: every counted column fits
    s_above = tot;
  }
  __syncthreads();
  if (before <= cap && before + mine > cap) {
    // the cut lies in this thread's group: the first bin from the top whose
    // columns, with those above, exceed the cap
    int64_t run = before;
    const int lo = g * kOmega > 1 ? g * kOmega : 1;
    for (int b = g * kOmega + kOmega - 1; b >= lo; --b) {
      if (run + hist[b] > cap) {
        s_cut = b;
        s_above = run;
        break;
      }
      run += hist[b];
    }
  }
  __syncthreads();
  const int32_t t = s_cut;
  const int64_t above = s_above;
  const int64_t extra = (t == 0 || whole_ties) ? 0 : cap - above;
  // covered: the sum of the taken columns' counts
  int64_t cov = 0;
  for (int g2 = wid; g2 < kCutGroups; g2 += W) {
    const int b = g2 * kOmega + lid;
    cov += b > t ? (int64_t)b * hist[b] : 0;
  }
  int64_t cov_tot = 0;
  (void)block_exscan_i64<kCutThreads>(cov, s_wave, &cov_tot);
  if (threadIdx.x == 0) {
    HotSel* sel = sel_all + blockIdx.x;
    sel->t = t;
    sel->extra = (int32_t)extra;
    sel->taken = above + extra;
    sel->covered = (double)(cov_tot + (int64_t)t * extra);
  }
}

__global__ __launch_bounds__(kSelThreads) void select_count_kernel(
    const int32_t* __restrict__ counts_all, const HotSeg* __restrict__ segs,
    const HotSel* __restrict__ sel_all, int32_t* __restrict__ block_counts) {
  const HotSeg sg = segs[blockIdx.y];
  const int64_t base = (int64_t)blockIdx.x * kSelSpan;
  if (base >= sg.span) return;  // uniform over the block
  __shared__ int32_t s_cnt[2][kSelThreads / kOmega];
  const int32_t* counts = counts_all + sg.coff;
  const int32_t threshold = sel_all[blockIdx.y].t;
  int above = 0, at = 0;
  for (int k = 0; k < kSelPerThread; ++k) {
    const int64_t col = base + (int64_t)k * kSelThreads + threadIdx.x;
    if (col < sg.span) {
      const int32_t c = min(counts[col], kHotHistBins - 1);  // as the histogram bins it
      above += c > threshold;
      at += c == threshold;
    }
  }
  above = wave_sum(above);
  at = wave_sum(at);
  if ((threadIdx.x & (kOmega - 1)) == 0) {
    s_cnt[0][threadIdx.x / kOmega] = above;
    s_cnt[1][threadIdx.x / kOmega] = at;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int ta = 0, tt = 0;
    for (int w = 0; w < kSelThreads / kOmega; ++w) {
      ta += s_cnt[0][w];
      tt += s_cnt[1][w];
    }
    const int64_t b = sg.boff + blockIdx.x;
    block_counts[2 * b] = ta;
    block_counts[2 * b + 1] = tt;
  }
}

// block_plan[2b] = first slot of block b, block_plan[2b + 1] = its tie
// budget: the ties go to the range's blocks in column order until `extra`
// are taken.
__global__ __launch_bounds__(kCutThreads) void select_plan_kernel(
    const int32_t* __restrict__ block_counts, const HotSeg* __restrict__ segs,
    const HotSel* __restrict__ sel_all, int32_t* __restrict__ block_plan) {
  __shared__ int64_t s_wave[kCutThreads / kOmega];
  const HotSeg sg = segs[blockIdx.x];
  const int64_t nb = select_blocks(sg.span);
  const int64_t extra = sel_all[blockIdx.x].extra;
  const int32_t* bc = block_counts + 2 * sg.boff;
  int32_t* bp = block_plan + 2 * sg.boff;
  int64_t slot_carry = 0, tie_carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kCutThreads) {
    const int64_t b = b0 + threadIdx.x;
    const int64_t above = b < nb ? bc[2 * b] : 0;
    const int64_t at = b < nb ? bc[2 * b + 1] : 0;
    int64_t ties_total = 0, slots_total = 0;
    const int64_t ties_before = tie_carry + block_exscan_i64<kCutThreads>(at, s_wave, &ties_total);
    int64_t take = extra - ties_before;
    take = take < 0 ? 0 : (take > at ? at : take);
    const int64_t slot_before = block_exscan_i64<kCutThreads>(above + take, s_wave, &slots_total);
    if (b < nb) {
      bp[2 * b] = (int32_t)(slot_carry + slot_before);
      bp[2 * b + 1] = (int32_t)take;
    }
    slot_carry += slots_total;
    tie_carry += ties_total;
  }
}

// The taken columns of range k go to hot_cols[k * cap + slot]; slot_of gets
// the slot of every column of the span (-1: not taken).
__global__ __launch_bounds__(kSelThreads) void select_assign_kernel(
    const int32_t* __restrict__ counts_all, const HotSeg* __restrict__ segs,
    const HotSel* __restrict__ sel_all, const int32_t* __restrict__ block_plan, int64_t cap,
    int32_t* __restrict__ slot_all, int32_t* __restrict__ hot_cols) {
  const HotSeg sg = segs[blockIdx.y];
  const int64_t base = (int64_t)blockIdx.x * kSelSpan;
  if (base >= sg.span) return;  // uniform over the block
  __shared__ int32_t s_sel[kSelThreads / kOmega], s_tie[kSelThreads / kOmega];
  const int32_t* counts = counts_all + sg.coff;
  int32_t* slot_of = slot_all + sg.coff;
  int32_t* out = hot_cols + (int64_t)blockIdx.y * cap;
  const int32_t threshold = sel_all[blockIdx.y].t;
  const int lid = threadIdx.x & (kOmega - 1), wid = threadIdx.x / kOmega;
  const unsigned long long below = (1ull << lid) - 1ull;
  const int64_t b = sg.boff + blockIdx.x;
  int32_t slot_base = block_plan[2 * b];
  int32_t ties_left = block_plan[2 * b + 1];
  for (int k = 0; k < kSelPerThread; ++k) {
    const int64_t col = base + (int64_t)k * kSelThreads + threadIdx.x;
    const bool in = col < sg.span;
    const int32_t c = in ? min(counts[col], kHotHistBins - 1) : -1;
    // rank of this tie among this step's ties (wavefronts in order)
    const bool tie = in && c == threshold;
    const unsigned long long tmask = __ballot(tie);
    if (lid == 0) s_tie[wid] = __popcll(tmask);
    __syncthreads();
    int tie_rank = __popcll(tmask & below), ties_step = 0;
    for (int w = 0; w < kSelThreads / kOmega; ++w) {
      if (w < wid) tie_rank += s_tie[w];
      ties_step += s_tie[w];
    }
    const bool sel_now = (in && c > threshold) || (tie && tie_rank < ties_left);
    const unsigned long long smask = __ballot(sel_now);
    if (lid == 0) s_sel[wid] = __popcll(smask);
    __syncthreads();
    int wave_off = 0, total = 0;
    for (int w = 0; w < kSelThreads / kOmega; ++w) {
      if (w < wid) wave_off += s_sel[w];
      total += s_sel[w];
    }
    if (in) {
      if (sel_now) {
        const int slot = slot_base + wave_off + __popcll(smask & below);
        slot_of[col] = slot;
        out[slot] = sg.c_lo + (int32_t)col;
      } else {
        slot_of[col] = -1;
      }
    }
    slot_base += total;
    ties_left -= ties_step < ties_left ? ties_step : ties_left;
    __syncthreads();  // s_sel / s_tie are rewritten by the next step
  }
}

// colx[lo + k] = -1 - slot(col[lo + k]) for a hot column of range
// blockIdx.y, col[lo + k] otherwise
__global__ void recode_ranges_kernel(const int32_t* __restrict__ col,
                                     const HotSeg* __restrict__ segs,
                                     const int32_t* __restrict__ slot_all,
                                     int32_t* __restrict__ colx) {
  const HotSeg sg = segs[blockIdx.y];
  const int32_t* in = col + sg.lo;
  int32_t* out = colx + sg.lo;
  const int32_t* slot_of = slot_all + sg.coff;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < sg.len; k += stride) {
    const int32_t c = in[k];
    const int32_t s = slot_of[c - sg.c_lo];
    out[k] = s >= 0 ? -1 - s : c;
  }
}

// colx[k] = -1 - col[k]: a cache of every column, slot = column
__global__ void recode_all_kernel(const int32_t* __restrict__ col, int64_t nnz,
                                  int32_t* __restrict__ colx) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += stride)
    colx[k] = -1 - col[k];
}

// packed[off_k + s] = stage[k * cap + s] for s < taken_k, off_k = the taken
// counts of the ranges before k
__global__ void pack_ranges_kernel(const int32_t* __restrict__ stage, int64_t cap,
                                   const HotSel* __restrict__ sel, int32_t* __restrict__ packed) {
  int64_t off = 0;
  for (int j = 0; j < (int)blockIdx.y; ++j) off += sel[j].taken;
  const int64_t taken = sel[blockIdx.y].taken;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < taken) packed[off + s] = stage[(int64_t)blockIdx.y * cap + s];
}

// out[i] = src[idx[i]] for i < n (n <= kMaxPeek)
struct PeekIdx {
  int64_t i[kMaxPeek];
};
__global__ void peek_kernel(const int32_t* __restrict__ src, PeekIdx idx, int n,
                            int32_t* __restrict__ out) {
  const int i = threadIdx.x;
  if (i < n) out[i] = src[idx.i[i]];
}

static unsigned grid_for(int64_t n, int64_t cap) {
  int64_t g = (n + 255) / 256;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Work-space layout: the range table, the histograms, the counts, the slot
// map, then the selection blocks' counts and plan.
struct HotLayout {
  size_t segs, hist, counts, slot, blocks, total;
};

static HotLayout hot_layout(int R, int64_t span_sum, int64_t nb_sum) {
  HotLayout l;
  l.segs = 0;
  l.hist = l.segs + align256(sizeof(HotSeg) * (size_t)R);
  l.counts = l.hist + align256(sizeof(int32_t) * kHotHistBins * (size_t)R);
  l.slot = l.counts + align256(sizeof(int32_t) * (size_t)span_sum);
  l.blocks = l.slot + align256(sizeof(int32_t) * (size_t)span_sum);
  l.total = l.blocks + align256(sizeof(int32_t) * 4 * (size_t)(nb_sum > 0 ? nb_sum : 1));
  return l;
}

static HotLayout hot_layout_of(const HotSeg* segs, int R) {
  const HotSeg& last = segs[R - 1];
  return hot_layout(R, last.coff + last.span, last.boff + select_blocks(last.span));
}

size_t hot_select_layout(HotSeg* segs, int R) {
  int64_t coff = 0, boff = 0;
  for (int k = 0; k < R; ++k) {
    segs[k].coff = coff;
    segs[k].boff = boff;
    coff += segs[k].span;
    boff += select_blocks(segs[k].span);
  }
  return hot_layout(R, coff, boff).total;
}

hipError_t hot_select_ranges(const int32_t* col, const HotSeg* segs, int R, int64_t cap,
                             bool whole_ties, void* work, int32_t* hot_cols, HotSel* sel,
                             hipStream_t st) {
  const HotLayout l = hot_layout_of(segs, R);
  unsigned char* w = static_cast<unsigned char*>(work);
  HotSeg* segs_dev = reinterpret_cast<HotSeg*>(w + l.segs);
  int32_t* hist = reinterpret_cast<int32_t*>(w + l.hist);
  int32_t* counts = reinterpret_cast<int32_t*>(w + l.counts);
  int32_t* slot_of = reinterpret_cast<int32_t*>(w + l.slot);
  int32_t* block_counts = reinterpret_cast<int32_t*>(w + l.blocks);
  const int64_t nb_sum = segs[R - 1].boff + select_blocks(segs[R - 1].span);
  int32_t* block_plan = block_counts + 2 * (nb_sum > 0 ? nb_sum : 1);
  int64_t max_ns = 0, max_span = 0;
  for (int k = 0; k < R; ++k) {
    max_ns = std::max(max_ns, (segs[k].len + segs[k].sample - 1) / segs[k].sample);
    max_span = std::max(max_span, segs[k].span);
  }
  const int64_t max_nb = select_blocks(max_span);
  hipError_t e = hipMemcpyAsync(segs_dev, segs, sizeof(HotSeg) * (size_t)R,
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(w + l.hist, 0, l.slot - l.hist, st);  // hist, counts
  if (e != hipSuccess) return e;
  if (max_ns > 0) {
    const int64_t gx = (max_ns + kCountPerBlock - 1) / kCountPerBlock;
    hipLaunchKernelGGL(col_count_kernel, dim3((unsigned)gx, (unsigned)R), dim3(kCountThreads), 0,
                       st, col, segs_dev, counts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(count_hist_kernel, dim3(grid_for(max_span, 512), (unsigned)R), dim3(256), 0,
                     st, counts, segs_dev, hist);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(select_cut_kernel, dim3((unsigned)R), dim3(kCutThreads), 0, st, hist, cap,
                     whole_ties ? 1 : 0, sel);
  if ((e = hipGetLastError()) != hipSuccess || max_nb == 0) return e;
  hipLaunchKernelGGL(select_count_kernel, dim3((unsigned)max_nb, (unsigned)R), dim3(kSelThreads),
                     0, st, counts, segs_dev, sel, block_counts);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(select_plan_kernel, dim3((unsigned)R), dim3(kCutThreads), 0, st,
                     block_counts, segs_dev, sel, block_plan);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(select_assign_kernel, dim3((unsigned)max_nb, (unsigned)R), dim3(kSelThreads),
                     0, st, counts, segs_dev, sel, block_plan, cap, slot_of, hot_cols);
  return hipGetLastError();
}

hipError_t hot_recode_ranges(const int32_t* col, const HotSeg* segs, int R, const void* work,
                             int32_t* colx, hipStream_t st) {
  const HotLayout l = hot_layout_of(segs, R);
  const unsigned char* w = static_cast<const unsigned char*>(work);
  int64_t max_len = 0;
  for (int k = 0; k < R; ++k) max_len = std::max(max_len, segs[k].len);
  if (max_len == 0) return hipSuccess;
  hipLaunchKernelGGL(recode_ranges_kernel, dim3(grid_for(max_len, 8192 / R > 0 ? 8192 / R : 1),
                                                (unsigned)R),
                     dim3(256), 0, st, col, reinterpret_cast<const HotSeg*>(w + l.segs),
                     reinterpret_cast<const int32_t*>(w + l.slot), colx);
  return hipGetLastError();
}

hipError_t hot_recode_all(const int32_t* col, int64_t nnz, int32_t* colx, hipStream_t st) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(recode_all_kernel, dim3(grid_for(nnz, 8192)), dim3(256), 0, st, col, nnz,
                     colx);
  return hipGetLastError();
}

hipError_t hot_pack_ranges(const int32_t* stage, int64_t cap, const HotSel* sel, int R,
                           int32_t* packed, hipStream_t st) {
  if (cap <= 0 || R <= 0) return hipSuccess;
  hipLaunchKernelGGL(pack_ranges_kernel, dim3(grid_for(cap, cap), (unsigned)R), dim3(256), 0, st,
                     stage, cap, sel, packed);
  return hipGetLastError();
}

hipError_t launch_peek(const int32_t* src, const int64_t* idx, int n, int32_t* out,
                       hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n > kMaxPeek) return hipErrorInvalidValue;
  PeekIdx pi{};
  for (int i = 0; i < n; ++i) pi.i[i] = idx[i];
  hipLaunchKernelGGL(peek_kernel, dim3(1), dim3(kMaxPeek), 0, st, src, pi, n, out);
  return hipGetLastError();
}

// x_hot[s] = x[hot_cols[s]]
template <typename V>
__global__ void hot_gather_kernel(const V* __restrict__ x, const int32_t* __restrict__ hot_cols,
                                  int32_t hot_n, V* __restrict__ x_hot) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < hot_n) x_hot[s] = x[hot_cols[s]];
}

hipError_t launch_hot_gather(int dtype, const void* x, const int32_t* hot_cols, int32_t hot_n,
                             void* x_hot, hipStream_t st) {
  if (hot_n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((hot_n + 255) / 256);
  if (dtype == 0)
    hipLaunchKernelGGL(hot_gather_kernel<float>, dim3(grid), dim3(256), 0, st,
                       static_cast<const float*>(x), hot_cols, hot_n, static_cast<float*>(x_hot));
  else
    hipLaunchKernelGGL(hot_gather_kernel<double>, dim3(grid), dim3(256), 0, st,
                       static_cast<const double*>(x), hot_cols, hot_n,
                       static_cast<double*>(x_hot));
  return hipGetLastError();
}

}  // namespace merbit
