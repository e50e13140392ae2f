// C ABI of libmerbit, column stripes (plan side): the stacked matrix A' of
// the non-empty (stripe, row) pairs, its MERBIT plan, and one hot-column set
// per tile range.  The kernels are in merbit_stripes.hip; the SpMV entry
// points reach them through run_fused.
#include <algorithm>
#include <functional>
#include <vector>

#include "merbit_host.hpp"

namespace merbit {

namespace {
// Device temporaries of a striped plan build: one allocation reserved up
// front and handed out in 256-byte aligned parts; reset() hands the space out
// again (the parts given before are dead: every user is on the build's one
// stream, so later work is ordered after earlier reads), and a request
// beyond the reserve gets an allocation of its own.  Everything is freed
// when the build leaves: a hipFree of a large block costs about 0.3 ms
// (R-MAT 22), so the build frees one.
class Arena {
 public:
  Arena() = default;
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  ~Arena() {
    if (base_) (void)hipFree(base_);
    for (void* b : extra_) (void)hipFree(b);
  }
  hipError_t reserve(size_t bytes) {
    const hipError_t e = hipMalloc(&base_, bytes > 0 ? bytes : 1);
    cap_ = e == hipSuccess ? bytes : 0;
    return e;
  }
  template <typename T>
  hipError_t get(T** out, size_t count) {
    const size_t b = (count * sizeof(T) + 255) & ~(size_t)255;
    if (used_ + b <= cap_) {
      *out = reinterpret_cast<T*>(base_ + used_);
      used_ += b;
      return hipSuccess;
    }
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, b > 0 ? b : 1);
    if (e == hipSuccess) extra_.push_back(q);
    *out = static_cast<T*>(q);
    return e;
  }
  void reset() { used_ = 0; }

 private:
  unsigned char* base_ = nullptr;
  size_t cap_ = 0, used_ = 0;
  std::vector<void*> extra_;
};

// vals[i] = src[idx[i]] (device array, host indices): one kernel, one copy
int peek(const int32_t* src, const std::vector<int64_t>& idx, int32_t* buf, int32_t* vals,
         hipStream_t st) {
  for (size_t i0 = 0; i0 < idx.size(); i0 += kMaxPeek) {
    const int n = (int)std::min(idx.size() - i0, (size_t)kMaxPeek);
    HIP_TRY(launch_peek(src, idx.data() + i0, n, buf, st));
    HIP_TRY(hipMemcpyAsync(vals + i0, buf, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost,
                           st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  return MERBIT_OK;
}
}  // namespace

int stripes_copy_values(merbit_plan* p, const void* values, hipStream_t st) {
  HIP_TRY(launch_gather_values(p->dtype, p->sperm, values, nullptr, p->svals, p->nnz, st));
  return MERBIT_OK;
}

static int build_stripes(merbit_plan* p, const int32_t* row_ptr, hipStream_t st, Arena& tmp) {
  const int64_t m = p->nnz, n = p->n_rows;
  const int sbits = ceil_log2(p->stripes);
  int cbits = 0;  // columns are < 2^cbits
  while (((int64_t)1 << cbits) < p->n_cols) ++cbits;
  StripeSplitArgs a;
  a.row_ptr = row_ptr;
  a.col = p->col;
  a.n_rows = n;
  a.m = m;
  a.shift = cbits > sbits ? cbits - sbits : 0;
  p->stripe_shift = a.shift;
  a.key_bits = sbits;  // stripe indices are < 2^sbits
  a.stripes = p->stripes;
  a.words = (n + kOmega - 1) / kOmega;
  p->words = a.words;
  const int64_t nw = a.stripes * a.words;
  // the reserve holds the split's temporaries and, for at most m pairs, the
  // stacked rows' arrays
  const auto part = [](size_t b) { return (b + 255) & ~(size_t)255; };
  HIP_TRY(tmp.reserve(part(stripe_temp_bytes(m, nw, sbits)) + 7 * part(sizeof(int32_t) * (size_t)m) +
                      2 * part(sizeof(int32_t) * (size_t)nw) + part(sizeof(int32_t) * kMaxPeek) + 256));
  unsigned char* split_temp = nullptr;
  HIP_TRY(tmp.get(&split_temp, stripe_temp_bytes(m, nw, sbits)));
  HIP_TRY(tmp.get(&a.rows, (size_t)m));
  HIP_TRY(tmp.get(&a.row_s, (size_t)m));
  HIP_TRY(tmp.get(&a.flag, (size_t)m));
  HIP_TRY(tmp.get(&a.vidx, (size_t)m));
  a.temp = split_temp;
  HIP_TRY(hipMalloc(&p->sperm, sizeof(int32_t) * (size_t)m));
  HIP_TRY(hipMalloc(&p->scol, sizeof(int32_t) * (size_t)m));
  a.perm = p->sperm;
  a.col_s = p->scol;
  HIP_TRY(launch_stripe_split(a, st));
  // number of pairs V = vidx[m - 1] + flag[m - 1]
  int32_t last[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(&last[0], a.vidx + (m - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&last[1], a.flag + (m - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const int64_t nv = (int64_t)last[0] + last[1];
  if (nv < 1 || nv > m) return fail(MERBIT_EHIP, "column stripes: bad pair count");
  p->plan_rows = nv;
  HIP_TRY(tmp.get(&a.vrow_ptr, (size_t)nv + 1));
  HIP_TRY(tmp.get(&a.vrow_row, (size_t)nv));
  HIP_TRY(tmp.get(&a.vrow_stripe, (size_t)nv));
  HIP_TRY(tmp.get(&a.wcnt, (size_t)nw));
  HIP_TRY(tmp.get(&a.rank, (size_t)nw));
  HIP_TRY(hipMalloc(&p->swords, sizeof(StripeWord) * (size_t)nw));
  a.sw = p->swords;
  HIP_TRY(launch_stripe_rows(a, nv, st));
  // values in stacked order, the plan of A', and its two result buffers
  HIP_TRY(hipMalloc(&p->svals, vsize(p->dtype) * (size_t)m));
  int rc = stripes_copy_values(p, p->values, st);
  if (rc != MERBIT_OK) return rc;
  rc = build_tile(p, a.vrow_ptr, st);
  if (rc != MERBIT_OK) return rc;
  const size_t yb = vsize(p->dtype) * (size_t)nv;
  HIP_TRY(hipMalloc(&p->yv[0], yb));
  HIP_TRY(hipMalloc(&p->yv[1], yb));
  // zero everywhere: in particular at every tile's first row (dual buffers)
  HIP_TRY(hipMemsetAsync(p->yv[0], 0, yb, st));
  HIP_TRY(hipMemsetAsync(p->yv[1], 0, yb, st));
  p->yv_cur = 0;
  return MERBIT_OK;
}

// Tile ranges and their hot sets.  The grid is sized for one block per CU
// with the largest cache (cap_req > 0: that many values), rounded to a
// multiple of the XCD count, and the tiles are cut into that many contiguous
// ranges; each range takes the (at most cap) most frequent columns of its own
// nonzeros (counted on every 4th nonzero of a long range), ties by
// increasing column, in slots of increasing column.  The ranges first get
// equal tile counts; with a cache they are then re-cut so that every range
// carries the same estimated cost, tiles plus the gathers its cache does not
// serve (kColdWeight tiles per gather: a range whose columns are less
// concentrated gets fewer tiles), and the hot sets are chosen again for the
// new ranges.  The weights were swept on R-MAT 22 at the tuned
// configurations (512-lane blocks, 64-bit descriptors, 8 stripes; us per
// SpMV): FP32 sigma 32 at 0 / 1/3072 / 1/2048 / 1/1536 / 1/1024 / 1/768 /
// 1/384 / 1/192: 227 / 220 / 218 / 217 / 220 / 224 / 229 / 236; FP64 sigma 20
// at 0 / 1/3072 / 1/1536 / 1/768 / 1/384: 306 / 302 / 299 / 297 / 301.
// (Per-wavefront end stamps at 1/384 in FP32: the ranges' wavefronts ended
// 168 to 207 us, on average per range, into a 212 us launch, the ranges
// given the most tiles last.)  The cache is dropped when cap_req < 0 and the
// hot columns hold under 20 % of the nonzeros.
constexpr double kColdWeightF32 = 1.0 / 1536.0, kColdWeightF64 = 1.0 / 768.0;

static int build_range_hot(merbit_plan* p, int cap_req, hipStream_t st, Arena& tmp) {
  const size_t vs = vsize(p->dtype);
  const int64_t cap_lds = hot_cap_lds(p);
  int64_t cap = cap_req > 0 ? cap_req : (cap_req < 0 ? cap_lds : 0);
  if (cap > cap_lds) return fail(MERBIT_EUNSUPPORTED, "hot_columns exceeds the LDS budget");
  if (cap > p->n_cols) cap = p->n_cols;
  if (cap > 0 && !spmv_wave_supported(p->dtype, p->sigma, p->waves, true, p->desc_bits == 64)) {
    if (cap_req > 0) return fail(MERBIT_EUNSUPPORTED, "hot cache not built for this block size");
    cap = 0;
  }
  p->hot_lds_bytes = (size_t)cap * vs;  // for the grid size
  int rc = size_grid(p);
  if (rc != MERBIT_OK) return rc;
  const int R = p->ranges;
  std::vector<int32_t> rt(R + 1), spans(R + 1), hoff(R + 1, 0);
  std::vector<double> cov(R, 0.0);
  for (int k = 0; k <= R; ++k) rt[k] = (int32_t)(p->tile_num * k / R);
  // the stacked matrix is built: its temporaries are dead
  tmp.reset();
  int32_t* peek_buf = nullptr;
  int32_t* stage = nullptr;  // each range's hot columns at k * cap, before packing
  HotSel* sel_dev = nullptr;
  HIP_TRY(tmp.get(&peek_buf, (size_t)kMaxPeek));
  if (cap > 0) {
    HIP_TRY(tmp.get(&stage, (size_t)(cap * R)));
    HIP_TRY(tmp.get(&sel_dev, (size_t)R));
  }
  // spans[k] = first nonzero of range k (the x coordinate of its first tile)
  auto read_spans = [&]() -> int {
    std::vector<int64_t> idx(rt.begin(), rt.end());
    return peek(p->tile_x, idx, peek_buf, spans.data(), st);
  };
  rc = read_spans();
  if (rc != MERBIT_OK) return rc;
  int64_t taken_max = 0;
  if (cap > 0) {
    const int64_t nc = p->n_cols;
    unsigned char* work = nullptr;  // the selection's work space, a new part when a cut needs more
    size_t work_bytes = 0;
    HIP_TRY(hipMalloc(&p->hot_cols, sizeof(int32_t) * (size_t)(cap * R)));
    HIP_TRY(hipMalloc(&p->colx, sizeof(int32_t) * (size_t)p->nnz));
    std::vector<HotSel> sel((size_t)R);
    std::vector<HotSeg> segs((size_t)R);
    // hot sets of the current ranges: hoff, cov (hot nonzeros per range).
    // The stripes of a range's first and last nonzero bound its columns (the
    // stacked stream is stripe-major): counts, selection and the slot map
    // cover that span only.  All ranges are selected, recoded and packed by
    // the same launches; one copy brings back what the host needs.
    auto select = [&](bool final_cut) -> int {
      taken_max = 0;
      // the first and last column of every non-empty range
      std::vector<int64_t> idx;
      for (int k = 0; k < R; ++k)
        if (spans[k] < spans[k + 1]) {
          idx.push_back(spans[k]);
          idx.push_back(spans[k + 1] - 1);
        }
      std::vector<int32_t> got(idx.size()), ends(2 * (size_t)R, 0);
      int rc2 = peek(p->scol, idx, peek_buf, got.data(), st);
      if (rc2 != MERBIT_OK) return rc2;
      for (int k = 0, j = 0; k < R; ++k)
        if (spans[k] < spans[k + 1]) {
          ends[2 * k] = got[j++];
          ends[2 * k + 1] = got[j++];
        }
      const int sh = p->stripe_shift;
      for (int k = 0; k < R; ++k) {
        HotSeg& g = segs[k];
        g = HotSeg{};
        g.lo = spans[k];
        g.len = (int64_t)spans[k + 1] - spans[k];
        g.c_lo = g.len > 0 ? (ends[2 * k] >> sh) << sh : 0;
        const int64_t c_hi = std::min((int64_t)((ends[2 * k + 1] >> sh) + 1) << sh, nc);
        g.span = g.len > 0 ? c_hi - g.c_lo : 1;
        // a 1-in-4 sample of a long range: the hot columns' counts are in
        // the hundreds.  A cut that is re-cut afterwards only estimates each
        // range's hot share for the new cut: 1 in 16 there
        g.sample = g.len > 64 * cap ? (final_cut ? 4 : 16) : 1;
      }
      const size_t need = hot_select_layout(segs.data(), R);
      if (need > work_bytes) {
        HIP_TRY(tmp.get(&work, need));
        work_bytes = need;
      }
      HIP_TRY(hot_select_ranges(p->scol, segs.data(), R, cap, false, work, stage, sel_dev, st));
      if (final_cut) HIP_TRY(hot_recode_ranges(p->scol, segs.data(), R, work, p->colx, st));
      HIP_TRY(hot_pack_ranges(stage, cap, sel_dev, R, p->hot_cols, st));
      HIP_TRY(hipMemcpyAsync(sel.data(), sel_dev, sizeof(HotSel) * (size_t)R,
                             hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      for (int k = 0; k < R; ++k) {
        const int64_t len = segs[k].len;
        const int64_t taken = sel[k].taken;
        const double covered = sel[k].covered;
        cov[k] = segs[k].sample > 1 ? std::min(segs[k].sample * covered, (double)len) : covered;
        hoff[k + 1] = hoff[k] + (int32_t)taken;  // range k's columns at hoff[k]
        taken_max = std::max(taken_max, taken);
      }
      return MERBIT_OK;
    };
    // the column stream is recoded for the final ranges only
    rc = select(R == 1);
    if (rc != MERBIT_OK) return rc;
    if (R > 1) {
      // equal estimated cost per range: the cost is spread evenly over the
      // tiles of each old range, and the new cuts invert its running sum
      std::vector<double> acc(R + 1, 0.0);
      const double kColdWeight = p->dtype == MERBIT_F64 ? kColdWeightF64 : kColdWeightF32;
      for (int k = 0; k < R; ++k) {
        const double cold = (double)(spans[k + 1] - spans[k]) - cov[k];
        acc[k + 1] = acc[k] + (double)(rt[k + 1] - rt[k]) + kColdWeight * cold;
      }
      std::vector<int32_t> cut(R + 1);
      cut[0] = 0;
      cut[R] = (int32_t)p->tile_num;
      int k = 0;
      for (int q = 1; q < R; ++q) {
        const double target = acc[R] * q / R;
        while (k < R - 1 && acc[k + 1] < target) ++k;
        const double span = acc[k + 1] - acc[k];
        const double f = span > 0.0 ? (target - acc[k]) / span : 0.0;
        int32_t c = rt[k] + (int32_t)(f * (double)(rt[k + 1] - rt[k]) + 0.5);
        cut[q] = std::max(cut[q - 1], std::min(c, (int32_t)p->tile_num));
      }
      rt = cut;
      rc = read_spans();
      if (rc == MERBIT_OK) rc = select(true);
      if (rc != MERBIT_OK) return rc;
    }
    double covered = 0.0;
    for (int k = 0; k < R; ++k) covered += cov[k];
    p->hot_coverage = p->nnz > 0 ? covered / (double)p->nnz : 0.0;
    if (cap_req < 0 && p->hot_coverage < 0.2) {
      (void)hipFree(p->hot_cols);
      (void)hipFree(p->colx);
      p->hot_cols = nullptr;
      p->colx = nullptr;
      std::fill(hoff.begin(), hoff.end(), 0);
      taken_max = 0;
    }
  }
  HIP_TRY(hipMalloc(&p->range_tile, sizeof(int32_t) * (size_t)(R + 1)));
  HIP_TRY(hipMemcpyAsync(p->range_tile, rt.data(), sizeof(int32_t) * (size_t)(R + 1),
                         hipMemcpyHostToDevice, st));
  HIP_TRY(hipMalloc(&p->hot_off, sizeof(int32_t) * (size_t)(R + 1)));
  HIP_TRY(hipMemcpyAsync(p->hot_off, hoff.data(), sizeof(int32_t) * (size_t)(R + 1),
                         hipMemcpyHostToDevice, st));
  p->hot_n = hoff[R];
  p->hot_lds_bytes = (size_t)taken_max * vs;
  if (p->hot_n > 0) {
    HIP_TRY(hipMalloc(&p->x_hot, vs * (size_t)p->hot_n));
    HIP_TRY(spmv_wave_set_hot_lds(p->dtype, p->sigma, p->waves, p->hot_lds_bytes,
                                  p->desc_bits == 64));
  } else {
    p->hot_coverage = 0.0;
  }
  // the grid for the LDS actually used (it stays a multiple of the ranges)
  const int ranges = p->ranges;
  rc = size_grid(p);
  if (rc != MERBIT_OK) return rc;
  if (p->ranges != ranges) return fail(MERBIT_EHIP, "column stripes: range count changed");
  HIP_TRY(hipStreamSynchronize(st));  // host vectors above are read by queued copies
  return MERBIT_OK;
}

int build_striped(merbit_plan* p, const int32_t* row_ptr, int hot_columns, hipStream_t st) {
  Arena tmp;
  int rc = build_stripes(p, row_ptr, st, tmp);
  if (rc == MERBIT_OK) rc = build_range_hot(p, hot_columns, st, tmp);
  // the temporaries are freed on return: finish the work that reads them
  const hipError_t e = hipStreamSynchronize(st);
  if (rc == MERBIT_OK && e != hipSuccess) rc = fail_hip("column-stripe plan build", e);
  return rc;
}

}  // namespace merbit
