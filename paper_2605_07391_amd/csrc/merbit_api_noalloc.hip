// C ABI of libmerbit: PageRank that allocates nothing, for callers that cannot
// allocate device memory (code under HIP graph capture set-up, serving loops,
// harnesses that forbid hipMalloc).  Same iteration and kernels as
// merbit_pagerank; its work buffers (the SpMV's dual output buffers, the
// second iterate, the per-block reduction pairs and, when the plan has none
// yet, the dangling mask) live in one file-scope device array instead of
// plan-owned allocations.
//
// Each GPU the library runs on holds its own copy of the array until the
// process ends.  Host code never passes the array's name to a kernel or copy:
// the name is a host-side stand-in, not a device address.  The device address
// is looked up once per device with that device current and kept.
#include <stdio.h>

#include <mutex>

#include "merbit_host.hpp"

static __device__ __align__(256) unsigned char scratch[MERBIT_NOALLOC_SCRATCH_BYTES];

namespace merbit {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device.
int scratch_address(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return fail(MERBIT_EUNSUPPORTED, "device index too large");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip("hipGetSymbolAddress(scratch)", e);
    if (!ptr) return fail(MERBIT_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[device] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
  return MERBIT_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace
}  // namespace merbit

using namespace merbit;

extern "C" {

int merbit_pagerank_noalloc(merbit_plan* p, double alpha, double tol, int max_iter,
                            int check_every, void* x_inout, int* iters_out, double* resid_out,
                            void* stream) try {
  if (iters_out) *iters_out = 0;
  if (resid_out) *resid_out = 0.0;
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->n_rows != p->n_cols) return fail(MERBIT_EINVAL, "PageRank needs a square matrix");
  if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(MERBIT_EINVAL, "alpha must be in [0, 1]");
  if (max_iter < 0) return fail(MERBIT_EINVAL, "max_iter < 0");
  if (p->n_rows == 0 || max_iter == 0) return MERBIT_OK;
  if (!x_inout) return fail(MERBIT_EINVAL, "x is NULL");
  int device = -1;
  HIP_TRY(hipGetDevice(&device));
  if (device != p->device)
    return fail(MERBIT_EINVAL, "merbit_pagerank_noalloc: the plan's device must be current");

  // layout of the work buffers in the array (256-byte aligned pieces)
  const int64_t n = p->n_rows;
  const int rg = pr_reduce_grid(n);
  constexpr int kMaxReduceGrid = 1024;  // the bound pr_reduce_grid() keeps
  if (rg > kMaxReduceGrid) return fail(MERBIT_EHIP, "reduction grid larger than expected");
  const size_t vec = align256(vsize(p->dtype) * (size_t)n);
  const size_t pairs = align256(2 * sizeof(double) * (size_t)rg);
  const bool own_mask = p->dmask == nullptr;
  const size_t mask = own_mask ? align256(sizeof(uint32_t) * (size_t)((p->n_cols + 31) / 32 + 1))
                               : 0;
  const size_t bytes = own_mask ? align256((size_t)p->n_cols) : 0;
  const size_t need = 3 * vec + 2 * pairs + mask + bytes;
  if (need > MERBIT_NOALLOC_SCRATCH_BYTES) {
    char msg[200];
    snprintf(msg, sizeof msg,
             "merbit_pagerank_noalloc: n = %lld needs %zu bytes of work space, more than the "
             "library's %zu",
             (long long)n, need, (size_t)MERBIT_NOALLOC_SCRATCH_BYTES);
    return fail(MERBIT_EINVAL, msg);
  }
  unsigned char* base = nullptr;
  int rc = scratch_address(device, &base);
  if (rc != MERBIT_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);

  PageRankWork w;
  size_t off = 0;
  w.ybuf[0] = base + off;
  off += vec;
  w.ybuf[1] = base + off;
  off += vec;
  w.xwork = base + off;
  off += vec;
  w.partials[0] = reinterpret_cast<double*>(base + off);
  off += pairs;
  w.partials[1] = reinterpret_cast<double*>(base + off);
  off += pairs;
  if (own_mask) {
    uint32_t* dm = reinterpret_cast<uint32_t*>(base + off);
    HIP_TRY(launch_dangling_mask(p->col, p->nnz, p->n_cols, base + off + mask, dm, st));
    w.dmask = dm;
  } else {
    w.dmask = p->dmask;
  }
  w.reduce_grid = rg;
  w.zeroed_buf = -1;  // the array holds whatever the last call left: zero the boundary rows
  w.graphs = false;   // instantiating a graph allocates
  w.timed = false;    // creating timing events allocates
  double host_pairs[2 * kMaxReduceGrid];
  w.host_pairs = host_pairs;
  return pagerank_loop(p, w, alpha, tol, max_iter, check_every, x_inout, iters_out, resid_out,
                       st);
} catch (...) {
  return merbit::host_exception();
}

}  // extern "C"
