// C ABI of libmerbit, autotuner: per-matrix sweep of sigma and block size.
#include <math.h>
#include <string.h>

#include "merbit_host.hpp"

using namespace merbit;

extern "C" {

// Autotuner: one plan per (sigma, block size) candidate, each timed over
// `reps` dual-buffer SpMV launches (the PageRank regime) after two warm-up
// launches; x is a constant nonzero vector.  Candidates the kernels do not
// build are reported as -1 and skipped.
int merbit_tune(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t* row_ptr,
                const int32_t* col_ind, const void* values, int dtype, const int32_t* sigmas,
                int n_sigmas, const int32_t* block_lanes, int n_blocks, int reps,
                merbit_opts_t* opts_inout, float* us_out, void* stream) try {
  if (!opts_inout) return fail(MERBIT_EINVAL, "opts is NULL");
  if (dtype != MERBIT_F32 && dtype != MERBIT_F64) return fail(MERBIT_EUNSUPPORTED, "dtype");
  if (reps < 1) return fail(MERBIT_EINVAL, "reps < 1");
  static const int32_t def_sigma_f32[] = {7, 8, 9, 10, 11, 12};
  static const int32_t def_sigma_f64[] = {4, 5, 6, 7, 8, 9, 10};
  static const int32_t def_blocks[] = {256, 512, 1024};
  if (!sigmas || n_sigmas <= 0) {
    sigmas = dtype == MERBIT_F32 ? def_sigma_f32 : def_sigma_f64;
    n_sigmas = dtype == MERBIT_F32 ? 6 : 7;
  }
  if (!block_lanes || n_blocks <= 0) {
    block_lanes = def_blocks;
    n_blocks = 3;
  }
  const int rhs = opts_inout->tune_rhs;
  if (rhs < 0 || rhs > 64) return fail(MERBIT_EINVAL, "tune_rhs must be in 0..64");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t vs = vsize(dtype);
  const size_t width = rhs > 0 ? (size_t)rhs : 1;  // values per row of x / y
  void *x = nullptr, *y0 = nullptr, *y1 = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (x) (void)hipFree(x);
    if (y0) (void)hipFree(y0);
    if (y1) (void)hipFree(y1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
#define TUNE_TRY(expr)                          \
  do {                                          \
    hipError_t _e = (expr);                     \
    if (_e != hipSuccess) {                     \
      cleanup();                                \
      return fail_hip(#expr, _e);               \
    }                                           \
  } while (0)
  TUNE_TRY(hipMalloc(&x, vs * width * (size_t)(n_cols > 0 ? n_cols : 1)));
  TUNE_TRY(hipMalloc(&y0, vs * width * (size_t)(n_rows > 0 ? n_rows : 1)));
  TUNE_TRY(hipMalloc(&y1, vs * width * (size_t)(n_rows > 0 ? n_rows : 1)));
  // x = 1.0f (F32) or the double with two 1.0f words (about 1.0000002, F64)
  TUNE_TRY(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(x), 0x3f800000u,
                             (vs / 4) * width * (size_t)(n_cols > 0 ? n_cols : 1), st));
  TUNE_TRY(hipEventCreate(&e0));
  TUNE_TRY(hipEventCreate(&e1));
  float best = -1.0f;
  int best_sigma = 0, best_b = 0;
  for (int i = 0; i < n_sigmas; ++i) {
    for (int j = 0; j < n_blocks; ++j) {
      if (us_out) us_out[i * n_blocks + j] = -1.0f;
      merbit_opts_t o = *opts_inout;
      o.sigma = sigmas[i];
      o.block_lanes = block_lanes[j];
      o.validate = 0;
      merbit_plan* p = nullptr;
      const int rc = merbit_plan_create(n_rows, n_cols, nnz, row_ptr, col_ind, values, dtype, &o,
                                        stream, &p);
      if (rc == MERBIT_EUNSUPPORTED) continue;
      if (rc != MERBIT_OK) {
        cleanup();
        return rc;
      }
      int r2 = rhs > 0 ? MERBIT_OK : merbit_zero_boundary(p, y0, stream);
      void* ys[2] = {y0, y1};
      for (int k = 0; r2 == MERBIT_OK && k < 2 + reps; ++k) {
        if (k == 2) {
          hipError_t e = hipEventRecord(e0, st);
          if (e != hipSuccess) r2 = fail_hip("hipEventRecord", e);
        }
        if (r2 != MERBIT_OK) break;
        r2 = rhs > 0 ? merbit_spmm(p, x, rhs, ys[k & 1], rhs, rhs, stream)
                     : run_fused(p, x, ys[k & 1], ys[(k + 1) & 1], st);
      }
      float ms = 0.0f;
      if (r2 == MERBIT_OK) {
        hipError_t e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) r2 = fail_hip("tune timing", e);
      }
      plan_free_all(p);
      if (r2 != MERBIT_OK) {
        cleanup();
        return r2;
      }
      const float us = ms * 1000.0f / (float)reps;
      if (us_out) us_out[i * n_blocks + j] = us;
      if (best < 0.0f || us < best) {
        best = us;
        best_sigma = sigmas[i];
        best_b = block_lanes[j];
      }
    }
  }
#undef TUNE_TRY
  cleanup();
  if (best < 0.0f) return fail(MERBIT_EUNSUPPORTED, "no candidate is built");
  opts_inout->sigma = best_sigma;
  opts_inout->block_lanes = best_b;
  return MERBIT_OK;
} catch (...) {
  return merbit::host_exception();
}

}  // extern "C"
