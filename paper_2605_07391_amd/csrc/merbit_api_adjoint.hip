// C ABI of libmerbit, adjoint pieces: the transpose with its permutation,
// per-nonzero products, gathers and column scaling.
#include <math.h>
#include <string.h>

#include "merbit_host.hpp"

using namespace merbit;

extern "C" {

// ------------------------------------------------------------- adjoint --

static TileRowsArgs tile_rows_args(const merbit_plan* p) {
  TileRowsArgs a;
  memset(&a, 0, sizeof a);
  a.tile_x = p->tile_x;
  a.tile_y = p->tile_y;
  a.lane_desc = p->lane_desc;
  a.tile_num = (int32_t)p->tile_num;
  a.lane_num = (int32_t)p->lane_num;
  a.path_len = (int32_t)(p->nnz + p->n_rows);
  a.col = p->col;
  return a;
}

int merbit_transpose(merbit_plan* p, int32_t* rowT_ptr, int32_t* colT, int32_t* perm,
                     void* stream) try {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->stripes > 1) return fail(MERBIT_EUNSUPPORTED, "not available on a striped plan");
  if (p->desc_bits != 32)
    return fail(MERBIT_EUNSUPPORTED, "this call needs a plan with 32-bit descriptors");
  if (!rowT_ptr || (p->nnz > 0 && (!colT || !perm)))
    return fail(MERBIT_EINVAL, "output array is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t m = p->nnz;
  int end_bit = 1;
  while (end_bit < 31 && ((int64_t)1 << end_bit) < p->n_cols) ++end_bit;
  int32_t* rows = nullptr;
  void* tmp = nullptr;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    if (rows) (void)hipFree(rows);
    if (tmp) (void)hipFree(tmp);
  };
  hipError_t e = hipSuccess;
  const size_t mm = (size_t)(m > 0 ? m : 1);
  if (e == hipSuccess) e = hipMalloc(&rows, sizeof(int32_t) * mm);
  if (e == hipSuccess) e = hipMalloc(&tmp, transpose_temp_bytes(m, end_bit));
  if (e == hipSuccess && m > 0) {
    TileRowsArgs a = tile_rows_args(p);
    a.rows = rows;
    e = launch_tile_rows(p->dtype, p->sigma, false, a, st);
  }
  if (e == hipSuccess)
    e = launch_transpose(p->col, rows, m, p->n_cols, end_bit, tmp, rowT_ptr, colT, perm, st);
  cleanup();
  if (e != hipSuccess) return fail_hip("transpose", e);
  p->last_stream = st;
  return MERBIT_OK;
} catch (...) {
  return merbit::host_exception();
}

int merbit_sddmm(merbit_plan* p, const void* g, const void* x, double scale, void* out,
                 void* stream) try {
  if (!p) return fail(MERBIT_EINVAL, "plan is NULL");
  if (p->stripes > 1) return fail(MERBIT_EUNSUPPORTED, "not available on a striped plan");
  if (p->desc_bits != 32)
    return fail(MERBIT_EUNSUPPORTED, "this call needs a plan with 32-bit descriptors");
  if (p->nnz == 0) return MERBIT_OK;
  if (!g || !x || !out) return fail(MERBIT_EINVAL, "g, x or out is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  TileRowsArgs a = tile_rows_args(p);
  a.g = g;
  a.x = x;
  a.scale = scale;
  a.out = out;
  HIP_TRY(launch_tile_rows(p->dtype, p->sigma, true, a, st));
  p->last_stream = st;
  return MERBIT_OK;
} catch (...) {
  return merbit::host_exception();
}

int merbit_gather_values(int dtype, int64_t nnz, const int32_t* perm, const void* src,
                         const void* src2, void* dst, void* stream) try {
  if (dtype != MERBIT_F32 && dtype != MERBIT_F64) return fail(MERBIT_EUNSUPPORTED, "dtype");
  if (nnz < 0) return fail(MERBIT_EINVAL, "nnz < 0");
  if (nnz == 0) return MERBIT_OK;
  if (!perm || !src || !dst) return fail(MERBIT_EINVAL, "perm, src or dst is NULL");
  if (dst == src || (src2 && dst == src2)) return fail(MERBIT_EINVAL, "dst aliases an input");
  HIP_TRY(launch_gather_values(dtype, perm, src, src2, dst, nnz, static_cast<hipStream_t>(stream)));
  return MERBIT_OK;
} catch (...) {
  return merbit::host_exception();
}

int merbit_column_scale(int dtype, int64_t nnz, const int32_t* col, const void* a, const void* t,
                        const void* s, void* out, void* stream) try {
  if (dtype != MERBIT_F32 && dtype != MERBIT_F64) return fail(MERBIT_EUNSUPPORTED, "dtype");
  if (nnz < 0) return fail(MERBIT_EINVAL, "nnz < 0");
  if (nnz == 0) return MERBIT_OK;
  if (!col || !a || !s || !out) return fail(MERBIT_EINVAL, "col, a, s or out is NULL");
  HIP_TRY(launch_column_scale(dtype, col, a, t, s, out, nnz, static_cast<hipStream_t>(stream)));
  return MERBIT_OK;
} catch (...) {
  return merbit::host_exception();
}

}  // extern "C"
