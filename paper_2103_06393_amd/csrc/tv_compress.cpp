// Truncated-HOSVD compression (Sec. II.B.1): host orchestration.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "tv_internal.h"

using namespace tv;

extern "C" {

tv_status tv_compress_begin(const tv_grid* grid, double tol, int32_t rank_min, int32_t rank_cap,
                            tv_precision precision, tv_plan* out) {
  clear_error();
  if (!out) return set_error(TV_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!grid) return set_error(TV_ERR_INVALID_ARG, "grid is NULL");
  if (grid->n1 < 1 || grid->n2 < 1 || grid->n3 < 1 || grid->q < 1 || grid->m < 1)
    return set_error(TV_ERR_SHAPE, "grid sizes must be >= 1");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return set_error(TV_ERR_INVALID_ARG, "tol must be >= 0");
  if (rank_min < 1 || rank_min > TV_MAX_RANK)
    return set_error(TV_ERR_RANK, "rank_min outside [1, TV_MAX_RANK]");
  if (rank_cap > 0 && rank_cap < rank_min) return set_error(TV_ERR_RANK, "rank_cap < rank_min");
  if (precision != TV_PREC_FP32 && precision != TV_PREC_BF16X3)
    return set_error(TV_ERR_INVALID_ARG, "unknown precision");
  tv_plan_s* p = new (std::nothrow) tv_plan_s;
  if (!p) return set_error(TV_ERR_OOM, "host allocation");
  p->grid = *grid;
  p->precision = precision;
  p->tol = tol;
  p->rank_min = rank_min;
  p->rank_cap = rank_cap;
  p->appended = 0;
  *out = p;
  return TV_OK;
}

tv_status tv_compress_append(tv_plan p, const void* cols, int64_t ncols, void* stream) {
  clear_error();
  (void)cols;
  (void)ncols;
  (void)stream;
  if (!p) return set_error(TV_ERR_INVALID_ARG, "plan is NULL");
  return set_error(TV_ERR_NOT_SUPPORTED, "device compression is not built yet");
}

tv_status tv_plan_finalize(tv_plan p, void* stream) {
  clear_error();
  (void)stream;
  if (!p) return set_error(TV_ERR_INVALID_ARG, "plan is NULL");
  if (p->appended != p->grid.m)
    return set_error(TV_ERR_INVALID_ARG, "not all columns have been appended");
  return set_error(TV_ERR_NOT_SUPPORTED, "device compression is not built yet");
}

tv_status tv_compress_discarded(tv_plan p, double* rel) {
  clear_error();
  if (!p || !rel) return set_error(TV_ERR_INVALID_ARG, "plan and output must be non-NULL");
  const size_t n = (size_t)3 * p->grid.q * p->appended;
  if (p->rel_discarded.size() < n) return set_error(TV_ERR_INVALID_ARG, "no compression data");
  std::memcpy(rel, p->rel_discarded.data(), n * sizeof(double));
  return TV_OK;
}

}  // extern "C"
