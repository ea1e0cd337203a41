// ACA + Tucker products.  The coupling matrix is held as Z ~= U V^* (cross
// approximation, Sec. II.B.2) with the r_c columns of U compressed as the
// plan's Tucker tensors.  Sec. III.B gives the substitution: Algorithm 1 on U
// with X replaced by V^* X yields Z X, and Algorithm 2 on U followed by V
// yields Z^* Y (Table III, row ACA+Tucker).  The Tucker products are the
// plan's fused kernels; the two coil-side products here are O(r_c m p),
// HBM-bound, and accumulate in FP64 in a fixed order (deterministic).
#include <cstdio>

#include "tv_internal.h"

namespace tv {
namespace {

constexpr int kThreads = 256;

// W[r + rc*c] = sum_j conj(V[j + ldv*r]) X[j + ldx*c].  One workgroup per
// (r, c): strided FP64 partial sums per lane (coalesced along j), a wave
// butterfly, then the four wave sums in order.
__global__ __launch_bounds__(kThreads) void aca_vhx_kernel(const float2* __restrict__ V,
                                                            int64_t m, int64_t ldv,
                                                            const float2* __restrict__ X,
                                                            int64_t ldx, float2* __restrict__ W,
                                                            int64_t rc) {
  const int64_t r = blockIdx.x, c = blockIdx.y;
  const float2* v = V + r * ldv;
  const float2* x = X + c * ldx;
  double sr = 0.0, si = 0.0;
  for (int64_t j = threadIdx.x; j < m; j += kThreads) {
    const float2 a = v[j], b = x[j];
    sr += (double)a.x * b.x + (double)a.y * b.y;
    si += (double)a.x * b.y - (double)a.y * b.x;
  }
  for (int off = 32; off >= 1; off >>= 1) {
    sr += __shfl_xor(sr, off);
    si += __shfl_xor(si, off);
  }
  __shared__ double red[2][kThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = sr;
    red[1][wave] = si;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tr = 0.0, ti = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) {
      tr += red[0][w];
      ti += red[1][w];
    }
    W[r + rc * c] = make_float2((float)tr, (float)ti);
  }
}

// X[j + ldx*c] = sum_r V[j + ldv*r] W[r + rc*c].  One lane per row j (loads
// of V coalesced along j), terms in the order of r.
__global__ __launch_bounds__(kThreads) void aca_vw_kernel(const float2* __restrict__ V, int64_t m,
                                                           int64_t ldv,
                                                           const float2* __restrict__ W,
                                                           int64_t rc, float2* __restrict__ X,
                                                           int64_t ldx) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (j >= m) return;
  const float2* w = W + rc * blockIdx.y;
  double sr = 0.0, si = 0.0;
  for (int64_t r = 0; r < rc; ++r) {
    const float2 a = V[j + ldv * r], b = w[r];
    sr += (double)a.x * b.x - (double)a.y * b.y;
    si += (double)a.x * b.y + (double)a.y * b.x;
  }
  X[j + ldx * blockIdx.y] = make_float2((float)sr, (float)si);
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

bool overlaps(const void* a, size_t alen, const void* b, size_t blen) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + blen && pb < pa + alen;
}

// Host-side validation shared by both directions: `in` (rows_in x nrhs) is
// read, `out` (rows_out x nrhs) written.
tv_status aca_check(tv_plan p, const void* v, int64_t m, int64_t ldv, const void* in,
                    int64_t ldin, int64_t rows_in, int32_t nrhs, const void* out, int64_t ldout,
                    int64_t rows_out, int op, const void* ws, size_t ws_bytes) {
  if (!p) return set_error(TV_ERR_INVALID_ARG, "plan is NULL");
  if (!p->finalized) return set_error(TV_ERR_INVALID_ARG, "plan is not finalized");
  if (!p->bound) return set_error(TV_ERR_INVALID_ARG, "plan has no device arena (tv_plan_bind_arena)");
  if (!v || !in || !out) return set_error(TV_ERR_INVALID_ARG, "V and vectors must be non-NULL");
  if (m < 1 || m > ((int64_t)1 << 31)) return set_error(TV_ERR_SHAPE, "m must be in [1, 2^31]");
  if (ldv < m) return set_error(TV_ERR_SHAPE, "ldv smaller than m");
  if (nrhs < 1 || nrhs > 65535)
    return set_error(TV_ERR_INVALID_ARG, "nrhs must be in [1, 65535]");
  if (ldin < rows_in || ldout < rows_out)
    return set_error(TV_ERR_SHAPE, "leading dimension smaller than the number of rows");
  if (((uintptr_t)v | (uintptr_t)in | (uintptr_t)out) % 8)
    return set_error(TV_ERR_INVALID_ARG, "complex64 arrays must be 8-byte aligned");
  const int64_t rc = p->grid.m;
  const size_t in_len = 8 * (size_t)(ldin * (nrhs - 1) + rows_in);
  const size_t out_len = 8 * (size_t)(ldout * (nrhs - 1) + rows_out);
  const size_t v_len = 8 * (size_t)(ldv * (rc - 1) + m);
  if (overlaps(in, in_len, out, out_len)) return set_error(TV_ERR_INVALID_ARG, "input and output overlap");
  if (overlaps(v, v_len, out, out_len)) return set_error(TV_ERR_INVALID_ARG, "V and output overlap");
  size_t need = 0;
  tv_status st = tv_aca_workspace_bytes(p, op, nrhs, &need);
  if (st != TV_OK) return st;
  if (!ws || ws_bytes < need) {
    char buf[128];
    snprintf(buf, sizeof buf, "workspace of %zu bytes needed, %zu given", need,
             ws ? ws_bytes : (size_t)0);
    return set_error(TV_ERR_WORKSPACE, buf);
  }
  if ((uintptr_t)ws % 16) return set_error(TV_ERR_INVALID_ARG, "workspace alignment");
  if (overlaps(ws, need, out, out_len) || overlaps(ws, need, in, in_len) ||
      overlaps(ws, need, v, v_len))
    return set_error(TV_ERR_INVALID_ARG, "workspace overlaps an operand");
  return TV_OK;
}

}  // namespace
}  // namespace tv

using namespace tv;

extern "C" {

tv_status tv_aca_workspace_bytes(tv_plan p, int32_t op, int32_t nrhs, size_t* bytes) {
  clear_error();
  if (!p || !bytes) return set_error(TV_ERR_INVALID_ARG, "plan and bytes must be non-NULL");
  size_t inner = 0;
  tv_status st = tv_workspace_bytes(p, op, nrhs, &inner);
  if (st != TV_OK) return st;
  *bytes = align256((size_t)8 * p->grid.m * nrhs) + inner;
  return TV_OK;
}

tv_status tv_aca_matvec(tv_plan p, const void* v, int64_t m, int64_t ldv, const void* x,
                        int64_t ldx, int32_t nrhs, void* y, int64_t ldy, void* ws,
                        size_t ws_bytes, void* stream) {
  clear_error();
  if (!p) return set_error(TV_ERR_INVALID_ARG, "plan is NULL");
  const int64_t rows = (int64_t)p->grid.q * p->grid.n1 * p->grid.n2 * p->grid.n3;
  tv_status st = aca_check(p, v, m, ldv, x, ldx, m, nrhs, y, ldy, rows, 0, ws, ws_bytes);
  if (st != TV_OK) return st;
  const int64_t rc = p->grid.m;
  const size_t off = align256((size_t)8 * rc * nrhs);
  float2* W = (float2*)ws;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(aca_vhx_kernel, dim3((unsigned)rc, (unsigned)nrhs), dim3(kThreads), 0, s,
                     (const float2*)v, m, ldv, (const float2*)x, ldx, W, rc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "ACA V^* X launch");
  return tv_matvec(p, W, rc, nrhs, y, ldy, (char*)ws + off, ws_bytes - off, stream);
}

tv_status tv_aca_rmatvec(tv_plan p, const void* v, int64_t m, int64_t ldv, const void* y,
                         int64_t ldy, int32_t nrhs, void* x, int64_t ldx, void* ws,
                         size_t ws_bytes, void* stream) {
  clear_error();
  if (!p) return set_error(TV_ERR_INVALID_ARG, "plan is NULL");
  const int64_t rows = (int64_t)p->grid.q * p->grid.n1 * p->grid.n2 * p->grid.n3;
  tv_status st = aca_check(p, v, m, ldv, y, ldy, rows, nrhs, x, ldx, m, 1, ws, ws_bytes);
  if (st != TV_OK) return st;
  const int64_t rc = p->grid.m;
  const size_t off = align256((size_t)8 * rc * nrhs);
  float2* W = (float2*)ws;
  st = tv_rmatvec(p, y, ldy, nrhs, W, rc, (char*)ws + off, ws_bytes - off, stream);
  if (st != TV_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t blocks = (m + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(aca_vw_kernel, dim3((unsigned)blocks, (unsigned)nrhs), dim3(kThreads), 0, s,
                     (const float2*)v, m, ldv, (const float2*)W, rc, (float2*)x, ldx);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TV_OK : hip_error(e, "ACA V W launch");
}

}  // extern "C"
