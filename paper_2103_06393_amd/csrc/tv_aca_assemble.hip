// Tucker-based ACA assembly (Algorithm 3, Sec. III.C) on the device.
//
// Adaptive cross approximation with partial pivoting of the point-current
// coupling matrix Z (q nv x m), in which every new column of U is split into
// its q voxel tensors and compressed at once by the truncated HOSVD, so that
// U never exists uncompressed.  Per step: a row of Z (field of every coil
// element at one voxel), minus the same row of U V^* with U's row read by
// single-element decompression (eq. 6); the pivot column j of the largest
// residual; y = conj(r / r_j); the column Z_{:j} minus U V_{j:}^* (the plan's
// forward product, Algorithm 1); the Frobenius-norm estimate, whose cross
// term needs U^* x (the adjoint product, Algorithm 2) and V^* y; the HOSVD of
// the new column; the stopping test; the next pivot row (largest |x| other
// than the current row).  Everything runs in FP64 on the device except the
// two products with U, which use the plan's FP32 (or BF16X3) kernels.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "tv_internal.h"

namespace tv {
namespace {

constexpr int kT = 256;

// Sum of a double over the workgroup in a fixed order (wave butterfly, then
// the four wave sums in order); the result is valid in thread 0.
__device__ double block_sum(double v, double* red) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kT / 64; ++w) t += red[w];
  return t;
}

__device__ inline double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// t[l] = G x1 U1[f1,:] x2 U2[f2,:] x3 U3[f3,:] for tensor (p, l) of a plan
// with mcols columns (single-element decompression); one workgroup per l.
__global__ __launch_bounds__(kT) void entry_kernel(const TensorMeta* __restrict__ meta,
                                                   const float2* __restrict__ cores,
                                                   const float2* __restrict__ u1t,
                                                   const float2* __restrict__ u2t,
                                                   const float2* __restrict__ u3t, int64_t mcols,
                                                   int p, int f1, int f2, int f3,
                                                   double2* __restrict__ t) {
  __shared__ double red[kT / 64];
  const int64_t l = blockIdx.x;
  const TensorMeta M = meta[(int64_t)p * mcols + l];
  const int r1 = M.r1, r2 = M.r2, n = M.r1 * M.r2 * M.r3;
  const float2* G = cores + M.g_off;
  const float2* a1 = u1t + M.u1_off + (int64_t)f1 * r1;
  const float2* a2 = u2t + M.u2_off + (int64_t)f2 * r2;
  const float2* a3 = u3t + M.u3_off + (int64_t)f3 * M.r3;
  double sr = 0.0, si = 0.0;
  for (int e = threadIdx.x; e < n; e += kT) {
    const int a = e % r1, b = (e / r1) % r2, c = e / (r1 * r2);
    const float2 g = G[e], u = a1[a], v = a2[b], w = a3[c];
    double2 z = zmul(make_double2(g.x, g.y), make_double2(u.x, u.y));
    z = zmul(z, make_double2(v.x, v.y));
    z = zmul(z, make_double2(w.x, w.y));
    sr += z.x;
    si += z.y;
  }
  sr = block_sum(sr, red);
  si = block_sum(si, red);
  if (threadIdx.x == 0) t[l] = make_double2(sr, si);
}

// r[n] -= sum_l t[l] conj(V[n + ldv l]), l < k: row i of Z minus row i of
// U V^*.  One lane per n, terms in the order of l.
__global__ __launch_bounds__(kT) void row_update_kernel(double2* __restrict__ r,
                                                        const double2* __restrict__ V, int64_t ldv,
                                                        const double2* __restrict__ t, int64_t m,
                                                        int k) {
  const int64_t n = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (n >= m) return;
  double2 acc = r[n];
  for (int l = 0; l < k; ++l) {
    const double2 v = V[n + ldv * l], a = t[l];
    acc.x -= a.x * v.x + a.y * v.y;  // t conj(v)
    acc.y -= a.y * v.x - a.x * v.y;
  }
  r[n] = acc;
}

// Largest |v|^2 and its index (smallest index among equal values), skipping
// index `skip`: per-workgroup candidates, then one workgroup over them.
__device__ inline bool better(double va, int64_t ia, double vb, int64_t ib) {
  return va > vb || (va == vb && ia < ib);
}

__device__ void block_argmax(double& v, int64_t& i, double* rv, int64_t* ri) {
  for (int off = 32; off >= 1; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int64_t oi = __shfl_xor(i, off);
    if (better(ov, oi, v, i)) {
      v = ov;
      i = oi;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    rv[wave] = v;
    ri[wave] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < kT / 64; ++w)
      if (better(rv[w], ri[w], v, i)) {
        v = rv[w];
        i = ri[w];
      }
}

__global__ __launch_bounds__(kT) void amax1_kernel(const double2* __restrict__ x, int64_t n,
                                                   int64_t skip, double* __restrict__ bv,
                                                   int64_t* __restrict__ bi) {
  __shared__ double rv[kT / 64];
  __shared__ int64_t ri[kT / 64];
  double v = -1.0;
  int64_t i = INT64_MAX;
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT) {
    const double2 z = x[e];
    const double a = e == skip ? -1.0 : z.x * z.x + z.y * z.y;
    if (better(a, e, v, i)) {
      v = a;
      i = e;
    }
  }
  block_argmax(v, i, rv, ri);
  if (threadIdx.x == 0) {
    bv[blockIdx.x] = v;
    bi[blockIdx.x] = i;
  }
}

__global__ __launch_bounds__(kT) void amax2_kernel(const double* __restrict__ bv,
                                                   const int64_t* __restrict__ bi, int nb,
                                                   double* __restrict__ ov,
                                                   int64_t* __restrict__ oi) {
  __shared__ double rv[kT / 64];
  __shared__ int64_t ri[kT / 64];
  double v = -1.0;
  int64_t i = INT64_MAX;
  for (int e = threadIdx.x; e < nb; e += kT)
    if (better(bv[e], bi[e], v, i)) {
      v = bv[e];
      i = bi[e];
    }
  block_argmax(v, i, rv, ri);
  if (threadIdx.x == 0) {
    *ov = v;
    *oi = i;
  }
}

// sum |x|^2: fixed-order partial sums per workgroup, then one workgroup.
__global__ __launch_bounds__(kT) void sumsq1_kernel(const double2* __restrict__ x, int64_t n,
                                                    double* __restrict__ part) {
  __shared__ double red[kT / 64];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT) {
    const double2 z = x[e];
    s += z.x * z.x + z.y * z.y;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kT) void sumsq2_kernel(const double* __restrict__ part, int nb,
                                                    double* __restrict__ out) {
  __shared__ double red[kT / 64];
  double s = 0.0;
  for (int e = threadIdx.x; e < nb; e += kT) s += part[e];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = s;
}

// y[n] = conj(r[n] / r[j])
__global__ __launch_bounds__(kT) void set_y_kernel(const double2* __restrict__ r, int64_t m,
                                                   int64_t j, double2* __restrict__ y) {
  const int64_t n = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (n >= m) return;
  const double2 rj = r[j], rn = r[n];
  const double d = rj.x * rj.x + rj.y * rj.y;
  const double qr = (rn.x * rj.x + rn.y * rj.y) / d, qi = (rn.y * rj.x - rn.x * rj.y) / d;
  y[n] = make_double2(qr, -qi);
}

// w[l] = conj(V[j + ldv l]) in complex64, l < k
__global__ __launch_bounds__(kT) void conj_row_kernel(const double2* __restrict__ V, int64_t ldv,
                                                      int64_t j, int k, float2* __restrict__ w) {
  const int l = blockIdx.x * kT + threadIdx.x;
  if (l >= k) return;
  const double2 v = V[j + ldv * l];
  w[l] = make_float2((float)v.x, (float)-v.y);
}

// x -= u (complex64 product result)
__global__ __launch_bounds__(kT) void sub_kernel(double2* __restrict__ x,
                                                 const float2* __restrict__ u, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (e >= n) return;
  const float2 a = u[e];
  x[e] = make_double2(x[e].x - a.x, x[e].y - a.y);
}

__global__ __launch_bounds__(kT) void to_c64_kernel(const double2* __restrict__ x,
                                                    float2* __restrict__ y, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (e >= n) return;
  y[e] = make_float2((float)x[e].x, (float)x[e].y);
}

// b[l] = sum_n conj(V[n + ldv l]) y[n] (V^* y), one workgroup per l.
__global__ __launch_bounds__(kT) void vhy_kernel(const double2* __restrict__ V, int64_t ldv,
                                                 const double2* __restrict__ y, int64_t m,
                                                 double2* __restrict__ b) {
  __shared__ double red[kT / 64];
  const int64_t l = blockIdx.x;
  double br = 0.0, bi = 0.0;
  for (int64_t n = threadIdx.x; n < m; n += kT) {
    const double2 v = V[n + ldv * l], w = y[n];
    br += v.x * w.x + v.y * w.y;
    bi += v.x * w.y - v.y * w.x;
  }
  br = block_sum(br, red);
  bi = block_sum(bi, red);
  if (threadIdx.x == 0) b[l] = make_double2(br, bi);
}

// out = 2 Re sum_l conj(b_l) a_l (the norm estimate's cross term), one
// workgroup, fixed order.
__global__ __launch_bounds__(kT) void cross_kernel(const double2* __restrict__ b,
                                                   const float2* __restrict__ a, int k,
                                                   double* __restrict__ out) {
  __shared__ double red[kT / 64];
  double acc = 0.0;
  for (int l = threadIdx.x; l < k; l += kT) acc += b[l].x * a[l].x + b[l].y * a[l].y;
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) *out = 2.0 * acc;
}

unsigned blocks(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

tv_status last(const char* what) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TV_OK : hip_error(e, what);
}

// Device buffers of one assembly, carved from the caller's workspace
// (256-byte aligned, in call order); with base == nullptr only the size is
// accumulated.
struct Buffers {
  char* base = nullptr;
  size_t cap = 0, off = 0;
  template <typename T>
  tv_status alloc(T** p, size_t count) {
    off = (off + 255) & ~(size_t)255;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (base && off + bytes > cap) return set_error(TV_ERR_WORKSPACE, "ACA assembly workspace");
    *p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += bytes;
    return TV_OK;
  }
};

// Largest rank per mode a new column of U may keep (the HOSVD's clamps).
constexpr size_t kGrowAdjBudget = (size_t)16 << 30;

void rank_bounds(const tv_grid& g, int rank_cap, int rmax[3]) {
  const int dims[3] = {g.n1, g.n2, g.n3};
  for (int d = 0; d < 3; ++d) {
    int r = std::min(dims[d], std::min(64, TV_MAX_RANK));
    if (rank_cap > 0) r = std::min(r, rank_cap);
    rmax[d] = std::max(r, 1);
  }
}

// Sizes of the regions of the assembly's workspace (see tv_aca_assemble):
// fixed buffers, one column's compression scratch, U's arena at K columns of
// the largest ranks, and the product workspace.
struct AcaSizes {
  size_t fixed, comp, uarena, prod, total;
};
AcaSizes aca_sizes(const tv_grid& g, int K, double htol, int rank_min, int rank_cap,
                   tv_precision prec) {
  AcaSizes z{};
  const int64_t nv = (int64_t)g.n1 * g.n2 * g.n3, rows = (int64_t)g.q * nv, m = g.m;
  Buffers B;
  double *d1;
  int64_t* i1;
  double2* z2;
  float2* f2;
  B.alloc(&d1, (size_t)6 * m);
  B.alloc(&d1, 1024);
  B.alloc(&i1, 1024);
  B.alloc(&d1, 8);
  B.alloc(&z2, m);
  B.alloc(&z2, (size_t)m * K);
  B.alloc(&z2, K);
  B.alloc(&z2, K);
  B.alloc(&z2, rows);
  B.alloc(&f2, K);
  B.alloc(&f2, rows);
  B.alloc(&f2, rows);
  B.alloc(&f2, K);
  z.fixed = (B.off + 255) & ~(size_t)255;
  tv_grid g1 = g;
  g1.m = 1;
  tv_plan cp = nullptr;
  if (tv_compress_begin(&g1, htol, rank_min, rank_cap, prec, &cp) == TV_OK) {
    z.comp = compress_scratch_bytes(cp, g.q);
    tv_plan_destroy(cp);
  }
  int rmax[3];
  rank_bounds(g, rank_cap, rmax);
  tv_grid gk = g;
  gk.m = K;
  z.uarena = plan_arena_bound(gk, rmax, prec);
  // forward split partials (at most 8 by default) or the adjoint's partial
  // inner products per (component, tile, column)
  Tiling Ta;
  make_tiling(g, 0, 2, &Ta);
  z.prod = std::max((size_t)8 * 8 * rows, (size_t)8 * g.q * Ta.tiles * K);
  // U's adjoint runs as the column GEMM once U has a few columns, in at most
  // kGrowAdjBudget bytes (the fused kernels again past that)
  z.prod = std::max(z.prod, std::min(grow_adjoint_ws_bytes(gk, rmax), kGrowAdjBudget));
  z.total = z.fixed + z.comp + z.uarena + z.prod + 4 * 256;
  return z;
}

// Host copies of U's Tucker factors in the layout of tv_plan_from_factors.
struct HostFactors {
  std::vector<int32_t> ranks;
  std::vector<double> cores, u1, u2, u3;
};

// Truncated HOSVD of one column (q tensors) on the device, factors appended
// to the host copies.
tv_status compress_column(const tv_grid& grid, const double2* d_x, double tol, int rank_min,
                          int rank_cap, tv_precision prec, HostFactors& F, void* cws,
                          size_t cws_bytes, void* stream, const HostStage& stage) {
  tv_grid g1 = grid;
  g1.m = 1;
  tv_plan cp = nullptr;
  tv_status s = tv_compress_begin(&g1, tol, rank_min, rank_cap, prec, &cp);
  if (s != TV_OK) return s;
  s = compress_append_staged(cp, d_x, 1, cws, cws_bytes, (hipStream_t)stream, stage);
  std::vector<int32_t> rk((size_t)3 * grid.q);
  if (s == TV_OK) s = tv_plan_export_factors(cp, rk.data(), nullptr, nullptr, nullptr, nullptr);
  if (s == TV_OK) {
    size_t ng = 0, n1 = 0, n2 = 0, n3 = 0;
    for (int k = 0; k < grid.q; ++k) {
      ng += (size_t)rk[3 * k] * rk[3 * k + 1] * rk[3 * k + 2];
      n1 += (size_t)grid.n1 * rk[3 * k];
      n2 += (size_t)grid.n2 * rk[3 * k + 1];
      n3 += (size_t)grid.n3 * rk[3 * k + 2];
    }
    const size_t o0 = F.cores.size(), o1 = F.u1.size(), o2 = F.u2.size(), o3 = F.u3.size();
    F.cores.resize(o0 + 2 * ng);
    F.u1.resize(o1 + 2 * n1);
    F.u2.resize(o2 + 2 * n2);
    F.u3.resize(o3 + 2 * n3);
    s = tv_plan_export_factors(cp, rk.data(), &F.cores[o0], &F.u1[o1], &F.u2[o2], &F.u3[o3]);
    F.ranks.insert(F.ranks.end(), rk.begin(), rk.end());
  }
  tv_plan_destroy(cp);
  return s;
}

}  // namespace
}  // namespace tv

namespace tv {

struct CopySegs {
  CopySeg s[kMaxCopySegs];
};

// blockIdx.y = segment; the workgroups of x stride over its 4-byte words
__global__ __launch_bounds__(256) void segment_copy_kernel(CopySegs S, const uint32_t* src) {
  const CopySeg g = S.s[blockIdx.y];
  uint32_t* dst = reinterpret_cast<uint32_t*>(g.dst);
  const uint32_t* from = src + g.src_off / 4;
  const int64_t n = g.bytes / 4;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    dst[e] = from[e];
}

tv_status launch_segment_copy(const CopySeg* segs, int nseg, const void* src, hipStream_t st) {
  if (nseg < 1) return TV_OK;
  if (nseg > kMaxCopySegs) return set_error(TV_ERR_INVALID_ARG, "segment copy: too many segments");
  CopySegs S{};
  int64_t most = 0;
  for (int i = 0; i < nseg; ++i) {
    if (((uintptr_t)segs[i].dst | (uint64_t)segs[i].src_off | (uint64_t)segs[i].bytes) % 4)
      return set_error(TV_ERR_INVALID_ARG, "segment copy: ranges must be 4-byte aligned");
    S.s[i] = segs[i];
    most = std::max(most, segs[i].bytes / 4);
  }
  const unsigned bx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, (most + 255) / 256));
  hipLaunchKernelGGL(segment_copy_kernel, dim3(bx, (unsigned)nseg), dim3(256), 0, st, S,
                     (const uint32_t*)src);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TV_OK : hip_error(e, "segment_copy_kernel");
}

}  // namespace tv

using namespace tv;

extern "C" tv_status tv_aca_assemble_workspace_bytes(const tv_grid* grid, int32_t max_terms,
                                                     double tol, double hosvd_tol,
                                                     int32_t rank_min, int32_t rank_cap,
                                                     tv_precision precision, size_t* bytes) {
  clear_error();
  if (!grid || !bytes) return set_error(TV_ERR_INVALID_ARG, "NULL argument");
  if (grid->n1 < 1 || grid->n2 < 1 || grid->n3 < 1 || grid->m < 1 || grid->q < 1)
    return set_error(TV_ERR_SHAPE, "grid sizes and m must be >= 1");
  if (max_terms < 1) return set_error(TV_ERR_INVALID_ARG, "max_terms must be >= 1");
  const double htol = hosvd_tol > 0.0 ? hosvd_tol : 3.0 * tol;
  *bytes = aca_sizes(*grid, max_terms, htol, rank_min, rank_cap, precision).total;
  return TV_OK;
}

extern "C" tv_status tv_aca_assemble(const tv_grid* grid, double h, double k0, int32_t basis,
                                     const double* pos, const double* ori, double tol,
                                     double hosvd_tol, int32_t rank_min, int32_t rank_cap,
                                     int32_t max_terms, tv_precision precision, void* ws,
                                     size_t ws_bytes, tv_plan* u_out, double* v_out,
                                     int32_t* rc_out, int32_t* converged_out, int64_t* pivots,
                                     double* s_out, void* stream) {
  clear_error();
  if (!grid || !pos || !ori || !u_out || !v_out || !rc_out || !converged_out)
    return set_error(TV_ERR_INVALID_ARG, "NULL argument");
  *u_out = nullptr;
  const tv_grid g = *grid;
  if (g.n1 < 1 || g.n2 < 1 || g.n3 < 1 || g.m < 1)
    return set_error(TV_ERR_SHAPE, "grid sizes and m must be >= 1");
  if (basis < 0 || basis > 3) return set_error(TV_ERR_INVALID_ARG, "basis must be in 0..3");
  if (g.q != ((basis & 1) ? 12 : 3))
    return set_error(TV_ERR_SHAPE, "q must be 3 (PWC) or 12 (PWL) to match the basis");
  if (!(tol > 0.0) || !std::isfinite(tol)) return set_error(TV_ERR_INVALID_ARG, "tol must be > 0");
  if (!(h > 0.0) || !(k0 > 0.0)) return set_error(TV_ERR_INVALID_ARG, "h and k0 must be > 0");
  const int64_t nv = (int64_t)g.n1 * g.n2 * g.n3, rows = (int64_t)g.q * nv, m = g.m;
  if (max_terms < 1 || max_terms > std::min<int64_t>(std::min(rows, m), 65535))
    return set_error(TV_ERR_INVALID_ARG, "max_terms must be in [1, min(q nv, m, 65535)]");
  const double htol = hosvd_tol > 0.0 ? hosvd_tol : 3.0 * tol;
  std::vector<double> src;
  tv_status s = stage_sources(g.n1, g.n2, g.n3, h, m, pos, ori, src);
  if (s != TV_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const int K = max_terms;
  const unsigned nb_rows = std::min<unsigned>(1024, blocks(rows));
  const unsigned nb_m = std::min<unsigned>(1024, blocks(m));

  const AcaSizes Z = aca_sizes(g, K, htol, rank_min, rank_cap, precision);
  if (!ws || ws_bytes < Z.total) {
    char buf[128];
    snprintf(buf, sizeof buf, "assembly workspace of %zu bytes needed, %zu given", Z.total,
             ws ? ws_bytes : (size_t)0);
    return set_error(TV_ERR_WORKSPACE, buf);
  }
  if ((uintptr_t)ws % 256) return set_error(TV_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  // regions: fixed buffers | column compression | U's arena | product workspace
  char* const wsb = (char*)ws;
  void* const cws = wsb + Z.fixed;
  char* const uarena = wsb + Z.fixed + Z.comp;
  void* const pws = uarena + Z.uarena;
  Buffers B;
  B.base = wsb;
  B.cap = Z.fixed;
  double *d_src, *d_bv, *d_scal;
  int64_t *d_bi, *d_row, *d_iscal;
  double2 *d_r, *d_V, *d_t, *d_b, *d_x;
  float2 *d_w32, *d_x32, *d_u32, *d_a32;
  if ((s = B.alloc(&d_src, src.size())) != TV_OK || (s = B.alloc(&d_bv, 1024)) != TV_OK ||
      (s = B.alloc(&d_bi, 1024)) != TV_OK || (s = B.alloc(&d_scal, 8)) != TV_OK ||
      (s = B.alloc(&d_r, m)) != TV_OK || (s = B.alloc(&d_V, (size_t)m * K)) != TV_OK ||
      (s = B.alloc(&d_t, K)) != TV_OK || (s = B.alloc(&d_b, K)) != TV_OK ||
      (s = B.alloc(&d_x, rows)) != TV_OK ||
      (s = B.alloc(&d_w32, K)) != TV_OK || (s = B.alloc(&d_x32, rows)) != TV_OK ||
      (s = B.alloc(&d_u32, rows)) != TV_OK || (s = B.alloc(&d_a32, K)) != TV_OK)
    return s;
  // pinned host staging of the loop's transfers: the scalars below, one
  // column's compression and U's growth (without it, host vectors serve)
  struct Pinned {
    char* p = nullptr;
    hipStream_t st = nullptr;
    ~Pinned() {
      if (!p) return;
      (void)hipStreamSynchronize(st);  // no copy may still read or write it
      (void)hipHostFree(p);
    }
  } pin;
  pin.st = st;
  HostStage cstage, gstage;
  double hs_vec[5];
  double* hs = hs_vec;
  {
    tv_grid g1 = g;
    g1.m = 1;
    tv_plan cp = nullptr;
    size_t cbytes = 0, gbytes = 0;
    if (tv_compress_begin(&g1, htol, rank_min, rank_cap, precision, &cp) == TV_OK) {
      cbytes = compress_stage_bytes(cp, g.q);
      tv_plan_destroy(cp);
    }
    int rmax[3];
    rank_bounds(g, rank_cap, rmax);
    tv_grid gk = g;
    gk.m = K;
    gbytes = (grow_stage_bytes(gk, rmax, precision) + 255) & ~(size_t)255;
    if (cbytes && gbytes &&
        hipHostMalloc((void**)&pin.p, 256 + gbytes + cbytes, hipHostMallocDefault) == hipSuccess) {
      hs = reinterpret_cast<double*>(pin.p);
      gstage = HostStage{pin.p + 256, gbytes};
      cstage = HostStage{pin.p + 256 + gbytes, cbytes};
    } else {
      pin.p = nullptr;
      (void)hipGetLastError();
    }
  }
  // scalar results in one small region read back with one copy: [0] argmax
  // value, [1], [2] sums of squares, [3] cross term, [4] argmax index (int64),
  // which is also the next pivot row that rows_kernel reads
  d_iscal = reinterpret_cast<int64_t*>(d_scal + 4);
  d_row = d_iscal;
  const int64_t row0 = 0;
  hipError_t e =
      hipMemcpyAsync(d_src, src.data(), src.size() * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_row, &row0, sizeof(int64_t), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_error(e, "source upload");
  auto readback = [&](int count, const char* what) -> tv_status {
    hipError_t he = hipMemcpyAsync(hs, d_scal, count * sizeof(double), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    return he == hipSuccess ? TV_OK : hip_error(he, what);
  };

  // scalar results back to the host: (value, index) of an argmax, or a sum
  auto argmax = [&](const double2* x, int64_t n, int64_t skip, unsigned nb, double* v,
                    int64_t* i) -> tv_status {
    hipLaunchKernelGGL(amax1_kernel, dim3(nb), dim3(kT), 0, st, x, n, skip, d_bv, d_bi);
    hipLaunchKernelGGL(amax2_kernel, dim3(1), dim3(kT), 0, st, d_bv, d_bi, (int)nb, d_scal,
                       d_iscal);
    tv_status r = last("argmax kernels");
    if (r == TV_OK) r = readback(5, "argmax readback");
    if (r != TV_OK) return r;
    *v = hs[0];
    std::memcpy(i, &hs[4], sizeof(int64_t));
    return TV_OK;
  };
  // sum of squares of x into d_scal[slot] (read back by the caller)
  auto sumsq = [&](const double2* x, int64_t n, unsigned nb, int slot) -> tv_status {
    hipLaunchKernelGGL(sumsq1_kernel, dim3(nb), dim3(kT), 0, st, x, n, d_bv);
    hipLaunchKernelGGL(sumsq2_kernel, dim3(1), dim3(kT), 0, st, d_bv, (int)nb, d_scal + slot);
    return last("norm kernels");
  };

  HostFactors F;
  // the compressed U of the steps so far: a growable plan in uarena
  tv_plan U = nullptr;
  {
    int rmax[3];
    rank_bounds(g, rank_cap, rmax);
    tv_grid gk = g;
    gk.m = K;
    if ((s = grow_plan_create(gk, rmax, precision, uarena, Z.uarena, st, &U)) != TV_OK) return s;
    grow_plan_set_stage(U, gstage, Z.prod);
  }
  auto fail = [&](tv_status r) {
    tv_plan_destroy(U);
    return r;
  };
  int64_t i = 0;
  double ssum = 0.0;
  int rc = 0;
  bool converged = false;
  for (int k = 0; k < K; ++k) {
    // r = Z_{i:} - (U V^*)_{i:} (row i is in d_row already)
    if ((s = launch_dipole_rows(g.n1, g.n2, g.n3, h, k0, basis, m, d_src, 1, d_row, d_r, st)) !=
        TV_OK)
      return fail(s);
    if (k > 0) {
      const int p = (int)(i / nv);
      const int64_t v = i - (int64_t)p * nv;
      const int f1 = (int)(v % g.n1), f2 = (int)((v / g.n1) % g.n2),
                f3 = (int)(v / ((int64_t)g.n1 * g.n2));
      hipLaunchKernelGGL(entry_kernel, dim3((unsigned)k), dim3(kT), 0, st, U->d_meta, U->d_cores,
                         U->d_u1t, U->d_u2t, U->d_u3t, (int64_t)k, p, f1, f2, f3, d_t);
      hipLaunchKernelGGL(row_update_kernel, dim3(blocks(m)), dim3(kT), 0, st, d_r, d_V, m, d_t,
                         m, k);
      if ((s = last("row kernels")) != TV_OK) return fail(s);
    }
    double rmax = 0.0;
    int64_t j = 0;
    if ((s = argmax(d_r, m, -1, nb_m, &rmax, &j)) != TV_OK) return fail(s);
    if (!(rmax > 0.0)) {
      converged = true;  // the residual row is exactly zero
      break;
    }
    double2* y = d_V + (size_t)m * k;
    hipLaunchKernelGGL(set_y_kernel, dim3(blocks(m)), dim3(kT), 0, st, d_r, m, j, y);
    // x = Z_{:j} - U V_{j:}^*
    if ((s = launch_dipole_columns(g.n1, g.n2, g.n3, h, k0, basis, 1, d_src + 6 * j, d_x, st)) !=
        TV_OK)
      return fail(s);
    if (k > 0) {
      hipLaunchKernelGGL(conj_row_kernel, dim3(blocks(k)), dim3(kT), 0, st, d_V, m, j, k, d_w32);
      if ((s = last("conj_row_kernel")) != TV_OK) return fail(s);
      if ((s = tv_matvec(U, d_w32, k, 1, d_u32, rows, pws, Z.prod, stream)) != TV_OK)
        return fail(s);
      hipLaunchKernelGGL(sub_kernel, dim3(blocks(rows)), dim3(kT), 0, st, d_x, d_u32, rows);
      if ((s = last("sub_kernel")) != TV_OK) return fail(s);
    }
    // s_{k+1} = s_k + (|x||y|)^2 + 2 Re sum conj(V^* y) (U^* x)
    if ((s = sumsq(d_x, rows, nb_rows, 1)) != TV_OK || (s = sumsq(y, m, nb_m, 2)) != TV_OK ||
        (s = readback(3, "norm readback")) != TV_OK)
      return fail(s);
    const double nx2 = hs[1], ny2 = hs[2];
    double s_next = ssum + nx2 * ny2;
    if (k > 0) {
      hipLaunchKernelGGL(to_c64_kernel, dim3(blocks(rows)), dim3(kT), 0, st, d_x, d_x32, rows);
      if ((s = last("to_c64_kernel")) != TV_OK) return fail(s);
      if ((s = tv_rmatvec(U, d_x32, rows, 1, d_a32, k, pws, Z.prod, stream)) != TV_OK)
        return fail(s);
      hipLaunchKernelGGL(vhy_kernel, dim3((unsigned)k), dim3(kT), 0, st, d_V, m, y, m, d_b);
      hipLaunchKernelGGL(cross_kernel, dim3(1), dim3(kT), 0, st, d_b, d_a32, k, d_scal + 3);
      if ((s = last("cross_kernel")) != TV_OK || (s = readback(4, "cross term readback")) != TV_OK)
        return fail(s);
      s_next += hs[3];
    }
    // U = [U HOSVD(x)] and V = [V y] (y is already in place); the products
    // above have been waited for (the cross-term readback), so U's arrays
    // may grow in place
    const size_t o0 = F.cores.size(), o1 = F.u1.size(), o2 = F.u2.size(), o3 = F.u3.size(),
                 orank = F.ranks.size();
    if ((s = compress_column(g, d_x, htol, rank_min, rank_cap, precision, F, cws, Z.comp,
                             stream, cstage)) != TV_OK)
      return fail(s);
    if ((s = grow_plan_append(U, &F.ranks[orank], &F.cores[o0], &F.u1[o1], &F.u2[o2], &F.u3[o3],
                              st)) != TV_OK)
      return fail(s);
    if (pivots) {
      pivots[2 * k] = i;
      pivots[2 * k + 1] = j;
    }
    ssum = s_next;
    if (s_out) s_out[k] = ssum;
    rc = k + 1;
    if (std::sqrt(nx2 * ny2) <= tol * std::sqrt(std::max(ssum, 0.0))) {
      converged = true;
      break;
    }
    // next pivot row: the largest |x| other than row i
    double xmax = 0.0;
    int64_t inext = 0;
    if ((s = argmax(d_x, rows, i, nb_rows, &xmax, &inext)) != TV_OK) return fail(s);
    if (!(xmax >= 0.0) || inext >= rows) break;
    i = inext;
  }
  if (rc == 0) {
    // the first row was zero: no term; report an empty approximation
    *rc_out = 0;
    *converged_out = 1;
    return fail(set_error(TV_ERR_NUMERIC, "the first pivot row of Z is zero"));
  }
  e = hipMemcpy(v_out, d_V, sizeof(double2) * (size_t)m * rc, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(hip_error(e, "V readback"));
  // the returned plan is unbound: the caller binds it to an arena of its own
  tv_plan Uout = nullptr;
  {
    tv_grid gk = g;
    gk.m = rc;
    s = tv_plan_from_factors(&gk, F.ranks.data(), F.cores.data(), F.u1.data(), F.u2.data(),
                             F.u3.data(), precision, &Uout);
    if (s != TV_OK) return fail(s);
  }
  tv_plan_destroy(U);
  *u_out = Uout;
  *rc_out = rc;
  *converged_out = converged ? 1 : 0;
  return TV_OK;
}
