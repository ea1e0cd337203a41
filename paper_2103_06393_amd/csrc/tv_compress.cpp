// Truncated-HOSVD compression (Sec. II.B.1): host orchestration.
//
// Per batch of columns: FP64 Gram matrices of the three unfoldings of every
// tensor and their eigendecomposition on the device; the rank rule on the
// host; the core A x1 U1^* x2 U2^* x3 U3^* on the device.  Factors are kept
// in FP64 on the host until tv_plan_finalize packs the plan.
//
// Rank rule (the paper leaves the tolerance-to-rank map open): per mode keep
// the smallest r whose discarded eigenvalues (squared singular values) sum to
// at most tol^2 ||A||^2 / 3, so the HOSVD error bound gives a relative error
// of at most tol; extend r across singular values equal to within 1e-10;
// clamp to [rank_min, min(rank_cap, n, TV_MAX_RANK)].
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>

#include "tv_internal.h"

namespace tv {
tv_status launch_gram(const double2* A, int ntens, int n1, int n2, int n3, int nmax, double2* S,
                      double2* P, hipStream_t st);
size_t gram_partial_count(int ntens, int nmax);
tv_status launch_jacobi(const double2* S, int nmat, int n, int64_t stride, double* W,
                        int64_t wstride, double2* V, int64_t vstride, hipStream_t st);
tv_status launch_proj(const double2* A, int ntens, int n1, int n2, int n3, const double2* u1,
                      const double2* u2, const double2* u3, const int64_t* offs,
                      const int* ranks, int r1max, int r2max, double2* T1, double2* T2,
                      double2* G, hipStream_t st);
tv_status launch_subspace_eig(const double2* S, int nmat, int n, int64_t sS, double* W,
                              double2* U, double* tr, double2* ws, hipStream_t st);
tv_status launch_jacobi_batch(const JacobiGroup* groups, int ng, hipStream_t st);
tv_status launch_subspace_prep_batch(const SubspaceJob* jobs, int nj, int nmat, hipStream_t st);
tv_status launch_subspace_finish(int nmat, int n, const double2* ws, const double2* V,
                                 double2* U, hipStream_t st);
double2* subspace_T(double2* ws, int nmat, int n);
double2* subspace_V(double2* ws, int nmat, int n);
tv_status finalize_plan(tv_plan_s* p);
tv_status validate_ranks_and_offsets(tv_plan_s* p);

// Device scratch of one append call, carved from the caller's workspace
// (256-byte aligned pieces, in call order).  With base == nullptr only the
// size is accumulated.
struct DevScratch {
  char* base = nullptr;
  size_t cap = 0, off = 0;
  template <typename T>
  tv_status alloc(T** p, size_t count) {
    off = (off + 255) & ~(size_t)255;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (base && off + bytes > cap) return set_error(TV_ERR_WORKSPACE, "compression workspace");
    *p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += bytes;
    return TV_OK;
  }
};

// Upper bound of the scratch of one append call of T tensors: Gram
// matrices (and their partial tiles when the columns are split), eigenpairs
// (and the subspace solver's work arrays for modes longer than 64), factors
// at the largest rank a mode can keep, and the partial projections and cores
// of the core computation.  The call carves some of these as one region (one
// copy each way), which never needs more than the separately aligned pieces.
size_t compress_scratch_bytes(const tv_plan_s* p, int T) {
  const tv_grid& g = p->grid;
  const int dims[3] = {g.n1, g.n2, g.n3};
  const int nmax = std::max(g.n1, std::max(g.n2, g.n3));
  int rmax[3];
  for (int d = 0; d < 3; ++d) {
    int r = std::min(dims[d], std::min(64, TV_MAX_RANK));
    if (p->rank_cap > 0) r = std::min(r, (int)p->rank_cap);
    rmax[d] = std::max(r, 1);
  }
  DevScratch ds;
  double2* z2;
  double* z1;
  int64_t* zi;
  int* zk;
  ds.alloc(&z2, (size_t)3 * T * nmax * nmax);
  ds.alloc(&z2, gram_partial_count(T, nmax));
  for (int d = 0; d < 3; ++d) {
    const int n = dims[d], L = n <= 64 ? n : 64;
    ds.alloc(&z2, (size_t)T * n * L);
    ds.alloc(&z1, (size_t)T * L);
    if (n > 64) {
      ds.alloc(&z1, (size_t)T);
      ds.alloc(&z2, (size_t)T * (3 * (size_t)n * 64 + 64 * 64));
    }
  }
  for (int d = 0; d < 3; ++d) ds.alloc(&z2, (size_t)T * dims[d] * rmax[d]);
  ds.alloc(&z2, (size_t)T * rmax[0] * g.n2 * g.n3);
  ds.alloc(&z2, (size_t)T * rmax[0] * rmax[1] * g.n3);
  ds.alloc(&z2, (size_t)T * rmax[0] * rmax[1] * rmax[2]);
  ds.alloc(&zi, (size_t)4 * T);
  ds.alloc(&zk, (size_t)3 * T);
  return (ds.off + 255) & ~(size_t)255;
}

// Rank of one mode from its leading eigenvalues lam (descending, L of the
// n_full eigenvalues of the Gram matrix) and the Gram trace: the tail of
// the spectrum beyond r is trace - sum_{i<r} lam_i.
int select_rank(const std::vector<double>& lam, double trace, int n_full, double tol,
                int rank_min, int rank_cap, double* rel_tail) {
  const int L = (int)lam.size();
  trace = std::max(trace, 0.0);
  std::vector<double> tail(L + 1, 0.0);
  double head = 0.0;
  for (int r = 0; r <= L; ++r) {
    tail[r] = std::max(trace - head, 0.0);
    if (r < L) head += std::max(lam[r], 0.0);
  }
  if (L == n_full) tail[L] = 0.0;
  const double budget = tol * tol * trace / 3.0;
  int r = L;
  for (int c = 0; c <= L; ++c)
    if (tail[c] <= budget) {
      r = c;
      break;
    }
  int cap = std::min(L, TV_MAX_RANK);
  if (rank_cap > 0) cap = std::min(cap, rank_cap);
  while (r > 0 && r < cap &&
         std::sqrt(std::max(lam[r], 0.0)) >= (1.0 - 1e-10) * std::sqrt(std::max(lam[r - 1], 0.0)))
    ++r;
  r = std::max(r, rank_min);
  r = std::min(r, cap);
  *rel_tail = trace > 0.0 ? tail[r] / trace : 0.0;
  return r;
}

}  // namespace tv

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
  const int nmax = std::max(grid->n1, std::max(grid->n2, grid->n3));
  // Gram scratch is 3 x tensors x nmax^2 complex128 per append call
  if (nmax > 1024)
    return set_error(TV_ERR_NOT_SUPPORTED, "device compression is built for n1, n2, n3 <= 1024");
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

tv_status tv_compress_workspace_bytes(tv_plan p, int64_t ncols, size_t* bytes) {
  clear_error();
  if (!p || !bytes) return set_error(TV_ERR_INVALID_ARG, "plan and bytes must be non-NULL");
  if (ncols < 0 || ncols * p->grid.q > 65535)
    return set_error(TV_ERR_NOT_SUPPORTED, "at most 65535 tensors per append call");
  *bytes = ncols ? compress_scratch_bytes(p, (int)(ncols * p->grid.q)) : 0;
  return TV_OK;
}

tv_status tv_compress_append(tv_plan p, const void* cols, int64_t ncols, void* ws,
                             size_t ws_bytes, void* stream) {
  clear_error();
  return compress_append_staged(p, cols, ncols, ws, ws_bytes, (hipStream_t)stream, HostStage{});
}

}  // extern "C"

namespace tv {

size_t compress_stage_bytes(const tv_plan_s* p, int T) {
  const tv_grid& g = p->grid;
  const int dims[3] = {g.n1, g.n2, g.n3};
  size_t n2 = 0;  // double2 units: eigenpair readback, factor upload, cores
  int rmax[3];
  for (int d = 0; d < 3; ++d) {
    const int n = dims[d], L = n <= 64 ? n : 64;
    n2 += (size_t)T * n * L + ((size_t)T * L + 1) / 2 + (n > 64 ? ((size_t)T + 1) / 2 : 0);
    int r = std::min(n, std::min(64, TV_MAX_RANK));
    if (p->rank_cap > 0) r = std::min(r, (int)p->rank_cap);
    rmax[d] = std::max(r, 1);
    n2 += (size_t)T * n * rmax[d];
  }
  n2 += (4 * (size_t)T + 1) / 2 + (3 * (size_t)T + 3) / 4;
  n2 += (size_t)T * rmax[0] * rmax[1] * rmax[2];
  return n2 * sizeof(double2) + 3 * 256;
}

tv_status compress_append_staged(tv_plan p, const void* cols, int64_t ncols, void* ws,
                                 size_t ws_bytes, hipStream_t st, const HostStage& stage) {
  if (!p) return set_error(TV_ERR_INVALID_ARG, "plan is NULL");
  if (p->finalized) return set_error(TV_ERR_INVALID_ARG, "plan is already finalized");
  if (ncols < 0 || p->appended + ncols > p->grid.m)
    return set_error(TV_ERR_SHAPE, "more columns than the plan holds");
  if (ncols == 0) return TV_OK;
  if (!cols) return set_error(TV_ERR_INVALID_ARG, "cols is NULL");
  if (ncols * p->grid.q > 65535)
    return set_error(TV_ERR_NOT_SUPPORTED, "at most 65535 tensors per append call");
  const tv_grid& g = p->grid;
  const int dims[3] = {g.n1, g.n2, g.n3};
  const int nmax = std::max(g.n1, std::max(g.n2, g.n3));
  const int64_t nv = (int64_t)g.n1 * g.n2 * g.n3;
  const int T = (int)(ncols * g.q);
  const double2* A = (const double2*)cols;
  // host side of the transfers: the caller's (pinned) staging when it covers
  // this call, else host vectors; carved in call order
  const bool staged = stage.ptr && stage.bytes >= compress_stage_bytes(p, T);
  size_t stage_off = 0;
  std::vector<double2> hv[3];
  auto host_buf = [&](int slot, size_t n) -> double2* {
    if (!staged) {
      hv[slot].resize(n);
      return hv[slot].data();
    }
    double2* q = reinterpret_cast<double2*>(stage.ptr + stage_off);
    stage_off = (stage_off + n * sizeof(double2) + 255) & ~(size_t)255;
    return q;
  };
  const size_t need = compress_scratch_bytes(p, T);
  if (!ws || ws_bytes < need) {
    char buf[128];
    snprintf(buf, sizeof buf, "compression workspace of %zu bytes needed, %zu given", need,
             ws ? ws_bytes : (size_t)0);
    return set_error(TV_ERR_WORKSPACE, buf);
  }
  if ((uintptr_t)ws % 256) return set_error(TV_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  DevScratch ds;
  ds.base = (char*)ws;
  ds.cap = ws_bytes;
  tv_status s;

  // 1. Gram matrices S_d (mode-major) and their (leading) eigenpairs: the
  //    full Jacobi eigendecomposition for modes of length <= 64, the leading
  //    64 pairs by subspace iteration otherwise
  const int64_t mat = (int64_t)nmax * nmax;
  double2* dS;
  double2* dP;  // partial Gram tiles of calls with few tensors
  if ((s = ds.alloc(&dS, (size_t)3 * T * mat)) != TV_OK) return s;
  if ((s = ds.alloc(&dP, gram_partial_count(T, nmax))) != TV_OK) return s;
  if ((s = launch_gram(A, T, g.n1, g.n2, g.n3, nmax, dS, dP, st)) != TV_OK) return s;
  int L[3];
  // the three modes' eigenproblems: subspace preparation for the long modes,
  // then one Jacobi launch over every mode's matrices (n x n directly for
  // modes <= 64, the 64 x 64 Rayleigh-Ritz matrices otherwise), the long
  // modes' vectors, and one readback: the eigenvectors, eigenvalues and the
  // long modes' Gram traces of all modes sit in one region (double2 units)
  size_t rb_off[3][3];
  size_t rb_n = 0;
  for (int d = 0; d < 3; ++d) {
    const int n = dims[d];
    L[d] = n <= 64 ? n : 64;
    rb_off[d][0] = rb_n;
    rb_n += (size_t)T * n * L[d];
    rb_off[d][1] = rb_n;
    rb_n += ((size_t)T * L[d] + 1) / 2;
    rb_off[d][2] = rb_n;
    rb_n += n > 64 ? ((size_t)T + 1) / 2 : 0;
  }
  double2* dRB;
  if ((s = ds.alloc(&dRB, rb_n)) != TV_OK) return s;
  double2* dV[3];
  double* dW[3];
  double* dTr[3] = {nullptr, nullptr, nullptr};
  double2* dWs[3] = {nullptr, nullptr, nullptr};
  JacobiGroup groups[3];
  SubspaceJob jobs[3];
  int nj = 0;
  for (int d = 0; d < 3; ++d) {
    const int n = dims[d];
    dV[d] = dRB + rb_off[d][0];
    dW[d] = reinterpret_cast<double*>(dRB + rb_off[d][1]);
    const double2* Sd = dS + (int64_t)d * T * mat;
    if (n <= 64) {
      // eigenvectors are written compactly, n x n per matrix
      groups[d] = JacobiGroup{Sd, dW[d], dV[d], mat, n, (int64_t)n * n, n, T};
    } else {
      dTr[d] = reinterpret_cast<double*>(dRB + rb_off[d][2]);
      if ((s = ds.alloc(&dWs[d], (size_t)T * (3 * (size_t)n * 64 + 64 * 64))) != TV_OK) return s;
      jobs[nj++] = SubspaceJob{Sd, mat, dTr[d], dWs[d], n};
      groups[d] = JacobiGroup{subspace_T(dWs[d], T, n), dW[d], subspace_V(dWs[d], T, n),
                              64 * 64, 64, 64 * 64, 64, T};
    }
  }
  if (nj > 0 && (s = launch_subspace_prep_batch(jobs, nj, T, st)) != TV_OK) return s;
  if ((s = launch_jacobi_batch(groups, 3, st)) != TV_OK) return s;
  for (int d = 0; d < 3; ++d)
    if (dims[d] > 64 &&
        (s = launch_subspace_finish(T, dims[d], dWs[d], subspace_V(dWs[d], T, dims[d]), dV[d],
                                    st)) != TV_OK)
      return s;
  const double2* RB = host_buf(0, rb_n);
  {
    hipError_t e = hipMemcpyAsync((void*)RB, dRB, rb_n * sizeof(double2), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_error(e, "eigenpair readback");
  }
  const double2* V[3];
  const double* W[3];
  const double* TR[3];
  for (int d = 0; d < 3; ++d) {
    V[d] = RB + rb_off[d][0];
    W[d] = reinterpret_cast<const double*>(RB + rb_off[d][1]);
    TR[d] = reinterpret_cast<const double*>(RB + rb_off[d][2]);
  }

  // 2. ranks and factors on the host
  std::vector<int> rk((size_t)3 * T);
  std::vector<double> reld((size_t)3 * T);
  std::vector<std::vector<double2>> U(3);
  std::vector<int64_t> offs((size_t)4 * T, 0);  // u1, u2, u3, g offsets (complex)
  int64_t tot[4] = {0, 0, 0, 0};
  for (int t = 0; t < T; ++t) {
    for (int d = 0; d < 3; ++d) {
      const int n = dims[d], Ld = L[d];
      const double* w = W[d] + (size_t)t * Ld;
      std::vector<int> idx(Ld);
      std::iota(idx.begin(), idx.end(), 0);
      std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return w[a] > w[b]; });
      std::vector<double> lam(Ld);
      double trace = 0.0;
      for (int i = 0; i < Ld; ++i) {
        lam[i] = w[idx[i]];
        trace += std::max(w[i], 0.0);
      }
      if (n > 64) trace = TR[d][t];
      double rt = 0.0;
      const int r = select_rank(lam, trace, n, p->tol, p->rank_min, p->rank_cap, &rt);
      rk[3 * t + d] = r;
      reld[3 * t + d] = rt;
      offs[(size_t)d * T + t] = tot[d];
      const double2* Vm = V[d] + (size_t)t * n * Ld;  // row-major n x Ld
      for (int a = 0; a < r; ++a)
        for (int i = 0; i < n; ++i) U[d].push_back(Vm[(size_t)i * Ld + idx[a]]);
      tot[d] += (int64_t)n * r;
    }
    offs[(size_t)3 * T + t] = tot[3];
    tot[3] += (int64_t)rk[3 * t] * rk[3 * t + 1] * rk[3 * t + 2];
  }
  int r1max = 1, r2max = 1;
  for (int t = 0; t < T; ++t) {
    r1max = std::max(r1max, rk[3 * t]);
    r2max = std::max(r2max, rk[3 * t + 1]);
  }

  // 3. core = A x1 U1^* x2 U2^* x3 U3^* on the device; the factors, offsets
  //    and ranks go up in one copy (one region, double2 units)
  const size_t up_off[5] = {0, U[0].size(), U[0].size() + U[1].size(),
                            U[0].size() + U[1].size() + U[2].size(),
                            U[0].size() + U[1].size() + U[2].size() + (offs.size() + 1) / 2};
  const size_t up_n = up_off[4] + (rk.size() + 3) / 4;
  double2 *dUp, *dT1, *dT2, *dG;
  if ((s = ds.alloc(&dUp, up_n)) != TV_OK ||
      (s = ds.alloc(&dT1, (size_t)T * r1max * g.n2 * g.n3)) != TV_OK ||
      (s = ds.alloc(&dT2, (size_t)T * r1max * r2max * g.n3)) != TV_OK ||
      (s = ds.alloc(&dG, (size_t)tot[3])) != TV_OK)
    return s;
  double2* up = host_buf(1, up_n);
  for (int d = 0; d < 3; ++d) std::copy(U[d].begin(), U[d].end(), up + up_off[d]);
  std::memcpy(up + up_off[3], offs.data(), offs.size() * sizeof(int64_t));
  std::memcpy(up + up_off[4], rk.data(), rk.size() * sizeof(int));
  double2 *dU1 = dUp + up_off[0], *dU2 = dUp + up_off[1], *dU3 = dUp + up_off[2];
  int64_t* dOffs = reinterpret_cast<int64_t*>(dUp + up_off[3]);
  int* dRk = reinterpret_cast<int*>(dUp + up_off[4]);
  hipError_t e = hipMemcpyAsync(dUp, up, up_n * sizeof(double2), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_error(e, "factor upload");
  if ((s = launch_proj(A, T, g.n1, g.n2, g.n3, dU1, dU2, dU3, dOffs, dRk, r1max, r2max, dT1, dT2,
                       dG, st)) != TV_OK)
    return s;
  double2* G = host_buf(2, (size_t)tot[3]);
  e = hipMemcpyAsync(G, dG, (size_t)tot[3] * sizeof(double2), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_error(e, "core readback");

  // 4. append to the plan's host factors (tensor order t = k + q j)
  try {
    for (int t = 0; t < T; ++t)
      for (int d = 0; d < 3; ++d) p->ranks.push_back(rk[3 * t + d]);
    p->rel_discarded.insert(p->rel_discarded.end(), reld.begin(), reld.end());
    auto put = [](std::vector<double>& dst, const double2* src, size_t n) {
      const size_t o = dst.size();
      dst.resize(o + 2 * n);
      std::memcpy(&dst[o], src, n * sizeof(double2));
    };
    put(p->cores, G, (size_t)tot[3]);
    put(p->u1, U[0].data(), U[0].size());
    put(p->u2, U[1].data(), U[1].size());
    put(p->u3, U[2].data(), U[2].size());
  } catch (const std::bad_alloc&) {
    return set_error(TV_ERR_OOM, "host factor storage");
  }
  p->appended += ncols;
  // offsets of what has been appended so far (for export before finalize)
  tv_grid part = p->grid;
  part.m = p->appended;
  const tv_grid full = p->grid;
  p->grid = part;
  s = validate_ranks_and_offsets(p);
  p->grid = full;
  return s;
}

}  // namespace tv

extern "C" {

tv_status tv_plan_finalize(tv_plan p, void* stream) {
  clear_error();
  (void)stream;
  if (!p) return set_error(TV_ERR_INVALID_ARG, "plan is NULL");
  if (p->finalized) return TV_OK;
  if (p->appended != p->grid.m)
    return set_error(TV_ERR_INVALID_ARG, "not all columns have been appended");
  tv_status s = validate_ranks_and_offsets(p);
  if (s != TV_OK) return s;
  return finalize_plan(p);
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
