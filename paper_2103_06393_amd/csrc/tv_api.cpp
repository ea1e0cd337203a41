// Host side of libtuckvsie: validation, plan packing, tiling and dispatch.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <type_traits>

#include "tv_internal.h"

namespace tv {

static thread_local std::string g_last_error;

tv_status set_error(tv_status s, const std::string& msg) {
  g_last_error = std::string(tv_status_string(s)) + ": " + msg;
  return s;
}
void clear_error() { g_last_error.clear(); }
tv_status hip_error(hipError_t e, const char* what) {
  return set_error(e == hipErrorOutOfMemory ? TV_ERR_OOM : TV_ERR_HIP,
                   std::string(what) + ": " + hipGetErrorString(e));
}


// bf16 bits of x, round to nearest even (via FP32; finite inputs)
static uint32_t bf16_bits(double x) {
  const float f = (float)x;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
static double bf16_value(uint32_t h) {
  const uint32_t u = h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

// Column tiling of the fused kernels: each workgroup owns every voxel row i1
// (2*n1 real rows, split over wm waves of nb 32-row MFMA blocks) and
// nwg = 32*wn columns (i2, i3) of the mode-1 unfolding, t2 values of i2 by
// t3 = nwg / t2 values of i3.  t2 = 0 picks the shape covering the fewest
// columns beyond the grid.
int nb_cap(const tv_plan_s* p, int op) {
  // the adjoint keeps the y tile in registers next to the accumulators: 2 row
  // blocks per wave keep two workgroups per CU resident; 3 pad short voxel
  // rows less (81 rows: 96 instead of 128) at one workgroup per CU, so the
  // autotuner times both
  return op == 1 ? (p ? p->nbcap_a : 2) : 8;
}

tv_status make_tiling(const tv_grid& g, int t2req, int nbcap, Tiling* T) {
  const int nbt0 = (g.n1 + 15) / 16;
  int wm = 1;
  while ((nbt0 + wm - 1) / wm > 8) wm *= 2;
  while ((nbt0 + wm - 1) / wm > nbcap && wm < 4) wm *= 2;
  if (wm > 4) return set_error(TV_ERR_NOT_SUPPORTED, "n1 > 512 is not built");
  T->wm = wm;
  T->nb = (nbt0 + wm - 1) / wm;
  T->nbt = T->nb * wm;
  T->n1p = 16 * T->nbt;
  T->wn = 4 / wm;
  T->nwg = 32 * T->wn;
  if (t2req) {
    if (t2req < 2 || t2req > T->nwg || (T->nwg % t2req) != 0)
      return set_error(TV_ERR_INVALID_ARG, "t2 must divide the workgroup's columns and be >= 2");
    T->t2 = t2req;
    T->t3 = T->nwg / t2req;
  } else {
    int64_t best = -1;
    for (int t2 = T->nwg; t2 >= 2; t2 /= 2) {  // column pairs share one i3
      const int t3 = T->nwg / t2;
      const int64_t cover =
          (int64_t)((g.n2 + t2 - 1) / t2) * t2 * ((g.n3 + t3 - 1) / t3) * t3;
      if (best < 0 || cover < best) {
        best = cover;
        T->t2 = t2;
        T->t3 = t3;
      }
    }
  }
  T->tiles2 = (g.n2 + T->t2 - 1) / T->t2;
  T->tiles3 = (g.n3 + T->t3 - 1) / T->t3;
  T->tiles = (int64_t)T->tiles2 * T->tiles3;
  return TV_OK;
}


static tv_status validate_grid(const tv_grid* g) {
  if (!g) return set_error(TV_ERR_INVALID_ARG, "grid is NULL");
  if (g->n1 < 1 || g->n2 < 1 || g->n3 < 1 || g->q < 1 || g->m < 1)
    return set_error(TV_ERR_SHAPE, "grid sizes must be >= 1");
  if ((int64_t)g->n1 * g->n2 * g->n3 * g->q > (int64_t)1 << 40)
    return set_error(TV_ERR_SHAPE, "grid too large");
  if (g->m > (int64_t)1 << 30) return set_error(TV_ERR_SHAPE, "too many columns");
  return TV_OK;
}

// Device arena of a plan: every packed array at a 256-byte aligned offset, in
// a fixed order.  With base == nullptr only the size is computed; otherwise
// the plan's device pointers are set into [base, base + size).
static size_t arena_layout(tv_plan_s* p, char* base) {
  size_t off = 0;
  auto carve = [&](auto** ptr, size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    typedef typename std::remove_reference<decltype(**ptr)>::type T;
    if (base) *ptr = bytes ? reinterpret_cast<T*>(base + off) : nullptr;
    off += bytes;
  };
  const HostPack& h = p->hp;
  const size_t splits = (size_t)p->grid.q * (TV_SPLIT_MAX + 1) * sizeof(int32_t);
  carve(&p->d_meta, h.meta.size() * sizeof(TensorMeta));
  carve(&p->d_cores, h.cores.size() * sizeof(float2));
  carve(&p->d_u1t, h.u1t.size() * sizeof(float2));
  carve(&p->d_u2t, h.u2t.size() * sizeof(float2));
  carve(&p->d_u3t, h.u3t.size() * sizeof(float2));
  carve(&p->d_apack, h.apack.size() * sizeof(float));
  carve(&p->d_apack_bf, h.apack_bf.size() * sizeof(uint4));
  carve(&p->d_apack_koff, p->apack_koff.size() * sizeof(int64_t));
  carve(&p->d_split_f, splits);
  carve(&p->d_split_a, splits);
  carve(&p->d_apack4, h.a4.size() * sizeof(float));
  carve(&p->d_abf, h.abf.size() * sizeof(uint4));
  carve(&p->d_drow, h.drow.size() * sizeof(int32_t));
  return (off + 255) & ~(size_t)255;
}

static void clear_device_pointers(tv_plan_s* p) {
  p->d_meta = nullptr;
  p->d_cores = p->d_u1t = p->d_u2t = p->d_u3t = nullptr;
  p->d_apack = nullptr;
  p->d_apack_bf = nullptr;
  p->d_apack_koff = nullptr;
  p->d_split_f = p->d_split_a = nullptr;
  p->d_apack4 = nullptr;
  p->d_abf = nullptr;
  p->d_drow = nullptr;
  p->bound = false;
}

// Offsets of every tensor's factors in the concatenated host arrays.
static tv_status compute_offsets(tv_plan_s* p) {
  const tv_grid& g = p->grid;
  const int64_t K = (int64_t)g.q * g.m;
  p->g_off.assign(K + 1, 0);
  p->u1_off.assign(K + 1, 0);
  p->u2_off.assign(K + 1, 0);
  p->u3_off.assign(K + 1, 0);
  const int dims[3] = {g.n1, g.n2, g.n3};
  for (int d = 0; d < 3; ++d) p->max_r[d] = 0;
  p->max_r12 = 0;
  p->max_core = 0;
  p->sum_r1 = 0;
  for (int64_t t = 0; t < K; ++t) {
    const int32_t* r = &p->ranks[3 * t];
    for (int d = 0; d < 3; ++d) {
      if (r[d] < 1 || r[d] > dims[d] || r[d] > TV_MAX_RANK) {
        char buf[160];
        snprintf(buf, sizeof buf, "tensor %lld mode %d rank %d outside [1, min(%d, %d)]",
                 (long long)t, d + 1, r[d], dims[d], TV_MAX_RANK);
        return set_error(TV_ERR_RANK, buf);
      }
      p->max_r[d] = std::max(p->max_r[d], (int)r[d]);
    }
    p->sum_r1 += r[0];
    p->max_r12 = std::max(p->max_r12, (int)(r[0] * r[1]));
    p->max_core = std::max(p->max_core, (int64_t)r[0] * r[1] * r[2]);
    p->g_off[t + 1] = p->g_off[t] + (int64_t)r[0] * r[1] * r[2];
    p->u1_off[t + 1] = p->u1_off[t] + (int64_t)g.n1 * r[0];
    p->u2_off[t + 1] = p->u2_off[t] + (int64_t)g.n2 * r[1];
    p->u3_off[t + 1] = p->u3_off[t] + (int64_t)g.n3 * r[2];
  }
  return TV_OK;
}

// Balanced column ranges per component: S contiguous ranges with about
// equal sum of r1 (the K extent of the stacked mode-1 GEMM).
static std::vector<int32_t> make_split(const tv_plan_s* p, int S) {
  const tv_grid& g = p->grid;
  std::vector<int32_t> out((size_t)g.q * (S + 1));
  for (int k = 0; k < g.q; ++k) {
    const int64_t total = p->sum_r1_k[k];
    int64_t acc = 0;
    int s = 1;
    out[(size_t)k * (S + 1)] = 0;
    for (int64_t j = 0; j < g.m && s < S; ++j) {
      acc += p->ranks[3 * (k + (int64_t)g.q * j)];
      while (s < S && acc * S >= total * s) out[(size_t)k * (S + 1) + s++] = (int32_t)(j + 1);
    }
    while (s < S) out[(size_t)k * (S + 1) + s++] = (int32_t)g.m;
    out[(size_t)k * (S + 1) + S] = (int32_t)g.m;
  }
  return out;
}

tv_status set_split(tv_plan_s* p, int op, int S) {
  S = (int)std::max<int64_t>(1, std::min<int64_t>(std::min(S, TV_SPLIT_MAX), p->grid.m));
  if (p->bound) {
    // [q][S + 1] first column of each split, within the region reserved for
    // TV_SPLIT_MAX splits
    std::vector<int32_t> sp = make_split(p, S);
    hipError_t e = hipMemcpy(op == 0 ? p->d_split_f : p->d_split_a, sp.data(),
                             sp.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "split table upload");
  }
  if (op == 0)
    p->split_f = S;
  else
    p->split_a = S;
  return TV_OK;
}

// FP32 copies of one tensor's factors (ranks r, FP64 interleaved inputs):
// the core as is, U1..U3 transposed to row-major (i, rank).
static void pack_tensor_f32(const tv_grid& g, const int32_t* r, const double* core,
                            const double* u1, const double* u2, const double* u3, float2* dc,
                            float2* d1, float2* d2, float2* d3) {
  const int64_t nc = (int64_t)r[0] * r[1] * r[2];
  for (int64_t i = 0; i < nc; ++i) dc[i] = make_float2((float)core[2 * i], (float)core[2 * i + 1]);
  auto transpose = [](int n, int rk, const double* u, float2* d) {
    for (int a = 0; a < rk; ++a)
      for (int i = 0; i < n; ++i) {
        const size_t src = i + (size_t)n * a;
        d[(size_t)i * rk + a] = make_float2((float)u[2 * src], (float)u[2 * src + 1]);
      }
  };
  transpose(g.n1, r[0], u1, d1);
  transpose(g.n2, r[1], u2, d2);
  transpose(g.n3, r[2], u3, d3);
}

// Stacked U1 rows of one tensor in MFMA A-operand lane order, as the real
// embedding A_emb[2 i1 + s][(a, p)] = Ar (s == p), -Ai (s = 0, p = 1),
// Ai (s = 1, p = 0) of U1 (n1 x r1, FP64 interleaved, column-major).
// FP32: r1 rows of nbt * 64 floats, rows[(a * nbt + blk) * 64 + lane] =
//   A_emb[32 blk + lane % 32][(a, lane / 32)]; voxel row i1 fills embedded
//   rows 2 i1 (Re) and 2 i1 + 1 (Im) of both K slots; rows past n1 are zero.
static void pack_apack_f32(const tv_grid& g, int r1, const double* u1, int nbt, float* rows) {
  std::fill(rows, rows + (size_t)r1 * nbt * 64, 0.f);
  const int n1 = std::min(g.n1, nbt * 16);
  for (int a = 0; a < r1; ++a) {
    float* row = rows + (size_t)a * nbt * 64;
    const double* u = u1 + 2 * (size_t)g.n1 * a;
    for (int i1 = 0; i1 < n1; ++i1) {
      const float ar = (float)u[2 * i1], ai = (float)u[2 * i1 + 1];
      float* rb = row + ((2 * i1) >> 5) * 64 + ((2 * i1) & 31);
      rb[0] = ar;    // (Re row, Re part)
      rb[32] = -ai;  // (Re row, Im part)
      rb[1] = ai;    // (Im row, Re part)
      rb[33] = ar;   // (Im row, Im part)
    }
  }
}

// BF16X3: ceil(r1 / 8) chunks of nbt * 128 uint4,
//   chunks[((c * nbt + blk) * 2 + hl) * 64 + lane] = 8 bf16 (hi or lo) for K
//   slots 8 (lane / 32) + i, i < 8, slot k = (row 8 c + k / 2, part k % 2).
static void pack_apack_bf(const tv_grid& g, int r1, const double* u1, int nbt, uint4* chunks) {
  const int nch = (r1 + 7) / 8;
  for (int c = 0; c < nch; ++c)
    for (int blk = 0; blk < nbt; ++blk)
      for (int lane = 0; lane < 64; ++lane) {
        const int mrow = 32 * blk + (lane & 31), i1 = mrow >> 1, srow = mrow & 1;
        uint32_t hi[8], lo[8];
        for (int i = 0; i < 8; ++i) {
          const int kk = 8 * (lane >> 5) + i, a = 8 * c + kk / 2, pp = kk % 2;
          double v = 0.0;
          if (i1 < g.n1 && a < r1) {
            const size_t src = i1 + (size_t)g.n1 * a;
            const double ar = u1[2 * src], ai = u1[2 * src + 1];
            v = srow == pp ? ar : (srow == 0 ? -ai : ai);
          }
          hi[i] = bf16_bits(v);
          lo[i] = bf16_bits(v - bf16_value(hi[i]));
        }
        uint4* dst = &chunks[((size_t)(c * nbt + blk) * 2) * 64 + lane];
        dst[0] = make_uint4(hi[0] | (hi[1] << 16), hi[2] | (hi[3] << 16), hi[4] | (hi[5] << 16),
                            hi[6] | (hi[7] << 16));
        dst[64] = make_uint4(lo[0] | (lo[1] << 16), lo[2] | (lo[3] << 16), lo[4] | (lo[5] << 16),
                             lo[6] | (lo[7] << 16));
      }
}

// Pack the FP64 host factors into the device layouts of the kernels (host
// side; the device copy is made by tv_plan_bind_arena).
static tv_status pack_plan(tv_plan_s* p) {
  const tv_grid& g = p->grid;
  const int64_t K = (int64_t)g.q * g.m;
  tv_status st = make_tiling(g, 0, nb_cap(p, 0), &p->tiling);
  if (st != TV_OK) return st;
  if ((st = make_tiling(g, 0, nb_cap(p, 1), &p->tiling_a)) != TV_OK) return st;
  if (fused_lds_bytes(p, p->tiling, false) > 160 * 1024 ||
      fused_lds_bytes(p, p->tiling_a, true) > 160 * 1024)
    return set_error(TV_ERR_NOT_SUPPORTED, "ranks too large for the LDS tile");
  // the stacked A operand is packed for the larger row-block count of the
  // two kernels; blocks past n1 are zero rows
  const int nbt = std::max(p->tiling.nbt, p->tiling_a.nbt);
  p->nbt_pack = nbt;

  // per-tensor metadata, component-major [k][j]
  const bool bf = p->precision == TV_PREC_BF16X3;
  std::vector<TensorMeta> meta((size_t)K);
  std::vector<int64_t> chunks_k(g.q, 0);
  p->sum_r1_k.assign(g.q, 0);
  for (int64_t j = 0; j < g.m; ++j)
    for (int k = 0; k < g.q; ++k) {
      const int64_t t = k + (int64_t)g.q * j;
      TensorMeta& M = meta[(size_t)k * g.m + j];
      M.r1 = p->ranks[3 * t];
      M.r2 = p->ranks[3 * t + 1];
      M.r3 = p->ranks[3 * t + 2];
      M.arow = (int32_t)(bf ? chunks_k[k] : p->sum_r1_k[k]);
      M.g_off = p->g_off[t];
      M.u2_off = p->u2_off[t];
      M.u3_off = p->u3_off[t];
      M.u1_off = p->u1_off[t];
      p->sum_r1_k[k] += M.r1;
      chunks_k[k] += (M.r1 + 7) / 8;
    }

  std::vector<float2> cores((size_t)p->g_off[K]);
  std::vector<float2> u1t((size_t)p->u1_off[K]), u2t((size_t)p->u2_off[K]),
      u3t((size_t)p->u3_off[K]);
  for (int64_t t = 0; t < K; ++t)
    pack_tensor_f32(g, &p->ranks[3 * t], &p->cores[2 * p->g_off[t]], &p->u1[2 * p->u1_off[t]],
                    &p->u2[2 * p->u2_off[t]], &p->u3[2 * p->u3_off[t]], &cores[p->g_off[t]],
                    &u1t[p->u1_off[t]], &u2t[p->u2_off[t]], &u3t[p->u3_off[t]]);

  p->apack_koff.assign(g.q + 1, 0);
  std::vector<float> apack;
  std::vector<uint4> apack_bf;
  for (int k = 0; k < g.q; ++k)
    p->apack_koff[k + 1] =
        p->apack_koff[k] + (bf ? chunks_k[k] * nbt * 128 : p->sum_r1_k[k] * nbt * 64);
  if (!bf)
    apack.resize((size_t)p->apack_koff[g.q]);
  else
    apack_bf.resize((size_t)p->apack_koff[g.q]);
  for (int64_t j = 0; j < g.m; ++j)
    for (int k = 0; k < g.q; ++k) {
      const int64_t t = k + (int64_t)g.q * j;
      const TensorMeta& M = meta[(size_t)k * g.m + j];
      const double* u1 = &p->u1[2 * p->u1_off[t]];
      if (!bf)
        pack_apack_f32(g, M.r1, u1, nbt, &apack[p->apack_koff[k] + (int64_t)M.arow * nbt * 64]);
      else
        pack_apack_bf(g, M.r1, u1, nbt,
                      &apack_bf[p->apack_koff[k] + (int64_t)M.arow * nbt * 128]);
    }

  // column splits: spread the work over enough workgroups to fill the chip
  const int64_t base_f = (int64_t)g.q * p->tiling.tiles, base_a = (int64_t)g.q * p->tiling_a.tiles;
  int sf = (int)std::min<int64_t>(8, std::max<int64_t>(1, (1024 + base_f - 1) / base_f));
  int sa = (int)std::min<int64_t>(64, std::max<int64_t>(1, (1024 + base_a - 1) / base_a));
  p->split_f = (int)std::max<int64_t>(1, std::min<int64_t>(sf, g.m));
  p->split_a = (int)std::max<int64_t>(1, std::min<int64_t>(sa, g.m));

  clear_device_pointers(p);
  p->hp.meta = std::move(meta);
  p->hp.cores = std::move(cores);
  p->hp.u1t = std::move(u1t);
  p->hp.u2t = std::move(u2t);
  p->hp.u3t = std::move(u3t);
  p->hp.apack = std::move(apack);
  p->hp.apack_bf = std::move(apack_bf);
  if (p->with_dtg && (st = dtg_pack(p, p->hp.meta)) != TV_OK) return st;
  p->device_bytes = arena_layout(p, nullptr);
  p->finalized = true;
  return TV_OK;
}

// Upload the packed plan into [arena, arena + bytes) (set-up call; waits for
// the copies, then releases the host-side packed copies).
static tv_status bind_arena(tv_plan_s* p, void* arena, size_t bytes, hipStream_t st) {
  arena_layout(p, (char*)arena);
  const HostPack& h = p->hp;
  hipError_t e = hipSuccess;
  auto put = [&](void* d, const void* src, size_t n) {
    if (e == hipSuccess && n) e = hipMemcpyAsync(d, src, n, hipMemcpyHostToDevice, st);
  };
  put(p->d_meta, h.meta.data(), h.meta.size() * sizeof(TensorMeta));
  put(p->d_cores, h.cores.data(), h.cores.size() * sizeof(float2));
  put(p->d_u1t, h.u1t.data(), h.u1t.size() * sizeof(float2));
  put(p->d_u2t, h.u2t.data(), h.u2t.size() * sizeof(float2));
  put(p->d_u3t, h.u3t.data(), h.u3t.size() * sizeof(float2));
  put(p->d_apack, h.apack.data(), h.apack.size() * sizeof(float));
  put(p->d_apack_bf, h.apack_bf.data(), h.apack_bf.size() * sizeof(uint4));
  put(p->d_apack_koff, p->apack_koff.data(), p->apack_koff.size() * sizeof(int64_t));
  put(p->d_apack4, h.a4.data(), h.a4.size() * sizeof(float));
  put(p->d_abf, h.abf.data(), h.abf.size() * sizeof(uint4));
  put(p->d_drow, h.drow.data(), h.drow.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    clear_device_pointers(p);
    return hip_error(e, "plan upload");
  }
  (void)bytes;
  p->bound = true;
  tv_status s = set_split(p, 0, p->split_f);
  if (s == TV_OK) s = set_split(p, 1, p->split_a);
  if (s != TV_OK) {
    clear_device_pointers(p);
    return s;
  }
  p->hp = HostPack();
  return TV_OK;
}

static bool all_finite(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

tv_status finalize_plan(tv_plan_s* p) { return pack_plan(p); }

tv_status validate_ranks_and_offsets(tv_plan_s* p) { return compute_offsets(p); }

}  // namespace tv

using namespace tv;

extern "C" {

const char* tv_status_string(tv_status s) {
  switch (s) {
    case TV_OK: return "TV_OK";
    case TV_ERR_INVALID_ARG: return "TV_ERR_INVALID_ARG";
    case TV_ERR_SHAPE: return "TV_ERR_SHAPE";
    case TV_ERR_RANK: return "TV_ERR_RANK";
    case TV_ERR_OOM: return "TV_ERR_OOM";
    case TV_ERR_HIP: return "TV_ERR_HIP";
    case TV_ERR_NOT_SUPPORTED: return "TV_ERR_NOT_SUPPORTED";
    case TV_ERR_NUMERIC: return "TV_ERR_NUMERIC";
    case TV_ERR_WORKSPACE: return "TV_ERR_WORKSPACE";
  }
  return "TV_ERR_UNKNOWN";
}

const char* tv_last_error(void) { return g_last_error.c_str(); }

tv_status tv_plan_from_factors(const tv_grid* grid, const int32_t* ranks, const double* cores,
                               const double* u1, const double* u2, const double* u3,
                               tv_precision precision, tv_plan* out) {
  clear_error();
  if (!out) return set_error(TV_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  tv_status st = validate_grid(grid);
  if (st != TV_OK) return st;
  if (!ranks || !cores || !u1 || !u2 || !u3)
    return set_error(TV_ERR_INVALID_ARG, "ranks and factor arrays must be non-NULL");
  if (precision != TV_PREC_FP32 && precision != TV_PREC_BF16X3)
    return set_error(TV_ERR_INVALID_ARG, "unknown precision");
  tv_plan_s* p = new (std::nothrow) tv_plan_s;
  if (!p) return set_error(TV_ERR_OOM, "host allocation");
  p->grid = *grid;
  p->precision = precision;
  p->with_dtg = true;
  p->appended = grid->m;
  const int64_t K = (int64_t)grid->q * grid->m;
  p->ranks.assign(ranks, ranks + 3 * K);
  if ((st = compute_offsets(p)) != TV_OK) {
    delete p;
    return st;
  }
  try {
    p->cores.assign(cores, cores + 2 * p->g_off[K]);
    p->u1.assign(u1, u1 + 2 * p->u1_off[K]);
    p->u2.assign(u2, u2 + 2 * p->u2_off[K]);
    p->u3.assign(u3, u3 + 2 * p->u3_off[K]);
  } catch (const std::bad_alloc&) {
    delete p;
    return set_error(TV_ERR_OOM, "host copy of factors");
  }
  if (!all_finite(p->cores.data(), p->cores.size()) || !all_finite(p->u1.data(), p->u1.size()) ||
      !all_finite(p->u2.data(), p->u2.size()) || !all_finite(p->u3.data(), p->u3.size())) {
    delete p;
    return set_error(TV_ERR_NUMERIC, "non-finite factor values");
  }
  if ((st = pack_plan(p)) != TV_OK) {
    delete p;
    return st;
  }
  *out = p;
  return TV_OK;
}

}  // extern "C"

namespace tv {

// Staging of one growable-plan append: the metadata of every tensor and one
// column's q tensors of every other array, each piece 16-byte aligned.
static size_t stage_size(const tv_grid& g, const int rmax[3], int nbt, tv_precision precision) {
  const size_t K = (size_t)g.q * g.m;
  const size_t r1 = rmax[0], r2 = rmax[1], r3 = rmax[2];
  const bool bf = precision == TV_PREC_BF16X3;
  return K * sizeof(TensorMeta) +
         (size_t)g.q * (r1 * r2 * r3 + g.n1 * r1 + g.n2 * r2 + g.n3 * r3) * sizeof(float2) +
         (bf ? (size_t)g.q * ((r1 + 7) / 8) * nbt * 128 * sizeof(uint4)
             : (size_t)g.q * r1 * nbt * 64 * sizeof(float)) +
         (size_t)2 * g.q * (TV_SPLIT_MAX + 1) * sizeof(int32_t) + K * sizeof(int32_t) +
         (size_t)(g.q + 9) * 16;
}

// Device layout of a plan holding up to g.m columns at ranks up to rmax, in
// the order of arena_layout, every array at its capacity; with p and base
// set, p's device pointers are carved from base.
static size_t capacity_layout(const tv_grid& g, const int rmax[3], int nbt,
                              tv_precision precision, tv_plan_s* p, char* base) {
  const size_t K = (size_t)g.q * g.m;
  const size_t r1 = rmax[0], r2 = rmax[1], r3 = rmax[2];
  const bool bf = precision == TV_PREC_BF16X3;
  size_t off = 0;
  auto carve = [&](auto** ptr, size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    typedef typename std::remove_reference<decltype(**ptr)>::type T;
    if (p && base) *ptr = bytes ? reinterpret_cast<T*>(base + off) : nullptr;
    off += bytes;
  };
  tv_plan_s dummy;
  tv_plan_s* d = p ? p : &dummy;
  carve(&d->d_meta, K * sizeof(TensorMeta));
  carve(&d->d_cores, K * r1 * r2 * r3 * sizeof(float2));
  carve(&d->d_u1t, K * g.n1 * r1 * sizeof(float2));
  carve(&d->d_u2t, K * g.n2 * r2 * sizeof(float2));
  carve(&d->d_u3t, K * g.n3 * r3 * sizeof(float2));
  carve(&d->d_apack, bf ? 0 : K * r1 * nbt * 64 * sizeof(float));
  carve(&d->d_apack_bf, bf ? K * ((r1 + 7) / 8) * nbt * 128 * sizeof(uint4) : 0);
  carve(&d->d_apack_koff, (size_t)(g.q + 1) * sizeof(int64_t));
  carve(&d->d_split_f, (size_t)g.q * (TV_SPLIT_MAX + 1) * sizeof(int32_t));
  carve(&d->d_split_a, (size_t)g.q * (TV_SPLIT_MAX + 1) * sizeof(int32_t));
  carve(&d->d_drow, K * sizeof(int32_t));
  const size_t stage = stage_size(g, rmax, nbt, precision);
  carve(&d->d_stage, stage);
  if (p && base) p->stage_bytes = stage;
  return (off + 255) & ~(size_t)255;
}

void grow_plan_set_stage(tv_plan p, const HostStage& stage, size_t adj_ws_bytes) {
  p->grow_pinned = stage.ptr;
  p->grow_pinned_bytes = stage.bytes;
  p->grow_adj_ws = adj_ws_bytes;
}

static int pack_nbt(const tv_grid& g, int nbcap_a) {
  // the packed U1 rows hold the larger row-block count of the forward (8
  // blocks per wave) and adjoint tilings
  Tiling Tf, Ta;
  if (make_tiling(g, 0, 8, &Tf) != TV_OK || make_tiling(g, 0, nbcap_a, &Ta) != TV_OK) return 0;
  return std::max(Tf.nbt, Ta.nbt);
}

size_t grow_stage_bytes(const tv_grid& g, const int rmax[3], tv_precision precision) {
  const int nbt = pack_nbt(g, 2);
  return nbt ? stage_size(g, rmax, nbt, precision) : 0;
}

// Growable plans run their adjoint as the column GEMM of tv_dtg.hip (its
// operands are the plan's U1 rows, cores, U2 and U3 and the caller's y, so
// only the stacked row layout follows the appends): set-up for the plan's
// geometry, then the padded rows per component after each append. Rows of
// A_k are padded to the GEMM's k-step of 16, as dtg_pack pads them.
constexpr int kDtgRowPad = 16;
static void dtg_grow_setup(tv_plan_s* p) {
  if (p->grid.q > DTG_MAXQ_HOST) return;
  const int MT = dtg_mt(p);
  p->dtg_nbtp = (p->nbt_pack + MT - 1) / MT * MT;
  p->dtg_rpad.assign(p->grid.q, 0);
  p->dtg_rows = 0;
  p->dtg_packed = true;
}

static void dtg_grow_rows(tv_plan_s* p) {
  if (!p->dtg_packed) return;
  p->dtg_rows = 0;
  for (int k = 0; k < p->grid.q; ++k) {
    p->dtg_rpad[k] = (p->sum_r1_k[k] + kDtgRowPad - 1) / kDtgRowPad * kDtgRowPad;
    p->dtg_rows += p->dtg_rpad[k];
  }
}

size_t grow_adjoint_ws_bytes(const tv_grid& g, const int rmax[3]) {
  const int nbt = pack_nbt(g, 2);
  if (!nbt || g.q > DTG_MAXQ_HOST) return 0;
  tv_plan_s t;
  t.grid = g;
  t.nbt_pack = nbt;
  dtg_grow_setup(&t);
  t.dtg_rows = (int64_t)g.q * (((int64_t)g.m * rmax[0] + kDtgRowPad - 1) / kDtgRowPad * kDtgRowPad);
  return dtg_workspace_bytes(&t, 1);
}

size_t plan_arena_bound(const tv_grid& g, const int rmax[3], tv_precision precision) {
  const int nbt = pack_nbt(g, 2);
  return nbt ? capacity_layout(g, rmax, nbt, precision, nullptr, nullptr) : 0;
}

tv_status grow_plan_create(const tv_grid& g, const int rmax[3], tv_precision precision,
                           void* arena, size_t bytes, hipStream_t st, tv_plan* out) {
  *out = nullptr;
  tv_status s = validate_grid(&g);
  if (s != TV_OK) return s;
  if (precision != TV_PREC_FP32 && precision != TV_PREC_BF16X3)
    return set_error(TV_ERR_INVALID_ARG, "unknown precision");
  const int dims[3] = {g.n1, g.n2, g.n3};
  for (int d = 0; d < 3; ++d)
    if (rmax[d] < 1 || rmax[d] > std::min(dims[d], TV_MAX_RANK))
      return set_error(TV_ERR_RANK, "growable plan: rank cap outside [1, min(n, TV_MAX_RANK)]");
  if (!arena || (uintptr_t)arena % 256)
    return set_error(TV_ERR_INVALID_ARG, "arena must be non-NULL and 256-byte aligned");
  if (g.q + 8 > kMaxCopySegs)
    return set_error(TV_ERR_NOT_SUPPORTED, "growable plan: too many components");
  tv_plan_s* p = new (std::nothrow) tv_plan_s;
  if (!p) return set_error(TV_ERR_OOM, "host allocation");
  p->grid = g;
  p->grid.m = 0;
  p->precision = precision;
  p->with_dtg = false;
  p->grow_mcap = g.m;
  for (int d = 0; d < 3; ++d) p->grow_rcap[d] = rmax[d];
  if ((s = make_tiling(g, 0, nb_cap(p, 0), &p->tiling)) != TV_OK ||
      (s = make_tiling(g, 0, nb_cap(p, 1), &p->tiling_a)) != TV_OK) {
    delete p;
    return s;
  }
  const int nbt = std::max(p->tiling.nbt, p->tiling_a.nbt);
  p->nbt_pack = nbt;
  const size_t need = capacity_layout(g, rmax, nbt, precision, nullptr, nullptr);
  if (bytes < need) {
    delete p;
    char buf[128];
    snprintf(buf, sizeof buf, "growable plan arena of %zu bytes needed, %zu given", need, bytes);
    return set_error(TV_ERR_WORKSPACE, buf);
  }
  capacity_layout(g, rmax, nbt, precision, p, (char*)arena);
  const bool bf = precision == TV_PREC_BF16X3;
  const int64_t cap_k = bf ? g.m * (int64_t)((rmax[0] + 7) / 8) * nbt * 128
                           : g.m * (int64_t)rmax[0] * nbt * 64;
  p->apack_koff.resize(g.q + 1);
  for (int k = 0; k <= g.q; ++k) p->apack_koff[k] = k * cap_k;
  p->sum_r1_k.assign(g.q, 0);
  p->grow_chunks_k.assign(g.q, 0);
  p->g_off.assign(1, 0);
  p->u1_off.assign(1, 0);
  p->u2_off.assign(1, 0);
  p->u3_off.assign(1, 0);
  dtg_grow_setup(p);
  hipError_t e = hipMemcpyAsync(p->d_apack_koff, p->apack_koff.data(),
                                p->apack_koff.size() * sizeof(int64_t), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete p;
    return hip_error(e, "growable plan set-up");
  }
  p->finalized = true;
  p->bound = true;
  *out = p;
  return TV_OK;
}

tv_status grow_plan_append(tv_plan p, const int32_t* ranks, const double* cores,
                           const double* u1, const double* u2, const double* u3,
                           hipStream_t st) {
  if (!p || !p->grow_mcap) return set_error(TV_ERR_INVALID_ARG, "not a growable plan");
  tv_grid& g = p->grid;
  const int64_t j = g.m;
  if (j >= p->grow_mcap) return set_error(TV_ERR_SHAPE, "growable plan is full");
  const int dims[3] = {g.n1, g.n2, g.n3};
  for (int k = 0; k < g.q; ++k)
    for (int d = 0; d < 3; ++d)
      if (ranks[3 * k + d] < 1 || ranks[3 * k + d] > p->grow_rcap[d] ||
          ranks[3 * k + d] > dims[d])
        return set_error(TV_ERR_RANK, "growable plan: rank above the plan's cap");
  const bool bf = p->precision == TV_PREC_BF16X3;
  const int nbt = p->nbt_pack;
  const int64_t t0 = (int64_t)g.q * j;
  // new tensors' offsets, ranks and running maxima
  int max_r[3] = {p->max_r[0], p->max_r[1], p->max_r[2]};
  int max_r12 = p->max_r12;
  int64_t max_core = p->max_core;
  for (int k = 0; k < g.q; ++k) {
    const int32_t* r = &ranks[3 * k];
    for (int d = 0; d < 3; ++d) max_r[d] = std::max(max_r[d], (int)r[d]);
    max_r12 = std::max(max_r12, (int)(r[0] * r[1]));
    max_core = std::max(max_core, (int64_t)r[0] * r[1] * r[2]);
  }
  {
    // the fused kernels' LDS tile at the new maxima
    tv_plan_s probe;
    for (int d = 0; d < 3; ++d) probe.max_r[d] = max_r[d];
    probe.max_r12 = max_r12;
    probe.max_core = max_core;
    if (fused_lds_bytes(&probe, p->tiling, false) > 160 * 1024 ||
        fused_lds_bytes(&probe, p->tiling_a, true) > 160 * 1024)
      return set_error(TV_ERR_NOT_SUPPORTED, "ranks too large for the LDS tile");
  }
  HostPack& H = p->grow_stage;
  int64_t nc = 0, n1 = 0, n2 = 0, n3 = 0;
  for (int k = 0; k < g.q; ++k) {
    const int32_t* r = &ranks[3 * k];
    nc += (int64_t)r[0] * r[1] * r[2];
    n1 += (int64_t)g.n1 * r[0];
    n2 += (int64_t)g.n2 * r[1];
    n3 += (int64_t)g.n3 * r[2];
  }
  if (!all_finite(cores, 2 * nc) || !all_finite(u1, 2 * n1) || !all_finite(u2, 2 * n2) ||
      !all_finite(u3, 2 * n3))
    return set_error(TV_ERR_NUMERIC, "non-finite factor values");
  H.cores.resize(nc);
  H.u1t.resize(n1);
  H.u2t.resize(n2);
  H.u3t.resize(n3);
  int64_t oc = 0, o1 = 0, o2 = 0, o3 = 0, arows = 0;
  for (int k = 0; k < g.q; ++k) {
    const int32_t* r = &ranks[3 * k];
    pack_tensor_f32(g, r, cores + 2 * oc, u1 + 2 * o1, u2 + 2 * o2, u3 + 2 * o3, &H.cores[oc],
                    &H.u1t[o1], &H.u2t[o2], &H.u3t[o3]);
    oc += (int64_t)r[0] * r[1] * r[2];
    o1 += (int64_t)g.n1 * r[0];
    o2 += (int64_t)g.n2 * r[1];
    o3 += (int64_t)g.n3 * r[2];
    arows += bf ? (r[0] + 7) / 8 : r[0];
  }
  // stacked U1 rows of the new tensors, component by component
  if (!bf)
    H.apack.resize((size_t)arows * nbt * 64);
  else
    H.apack_bf.resize((size_t)arows * nbt * 128);
  std::vector<int64_t> arow_new(g.q);
  o1 = 0;
  arows = 0;
  for (int k = 0; k < g.q; ++k) {
    const int r1 = ranks[3 * k];
    arow_new[k] = bf ? p->grow_chunks_k[k] : p->sum_r1_k[k];
    if (!bf)
      pack_apack_f32(g, r1, u1 + 2 * o1, nbt, &H.apack[(size_t)arows * nbt * 64]);
    else
      pack_apack_bf(g, r1, u1 + 2 * o1, nbt, &H.apack_bf[(size_t)arows * nbt * 128]);
    o1 += (int64_t)g.n1 * r1;
    arows += bf ? (r1 + 7) / 8 : r1;
  }
  // commit the host state
  for (int k = 0; k < g.q; ++k) {
    const int32_t* r = &ranks[3 * k];
    p->ranks.insert(p->ranks.end(), r, r + 3);
    const int64_t t = t0 + k;
    p->g_off.push_back(p->g_off[t] + (int64_t)r[0] * r[1] * r[2]);
    p->u1_off.push_back(p->u1_off[t] + (int64_t)g.n1 * r[0]);
    p->u2_off.push_back(p->u2_off[t] + (int64_t)g.n2 * r[1]);
    p->u3_off.push_back(p->u3_off[t] + (int64_t)g.n3 * r[2]);
    p->sum_r1_k[k] += r[0];
    p->grow_chunks_k[k] += (r[0] + 7) / 8;
    p->sum_r1 += r[0];
  }
  for (int d = 0; d < 3; ++d) p->max_r[d] = max_r[d];
  p->max_r12 = max_r12;
  p->max_core = max_core;
  g.m = j + 1;
  const int64_t K = (int64_t)g.q * g.m;
  // metadata, component-major [k][j]
  H.meta.resize(K);
  {
    std::vector<int64_t> row(g.q, 0);
    for (int64_t jj = 0; jj < g.m; ++jj)
      for (int k = 0; k < g.q; ++k) {
        const int64_t t = k + (int64_t)g.q * jj;
        TensorMeta& M = H.meta[(size_t)k * g.m + jj];
        M.r1 = p->ranks[3 * t];
        M.r2 = p->ranks[3 * t + 1];
        M.r3 = p->ranks[3 * t + 2];
        M.arow = (int32_t)row[k];
        M.g_off = p->g_off[t];
        M.u2_off = p->u2_off[t];
        M.u3_off = p->u3_off[t];
        M.u1_off = p->u1_off[t];
        row[k] += bf ? (M.r1 + 7) / 8 : M.r1;
      }
  }
  // stacked row of each tensor's first U1 column in A_k, [k][j] (the column
  // GEMM's layout: no padding between tensors), and the adjoint's path
  H.drow.resize(K);
  {
    std::vector<int64_t> row(g.q, 0);
    for (int64_t jj = 0; jj < g.m; ++jj)
      for (int k = 0; k < g.q; ++k) {
        H.drow[(size_t)k * g.m + jj] = (int32_t)row[k];
        row[k] += p->ranks[3 * (k + (int64_t)g.q * jj)];
      }
  }
  dtg_grow_rows(p);
  if (p->dtg_packed) {
    // column splits of the adjoint's column GEMM: U holds a few stacked rows
    // per component, so split the voxel columns towards 1024 workgroups (each
    // split at least 4 k-steps), at most 16 ways (the reduction, one
    // workgroup per column of U, reads every split's partials: at 64 splits
    // it took longer than the GEMM), fewer where the workspace would not hold
    // their partials
    const int64_t tiles = std::max<int64_t>(1, dtg_colgemm_tiles(p, p->dtg_nbw_a));
    const int64_t nst = ((int64_t)g.n2 * g.n3 + kDtgRowPad - 1) / kDtgRowPad;
    int S = (int)std::max<int64_t>(
        1, std::min<int64_t>({(1024 + tiles - 1) / tiles, 16, nst / 4}));
    p->dtg_split_a = S;
    while (S > 1 && dtg_workspace_bytes(p, 1) > p->grow_adj_ws) p->dtg_split_a = S /= 2;
  }
  p->use_dtg[1] = p->dtg_packed && g.m >= kGrowColGemmMin &&
                  dtg_workspace_bytes(p, 1) <= p->grow_adj_ws;
  // column splits as pack_plan sets them
  const int64_t base_f = (int64_t)g.q * p->tiling.tiles, base_a = (int64_t)g.q * p->tiling_a.tiles;
  const int sf = (int)std::min<int64_t>(8, std::max<int64_t>(1, (1024 + base_f - 1) / base_f));
  const int sa = (int)std::min<int64_t>(64, std::max<int64_t>(1, (1024 + base_a - 1) / base_a));
  p->split_f = (int)std::max<int64_t>(1, std::min<int64_t>(sf, g.m));
  p->split_a = (int)std::max<int64_t>(1, std::min<int64_t>(sa, g.m));
  {
    std::vector<int32_t> a = make_split(p, p->split_f), b = make_split(p, p->split_a);
    p->grow_split.assign(a.begin(), a.end());
    p->grow_split.insert(p->grow_split.end(), b.begin(), b.end());
  }
  // the pieces go up in one copy to the arena's staging region and one
  // kernel scatters them; then wait, so that the host buffer may be reused
  CopySeg segs[kMaxCopySegs];
  int nseg = 0;
  size_t off = 0;
  const bool pinned = p->grow_pinned && p->grow_pinned_bytes >= p->stage_bytes;
  if (!pinned && p->grow_buf.size() < p->stage_bytes) p->grow_buf.resize(p->stage_bytes);
  char* const hbuf = pinned ? p->grow_pinned : p->grow_buf.data();
  bool overflow = false;
  auto add = [&](void* dst, const void* src, size_t n) {
    if (!n) return;
    off = (off + 15) & ~(size_t)15;
    if (nseg == kMaxCopySegs || off + n > p->stage_bytes) {
      overflow = true;
      return;
    }
    std::memcpy(hbuf + off, src, n);
    segs[nseg++] = CopySeg{dst, (int64_t)off, (int64_t)n};
    off += n;
  };
  add(p->d_meta, H.meta.data(), H.meta.size() * sizeof(TensorMeta));
  add(p->d_drow, H.drow.data(), H.drow.size() * sizeof(int32_t));
  add(p->d_cores + p->g_off[t0], H.cores.data(), H.cores.size() * sizeof(float2));
  add(p->d_u1t + p->u1_off[t0], H.u1t.data(), H.u1t.size() * sizeof(float2));
  add(p->d_u2t + p->u2_off[t0], H.u2t.data(), H.u2t.size() * sizeof(float2));
  add(p->d_u3t + p->u3_off[t0], H.u3t.data(), H.u3t.size() * sizeof(float2));
  arows = 0;
  for (int k = 0; k < g.q; ++k) {
    const int r1 = ranks[3 * k];
    const int64_t nr = bf ? (r1 + 7) / 8 : r1;
    if (!bf)
      add(p->d_apack + p->apack_koff[k] + arow_new[k] * nbt * 64, &H.apack[arows * nbt * 64],
          (size_t)nr * nbt * 64 * sizeof(float));
    else
      add(p->d_apack_bf + p->apack_koff[k] + arow_new[k] * nbt * 128,
          &H.apack_bf[arows * nbt * 128], (size_t)nr * nbt * 128 * sizeof(uint4));
    arows += nr;
  }
  const size_t nsf = (size_t)g.q * (p->split_f + 1);
  add(p->d_split_f, p->grow_split.data(), nsf * sizeof(int32_t));
  add(p->d_split_a, p->grow_split.data() + nsf, (size_t)g.q * (p->split_a + 1) * sizeof(int32_t));
  if (overflow) return set_error(TV_ERR_WORKSPACE, "growable plan staging overflow");
  hipError_t e = hipMemcpyAsync(p->d_stage, hbuf, off, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_error(e, "growable plan upload");
  tv_status cs = launch_segment_copy(segs, nseg, p->d_stage, st);
  if (cs != TV_OK) return cs;
  e = hipStreamSynchronize(st);
  return e == hipSuccess ? TV_OK : hip_error(e, "growable plan upload");
}

}  // namespace tv

extern "C" {

tv_status tv_plan_destroy(tv_plan p) {
  clear_error();
  if (!p) return TV_OK;
  delete p;  // the device arena belongs to the caller
  return TV_OK;
}

tv_status tv_plan_required_bytes(tv_plan p, size_t* bytes) {
  clear_error();
  if (!p || !bytes) return set_error(TV_ERR_INVALID_ARG, "plan and bytes must be non-NULL");
  if (!p->finalized) return set_error(TV_ERR_INVALID_ARG, "plan is not finalized");
  *bytes = p->device_bytes;
  return TV_OK;
}

tv_status tv_plan_bind_arena(tv_plan p, void* arena, size_t bytes, void* stream) {
  clear_error();
  if (!p) return set_error(TV_ERR_INVALID_ARG, "plan is NULL");
  if (!p->finalized) return set_error(TV_ERR_INVALID_ARG, "plan is not finalized");
  if (p->bound) return set_error(TV_ERR_INVALID_ARG, "plan is already bound to an arena");
  if (!arena) return set_error(TV_ERR_INVALID_ARG, "arena is NULL");
  if ((uintptr_t)arena % 256) return set_error(TV_ERR_INVALID_ARG, "arena must be 256-byte aligned");
  if (bytes < p->device_bytes) {
    char buf[128];
    snprintf(buf, sizeof buf, "arena of %zu bytes needed, %zu given", p->device_bytes, bytes);
    return set_error(TV_ERR_WORKSPACE, buf);
  }
  return bind_arena(p, arena, bytes, (hipStream_t)stream);
}

tv_status tv_plan_info(tv_plan p, tv_plan_info_t* info) {
  clear_error();
  if (!p || !info) return set_error(TV_ERR_INVALID_ARG, "plan and info must be non-NULL");
  std::memset(info, 0, sizeof *info);
  info->grid = p->grid;
  info->precision = p->precision;
  const int64_t K = (int64_t)p->grid.q * p->appended_or_all();
  double sum[3] = {0, 0, 0};
  double fl = 0.0, dot = 0.0;
  const double n1 = p->grid.n1, n2 = p->grid.n2, n3 = p->grid.n3;
  for (int64_t t = 0; t < K; ++t) {
    const double r1 = p->ranks[3 * t], r2 = p->ranks[3 * t + 1], r3 = p->ranks[3 * t + 2];
    for (int d = 0; d < 3; ++d) {
      sum[d] += p->ranks[3 * t + d];
      info->max_rank[d] = std::max(info->max_rank[d], p->ranks[3 * t + d]);
    }
    info->factor_bytes += (size_t)8 * (size_t)(r1 * r2 * r3 + n1 * r1 + n2 * r2 + n3 * r3);
    info->sum_r1 += (int64_t)r1;
    // modes 2, 3 then 1 (Table III's decompression term r q nv m dominates)
    fl += 8.0 * (r1 * r2 * r3 * n2 + r1 * r3 * n2 * n3 + r1 * n1 * n2 * n3);
    // the adjoint's inner product is taken at the mode-1 output: the
    // conjugated mode-2/3 decompression (r1 x n2 n3) against U1^* y's block
    dot += 8.0 * r1 * n2 * n3;
  }
  for (int d = 0; d < 3; ++d) info->mean_rank[d] = K ? sum[d] / (double)K : 0.0;
  info->device_bytes = p->device_bytes;
  info->flops_matvec = fl;
  info->flops_rmatvec = fl + dot;
  for (int o = 0; o < 2; ++o) {
    const Tiling& T = o == 0 ? p->tiling : p->tiling_a;
    info->tile_t2[o] = T.t2;
    info->tile_t3[o] = T.t3;
    info->splits[o] = o == 0 ? p->split_f : p->split_a;
    info->kernel[o] = (p->finalized && p->kernel_ws[o] && ws_supported(p, T, o == 1)) ? 1 : 0;
    if (p->use_dtg[o] && dtg_supported(p)) {
      info->kernel[o] = 2;
      info->splits[o] = o == 0 ? p->dtg_split
                               : dtg_colgemm_splits(p, std::min(p->dtg_s3_a, p->grid.n3));
      info->tile_t2[o] = std::min(o == 0 ? p->dtg_s3 : p->dtg_s3_a, p->grid.n3);  // slab
      info->tile_t3[o] = o == 0 ? p->dtg_nbw : p->dtg_nbw_a;
    }
  }
  return TV_OK;
}

tv_status tv_plan_export_factors(tv_plan p, int32_t* ranks, double* cores, double* u1,
                                 double* u2, double* u3) {
  clear_error();
  if (!p || !ranks) return set_error(TV_ERR_INVALID_ARG, "plan and ranks must be non-NULL");
  const int64_t K = (int64_t)p->grid.q * p->appended_or_all();
  std::memcpy(ranks, p->ranks.data(), sizeof(int32_t) * 3 * K);
  if (cores) std::memcpy(cores, p->cores.data(), sizeof(double) * 2 * p->g_off[K]);
  if (u1) std::memcpy(u1, p->u1.data(), sizeof(double) * 2 * p->u1_off[K]);
  if (u2) std::memcpy(u2, p->u2.data(), sizeof(double) * 2 * p->u2_off[K]);
  if (u3) std::memcpy(u3, p->u3.data(), sizeof(double) * 2 * p->u3_off[K]);
  return TV_OK;
}

tv_status tv_workspace_bytes(tv_plan p, int32_t op, int32_t nrhs, size_t* bytes) {
  clear_error();
  if (!p || !bytes) return set_error(TV_ERR_INVALID_ARG, "plan and bytes must be non-NULL");
  if (op != 0 && op != 1) return set_error(TV_ERR_INVALID_ARG, "op must be 0 or 1");
  if (nrhs < 1) return set_error(TV_ERR_INVALID_ARG, "nrhs must be >= 1");
  if (!p->finalized) return set_error(TV_ERR_INVALID_ARG, "plan is not finalized");
  const tv_grid& g = p->grid;
  const int64_t nv = (int64_t)g.n1 * g.n2 * g.n3;
  if (p->use_dtg[op] && dtg_supported(p))
    *bytes = dtg_workspace_bytes(p, op);
  else if (op == 0)
    *bytes = p->split_f > 1 ? (size_t)8 * p->split_f * g.q * nv : 0;
  else
    *bytes = (size_t)8 * g.q * p->tiling_a.tiles * g.m;
  return TV_OK;
}

static tv_status check_call(tv_plan p, const void* in, int64_t ldin, int64_t rows_in,
                            int32_t nrhs, const void* out, int64_t ldout, int64_t rows_out,
                            int op, const void* ws, size_t ws_bytes) {
  if (!p) return set_error(TV_ERR_INVALID_ARG, "plan is NULL");
  if (!p->finalized) return set_error(TV_ERR_INVALID_ARG, "plan is not finalized");
  if (!p->bound)
    return set_error(TV_ERR_INVALID_ARG, "plan has no device arena (tv_plan_bind_arena)");
  if (!in || !out) return set_error(TV_ERR_INVALID_ARG, "vector pointers must be non-NULL");
  if (nrhs < 1) return set_error(TV_ERR_INVALID_ARG, "nrhs must be >= 1");
  if (ldin < rows_in || ldout < rows_out)
    return set_error(TV_ERR_SHAPE, "leading dimension smaller than the number of rows");
  if (((uintptr_t)in | (uintptr_t)out) % 8)
    return set_error(TV_ERR_INVALID_ARG, "complex64 vectors must be 8-byte aligned");
  const char* ib = (const char*)in;
  const char* ob = (const char*)out;
  const size_t in_len = 8 * (size_t)(ldin * (nrhs - 1) + rows_in);
  const size_t out_len = 8 * (size_t)(ldout * (nrhs - 1) + rows_out);
  if (ib < ob + out_len && ob < ib + in_len)
    return set_error(TV_ERR_INVALID_ARG, "input and output overlap");
  size_t need = 0;
  tv_status st = tv_workspace_bytes(p, op, nrhs, &need);
  if (st != TV_OK) return st;
  if (need && (!ws || ws_bytes < need)) {
    char buf[128];
    snprintf(buf, sizeof buf, "workspace of %zu bytes needed, %zu given", need,
             ws ? ws_bytes : (size_t)0);
    return set_error(TV_ERR_WORKSPACE, buf);
  }
  if (need && (uintptr_t)ws % 16) return set_error(TV_ERR_INVALID_ARG, "workspace alignment");
  return TV_OK;
}

tv_status tv_matvec(tv_plan p, const void* x, int64_t ldx, int32_t nrhs, void* y, int64_t ldy,
                    void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (!p) return set_error(TV_ERR_INVALID_ARG, "plan is NULL");
  const int64_t rows = (int64_t)p->grid.q * p->grid.n1 * p->grid.n2 * p->grid.n3;
  tv_status st = check_call(p, x, ldx, p->grid.m, nrhs, y, ldy, rows, 0, ws, ws_bytes);
  if (st != TV_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  for (int32_t c = 0; c < nrhs; ++c) {
    const float2* xc = (const float2*)x + (int64_t)c * ldx;
    float2* yc = (float2*)y + (int64_t)c * ldy;
    if (p->use_dtg[0] && dtg_supported(p)) {
      st = launch_dtg_forward(p, xc, yc, ws, s);
    } else if (p->split_f > 1) {
      st = launch_forward_f32(p, xc, (float2*)ws, p->split_f, p->d_split_f, rows, s);
      if (st == TV_OK) st = launch_sum_partials((const float2*)ws, p->split_f, rows, yc, s);
    } else {
      st = launch_forward_f32(p, xc, yc, 1, p->d_split_f, rows, s);
    }
    if (st != TV_OK) return st;
  }
  return TV_OK;
}

tv_status tv_rmatvec(tv_plan p, const void* y, int64_t ldy, int32_t nrhs, void* x, int64_t ldx,
                     void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (!p) return set_error(TV_ERR_INVALID_ARG, "plan is NULL");
  const int64_t rows = (int64_t)p->grid.q * p->grid.n1 * p->grid.n2 * p->grid.n3;
  tv_status st = check_call(p, y, ldy, rows, nrhs, x, ldx, p->grid.m, 1, ws, ws_bytes);
  if (st != TV_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  for (int32_t c = 0; c < nrhs; ++c) {
    const float2* yc = (const float2*)y + (int64_t)c * ldy;
    float2* xc = (float2*)x + (int64_t)c * ldx;
    if (p->use_dtg[1] && dtg_supported(p)) {
      st = launch_dtg_adjoint(p, yc, xc, ws, s);
      if (st != TV_OK) return st;
      continue;
    }
    st = launch_adjoint_f32(p, yc, (float2*)ws, p->split_a, p->d_split_a, s);
    if (st == TV_OK)
      st = launch_reduce_adjoint((const float2*)ws, p->grid.q, p->tiling_a.tiles, p->grid.m, xc,
                                 s);
    if (st != TV_OK) return st;
  }
  return TV_OK;
}

}  // extern "C"
