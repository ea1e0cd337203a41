// Batched products with many right-hand sides: several plans on one voxel
// grid, each with p_c right-hand sides, in one persistent launch.
//
// Table III prices a Tucker product with p right-hand sides as
// O(r q nv m) to decompress plus O(q nv m p) to apply.  These kernels keep
// that split: every tensor is decompressed once per voxel tile and then
// applied to all right-hand sides on MFMA,
//   forward  Y_tile(V x p) += T(V x 4) X(4 x p), four tensors per step,
//   adjoint  W(p x 32)     += Y_tile^T(p x V) conj(T)(V x 32), 32 tensors,
// where T holds decompressed tensor values Z^{kj} on the tile's V voxels.
// Decompression is wave-local (each wave takes whole tensors: mode-3 on the
// core, mode-2 per column, mode-1 per voxel row, eq. 6/7) so that a work
// item needs only two workgroup barriers per step.  Work items are pulled
// from a queue ordered longest first (most tensors), and the workgroups stay
// resident until the queue is empty.
//
// Complex products on real MFMA (v_mfma_f32_32x32x2f32) use the real forms
//   [Yr | Yi] = [Tr Ti] [[Xr, Xi], [-Xi, Xr]]
//   [Wr; Wi]  = [[Yr^T, -Yi^T], [Yi^T, Yr^T]] [Tr; -Ti].
#include <algorithm>
#include <climits>
#include <new>

#include "tv_internal.h"

namespace tv {

typedef float v16f __attribute__((ext_vector_type(16)));

struct BatchStatic {  // per plan, uploaded once
  const TensorMeta* meta;
  const float2* cores;
  const float2* u1t;
  const float2* u2t;
  const float2* u3t;
  int64_t m;
};

struct BatchArgs {
  const BatchStatic* plans;
  const int4* items;  // forward {plan, component, tile, rhs group};
                      // adjoint {plan, component * tsplit + slice, chunk, rhs group}
  int nitems;
  int* counter;
  float2* partial;    // adjoint: one 32 x 32 block per item
  int tsplit;         // adjoint: voxel-tile slices per (plan, component, chunk)
  int n1, n2, n3, n1p32, tiles2;
  int64_t nv;
  int r1max, r2max;
  const float2* in[TV_BATCH_MAX_PLANS];
  float2* out[TV_BATCH_MAX_PLANS];
  int64_t ld_in[TV_BATCH_MAX_PLANS];
  int64_t ld_out[TV_BATCH_MAX_PLANS];
  int nrhs[TV_BATCH_MAX_PLANS];
};

__device__ __forceinline__ float2 bcfma(float2 a, float2 b, float2 c) {
  c.x = fmaf(a.x, b.x, c.x);
  c.x = fmaf(-a.y, b.y, c.x);
  c.y = fmaf(a.x, b.y, c.y);
  c.y = fmaf(a.y, b.x, c.y);
  return c;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave decompresses tensor t on the tile (NCOL columns i2_0.., one i3,
// all n1 rows) and writes T[v], v = col * n1p32 + i1, to dst[v * dstride];
// rows i1 >= n1 and columns i2 >= n2 are written as zeros.
template <int NCOL>
__device__ void decompress_tile(const TensorMeta& t, const BatchStatic& S, int i2_0, int i3,
                                int n1, int n1p32, int n2, float2* Hw, float2* Bw, float2* dst,
                                int dstride, int lane) {
  const int r1 = t.r1, r2 = t.r2, r3 = t.r3;
  const int r12 = r1 * r2;
  // mode 3 on the core: H[a + r1 b] = sum_c G[a,b,c] U3[i3,c]
  const float2* u3 = S.u3t + t.u3_off + (int64_t)i3 * r3;
  for (int task = lane; task < r12; task += 64) {
    const float2* g = S.cores + t.g_off + task;
    float2 h = make_float2(0.f, 0.f);
    for (int c = 0; c < r3; ++c) h = bcfma(g[(int64_t)c * r12], u3[c], h);
    Hw[task] = h;
  }
  wave_sync();
  // mode 2 per column: B[a][col] = sum_b H[a + r1 b] U2[i2_0 + col, b]
  for (int task = lane; task < r1 * NCOL; task += 64) {
    const int col = task % NCOL, a = task / NCOL;
    const int i2 = i2_0 + col;
    float2 v = make_float2(0.f, 0.f);
    if (i2 < n2) {
      const float2* u2 = S.u2t + t.u2_off + (int64_t)i2 * r2;
      for (int b = 0; b < r2; ++b) v = bcfma(Hw[a + r1 * b], u2[b], v);
    }
    Bw[task] = v;
  }
  wave_sync();
  // mode 1 per voxel row: T[i1][col] = sum_a U1[i1, a] B[a][col]
  for (int i1 = lane; i1 < n1p32; i1 += 64) {
    float2 acc[NCOL];
#pragma unroll
    for (int c = 0; c < NCOL; ++c) acc[c] = make_float2(0.f, 0.f);
    if (i1 < n1) {
      const float2* u1 = S.u1t + t.u1_off + (int64_t)i1 * r1;
      for (int a = 0; a < r1; ++a) {
        const float2 u = u1[a];
#pragma unroll
        for (int c = 0; c < NCOL; ++c) acc[c] = bcfma(u, Bw[a * NCOL + c], acc[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < NCOL; ++c) dst[(int64_t)(c * n1p32 + i1) * dstride] = acc[c];
  }
  wave_sync();
}

__device__ __forceinline__ int next_item(int* counter, int* s_item) {
  __syncthreads();
  if (threadIdx.x == 0) *s_item = atomicAdd(counter, 1);
  __syncthreads();
  return *s_item;
}

// Forward: item = (plan, component, column tile, right-hand-side group of 32).
// Each wave owns BPW blocks of 32 voxels of the tile's V = n1p32 * NCOL.
template <int NCOL, int BPW>
__global__ __launch_bounds__(256) void batch_fwd(BatchArgs A) {
  extern __shared__ float4 bsm4[];
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int V = A.n1p32 * NCOL;
  float2* Hw = reinterpret_cast<float2*>(bsm4) + wave * (A.r1max * A.r2max);
  float2* Bw = reinterpret_cast<float2*>(bsm4) + 4 * A.r1max * A.r2max + wave * (A.r1max * NCOL);
  float2* Ts = reinterpret_cast<float2*>(bsm4) + 4 * (A.r1max * A.r2max + A.r1max * NCOL);
  for (;;) {
    const int it = next_item(A.counter, &s_item);
    if (it >= A.nitems) break;
    const int4 I = A.items[it];
    const BatchStatic S = A.plans[I.x];
    const int k = I.y;
    const int i2_0 = (I.z % A.tiles2) * NCOL, i3 = I.z / A.tiles2;
    const int rhs = I.w * 32 + (lane & 31);
    const float2* X = A.in[I.x];
    const int64_t ldx = A.ld_in[I.x];
    const bool rok = rhs < A.nrhs[I.x];
    const TensorMeta* meta = S.meta + (int64_t)k * S.m;
    v16f acc[BPW][2];
#pragma unroll
    for (int b = 0; b < BPW; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[b][0][i] = acc[b][1][i] = 0.f;
    for (int64_t j0 = 0; j0 < S.m; j0 += 4) {
      const int64_t j = j0 + wave;
      float2* mine = Ts + wave * V;
      if (j < S.m) {
        const TensorMeta t = meta[j];
        decompress_tile<NCOL>(t, S, i2_0, i3, A.n1, A.n1p32, A.n2, Hw, Bw, mine, 1, lane);
      } else {
        for (int v = lane; v < V; v += 64) mine[v] = make_float2(0.f, 0.f);
      }
      __syncthreads();
      const int nj = (int)min((int64_t)4, S.m - j0);
      for (int jj = 0; jj < nj; ++jj) {
        float2 xv = make_float2(0.f, 0.f);
        if (rok) xv = X[(j0 + jj) + ldx * rhs];
        const float b0 = lane < 32 ? xv.x : -xv.y;
        const float b1 = lane < 32 ? xv.y : xv.x;
        const float2* tj = Ts + jj * V + wave * BPW * 32 + (lane & 31);
#pragma unroll
        for (int b = 0; b < BPW; ++b) {
          const float2 tv = tj[b * 32];
          const float a = lane < 32 ? tv.x : tv.y;
          acc[b][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b0, acc[b][0], 0, 0, 0);
          acc[b][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b1, acc[b][1], 0, 0, 0);
        }
      }
      __syncthreads();
    }
    if (rok) {
      float2* Y = A.out[I.x] + A.ld_out[I.x] * rhs + (int64_t)k * A.nv;
#pragma unroll
      for (int b = 0; b < BPW; ++b)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int v = (wave * BPW + b) * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
          const int col = v / A.n1p32, i1 = v % A.n1p32;
          const int i2 = i2_0 + col;
          if (i1 < A.n1 && i2 < A.n2)
            Y[i1 + (int64_t)A.n1 * (i2 + (int64_t)A.n2 * i3)] =
                make_float2(acc[b][0][i], acc[b][1][i]);
        }
    }
  }
}

// Adjoint: item = (plan, component and slice of the voxel tiles, chunk of 32
// columns, right-hand-side group of 32).  The item sweeps its slice of tiles
// and stores its 32 x 32 share of W; batch_adj_reduce then sums the shares of
// every component and slice in a fixed order (Algorithm 2 sums over k).
template <int NCOL>
__global__ __launch_bounds__(256) void batch_adj(BatchArgs A) {
  extern __shared__ float4 bsm4[];
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int V = A.n1p32 * NCOL;
  const int tiles = A.tiles2 * A.n3;
  float2* Hw = reinterpret_cast<float2*>(bsm4) + wave * (A.r1max * A.r2max);
  float2* Bw = reinterpret_cast<float2*>(bsm4) + 4 * A.r1max * A.r2max + wave * (A.r1max * NCOL);
  float2* Tb = reinterpret_cast<float2*>(bsm4) + 4 * (A.r1max * A.r2max + A.r1max * NCOL);
  for (;;) {
    const int it = next_item(A.counter, &s_item);
    if (it >= A.nitems) break;
    const int4 I = A.items[it];
    const BatchStatic S = A.plans[I.x];
    const int k = I.y / A.tsplit, slice = I.y % A.tsplit;
    const int tb0 = (int)((int64_t)tiles * slice / A.tsplit);
    const int tb1 = (int)((int64_t)tiles * (slice + 1) / A.tsplit);
    const int64_t j0 = (int64_t)I.z * 32;
    const int jc = (int)min((int64_t)32, S.m - j0);
    const int rhs = I.w * 32 + (lane & 31);
    const bool rok = rhs < A.nrhs[I.x];
    const float2* Y = A.in[I.x] + A.ld_in[I.x] * rhs + (int64_t)k * A.nv;
    const TensorMeta* meta = S.meta + (int64_t)k * S.m;
    v16f acc[2];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[0][i] = acc[1][i] = 0.f;
    for (int tile = tb0; tile < tb1; ++tile) {
      const int i2_0 = (tile % A.tiles2) * NCOL, i3 = tile / A.tiles2;
      for (int e = 0; e < 8; ++e) {
        const int jj = wave * 8 + e;
        if (jj < jc) {
          const TensorMeta t = meta[j0 + jj];
          decompress_tile<NCOL>(t, S, i2_0, i3, A.n1, A.n1p32, A.n2, Hw, Bw, Tb + jj, 32, lane);
        } else {
          for (int v = lane; v < V; v += 64) Tb[v * 32 + jj] = make_float2(0.f, 0.f);
        }
      }
      __syncthreads();
      const int vq = V / 4;
      for (int v = wave * vq; v < (wave + 1) * vq; ++v) {
        const int col = v / A.n1p32, i1 = v % A.n1p32;
        const int i2 = i2_0 + col;
        float2 yv = make_float2(0.f, 0.f);
        if (rok && i1 < A.n1 && i2 < A.n2)
          yv = Y[i1 + (int64_t)A.n1 * (i2 + (int64_t)A.n2 * i3)];
        const float a0 = lane < 32 ? yv.x : -yv.y;
        const float a1 = lane < 32 ? yv.y : yv.x;
        const float2 tb = Tb[v * 32 + (lane & 31)];
        const float b = lane < 32 ? tb.x : -tb.y;
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b, acc[1], 0, 0, 0);
      }
      __syncthreads();
    }
    // sum the four waves' voxel quarters in a fixed order
    float* red = reinterpret_cast<float*>(Tb);
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int i = 0; i < 16; ++i) red[((wave * 2 + mb) * 16 + i) * 64 + lane] = acc[mb][i];
    __syncthreads();
    if (wave == 0) {
      // this item's share of W (32 right-hand sides x 32 columns), [rl][jj]
      float2* blk = A.partial + (int64_t)it * 1024;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        float wr = 0.f, wi = 0.f;
        for (int w = 0; w < 4; ++w) {
          wr += red[((w * 2 + 0) * 16 + i) * 64 + lane];
          wi += red[((w * 2 + 1) * 16 + i) * 64 + lane];
        }
        const int rl = 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        blk[rl * 32 + (lane & 31)] = make_float2(wr, wi);
      }
    }
  }
}

// Adjoint epilogue: X_c[j0 + jj][32 g + rl] = sum of the partial blocks of
// all components and tile slices of (plan, chunk, group), in list order.
// One workgroup per output block; red_list[b*nper .. (b+1)*nper) are item
// indices, red_out[b] = {plan, chunk, group}.
__global__ __launch_bounds__(256) void batch_adj_reduce(BatchArgs A, const int* red_list,
                                                        const int4* red_out, int nper) {
  const int4 O = red_out[blockIdx.x];
  const int* lst = red_list + (int64_t)blockIdx.x * nper;
  const int64_t m = A.plans[O.x].m;
  const int64_t j0 = (int64_t)O.y * 32;
  float2* Xo = A.out[O.x];
  const int64_t ldx = A.ld_out[O.x];
  for (int e = threadIdx.x; e < 1024; e += 256) {
    const int rl = e / 32, jj = e % 32;
    float2 acc = make_float2(0.f, 0.f);
    for (int i = 0; i < nper; ++i) {
      const float2 v = A.partial[(int64_t)lst[i] * 1024 + e];
      acc.x += v.x;
      acc.y += v.y;
    }
    const int r = O.z * 32 + rl;
    if (j0 + jj < m && r < A.nrhs[O.x]) Xo[(j0 + jj) + ldx * r] = acc;
  }
}

__global__ void reset_counter(int* c) { *c = 0; }

size_t batch_lds_bytes(int op, int ncol, int n1p32, int r1max, int r2max) {
  const size_t per = (size_t)4 * (r1max * r2max + r1max * ncol);
  const size_t V = (size_t)n1p32 * ncol;
  const size_t shared = op == 0 ? 4 * V : 32 * V;
  size_t need = 8 * (per + shared);
  if (op == 1) need = std::max(need, 8 * per + (size_t)2 * 2 * 16 * 64 * 4 * 2);
  return need;
}

typedef void (*batch_fn)(BatchArgs);

static batch_fn pick_fwd(int ncol, int bpw) {
#define TV_BF(NC)                                   \
  if (ncol == NC) {                                 \
    if (bpw == 1) return batch_fwd<NC, 1>;          \
    if (bpw == 2) return batch_fwd<NC, 2>;          \
    if (bpw == 3) return batch_fwd<NC, 3>;          \
  }
  TV_BF(1) TV_BF(2) TV_BF(4) TV_BF(8) TV_BF(16)
#undef TV_BF
  return nullptr;
}

static batch_fn pick_adj(int ncol) {
  switch (ncol) {
    case 8: return batch_adj<8>;
    case 4: return batch_adj<4>;
    case 2: return batch_adj<2>;
    case 1: return batch_adj<1>;
  }
  return nullptr;
}

}  // namespace tv

// --------------------------------------------------------------------------
// Host side
using namespace tv;

struct tv_batch_s {
  int op = 0;
  int nplans = 0;
  tv_grid grid{};
  int n1p32 = 0, ncol = 0, bpw = 0, tiles2 = 0;
  int r1max = 1, r2max = 1;
  int nitems = 0;
  int grid_blocks = 0;
  size_t lds = 0;
  std::vector<int64_t> m;
  std::vector<int32_t> nrhs;
  BatchStatic* d_plans = nullptr;
  int4* d_items = nullptr;
  batch_fn fn = nullptr;
  // adjoint: voxel-tile slices per item and the fixed-order reduction lists
  int tsplit = 1;
  int nred = 0, nper = 0;
  int* d_red_list = nullptr;
  int4* d_red_out = nullptr;
};

extern "C" {

tv_status tv_batch_create(int32_t nplans, const tv_plan* plans, int32_t op, const int32_t* nrhs,
                          tv_batch* out) {
  clear_error();
  if (!out) return set_error(TV_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (nplans < 1 || nplans > TV_BATCH_MAX_PLANS)
    return set_error(TV_ERR_INVALID_ARG, "nplans outside [1, TV_BATCH_MAX_PLANS]");
  if (!plans || !nrhs) return set_error(TV_ERR_INVALID_ARG, "plans and nrhs must be non-NULL");
  if (op != 0 && op != 1) return set_error(TV_ERR_INVALID_ARG, "op must be 0 or 1");
  for (int c = 0; c < nplans; ++c) {
    if (!plans[c] || !plans[c]->finalized)
      return set_error(TV_ERR_INVALID_ARG, "every plan must be finalized");
    if (nrhs[c] < 1 || nrhs[c] > (1 << 20)) return set_error(TV_ERR_INVALID_ARG, "nrhs < 1");
    const tv_grid& g0 = plans[0]->grid;
    const tv_grid& g = plans[c]->grid;
    if (g.n1 != g0.n1 || g.n2 != g0.n2 || g.n3 != g0.n3 || g.q != g0.q)
      return set_error(TV_ERR_SHAPE, "all plans of a batch must share the voxel grid and q");
  }
  const tv_grid g = plans[0]->grid;
  if (g.n1 > 256) return set_error(TV_ERR_NOT_SUPPORTED, "batched products need n1 <= 256");
  tv_batch_s* b = new (std::nothrow) tv_batch_s;
  if (!b) return set_error(TV_ERR_OOM, "host allocation");
  b->op = op;
  b->nplans = nplans;
  b->grid = g;
  b->n1p32 = (g.n1 + 31) / 32 * 32;
  const int nb1 = b->n1p32 / 32;
  if (op == 0) {
    // columns per tile: the widest power of two whose nb1 * ncol 32-voxel
    // blocks split evenly over the 4 waves with at most 3 blocks per wave
    // (each block holds 32 accumulator registers per real/imaginary half)
    int ncol = 0;
    for (int c = 16; c >= 1 && !ncol; c /= 2)
      if ((nb1 * c) % 4 == 0 && nb1 * c / 4 <= 3) ncol = c;
    if (!ncol) {
      delete b;
      return set_error(TV_ERR_NOT_SUPPORTED, "no batched tile for this n1");
    }
    b->ncol = ncol;
    b->bpw = nb1 * ncol / 4;
  } else {
    int ncol = 1;
    while (ncol * 2 * b->n1p32 <= 384) ncol *= 2;
    b->ncol = ncol;
  }
  b->tiles2 = (g.n2 + b->ncol - 1) / b->ncol;
  for (int c = 0; c < nplans; ++c) {
    b->r1max = std::max(b->r1max, plans[c]->max_r[0]);
    b->r2max = std::max(b->r2max, plans[c]->max_r[1]);
    b->m.push_back(plans[c]->grid.m);
    b->nrhs.push_back(nrhs[c]);
  }
  b->lds = batch_lds_bytes(op, b->ncol, b->n1p32, b->r1max, b->r2max);
  b->fn = op == 0 ? pick_fwd(b->ncol, b->bpw) : pick_adj(b->ncol);
  if (!b->fn || b->lds > 160 * 1024) {
    delete b;
    return set_error(TV_ERR_NOT_SUPPORTED, "no batched kernel for these sizes and ranks");
  }
  // work items, longest first (most tensors per item); the adjoint splits
  // the voxel tiles of each (plan, component, chunk) into tsplit slices so
  // that there are enough items to fill the device
  std::vector<int> order(nplans);
  for (int c = 0; c < nplans; ++c) order[c] = c;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->m[x] > b->m[y]; });
  const int tiles = b->tiles2 * g.n3;
  if (op == 1) {
    int64_t base = 0;
    for (int c = 0; c < nplans; ++c) base += (int64_t)g.q * ((b->m[c] + 31) / 32) * ((nrhs[c] + 31) / 32);
    b->tsplit = (int)std::max<int64_t>(1, std::min<int64_t>(tiles, (2048 + base - 1) / base));
  }
  std::vector<int4> items;
  std::vector<int> red_list;
  std::vector<int4> red_out;
  for (int c : order) {
    const int groups = (nrhs[c] + 31) / 32;
    if (op == 0) {
      for (int k = 0; k < g.q; ++k)
        for (int64_t u = 0; u < (int64_t)tiles; ++u)
          for (int gr = 0; gr < groups; ++gr) items.push_back(make_int4(c, k, (int)u, gr));
    } else {
      const int64_t chunks = (b->m[c] + 31) / 32;
      for (int64_t u = 0; u < chunks; ++u)
        for (int gr = 0; gr < groups; ++gr) {
          red_out.push_back(make_int4(c, (int)u, gr, 0));
          for (int k = 0; k < g.q; ++k)
            for (int sl = 0; sl < b->tsplit; ++sl) {
              red_list.push_back((int)items.size());
              items.push_back(make_int4(c, k * b->tsplit + sl, (int)u, gr));
            }
        }
    }
  }
  b->nred = (int)red_out.size();
  b->nper = g.q * b->tsplit;
  if (items.size() > (size_t)INT32_MAX) {
    delete b;
    return set_error(TV_ERR_NOT_SUPPORTED, "too many work items");
  }
  b->nitems = (int)items.size();
  std::vector<BatchStatic> st(nplans);
  for (int c = 0; c < nplans; ++c)
    st[c] = BatchStatic{plans[c]->d_meta, plans[c]->d_cores, plans[c]->d_u1t, plans[c]->d_u2t,
                        plans[c]->d_u3t, plans[c]->grid.m};
  hipError_t e = hipMalloc((void**)&b->d_plans, st.size() * sizeof(BatchStatic));
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_items, items.size() * sizeof(int4));
  if (e == hipSuccess)
    e = hipMemcpy(b->d_plans, st.data(), st.size() * sizeof(BatchStatic), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_items, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice);
  if (e == hipSuccess && op == 1) {
    e = hipMalloc((void**)&b->d_red_list, red_list.size() * sizeof(int));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_red_out, red_out.size() * sizeof(int4));
    if (e == hipSuccess)
      e = hipMemcpy(b->d_red_list, red_list.data(), red_list.size() * sizeof(int),
                    hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(b->d_red_out, red_out.data(), red_out.size() * sizeof(int4),
                    hipMemcpyHostToDevice);
  }
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)b->fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)b->lds);
  int dev = 0, cus = 256, per_cu = 1;
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)b->fn, 256, b->lds);
  if (e != hipSuccess) {
    hipFree(b->d_plans);
    hipFree(b->d_items);
    hipFree(b->d_red_list);
    hipFree(b->d_red_out);
    delete b;
    return hip_error(e, "tv_batch_create");
  }
  b->grid_blocks = std::max(1, std::min(b->nitems, cus * std::max(per_cu, 1)));
  *out = b;
  return TV_OK;
}

tv_status tv_batch_workspace_bytes(tv_batch b, size_t* bytes) {
  clear_error();
  if (!b || !bytes) return set_error(TV_ERR_INVALID_ARG, "batch and bytes must be non-NULL");
  // the work-queue counter, then (adjoint) one 32 x 32 complex64 block per item
  *bytes = 256 + (b->op == 1 ? (size_t)b->nitems * 1024 * 8 : 0);
  return TV_OK;
}

tv_status tv_batch_run(tv_batch b, const void* const* in, const int64_t* ld_in, void* const* out,
                       const int64_t* ld_out, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (!b || !in || !ld_in || !out || !ld_out)
    return set_error(TV_ERR_INVALID_ARG, "NULL argument");
  size_t need = 0;
  tv_batch_workspace_bytes(b, &need);
  if (!ws || ws_bytes < need || (uintptr_t)ws % 16)
    return set_error(TV_ERR_WORKSPACE, "workspace missing, too small or not 16-byte aligned");
  BatchArgs A;
  A.plans = b->d_plans;
  A.items = b->d_items;
  A.nitems = b->nitems;
  A.counter = (int*)ws;
  A.partial = (float2*)((char*)ws + 256);
  A.tsplit = b->tsplit;
  A.n1 = b->grid.n1;
  A.n2 = b->grid.n2;
  A.n3 = b->grid.n3;
  A.n1p32 = b->n1p32;
  A.tiles2 = b->tiles2;
  A.nv = (int64_t)b->grid.n1 * b->grid.n2 * b->grid.n3;
  A.r1max = b->r1max;
  A.r2max = b->r2max;
  const int64_t rows = (int64_t)b->grid.q * A.nv;
  for (int c = 0; c < b->nplans; ++c) {
    const int64_t rin = b->op == 0 ? b->m[c] : rows, rout = b->op == 0 ? rows : b->m[c];
    if (!in[c] || !out[c]) return set_error(TV_ERR_INVALID_ARG, "NULL vector pointer");
    if (ld_in[c] < rin || ld_out[c] < rout)
      return set_error(TV_ERR_SHAPE, "leading dimension smaller than the number of rows");
    if (((uintptr_t)in[c] | (uintptr_t)out[c]) % 8)
      return set_error(TV_ERR_INVALID_ARG, "complex64 vectors must be 8-byte aligned");
    A.in[c] = (const float2*)in[c];
    A.out[c] = (float2*)out[c];
    A.ld_in[c] = ld_in[c];
    A.ld_out[c] = ld_out[c];
    A.nrhs[c] = b->nrhs[c];
  }
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, st, A.counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "reset_counter launch");
  hipLaunchKernelGGL(b->fn, dim3((unsigned)b->grid_blocks), dim3(256), b->lds, st, A);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "batched kernel launch");
  if (b->op == 1) {
    hipLaunchKernelGGL(batch_adj_reduce, dim3((unsigned)b->nred), dim3(256), 0, st, A,
                       b->d_red_list, b->d_red_out, b->nper);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "batched reduction launch");
  }
  return TV_OK;
}

tv_status tv_batch_destroy(tv_batch b) {
  clear_error();
  if (!b) return TV_OK;
  hipFree(b->d_plans);
  hipFree(b->d_items);
  hipFree(b->d_red_list);
  hipFree(b->d_red_out);
  delete b;
  return TV_OK;
}

}  // extern "C"
