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
// Two generations of kernels:
//  * ranks <= 32: decompression on MFMA as well (batch_mode3, then
//    batch_fwd_mfma / batch_adj_mfma below), eight waves per workgroup;
//  * otherwise wave-local VALU decompression (each wave takes whole
//    tensors: mode-3 on the core, mode-2 per column, mode-1 per voxel row,
//    eq. 6/7), two workgroup barriers per step.
// Work items are pulled from a queue ordered longest first (most tensors),
// and the workgroups stay resident until the queue is empty.
//
// Complex products on real MFMA (v_mfma_f32_32x32x2f32) use the real forms
//   [Yr | Yi] = [Tr Ti] [[Xr, Xi], [-Xi, Xr]]
//   [Wr; Wi]  = [[Yr^T, -Yi^T], [Yi^T, Yr^T]] [Tr; -Ti].
#include <algorithm>
#include <cstdio>
#include <type_traits>
#include <climits>
#include <new>

#include "tv_internal.h"

namespace tv {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Per tensor, for the MFMA decompression kernels ([k][j] like TensorMeta).
// Operands are stored in the MFMA lane order of the kernels, four K steps
// per lane in 16 bytes ("quads"): a block of 64 lanes x 4 floats = 1 KB.
struct BTensor {
  int32_t r1, r2;
  int64_t h_off;    // float offset of H(i3 = 0) in the mode-3 cache
  int64_t u1p_off;  // float offset of the packed U1 blocks
  int64_t u2p_off;  // float offset of the packed U2 blocks
};

struct BatchStatic {  // per plan, uploaded once
  const TensorMeta* meta;
  const float2* cores;
  const float2* u1t;
  const float2* u2t;
  const float2* u3t;
  int64_t m;
  const BTensor* bt;  // MFMA kernels only
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
  // MFMA kernels: mode-3 cache (workspace), packed U1, 16-row chunks per
  // tensor in the packed U1, 16-row chunks per adjoint tile
  float* hcache;
  const float* u1p;
  const float* u2p;
  int nch, nic;
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

// ---------------------------------------------------------------------------
// MFMA decompression (batched kernels for ranks up to 32)
//
// On a voxel tile at one i3 and 8 consecutive i2 columns c0.., tensor j is
//   T[i1][f] = sum_a U1[i1][a] B[a][f],  B[a][f] = sum_b H[a][b] U2[c0+f][b],
//   H = G x3 U3[i3]                                   (eq. 6/7, modes 3, 2, 1).
// H for every (tensor, i3) is computed once per run into the workspace
// (batch_mode3), so a tile reads r1 r2 values instead of the whole core.
// Modes 2 and 1 run on v_mfma_f32_16x16x4f32 (A lane l = A[l%16][l/16],
// B lane l = B[l/16][l%16], D register r = D[4(l/16) + r][l%16]) with the
// complex products in real form.  Columns are (f, part) = f + 8 part; the K
// index k = l/16 is (pair member k/2, real/imaginary selector s = k%2), so
// a K step t covers b (or a) = 2t and 2t + 1:
//   mode 2: rows a,  A[a][(b,s)]  = s ? Hi : Hr,
//           B[(b,s)][(f,p)] = p ? (s ? U2r : U2i) : (s ? -U2i : U2r)
//   mode 1: rows i1, A[i1][(a,s)] = s ? U1i : U1r   (packed: batch_pack_u1),
//           B[(a,s)][(f,p)] = p ? (s ? Br : Bi) : (s ? -Bi : Br)
// so D[a][(f,p)] = Re/Im of (H U2^T)[a][f] and D[i1][(f,p)] = Re/Im T[i1][f].

__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// BF16X3 apply: bf16 round to nearest even (finite values), hi/lo split
typedef __bf16 bv8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ uint32_t bt_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bt_f(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ uint32_t bt_pack(uint32_t lo16, uint32_t hi16) {
  return (lo16 & 0xFFFFu) | (hi16 << 16);
}
__device__ __forceinline__ v16f mfma_bf(uint4 a, uint4 b, v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bv8, a),
                                                 __builtin_bit_cast(bv8, b), c, 0, 0, 0);
}

// Packed operand layouts (np = (r + 1) / 2 K steps, nq = (np + 3) / 4 quads,
// nab = (r1 + 15) / 16 row blocks of 16; value 0 outside the ranks/grid):
//   H   [i3][ab < nab][q < nq2][lane][4]: step t = 4q + i of lane l holds
//       Re/Im (s = (l/16)%2) of H[16 ab + l%16][2t + l/32]          (mode 2 A)
//   U2  [cg][q < nq2][lane][4]: Re/Im (part ^ s) of U2[8 cg + l%8][2t + l/32],
//       part = (l/8)%2; the sign of -U2i is applied at the MFMA      (mode 2 B)
//   U1  [ic][q < nq1][lane][4]: Re/Im (s) of U1[16 ic + l%16][2t + l/32]   (mode 1 A)

// Mode 3 for every tensor of the batch and every i3, written in the packed
// H layout: H[a, b] = sum_c G[a, b, c] U3[i3][c].  One workgroup per tensor,
// tlist[x] = {plan, k m + j}.  A thread computes one complex entry (both of
// its packed floats) for 16 consecutive i3 from the core fibre G[a, b, :]
// held in registers; U3 (n3 x r3) is staged in LDS when it fits (LDSU3).
template <bool LDSU3>
__global__ __launch_bounds__(256) void batch_mode3(BatchArgs A, const int2* tlist) {
  extern __shared__ float2 u3s[];
  const int2 T = tlist[blockIdx.x];
  const BatchStatic S = A.plans[T.x];
  const TensorMeta M = S.meta[T.y];
  const int64_t ho = S.bt[T.y].h_off;
  const int r1 = M.r1, r2 = M.r2, r12 = r1 * r2, r3 = M.r3, n3 = A.n3;
  const int nq2 = (((r2 + 1) >> 1) + 3) >> 2, hq = ((r1 + 15) >> 4) * nq2;
  const float2* u3 = S.u3t + M.u3_off;
  if (LDSU3) {
    for (int i = threadIdx.x; i < n3 * r3; i += 256) u3s[i] = u3[i];
    __syncthreads();
  }
  const int nblk = (n3 + 15) / 16;
  // entry e: block e / 128 (= ab nq2 + q), lane l with bit 4 (s) clear, step
  // in quad i; the real part goes to lane l, the imaginary part to l + 16
  for (int item = threadIdx.x; item < hq * 128 * nblk; item += 256) {
    const int e = item % (hq * 128), i30 = 16 * (item / (hq * 128));
    const int blk = e >> 7, rem = e & 127, i = rem & 3, lo = rem >> 2;
    const int l = (lo & 15) | ((lo >> 4) << 5);
    const int ab = blk / nq2, q = blk % nq2;
    const int a = 16 * ab + (l & 15), bb = 2 * (4 * q + i) + (l >> 5);
    const bool ok = a < r1 && bb < r2;
    float2 g[32];
#pragma unroll
    for (int c = 0; c < 32; ++c)
      g[c] = ok && c < r3 ? S.cores[M.g_off + a + r1 * bb + (int64_t)r12 * c] : make_float2(0.f, 0.f);
    const int64_t p0 = ho + (int64_t)blk * 256 + l * 4 + i;
    const int i3e = min(i30 + 16, n3);
    for (int i3 = i30; i3 < i3e; ++i3) {
      float2 h = make_float2(0.f, 0.f);
#pragma unroll
      for (int c = 0; c < 32; ++c)
        if (c < r3) h = bcfma(g[c], LDSU3 ? u3s[i3 * r3 + c] : u3[i3 * r3 + c], h);
      float* dst = A.hcache + p0 + (int64_t)i3 * hq * 256;
      dst[0] = h.x;
      dst[64] = h.y;
    }
  }
}

// Operands of one tensor on one tile, loaded a step before they are used:
// mode-2 A (H) and B (U2 rows c0..c0+7) lane values, x_j for this lane's
// right-hand side, and what mode 1 needs of the metadata.
struct DecOps {
  float ha[2][16];
  float ub[16];
  float2 xv;
  int r1, r2;
  int64_t u1p;
};

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)(uint64_t)v);
  const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ int4 uni_item(int4 v) {
  return make_int4(uni(v.x), uni(v.y), uni(v.z), uni(v.w));
}

// Raw buffer loads with the hardware range check: an offset at or beyond
// num_records bytes reads zero, so masked operands need neither a branch
// nor a select after the load.  Word 3 is the gfx9 raw-dword format.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t brsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, int off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
// four K steps t = 4q .. 4q + 3 of one packed quad block into dst[4q ..]
__device__ __forceinline__ void bload4(__amdgpu_buffer_rsrc_t r, int off, float* dst) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
  dst[0] = __uint_as_float(v[0]);
  dst[1] = __uint_as_float(v[1]);
  dst[2] = __uint_as_float(v[2]);
  dst[3] = __uint_as_float(v[3]);
}
#define TV_OOB 0x40000000

// Loads are unconditional and land in their final registers, so the
// compiler neither branches around them nor waits for each one.  Callers
// pass an index that is always valid (clamped) and discard what they do not
// use: every path through a loop then issues the same loads in the same
// order, which keeps the wait counts exact at the joins.  The x_j load (WX)
// clamps the right-hand side (lanes beyond nrhs are never stored).
template <bool WX>
__device__ __forceinline__ void dec_load(DecOps& o, const BTensor* bt, int64_t j,
                                         const float* hc, const float* u2p, int i3, int c0,
                                         const float2* X, int64_t ldx, int xr, int lane) {
  // read-only for the kernel's lifetime: constant address space, uniform
  // index, so these are scalar loads (lgkmcnt, no drain of vector loads)
  typedef const __attribute__((address_space(4))) BTensor CBT;
  CBT* T = reinterpret_cast<CBT*>(reinterpret_cast<uintptr_t>(bt)) + j;
  const int r1 = uni(T->r1), r2 = uni(T->r2);
  const int64_t h_off = uni64(T->h_off), u2p_off = uni64(T->u2p_off);
  o.r1 = r1;
  o.r2 = r2;
  o.u1p = uni64(T->u1p_off);
  const int nab = (r1 + 15) >> 4, nq2 = (((r2 + 1) >> 1) + 3) >> 2;
  // packed H(i3): nab x nq2 blocks; quads beyond are out of range (zero)
  const __amdgpu_buffer_rsrc_t rh =
      brsrc(hc + h_off + (int64_t)i3 * nab * nq2 * 256, 1024u * nab * nq2);
#pragma unroll
  for (int ab = 0; ab < 2; ++ab)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      bload4(rh, ab < nab && q < nq2 ? ((ab * nq2 + q) * 64 + lane) * 16 : TV_OOB, &o.ha[ab][4 * q]);
  // packed U2 of column group c0 / 8
  const __amdgpu_buffer_rsrc_t ru = brsrc(u2p + u2p_off + (int64_t)(c0 >> 3) * nq2 * 256, 1024u * nq2);
#pragma unroll
  for (int q = 0; q < 4; ++q) bload4(ru, q < nq2 ? (q * 64 + lane) * 16 : TV_OOB, &o.ub[4 * q]);
  if (WX) o.xv = X[j + ldx * xr];
}

// sum_t a[t] b[t] over NP K steps on two accumulators; NP is a template
// argument so that the chain is straight-line code (the wait counters then
// stay exact instead of dropping to zero at branch joins).
template <int NP>
__device__ __forceinline__ v4f chain16(const float* a, const float* b) {
  v4f d0 = {0.f, 0.f, 0.f, 0.f}, d1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < NP; t += 2) {
    d0 = mfma16(a[t], b[t], d0);
    if (t + 1 < NP) d1 = mfma16(a[t + 1], b[t + 1], d1);
  }
  return d0 + d1;
}

__device__ __forceinline__ v4f chain16_n(int np, const float* a, const float* b) {
  switch (np) {
#define TV_CH(N) \
  case N: return chain16<N>(a, b);
    TV_CH(1) TV_CH(2) TV_CH(3) TV_CH(4) TV_CH(5) TV_CH(6) TV_CH(7) TV_CH(8)
    TV_CH(9) TV_CH(10) TV_CH(11) TV_CH(12) TV_CH(13) TV_CH(14) TV_CH(15) TV_CH(16)
#undef TV_CH
  }
  return v4f{0.f, 0.f, 0.f, 0.f};
}

// Mode 2 on MFMA into the wave's Bc[a][32]: columns f (Re), 8 + f (Im),
// 16 + f (-Re, unused) and 24 + f (-Im), so that the mode-1 B operand is a
// plain read.  The U2 operand's sign (-U2i at part 0, s = 1) is applied here.
__device__ __forceinline__ void dec_mode2(const DecOps& o, float* Bc, int lane) {
  const int np2 = (o.r2 + 1) >> 1;
  const bool neg = ((lane >> 3) & 1) == 0 && ((lane >> 4) & 1) == 1;
  float ub[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) ub[t] = neg ? -o.ub[t] : o.ub[t];
#pragma unroll
  for (int ab = 0; ab < 2; ++ab) {
    if (16 * ab < o.r1) {
      const v4f d = chain16_n(np2, o.ha[ab], ub);
      float* dst = Bc + (16 * ab + 4 * (lane >> 4)) * 32 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        dst[32 * r] = d[r];
        dst[32 * r + 16] = -d[r];
      }
    }
  }
}

// Mode-1 B operand (the embedded B = H U2^T) for every K step, from Bc;
// steps t >= (r1 + 1) / 2 are never issued.
__device__ __forceinline__ void dec_bops(const float* Bc, float* bb, int lane) {
  const int f = lane & 7, part = (lane >> 3) & 1, s = (lane >> 4) & 1;
  const int col = f + (part == 0 ? (s ? 24 : 0) : (s ? 0 : 8));
#pragma unroll
  for (int t = 0; t < 16; ++t) bb[t] = Bc[(2 * t + (lane >> 5)) * 32 + col];
}

// U1 operand of 16-row chunk ic for every K step (packed quads; quads
// beyond nq1 are out of range and read zero; steps t >= np1 are never
// issued as MFMAs).  All loads are issued on every path so that the wait
// counts stay exact.
__device__ __forceinline__ void dec_u1ops(const float* u1p, int64_t off, int r1, int ic,
                                          float* ua, int lane) {
  const int nq1 = (((r1 + 1) >> 1) + 3) >> 2;
  const __amdgpu_buffer_rsrc_t r = brsrc(u1p + off + (int64_t)ic * nq1 * 256, 1024u * nq1);
#pragma unroll
  for (int q = 0; q < 4; ++q) bload4(r, q < nq1 ? (q * 64 + lane) * 16 : TV_OOB, &ua[4 * q]);
}

// Forward, MFMA decompression.  Item = (plan, component, tile of 8 columns
// at one i3, right-hand-side group of 32); NB1 = n1p32 / 32 <= 3.  Waves
// 4..7 produce: in step s wave 4 + w decompresses tensor 4s + w into
// Ts[s&1][w], its operands loaded one step ahead (U1 chunk by chunk as the
// previous tensor's chunks retire).  Waves 0..3 consume: in step s wave w
// applies tensors 4(s-1).. to columns 2w, 2w+1 of the tile (2 NB1 blocks of
// 32 voxels x 32 right-hand sides on v_mfma_f32_32x32x2f32).  One barrier
// per step.
template <int NB1, bool BF>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
void batch_fwd_mfma(BatchArgs A) {
  constexpr int NPW = 4, N1P = 32 * NB1, V = 8 * N1P, NCH = 2 * NB1, BPC = 2 * NB1;
  extern __shared__ float4 bsm4[];
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & 63, wave = uni(tid >> 6);
  const bool producer = wave >= 4;
  const int w = wave & 3;
  float* Ts = reinterpret_cast<float*>(bsm4);                    // [2][NPW][2][V]
  float2* Xs = reinterpret_cast<float2*>(Ts + 2 * NPW * 2 * V);  // [2][NPW][32]
  float* Bc = reinterpret_cast<float*>(Xs + 2 * NPW * 32) + w * 1024;  // [2][NPW][1024]
  // The two roles run separate item loops (same items, same barrier count
  // per item), so that neither keeps the other's per-lane constants live.
  if (!producer) {
    for (;;) {
      const int it = next_item(A.counter, &s_item);
      if (it >= A.nitems) break;
      const int4 I = uni_item(A.items[it]);
      const int64_t m = A.plans[I.x].m;
      const int nbat = (int)((m + 3) / 4);
      v16f acc[BPC][2];
#pragma unroll
      for (int b = 0; b < BPC; ++b)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[b][0][i] = acc[b][1][i] = 0.f;
      for (int s = 0; s <= nbat; ++s) {
        if (BF && s > 0) {
          // BF16X3: one v_mfma_f32_32x32x16_bf16 pair per output covers the
          // four tensors of the step.  K slot 8h + 4p + t holds the hi (h = 0,
          // lanes < 32) or lo (h = 1) half of part p of tensor t's value; the
          // B operands hold x in the real form of the output (Re: xr, -xi;
          // Im: xi, xr), hi in both halves for the first MFMA and lo against
          // the hi halves of T for the second: Th Xh + Tl Xh + Th Xl.
          const int pb = (s - 1) & 1;
          const int nj = (int)min((int64_t)4, m - 4 * (int64_t)(s - 1));
          uint32_t xr_h[4], xr_l[4], xi_h[4], xi_l[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const float2 xv = t < nj ? Xs[(pb * NPW + t) * 32 + (lane & 31)] : make_float2(0.f, 0.f);
            xr_h[t] = bt_rne(xv.x);
            xr_l[t] = bt_rne(xv.x - bt_f(xr_h[t]));
            xi_h[t] = bt_rne(xv.y);
            xi_l[t] = bt_rne(xv.y - bt_f(xi_h[t]));
          }
          const bool lo = lane < 32;
          const uint32_t sg = 0x8000u;  // bf16 sign bit
          const uint4 b1r = make_uint4(bt_pack(xr_h[0], xr_h[1]), bt_pack(xr_h[2], xr_h[3]),
                                       bt_pack(xi_h[0] ^ sg, xi_h[1] ^ sg),
                                       bt_pack(xi_h[2] ^ sg, xi_h[3] ^ sg));
          const uint4 b1i = make_uint4(bt_pack(xi_h[0], xi_h[1]), bt_pack(xi_h[2], xi_h[3]),
                                       bt_pack(xr_h[0], xr_h[1]), bt_pack(xr_h[2], xr_h[3]));
          const uint4 b2r = lo ? make_uint4(bt_pack(xr_l[0], xr_l[1]), bt_pack(xr_l[2], xr_l[3]),
                                            bt_pack(xi_l[0] ^ sg, xi_l[1] ^ sg),
                                            bt_pack(xi_l[2] ^ sg, xi_l[3] ^ sg))
                               : make_uint4(0u, 0u, 0u, 0u);
          const uint4 b2i = lo ? make_uint4(bt_pack(xi_l[0], xi_l[1]), bt_pack(xi_l[2], xi_l[3]),
                                            bt_pack(xr_l[0], xr_l[1]), bt_pack(xr_l[2], xr_l[3]))
                               : make_uint4(0u, 0u, 0u, 0u);
          const uint4* ta = reinterpret_cast<const uint4*>(Ts) + (pb * 2 + (lane >> 5)) * V +
                            2 * w * N1P + (lane & 31);
#pragma unroll
          for (int b = 0; b < BPC; ++b) {
            const uint4 a = ta[32 * b];
            acc[b][0] = mfma_bf(a, b1r, acc[b][0]);
            acc[b][0] = mfma_bf(a, b2r, acc[b][0]);
            acc[b][1] = mfma_bf(a, b1i, acc[b][1]);
            acc[b][1] = mfma_bf(a, b2i, acc[b][1]);
          }
        } else if (s > 0) {
          const int pb = (s - 1) & 1;
          const int nj = (int)min((int64_t)4, m - 4 * (int64_t)(s - 1));
          for (int jj = 0; jj < nj; ++jj) {
            const float2 xv = Xs[(pb * NPW + jj) * 32 + (lane & 31)];
            const float b0 = lane < 32 ? xv.x : -xv.y;
            const float b1 = lane < 32 ? xv.y : xv.x;
            const float* tj = Ts + ((pb * NPW + jj) * 2 + (lane >> 5)) * V + 2 * w * N1P + (lane & 31);
#pragma unroll
            for (int b = 0; b < BPC; ++b) {
              const float a = tj[32 * b];
              acc[b][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b0, acc[b][0], 0, 0, 0);
              acc[b][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b1, acc[b][1], 0, 0, 0);
            }
          }
        }
        __syncthreads();
      }
      const int rhs = I.w * 32 + (lane & 31);
      if (rhs < A.nrhs[I.x]) {
        const int k = I.y;
        const int c0 = (I.z % A.tiles2) * 8, i3 = I.z / A.tiles2;
        float2* Y = A.out[I.x] + A.ld_out[I.x] * rhs + (int64_t)k * A.nv +
                    (int64_t)A.n1 * ((int64_t)A.n2 * i3) + 4 * (lane >> 5);
#pragma unroll
        for (int b = 0; b < BPC; ++b) {
          const int col = c0 + 2 * w + b / NB1;
          if (col < A.n2) {
            float2* yb = Y + (int64_t)A.n1 * col + 32 * (b % NB1);
            const int lim = A.n1 - 32 * (b % NB1) - 4 * (lane >> 5);
#pragma unroll
            for (int i = 0; i < 16; ++i)
              if (8 * (i >> 2) + (i & 3) < lim)
                yb[8 * (i >> 2) + (i & 3)] = make_float2(acc[b][0][i], acc[b][1][i]);
          }
        }
      }
    }
  } else {
    float* tdst = Ts + (w * 2 + ((lane >> 3) & 1)) * V + (lane & 7) * N1P + 4 * (lane >> 4);
    for (;;) {
      const int it = next_item(A.counter, &s_item);
      if (it >= A.nitems) break;
      const int4 I = uni_item(A.items[it]);
      const BatchStatic S = A.plans[I.x];
      const int k = I.y;
      const int c0 = (I.z % A.tiles2) * 8, i3 = I.z / A.tiles2;
      const int64_t m = S.m;
      const int nbat = (int)((m + 3) / 4);
      const float2* X = A.in[I.x];
      const int64_t ldx = A.ld_in[I.x];
      const int xr = min(I.w * 32 + (lane & 31), A.nrhs[I.x] - 1);
      const BTensor* bt = S.bt + (int64_t)k * S.m;
      DecOps op;
      float ua[NCH][16];
      // Tensor j = 4s + w is decompressed in step s: its mode 2 ran in step
      // s - 1 (into Bc[s & 1]), so that step s starts mode 1 at once and runs
      // the next tensor's mode 2 alongside.  Tensor indices are clamped to
      // m - 1: loads are always issued, and only the MFMA and LDS work is
      // skipped for tensors beyond m.
      dec_load<true>(op, bt, min((int64_t)w, m - 1), A.hcache, A.u2p, i3, c0, X, ldx, xr, lane);
#pragma unroll
      for (int c = 0; c < NCH; ++c) dec_u1ops(A.u1p, op.u1p, op.r1, c, ua[c], lane);
      float2 xcur = op.xv;
      int r1cur = op.r1;
      if (w < m) dec_mode2(op, Bc, lane);
      dec_load<true>(op, bt, min((int64_t)w + 4, m - 1), A.hcache, A.u2p, i3, c0, X, ldx, xr, lane);
      for (int s = 0; s <= nbat; ++s) {
        const int buf = s & 1;
        const int64_t j = 4 * (int64_t)s + w;
        const bool have = s < nbat && j < m;
        const int np1 = (r1cur + 1) >> 1;
        if (have && lane < 32) Xs[(buf * NPW + w) * 32 + lane] = xcur;
        wave_sync();
        float bb[16];
        if (have) dec_bops(Bc + buf * NPW * 1024, bb, lane);
        // mode 2 of tensor j + 4 (operands in op) into the other Bc buffer
        if (s + 1 < nbat && j + 4 < m) dec_mode2(op, Bc + (buf ^ 1) * NPW * 1024, lane);
        const float2 x4 = op.xv;
        const int r1n = op.r1;
        const int64_t u1n = op.u1p;
        dec_load<true>(op, bt, min(j + 8, m - 1), A.hcache, A.u2p, i3, c0, X, ldx, xr, lane);
        float* dst = tdst + buf * NPW * 2 * V;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          if constexpr (BF) {
            // hi and lo halves into K slot 4 part + w of the 16-byte records
            // [buf][h][voxel]; a tensor beyond m writes zeros (its slot is
            // part of every MFMA's K)
            v4f d = {0.f, 0.f, 0.f, 0.f};
            if (have) d = chain16_n(np1, ua[c], bb);
            unsigned short* rec = reinterpret_cast<unsigned short*>(Ts) +
                                  ((size_t)(buf * 2) * V + (lane & 7) * N1P + 16 * c +
                                   4 * (lane >> 4)) * 8 + 4 * ((lane >> 3) & 1) + w;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const uint32_t h = bt_rne(d[r]);
              rec[r * 8] = (unsigned short)h;
              rec[(size_t)V * 8 + r * 8] = (unsigned short)bt_rne(d[r] - bt_f(h));
            }
          } else if (have) {
            const v4f d = chain16_n(np1, ua[c], bb);
            *reinterpret_cast<float4*>(dst + 16 * c) = make_float4(d[0], d[1], d[2], d[3]);
          }
          dec_u1ops(A.u1p, u1n, r1n, c, ua[c], lane);  // U1 of tensor j + 4
        }
        xcur = x4;
        r1cur = r1n;
        __syncthreads();
      }
    }
  }
}

// Adjoint, MFMA decompression.  Item = (plan, component and slice of the
// tiles, chunk of 32 columns, right-hand-side group); a tile is 16 NI rows
// of i1 x 8 columns at one i3.  Per tile each wave decompresses four of the
// 32 tensors into Tb[f][i1][jj] (row stride 33 complex, column stride
// 16 NI + 1 rows, against LDS bank conflicts); then wave w contracts column
// f = w: W(32 rhs x 32 columns) += Y^T conj(T) on v_mfma_f32_32x32x2f32, one
// voxel per pair of MFMAs.  The eight waves' W are summed in a fixed order.
template <int NI, bool BF>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
void batch_adj_mfma(BatchArgs A) {
  constexpr int NW = 8, IB = 16 * NI, RS = IB + 1, TS = 33;
  extern __shared__ float4 bsm4[];
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & 63, wave = uni(tid >> 6);
  float2* Tb = reinterpret_cast<float2*>(bsm4);  // [8][RS][TS]
  float* Bc = reinterpret_cast<float*>(Tb + 8 * RS * TS) + wave * 1024;
  // y window of this wave: 8 voxels x 32 right-hand sides, row stride 33
  float2* Ysw = reinterpret_cast<float2*>(reinterpret_cast<float*>(Tb + 8 * RS * TS) + 8 * 1024) +
                wave * 8 * 33;
  const int tiles = A.nic * A.tiles2 * A.n3;
  for (;;) {
    const int it = next_item(A.counter, &s_item);
    if (it >= A.nitems) break;
    const int4 I = uni_item(A.items[it]);
    const BatchStatic S = A.plans[I.x];
    const int k = I.y / A.tsplit, slice = I.y % A.tsplit;
    const int tb0 = (int)((int64_t)tiles * slice / A.tsplit);
    const int tb1 = (int)((int64_t)tiles * (slice + 1) / A.tsplit);
    const int64_t j0 = (int64_t)I.z * 32;
    const int jc = (int)min((int64_t)32, S.m - j0);
    // y is read in windows of 8 voxels of the wave's column: lane l loads
    // voxel l % 8 of right-hand sides l / 8 + 8 q (q < 4), so that a load
    // instruction touches 8 half cache lines instead of 32 lines; the window
    // is transposed through LDS.  Rows >= n1, columns >= n2 and right-hand
    // sides >= nrhs are read clamped: T is zero there, and lanes beyond nrhs
    // are never stored.
    const float2* yq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      yq[q] = A.in[I.x] + (int64_t)k * A.nv +
              A.ld_in[I.x] * min(I.w * 32 + (lane >> 3) + 8 * q, A.nrhs[I.x] - 1);
    const BTensor* bt = S.bt + (int64_t)k * S.m + j0;
    v16f acc[2];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[0][i] = acc[1][i] = 0.f;
    // tile t: i1 chunk (t % nic), column group ((t / nic) % tiles2), i3
    auto tile_pos = [&](int t, int& ic0, int& c0, int& i3) {
      ic0 = (t % A.nic) * NI;
      const int rest = t / A.nic;
      c0 = (rest % A.tiles2) * 8;
      i3 = rest / A.tiles2;
    };
    // this wave's columns of the chunk are 4 wave + e, e < 4, valid below
    // jc; the operands of the next slot (or of slot 0 on the next tile) are
    // loaded while the current one is decompressed, U1 chunk by chunk as
    // each chunk's registers retire.  Slot indices are clamped to jc - 1 so
    // that every slot issues the same loads; invalid slots skip the work.
    auto wload = [&](int wic0, int wc0, int wi3, int w, float2* yr) {
      const int col = min(wc0 + wave, A.n2 - 1);
      const int i1 = min(16 * wic0 + 8 * w + (lane & 7), A.n1 - 1);
      const int64_t off = (int64_t)A.n1 * (col + (int64_t)A.n2 * wi3) + i1;
#pragma unroll
      for (int q = 0; q < 4; ++q) yr[q] = yq[q][off];
    };
    float2 yr[4];
    DecOps op;
    float ua[NI][16];
    {
      int ic0, c0, i3;
      tile_pos(tb0, ic0, c0, i3);
      wload(ic0, c0, i3, 0, yr);
      dec_load<false>(op, bt, min(4 * wave, jc - 1), A.hcache, A.u2p, i3, c0, nullptr, 0, 0,
                      lane);
#pragma unroll
      for (int ic = 0; ic < NI; ++ic) dec_u1ops(A.u1p, op.u1p, op.r1, ic0 + ic, ua[ic], lane);
    }
    for (int tile = tb0; tile < tb1; ++tile) {
      int ic0, c0, i3;
      tile_pos(tile, ic0, c0, i3);
      int nic0, nc0, ni3;
      tile_pos(min(tile + 1, tb1 - 1), nic0, nc0, ni3);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int jj = 4 * wave + e;
        const bool have = jj < jc;
        const int np1 = (op.r1 + 1) >> 1;
        if (have) dec_mode2(op, Bc, lane);
        const int pj = e < 3 ? min(jj + 1, jc - 1) : min(4 * wave, jc - 1);
        const int pi3 = e < 3 ? i3 : ni3, pc0 = e < 3 ? c0 : nc0, pic0 = e < 3 ? ic0 : nic0;
        dec_load<false>(op, bt, pj, A.hcache, A.u2p, pi3, pc0, nullptr, 0, 0, lane);
        float bb[16];
        if (have) {
          wave_sync();
          dec_bops(Bc, bb, lane);
        }
        float* dst = reinterpret_cast<float*>(Tb) +
                     (((lane & 7) * RS + 4 * (lane >> 4)) * TS + jj) * 2 + ((lane >> 3) & 1);
        // BF16X3: 16-byte records [h][quad][jj] of four voxels x (Re, Im);
        // quad = f (IB / 4) + i1 / 4 within the tile
        unsigned short* dsb = reinterpret_cast<unsigned short*>(Tb) +
                              (((lane & 7) * (IB / 4) + (lane >> 4)) * 32 + jj) * 8 +
                              ((lane >> 3) & 1);
#pragma unroll
        for (int ic = 0; ic < NI; ++ic) {
          if (have) {
            const v4f d = chain16_n(np1, ua[ic], bb);
            if constexpr (BF) {
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const uint32_t h = bt_rne(d[r]);
                dsb[ic * 4 * 32 * 8 + 2 * r] = (unsigned short)h;
                dsb[2 * IB * 32 * 8 + ic * 4 * 32 * 8 + 2 * r] =
                    (unsigned short)bt_rne(d[r] - bt_f(h));
              }
            } else {
#pragma unroll
              for (int r = 0; r < 4; ++r) dst[(16 * ic + r) * TS * 2] = d[r];
            }
          }
          dec_u1ops(A.u1p, op.u1p, op.r1, pic0 + ic, ua[ic], lane);
        }
      }
      __syncthreads();
      // column f = wave of the tile, window by window
      if constexpr (BF) {
        // BF16X3: K slot 8h + 2v + p of a quad of four voxels; A = y of the
        // quad (hi for lanes < 32, lo for the others), A' = (Im, -Re) of the
        // same, B = T's hi halves in both slot halves (Yh Th + Yl Th) or its
        // lo halves against y's hi (Yh Tl): Wr from A, Wi from A'.
        const uint4* tq = reinterpret_cast<const uint4*>(Tb) + wave * (IB / 4) * 32 + (lane & 31);
        uint32_t* yw = reinterpret_cast<uint32_t*>(Ysw);  // [h][2 quads][32 rhs][4 words]
#pragma unroll
        for (int w = 0; w < IB / 8; ++w) {
          wave_sync();
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float2 y = yr[q];
            const uint32_t hr = bt_rne(y.x), hi = bt_rne(y.y);
            const uint32_t lr = bt_rne(y.x - bt_f(hr)), li = bt_rne(y.y - bt_f(hi));
            const int i = lane & 7, rhs = (lane >> 3) + 8 * q;
            const int o = ((i >> 2) * 32 + rhs) * 4 + (i & 3);
            yw[o] = bt_pack(hr, hi);
            yw[2 * 32 * 4 + o] = bt_pack(lr, li);
          }
          wave_sync();
          if (w + 1 < IB / 8)
            wload(ic0, c0, i3, w + 1, yr);
          else
            wload(nic0, nc0, ni3, 0, yr);  // first window of the next tile
#pragma unroll
          for (int qd = 0; qd < 2; ++qd) {
            const uint4 a = reinterpret_cast<const uint4*>(yw)[((lane >> 5) * 2 + qd) * 32 + (lane & 31)];
            uint4 a2;  // (Im, -Re) per voxel
            a2.x = (a.x >> 16) | ((a.x ^ 0x8000u) << 16);
            a2.y = (a.y >> 16) | ((a.y ^ 0x8000u) << 16);
            a2.z = (a.z >> 16) | ((a.z ^ 0x8000u) << 16);
            a2.w = (a.w >> 16) | ((a.w ^ 0x8000u) << 16);
            const int quad = 2 * w + qd;
            const uint4 b1 = tq[quad * 32];
            const uint4 b2 = lane < 32 ? tq[2 * IB * 32 + quad * 32] : make_uint4(0u, 0u, 0u, 0u);
            acc[0] = mfma_bf(a, b1, acc[0]);
            acc[0] = mfma_bf(a, b2, acc[0]);
            acc[1] = mfma_bf(a2, b1, acc[1]);
            acc[1] = mfma_bf(a2, b2, acc[1]);
          }
        }
      } else {
      const float2* tc = Tb + wave * RS * TS + (lane & 31);
#pragma unroll
      for (int w = 0; w < IB / 8; ++w) {
        wave_sync();
#pragma unroll
        for (int q = 0; q < 4; ++q) Ysw[(lane & 7) * 33 + (lane >> 3) + 8 * q] = yr[q];
        wave_sync();
        if (w + 1 < IB / 8)
          wload(ic0, c0, i3, w + 1, yr);
        else
          wload(nic0, nc0, ni3, 0, yr);  // first window of the next tile
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float2 yv = Ysw[i * 33 + (lane & 31)];
          const float2 tb = tc[(8 * w + i) * TS];
          const float bv = lane < 32 ? tb.x : -tb.y;
          const float a0 = lane < 32 ? yv.x : -yv.y;
          const float a1 = lane < 32 ? yv.y : yv.x;
          acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, bv, acc[0], 0, 0, 0);
          acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, bv, acc[1], 0, 0, 0);
        }
      }
      }
      __syncthreads();
    }
    // sum the eight waves' W in a fixed order
    float* red = reinterpret_cast<float*>(Tb);
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int i = 0; i < 16; ++i) red[((wave * 2 + mb) * 16 + i) * 64 + lane] = acc[mb][i];
    __syncthreads();
    if (wave == 0) {
      float2* blk = A.partial + (int64_t)it * 1024;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        float wr = 0.f, wi = 0.f;
        for (int w = 0; w < NW; ++w) {
          wr += red[((w * 2 + 0) * 16 + i) * 64 + lane];
          wi += red[((w * 2 + 1) * 16 + i) * 64 + lane];
        }
        const int rl = 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        blk[rl * 32 + (lane & 31)] = make_float2(wr, wi);
      }
    }
  }
}

size_t batch_mfma_lds_bytes(int op, int nb) {
  if (op == 0) return sizeof(float) * (2 * 4 * 2 * (8 * 32 * nb) + 2 * 4 * 64 + 2 * 4 * 1024);
  // Tb, then Bc, then the y windows; the final reduction reuses the start
  const size_t tb = sizeof(float2) * 8 * (16 * nb + 1) * 33;
  const size_t all = tb + sizeof(float) * 8 * 1024 + sizeof(float2) * 8 * 8 * 33;
  return std::max(all, sizeof(float) * 8 * 2 * 16 * 64);
}

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
  int r1max = 1, r2max = 1, r3max = 1;
  int nitems = 0;
  int grid_blocks = 0;
  int per_cu = 1;           // persistent workgroups per compute unit
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
  // MFMA decompression kernels (ranks <= 32): per-tensor records, packed U1
  // and U2, tensor list of the mode-3 kernel, mode-3 cache size in floats
  bool mfma = false;
  bool bf = false;          // forward apply in BF16X3 (all plans BF16X3)
  int nch = 0, nic = 0;
  int ntensors = 0;
  int64_t hcache = 0;
  BTensor* d_bt = nullptr;
  float* d_u1p = nullptr;
  float* d_u2p = nullptr;
  int2* d_tlist = nullptr;
  // host copies awaiting tv_batch_bind_arena (the arena is the caller's)
  std::vector<BTensor> h_bt;
  std::vector<size_t> h_bt_off;      // first record of each plan in h_bt
  std::vector<float> h_u1p, h_u2p;
  std::vector<int2> h_tlist;
  std::vector<BatchStatic> h_plans;
  std::vector<int4> h_items, h_red_out;
  std::vector<int> h_red_list;
  bool bound = false;
  size_t arena_bytes = 0;
};

static void batch_free(tv_batch_s* b) { delete b; }

// Device arena of a batch object: the per-plan records, work items,
// reduction lists and packed operands at 256-byte aligned offsets.  With
// base == nullptr only the size is computed.
static size_t batch_layout(tv_batch_s* b, char* base) {
  size_t off = 0;
  auto carve = [&](auto** ptr, size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    typedef typename std::remove_reference<decltype(**ptr)>::type T;
    if (base) *ptr = bytes ? reinterpret_cast<T*>(base + off) : nullptr;
    off += bytes;
  };
  carve(&b->d_plans, b->h_plans.size() * sizeof(BatchStatic));
  carve(&b->d_items, b->h_items.size() * sizeof(int4));
  carve(&b->d_red_list, b->h_red_list.size() * sizeof(int));
  carve(&b->d_red_out, b->h_red_out.size() * sizeof(int4));
  carve(&b->d_bt, b->h_bt.size() * sizeof(BTensor));
  carve(&b->d_u1p, b->h_u1p.size() * sizeof(float));
  carve(&b->d_u2p, b->h_u2p.size() * sizeof(float));
  carve(&b->d_tlist, b->h_tlist.size() * sizeof(int2));
  return (off + 255) & ~(size_t)255;
}

static size_t batch_hcache_offset(const tv_batch_s* b) {
  const size_t head = 256 + (b->op == 1 ? (size_t)b->nitems * 1024 * 8 : 0);
  return (head + 255) / 256 * 256;
}

extern "C" {

tv_status tv_batch_create(int32_t nplans, const tv_plan* plans, int32_t op, const int32_t* nrhs,
                          const tv_batch_config* cfg, tv_batch* out) {
  clear_error();
  if (!out) return set_error(TV_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (nplans < 1 || nplans > TV_BATCH_MAX_PLANS)
    return set_error(TV_ERR_INVALID_ARG, "nplans outside [1, TV_BATCH_MAX_PLANS]");
  if (!plans || !nrhs) return set_error(TV_ERR_INVALID_ARG, "plans and nrhs must be non-NULL");
  if (op != 0 && op != 1) return set_error(TV_ERR_INVALID_ARG, "op must be 0 or 1");
  if (cfg && (cfg->tsplit < 0 || cfg->blocks_per_cu < 0))
    return set_error(TV_ERR_INVALID_ARG, "batch configuration values must be >= 0");
  for (int c = 0; c < nplans; ++c) {
    if (!plans[c] || !plans[c]->finalized || !plans[c]->bound)
      return set_error(TV_ERR_INVALID_ARG, "every plan must be finalized and bound to its arena");
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
  int& r3max = b->r3max;
  for (int c = 0; c < nplans; ++c) {
    b->r1max = std::max(b->r1max, plans[c]->max_r[0]);
    b->r2max = std::max(b->r2max, plans[c]->max_r[1]);
    r3max = std::max(r3max, plans[c]->max_r[2]);
    b->m.push_back(plans[c]->grid.m);
    b->nrhs.push_back(nrhs[c]);
  }
  // MFMA decompression for ranks up to 32 (forward: n1 <= 96); otherwise the
  // wave-local VALU decompression kernels
  b->mfma = b->r1max <= 32 && b->r2max <= 32 && r3max <= 32 && (op == 1 || nb1 <= 3);
  if (b->mfma) {
    b->ncol = 8;
    if (op == 0) {
      b->bpw = nb1;
      bool bf = true;
      for (int c = 0; c < nplans; ++c) bf = bf && plans[c]->precision == TV_PREC_BF16X3;
      b->bf = bf;
      if (bf)
        b->fn = nb1 == 1 ? batch_fwd_mfma<1, true> : nb1 == 2 ? batch_fwd_mfma<2, true>
                                                              : batch_fwd_mfma<3, true>;
      else
        b->fn = nb1 == 1 ? batch_fwd_mfma<1, false> : nb1 == 2 ? batch_fwd_mfma<2, false>
                                                               : batch_fwd_mfma<3, false>;
    } else {
      const int ni = std::min(3, (g.n1 + 15) / 16);
      b->bpw = ni;
      b->nic = (g.n1 + 16 * ni - 1) / (16 * ni);
      bool bf = true;
      for (int c = 0; c < nplans; ++c) bf = bf && plans[c]->precision == TV_PREC_BF16X3;
      b->bf = bf;
      if (bf)
        b->fn = ni == 1 ? batch_adj_mfma<1, true> : ni == 2 ? batch_adj_mfma<2, true>
                                                            : batch_adj_mfma<3, true>;
      else
        b->fn = ni == 1 ? batch_adj_mfma<1, false> : ni == 2 ? batch_adj_mfma<2, false>
                                                             : batch_adj_mfma<3, false>;
    }
    b->nch = std::max(b->n1p32 / 16, op == 1 ? b->nic * b->bpw : 0);
    b->lds = batch_mfma_lds_bytes(op, b->bpw);
  } else if (op == 0) {
    // columns per tile: the widest power of two whose nb1 * ncol 32-voxel
    // blocks split evenly over the 4 waves with at most 3 blocks per wave
    // (each block holds 32 accumulator registers per real/imaginary half)
    int ncol = 0;
    for (int c = 16; c >= 1 && !ncol; c /= 2)
      if ((nb1 * c) % 4 == 0 && nb1 * c / 4 <= 3) ncol = c;
    b->ncol = ncol;
    b->bpw = ncol ? nb1 * ncol / 4 : 0;
    b->fn = ncol ? pick_fwd(b->ncol, b->bpw) : nullptr;
    b->lds = batch_lds_bytes(op, b->ncol, b->n1p32, b->r1max, b->r2max);
  } else {
    int ncol = 1;
    while (ncol * 2 * b->n1p32 <= 384) ncol *= 2;
    b->ncol = ncol;
    b->fn = pick_adj(b->ncol);
    b->lds = batch_lds_bytes(op, b->ncol, b->n1p32, b->r1max, b->r2max);
  }
  if (!b->fn || b->lds > 160 * 1024) {
    delete b;
    return set_error(TV_ERR_NOT_SUPPORTED, "no batched kernel for these sizes and ranks");
  }
  const int threads = b->mfma ? 512 : 256;
  b->tiles2 = (g.n2 + b->ncol - 1) / b->ncol;
  // work items, longest first (most tensors per item); the adjoint splits
  // the voxel tiles of each (plan, component, chunk) into tsplit slices so
  // that there are enough items to fill the device
  std::vector<int> order(nplans);
  for (int c = 0; c < nplans; ++c) order[c] = c;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->m[x] > b->m[y]; });
  const int tiles = b->tiles2 * g.n3 * (b->mfma && op == 1 ? b->nic : 1);
  if (op == 1) {
    const int64_t target = b->mfma ? 4096 : 2048;
    int64_t base = 0;
    for (int c = 0; c < nplans; ++c) base += (int64_t)g.q * ((b->m[c] + 31) / 32) * ((nrhs[c] + 31) / 32);
    b->tsplit = (int)std::max<int64_t>(1, std::min<int64_t>(tiles, (target + base - 1) / base));
    if (cfg && cfg->tsplit > 0) b->tsplit = std::min(cfg->tsplit, tiles);
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
  // MFMA kernels: per-tensor records, the mode-3 cache layout, and U1 and U2
  // packed in the kernels' operand order (quads of four K steps per lane)
  std::vector<std::vector<BTensor>> bts(nplans);
  std::vector<float> u1p, u2p;
  std::vector<int2> tlist;
  if (b->mfma) {
    const int ncg = (g.n2 + 7) / 8;
    size_t u1n = 0, u2n = 0;
    for (int c = 0; c < nplans; ++c) {
      const tv_plan_s* P = plans[c];
      for (int64_t t = 0; t < (int64_t)g.q * P->grid.m; ++t) {
        u1n += (size_t)b->nch * (((P->ranks[3 * t] + 1) / 2 + 3) / 4) * 256;
        u2n += (size_t)ncg * (((P->ranks[3 * t + 1] + 1) / 2 + 3) / 4) * 256;
      }
    }
    u1p.assign(u1n, 0.f);
    u2p.assign(u2n, 0.f);
    size_t u1o = 0, u2o = 0;
    for (int c = 0; c < nplans; ++c) {
      const tv_plan_s* P = plans[c];
      const int64_t m = P->grid.m;
      bts[c].resize((size_t)g.q * m);
      for (int k = 0; k < g.q; ++k)
        for (int64_t j = 0; j < m; ++j) {
          const int64_t t = k + (int64_t)g.q * j;
          const int r1 = P->ranks[3 * t], r2 = P->ranks[3 * t + 1];
          const int nq1 = ((r1 + 1) / 2 + 3) / 4, nq2 = ((r2 + 1) / 2 + 3) / 4;
          BTensor& T = bts[c][(size_t)k * m + j];
          T.r1 = r1;
          T.r2 = r2;
          T.h_off = b->hcache;
          T.u1p_off = (int64_t)u1o;
          T.u2p_off = (int64_t)u2o;
          b->hcache += (int64_t)g.n3 * ((r1 + 15) / 16) * nq2 * 256;
          // block (ic, q), lane l, step t = 4q + i: Re/Im (l/16 % 2) of U1[16 ic + l%16][2t + l/32]
          for (int ic = 0; ic < b->nch; ++ic)
            for (int q = 0; q < nq1; ++q)
              for (int l = 0; l < 64; ++l)
                for (int i = 0; i < 4; ++i) {
                  const int i1 = 16 * ic + (l & 15), a = 2 * (4 * q + i) + (l >> 5);
                  if (i1 < g.n1 && a < r1)
                    u1p[u1o + (((size_t)ic * nq1 + q) * 64 + l) * 4 + i] = (float)
                        P->u1[2 * (P->u1_off[t] + i1 + (size_t)g.n1 * a) + ((l >> 4) & 1)];
                }
          // block (cg, q), lane l, step t: Re/Im (part ^ s) of U2[8 cg + l%8][2t + l/32]
          for (int cg = 0; cg < ncg; ++cg)
            for (int q = 0; q < nq2; ++q)
              for (int l = 0; l < 64; ++l)
                for (int i = 0; i < 4; ++i) {
                  const int i2 = 8 * cg + (l & 7), bb = 2 * (4 * q + i) + (l >> 5);
                  const int comp = ((l >> 3) ^ (l >> 4)) & 1;
                  if (i2 < g.n2 && bb < r2)
                    u2p[u2o + (((size_t)cg * nq2 + q) * 64 + l) * 4 + i] =
                        (float)P->u2[2 * (P->u2_off[t] + i2 + (size_t)g.n2 * bb) + comp];
                }
          u1o += (size_t)b->nch * nq1 * 256;
          u2o += (size_t)ncg * nq2 * 256;
          tlist.push_back(make_int2(c, (int)(k * m + j)));
        }
    }
    b->ntensors = (int)tlist.size();
  }
  std::vector<BatchStatic> st(nplans);
  for (int c = 0; c < nplans; ++c)
    st[c] = BatchStatic{plans[c]->d_meta, plans[c]->d_cores, plans[c]->d_u1t, plans[c]->d_u2t,
                        plans[c]->d_u3t, plans[c]->grid.m, nullptr};
  if (b->mfma) {
    for (int c = 0; c < nplans; ++c) {
      b->h_bt_off.push_back(b->h_bt.size());
      b->h_bt.insert(b->h_bt.end(), bts[c].begin(), bts[c].end());
    }
    b->h_u1p = std::move(u1p);
    b->h_u2p = std::move(u2p);
    b->h_tlist = std::move(tlist);
  }
  b->h_plans = std::move(st);
  b->h_items = std::move(items);
  if (op == 1) {
    b->h_red_list = std::move(red_list);
    b->h_red_out = std::move(red_out);
  }
  b->arena_bytes = batch_layout(b, nullptr);
  hipError_t e = hipSuccess;
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)b->fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)b->lds);
  int dev = 0, cus = 256, per_cu = 1;
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)b->fn, threads, b->lds);
  if (e != hipSuccess) {
    batch_free(b);
    return hip_error(e, "tv_batch_create");
  }
  per_cu = std::max(per_cu, 1);
  if (cfg && cfg->blocks_per_cu > 0) per_cu = std::min(per_cu, (int)cfg->blocks_per_cu);
  b->per_cu = per_cu;
  b->grid_blocks = std::max(1, std::min(b->nitems, cus * per_cu));
  *out = b;
  return TV_OK;
}

tv_status tv_batch_required_bytes(tv_batch b, size_t* bytes) {
  clear_error();
  if (!b || !bytes) return set_error(TV_ERR_INVALID_ARG, "batch and bytes must be non-NULL");
  *bytes = b->arena_bytes;
  return TV_OK;
}

tv_status tv_batch_bind_arena(tv_batch b, void* arena, size_t bytes, void* stream) {
  clear_error();
  if (!b) return set_error(TV_ERR_INVALID_ARG, "batch is NULL");
  if (b->bound) return set_error(TV_ERR_INVALID_ARG, "batch is already bound to an arena");
  if (!arena) return set_error(TV_ERR_INVALID_ARG, "arena is NULL");
  if ((uintptr_t)arena % 256) return set_error(TV_ERR_INVALID_ARG, "arena must be 256-byte aligned");
  if (bytes < b->arena_bytes) {
    char buf[128];
    snprintf(buf, sizeof buf, "arena of %zu bytes needed, %zu given", b->arena_bytes, bytes);
    return set_error(TV_ERR_WORKSPACE, buf);
  }
  batch_layout(b, (char*)arena);
  for (size_t c = 0; c < b->h_bt_off.size(); ++c) b->h_plans[c].bt = b->d_bt + b->h_bt_off[c];
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  auto put = [&](void* d, const void* src, size_t n) {
    if (e == hipSuccess && n) e = hipMemcpyAsync(d, src, n, hipMemcpyHostToDevice, st);
  };
  put(b->d_plans, b->h_plans.data(), b->h_plans.size() * sizeof(BatchStatic));
  put(b->d_items, b->h_items.data(), b->h_items.size() * sizeof(int4));
  put(b->d_red_list, b->h_red_list.data(), b->h_red_list.size() * sizeof(int));
  put(b->d_red_out, b->h_red_out.data(), b->h_red_out.size() * sizeof(int4));
  put(b->d_bt, b->h_bt.data(), b->h_bt.size() * sizeof(BTensor));
  put(b->d_u1p, b->h_u1p.data(), b->h_u1p.size() * sizeof(float));
  put(b->d_u2p, b->h_u2p.data(), b->h_u2p.size() * sizeof(float));
  put(b->d_tlist, b->h_tlist.data(), b->h_tlist.size() * sizeof(int2));
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_error(e, "batch upload");
  b->bound = true;
  b->h_bt.clear();
  b->h_u1p.clear();
  b->h_u2p.clear();
  b->h_tlist.clear();
  b->h_items.clear();
  b->h_red_list.clear();
  b->h_red_out.clear();
  b->h_bt.shrink_to_fit();
  b->h_u1p.shrink_to_fit();
  b->h_u2p.shrink_to_fit();
  b->h_items.shrink_to_fit();
  return TV_OK;
}

tv_status tv_batch_workspace_bytes(tv_batch b, size_t* bytes) {
  clear_error();
  if (!b || !bytes) return set_error(TV_ERR_INVALID_ARG, "batch and bytes must be non-NULL");
  // the work-queue counter, (adjoint) one 32 x 32 complex64 block per item,
  // then (MFMA kernels) the packed mode-3 cache, about r1 r2 n3 complex64 per
  // tensor (row blocks of 16 and quads of four K steps rounded up)
  *bytes = b->mfma ? batch_hcache_offset(b) + (size_t)b->hcache * 4
                   : 256 + (b->op == 1 ? (size_t)b->nitems * 1024 * 8 : 0);
  return TV_OK;
}

tv_status tv_batch_run(tv_batch b, const void* const* in, const int64_t* ld_in, void* const* out,
                       const int64_t* ld_out, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (!b || !in || !ld_in || !out || !ld_out)
    return set_error(TV_ERR_INVALID_ARG, "NULL argument");
  if (!b->bound) return set_error(TV_ERR_INVALID_ARG, "batch has no device arena (tv_batch_bind_arena)");
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
  A.hcache = b->mfma ? (float*)((char*)ws + batch_hcache_offset(b)) : nullptr;
  A.u1p = b->d_u1p;
  A.u2p = b->d_u2p;
  A.nch = b->nch;
  A.nic = b->nic;
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
  if (b->mfma) {
    const size_t u3b = sizeof(float2) * b->grid.n3 * b->r3max;
    if (u3b <= 64 * 1024)
      hipLaunchKernelGGL(batch_mode3<true>, dim3((unsigned)b->ntensors), dim3(256), u3b, st, A,
                         (const int2*)b->d_tlist);
    else
      hipLaunchKernelGGL(batch_mode3<false>, dim3((unsigned)b->ntensors), dim3(256), 0, st, A,
                         (const int2*)b->d_tlist);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "mode-3 kernel launch");
  }
  hipLaunchKernelGGL(b->fn, dim3((unsigned)b->grid_blocks), dim3(b->mfma ? 512 : 256), b->lds,
                     st, A);
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
  batch_free(b);
  return TV_OK;
}

tv_status tv_batch_info(tv_batch b, tv_batch_config* cfg) {
  clear_error();
  if (!b || !cfg) return set_error(TV_ERR_INVALID_ARG, "batch and cfg must be non-NULL");
  cfg->tsplit = b->op == 1 ? b->tsplit : 0;
  cfg->blocks_per_cu = b->per_cu;
  return TV_OK;
}

// Times batch configurations (adjoint voxel-tile slices, persistent
// workgroups per CU) on zero-filled vectors with timing buffers of its own
// (set-up call: allocates and synchronises) and returns the fastest; results
// are cached in the JSON file shared with tv_autotune.
tv_status tv_batch_autotune(int32_t nplans, const tv_plan* plans, int32_t op,
                            const int32_t* nrhs, const char* cache_path, void* stream,
                            tv_batch_config* best) {
  clear_error();
  if (!best || !plans || !nrhs || nplans < 1 || nplans > TV_BATCH_MAX_PLANS)
    return set_error(TV_ERR_INVALID_ARG, "invalid batch autotune arguments");
  *best = tv_batch_config{0, 0};
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the plans' ranks and nrhs
  for (int c = 0; c < nplans; ++c) {
    if (!plans[c]) return set_error(TV_ERR_INVALID_ARG, "NULL plan");
    for (int32_t r : plans[c]->ranks) {
      h ^= (uint32_t)r;
      h *= 1099511628211ull;
    }
    h ^= (uint32_t)nrhs[c];
    h *= 1099511628211ull;
  }
  const tv_grid g0 = plans[0]->grid;
  char key[256];
  snprintf(key, sizeof key, "b1|%s|%dx%dx%d|q%d|n%d|h%016llx|op%d", device_arch().c_str(), g0.n1,
           g0.n2, g0.n3, g0.q, nplans, (unsigned long long)h, op);
  auto cache = read_tune_cache(cache_path);
  auto it = cache.find(key);
  if (it != cache.end() && it->second.size() == 2) {
    *best = tv_batch_config{it->second[0], it->second[1]};
    return TV_OK;
  }
  // the default configuration fixes the candidates' ranges
  tv_batch b0 = nullptr;
  tv_status s = tv_batch_create(nplans, plans, op, nrhs, nullptr, &b0);
  if (s != TV_OK) return s;
  const int ts0 = b0->tsplit, pc0 = b0->per_cu;
  const int tiles = b0->tiles2 * g0.n3 * (b0->mfma && op == 1 ? b0->nic : 1);
  tv_batch_destroy(b0);
  std::vector<tv_batch_config> cands;
  for (int pc = 1; pc <= pc0; ++pc) {
    if (op == 0) {
      cands.push_back(tv_batch_config{0, pc});
      continue;
    }
    for (int ts = std::max(1, ts0 / 4); ts <= std::min(tiles, 4 * ts0); ts *= 2)
      cands.push_back(tv_batch_config{ts, pc});
  }
  // zero-filled vectors and the largest workspace
  const int64_t nv = (int64_t)g0.n1 * g0.n2 * g0.n3, rows = (int64_t)g0.q * nv;
  std::vector<void*> vin(nplans, nullptr), vout(nplans, nullptr);
  std::vector<int64_t> ldi(nplans), ldo(nplans);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  for (int c = 0; c < nplans && e == hipSuccess; ++c) {
    const int64_t m = plans[c]->grid.m;
    ldi[c] = op == 0 ? m : rows;
    ldo[c] = op == 0 ? rows : m;
    e = hipMalloc(&vin[c], (size_t)8 * ldi[c] * nrhs[c]);
    if (e == hipSuccess) e = hipMalloc(&vout[c], (size_t)8 * ldo[c] * nrhs[c]);
    if (e == hipSuccess) e = hipMemsetAsync(vin[c], 0, (size_t)8 * ldi[c] * nrhs[c], st);
  }
  float bestms = -1.f;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (size_t a = 0; e == hipSuccess && a < cands.size(); ++a) {
    tv_batch b = nullptr;
    if (tv_batch_create(nplans, plans, op, nrhs, &cands[a], &b) != TV_OK) continue;
    size_t ab = 0, wb = 0;
    void *arena = nullptr, *ws = nullptr;
    tv_batch_required_bytes(b, &ab);
    tv_batch_workspace_bytes(b, &wb);
    e = hipMalloc(&arena, std::max<size_t>(ab, 256));
    if (e == hipSuccess) e = hipMalloc(&ws, std::max<size_t>(wb, 256));
    bool ok = e == hipSuccess && tv_batch_bind_arena(b, arena, ab, stream) == TV_OK;
    auto run = [&]() {
      return tv_batch_run(b, (const void* const*)vin.data(), ldi.data(), vout.data(), ldo.data(),
                          ws, wb, stream) == TV_OK;
    };
    if (ok) ok = run();
    float ms = 0.f;
    if (ok && e == hipSuccess) e = hipEventRecord(e0, st);
    if (ok && e == hipSuccess) ok = run();
    if (ok && e == hipSuccess) e = hipEventRecord(e1, st);
    if (ok && e == hipSuccess) e = hipEventSynchronize(e1);
    if (ok && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (ok && e == hipSuccess && (bestms < 0.f || ms < bestms)) {
      bestms = ms;
      *best = cands[a];
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    tv_batch_destroy(b);
    hipFree(arena);
    hipFree(ws);
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  for (int c = 0; c < nplans; ++c) {
    hipFree(vin[c]);
    hipFree(vout[c]);
  }
  if (e != hipSuccess) return hip_error(e, "tv_batch_autotune");
  if (bestms < 0.f) return set_error(TV_ERR_NOT_SUPPORTED, "no batch configuration ran");
  cache[key] = {best->tsplit, best->blocks_per_cu};
  write_tune_cache(cache_path, cache);
  clear_error();
  return TV_OK;
}

}  // extern "C"
