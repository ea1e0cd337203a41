// Fused Tucker-decompress-and-multiply kernels, FP32 on MFMA (gfx950).
//
// For component k the product Y^k = sum_j x_j Z^{kj}(:) (Algorithm 1) is the
// stacked GEMM Y^k_(1) = [U1_1 ... U1_m] [x_1 M_1; ...; x_m M_m], where
// Y^k_(1) is the n1 x (n2 n3) mode-1 unfolding and M_j = G_j x2 U2_j x3 U3_j
// unfolded along mode 1 (r1 x n2 n3), from eq. (6)/(7).  Each workgroup owns
// all n1 rows of a tile of t2 x t3 columns (i2, i3) and a contiguous range of
// columns j; per tensor it
//   A) contracts the core with the tile's U3 rows (mode 3, eq. 7), scaling by
//      x_j: H[t3][a][b] = x_j sum_c G[a,b,c] U3[i3,c]            -> LDS
//   B) applies U2 per column (mode 2): B[a][(i2,i3)] = sum_b H U2[i2,b] -> LDS
//   C) accumulates the mode-1 product on v_mfma_f32_32x32x2f32 with the
//      complex product in real form: rows 2*i1 + {0,1} hold (Re, Im) of
//      output row i1, K step {0,1} carries (Re, Im) of B's row a, and the
//      A operand is [[Ar, -Ai], [Ai, Ar]] pre-packed in lane order.
// The adjoint (Algorithm 2) reuses A-C without the x_j scaling: it forms the
// tile of Z^{kj} = U1_j M_j, takes its conjugated dot product with the
// matching tile of y (held in registers) and writes one partial per
// (component, tile, column); a second kernel sums them in a fixed order.
//
// MFMA 32x32x2 f32 lane layout: A operand lane l = A[l%32][l/32], B operand
// lane l = B[l/32][l%32], accumulator register i of lane l =
// D[8*(i/4) + 4*(l/32) + i%4][l%32].
#include "tv_internal.h"

namespace tv {

typedef float v16f __attribute__((ext_vector_type(16)));

struct KParams {
  const TensorMeta* meta;
  const float2* cores;
  const float2* u2t;
  const float2* u3t;
  const float* apack;
  const int64_t* apack_koff;
  const int32_t* split;  // [q][S+1] first column of each split
  const float2* vec;     // x (forward) or one column of y (adjoint)
  float2* out;           // forward: y or its split partials; adjoint: partials
  int64_t out_stride;    // forward: complex stride between split partials
  int64_t m;
  int64_t nv;
  int n1, n2, n3, q;
  int nbt, t2, t3, tiles2;
  int64_t tiles;         // column tiles per component
  int S;
  int64_t nitems;        // q * S * tiles
  int r1max, r2max;
  int vec4;              // forward output may use 16-byte stores
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 c) {
  c.x = fmaf(a.x, b.x, c.x);
  c.x = fmaf(-a.y, b.y, c.x);
  c.y = fmaf(a.x, b.y, c.y);
  c.y = fmaf(a.y, b.x, c.y);
  return c;
}

// LDS carve-up shared by host sizing and the kernel.
__host__ __device__ inline size_t lds_hs_elems(int t3, int r1, int r2) {
  return (size_t)t3 * r1 * r2;  // float2
}
__host__ __device__ inline size_t lds_u2_elems(int t2, int r2) {
  return (size_t)t2 * r2;  // float2
}
__host__ __device__ inline size_t lds_bs_elems(int r1, int nwg) {
  return (size_t)r1 * 2 * nwg;  // float
}
size_t fused_lds_bytes(int t2, int t3, int r1max, int r2max, int nwg) {
  return 8 * lds_hs_elems(t3, r1max, r2max) + 8 * lds_u2_elems(t2, r2max) +
         4 * lds_bs_elems(r1max, nwg) + 64;
}

template <int NB, int WN, bool ADJ>
__global__ __launch_bounds__(256) void fused_f32(KParams P) {
  extern __shared__ float4 smem4[];
  constexpr int NWG = 32 * WN;
  constexpr int AG = 256 / NWG;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;

  // Consecutive work items (same component and column split, neighbouring
  // tiles) go to the same XCD: hardware deals blocks round-robin over 8.
  const int64_t G8 = gridDim.x / 8;
  const int64_t item = (int64_t)(blockIdx.x % 8) * G8 + blockIdx.x / 8;
  if (item >= P.nitems) return;
  const int64_t tile = item % P.tiles;
  const int64_t ks = item / P.tiles;
  const int s = (int)(ks % P.S);
  const int k = (int)(ks / P.S);
  const int i2_0 = (int)(tile % P.tiles2) * P.t2;
  const int i3_0 = (int)(tile / P.tiles2) * P.t3;
  const int jb = P.split[k * (P.S + 1) + s];
  const int je = P.split[k * (P.S + 1) + s + 1];
  const int T2 = P.t2;

  float2* Hs = reinterpret_cast<float2*>(smem4);
  float2* U2s = Hs + lds_hs_elems(P.t3, P.r1max, P.r2max);
  float* Bs = reinterpret_cast<float*>(U2s + lds_u2_elems(T2, P.r2max));
  float2* red = reinterpret_cast<float2*>(Bs + lds_bs_elems(P.r1max, NWG));

  // this lane's output column (mode-1 fibre) inside the tile
  const int ncol = wn * 32 + (lane & 31);
  const int i2 = i2_0 + ncol % T2;
  const int i3 = i3_0 + ncol / T2;
  const bool colok = (i2 < P.n2) && (i3 < P.n3);
  const int64_t fibre = (int64_t)k * P.nv + (int64_t)P.n1 * (i2 + (int64_t)P.n2 * i3);

  v16f acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[b][i] = 0.f;

  v16f yv[ADJ ? NB : 1];
  if (ADJ) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int m0 = (wm * NB + b) * 32 + 8 * g + 4 * (lane >> 5);
        const int i1 = m0 >> 1;
        float2 v0 = make_float2(0.f, 0.f), v1 = v0;
        if (colok && i1 < P.n1) v0 = P.vec[fibre + i1];
        if (colok && i1 + 1 < P.n1) v1 = P.vec[fibre + i1 + 1];
        yv[ADJ ? b : 0][4 * g + 0] = v0.x;
        yv[ADJ ? b : 0][4 * g + 1] = v0.y;
        yv[ADJ ? b : 0][4 * g + 2] = v1.x;
        yv[ADJ ? b : 0][4 * g + 3] = v1.y;
      }
  }

  const TensorMeta* meta = P.meta + (int64_t)k * P.m;
  const float* Ak = P.apack + P.apack_koff[k];

  for (int j = jb; j < je; ++j) {
    const TensorMeta t = meta[j];
    const int r1 = t.r1, r2 = t.r2, r3 = t.r3;
    const float2 xj = ADJ ? make_float2(1.f, 0.f) : P.vec[j];

    // stage the tile's U2 rows, b-major so a wave reads consecutive i2
    for (int idx = tid; idx < r2 * T2; idx += 256) {
      const int t2 = idx % T2, b = idx / T2;
      const int ii = i2_0 + t2;
      U2s[idx] = (ii < P.n2) ? P.u2t[t.u2_off + (int64_t)ii * r2 + b]
                             : make_float2(0.f, 0.f);
    }
    // A) mode-3 contraction of the core for the tile's i3 values
    const int r12 = r1 * r2;
    for (int idx = tid; idx < P.t3 * r12; idx += 256) {
      const int t3 = idx / r12, rem = idx - t3 * r12;  // rem = a + r1*b
      const int a = rem % r1, b = rem / r1;
      const int ii = i3_0 + t3;
      float2 h = make_float2(0.f, 0.f);
      if (ii < P.n3) {
        const float2* g = P.cores + t.g_off + rem;
        const float2* u3 = P.u3t + t.u3_off + (int64_t)ii * r3;
        for (int c = 0; c < r3; ++c) h = cfma(g[(int64_t)c * r12], u3[c], h);
        if (!ADJ) h = cmul(xj, h);
      }
      Hs[(t3 * r1 + a) * r2 + b] = h;
    }
    __syncthreads();

    // B) mode-2 product per column into the MFMA B tile
    {
      const int n = tid % NWG, ag = tid / NWG;
      const int t2n = n % T2, t3n = n / T2;
      const float2* hrow = Hs + (t3n * r1) * r2;
      for (int a = ag; a < r1; a += AG) {
        float2 v = make_float2(0.f, 0.f);
        for (int b = 0; b < r2; ++b) v = cfma(hrow[a * r2 + b], U2s[b * T2 + t2n], v);
        Bs[(2 * a) * NWG + n] = v.x;
        Bs[(2 * a + 1) * NWG + n] = v.y;
      }
    }
    __syncthreads();

    // adjoint: publish the previous column's partial (its wave sums were
    // written before the barrier above)
    if (ADJ && tid == 0 && j > jb) {
      const float2* rr = red + ((j - 1) & 1) * 4;
      float2 sum = rr[0];
      for (int w = 1; w < 4; ++w) { sum.x += rr[w].x; sum.y += rr[w].y; }
      P.out[((int64_t)k * P.tiles + tile) * P.m + (j - 1)] = sum;
    }

    // C) stacked mode-1 product on MFMA
    if (ADJ) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[b][i] = 0.f;
    }
    const float* Arow = Ak + ((int64_t)t.arow * P.nbt + wm * NB) * 64 + lane;
    const float* Brow = Bs + (lane >> 5) * NWG + wn * 32 + (lane & 31);
    for (int a = 0; a < r1; ++a) {
      const float bv = Brow[2 * a * NWG];
      const float* ap = Arow + (int64_t)a * P.nbt * 64;
#pragma unroll
      for (int b = 0; b < NB; ++b)
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ap[b * 64], bv, acc[b], 0, 0, 0);
    }

    if (ADJ) {
      // conjugated dot product of the Z^{kj} tile with the y tile
      float dr = 0.f, di = 0.f;
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 16; i += 2) {
          const float tr = acc[b][i], ti = acc[b][i + 1];
          const float yr = yv[ADJ ? b : 0][i], yi = yv[ADJ ? b : 0][i + 1];
          dr = fmaf(tr, yr, dr);
          dr = fmaf(ti, yi, dr);
          di = fmaf(tr, yi, di);
          di = fmaf(-ti, yr, di);
        }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        dr += __shfl_xor(dr, off);
        di += __shfl_xor(di, off);
      }
      if (lane == 0) red[(j & 1) * 4 + wave] = make_float2(dr, di);
    }
  }

  if (ADJ) {
    __syncthreads();
    if (tid == 0 && je > jb) {
      const float2* rr = red + ((je - 1) & 1) * 4;
      float2 sum = rr[0];
      for (int w = 1; w < 4; ++w) { sum.x += rr[w].x; sum.y += rr[w].y; }
      P.out[((int64_t)k * P.tiles + tile) * P.m + (je - 1)] = sum;
    }
    return;
  }

  // forward epilogue: rows (2 i1, 2 i1 + 1, 2 i1 + 2, 2 i1 + 3) of a lane's
  // register quad are (Re, Im) of voxels i1 and i1 + 1 of its fibre
  if (!colok) return;
  float2* dst = P.out + (int64_t)s * P.out_stride + fibre;
  const bool vec4 = P.vec4 != 0;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int m0 = (wm * NB + b) * 32 + 8 * g + 4 * (lane >> 5);
      const int i1 = m0 >> 1;
      if (i1 >= P.n1) continue;
      if (vec4 && i1 + 1 < P.n1) {
        *reinterpret_cast<float4*>(dst + i1) =
            make_float4(acc[b][4 * g], acc[b][4 * g + 1], acc[b][4 * g + 2], acc[b][4 * g + 3]);
      } else {
        dst[i1] = make_float2(acc[b][4 * g], acc[b][4 * g + 1]);
        if (i1 + 1 < P.n1) dst[i1 + 1] = make_float2(acc[b][4 * g + 2], acc[b][4 * g + 3]);
      }
    }
}

__global__ void sum_partials_kernel(const float2* __restrict__ ws, int split, int64_t n,
                                    float2* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float2 s = ws[i];
  for (int p = 1; p < split; ++p) {
    const float2 v = ws[(int64_t)p * n + i];
    s.x += v.x;
    s.y += v.y;
  }
  y[i] = s;
}

__global__ void reduce_adjoint_kernel(const float2* __restrict__ partial, int64_t rows,
                                      int64_t m, float2* __restrict__ x) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  double sr = 0.0, si = 0.0;
  for (int64_t r = 0; r < rows; ++r) {
    const float2 v = partial[r * m + j];
    sr += v.x;
    si += v.y;
  }
  x[j] = make_float2((float)sr, (float)si);
}

typedef void (*fused_fn)(KParams);

template <bool ADJ>
static fused_fn pick(int nb, int wn) {
#define TV_CASE(NB)                                        \
  case NB:                                                 \
    return wn == 4 ? fused_f32<NB, 4, ADJ>                 \
                   : (wn == 2 ? fused_f32<NB, 2, ADJ> : fused_f32<NB, 1, ADJ>);
  switch (nb) {
    TV_CASE(1) TV_CASE(2) TV_CASE(3) TV_CASE(4)
    TV_CASE(5) TV_CASE(6) TV_CASE(7) TV_CASE(8)
  }
#undef TV_CASE
  return nullptr;
}

static tv_status launch_fused(const tv_plan_s* p, bool adj, const float2* vec, float2* out,
                              int split, const int32_t* d_split, int64_t out_stride,
                              hipStream_t st) {
  const Tiling& T = p->tiling;
  KParams P;
  P.meta = p->d_meta;
  P.cores = p->d_cores;
  P.u2t = p->d_u2t;
  P.u3t = p->d_u3t;
  P.apack = p->d_apack;
  P.apack_koff = p->d_apack_koff;
  P.split = d_split;
  P.vec = vec;
  P.out = out;
  P.out_stride = out_stride;
  P.m = p->grid.m;
  P.nv = (int64_t)p->grid.n1 * p->grid.n2 * p->grid.n3;
  P.n1 = p->grid.n1;
  P.n2 = p->grid.n2;
  P.n3 = p->grid.n3;
  P.q = p->grid.q;
  P.nbt = T.nbt;
  P.t2 = T.t2;
  P.t3 = T.t3;
  P.tiles2 = T.tiles2;
  P.tiles = T.tiles;
  P.S = split;
  P.nitems = (int64_t)p->grid.q * split * T.tiles;
  P.r1max = p->max_r[0];
  P.r2max = p->max_r[1];
  P.vec4 = (p->grid.n1 % 2 == 0) && ((uintptr_t)out % 16 == 0) && (out_stride % 2 == 0);
  fused_fn fn = adj ? pick<true>(T.nb, T.wn) : pick<false>(T.nb, T.wn);
  if (!fn) return set_error(TV_ERR_NOT_SUPPORTED, "no kernel instance for this tiling");
  const size_t lds = fused_lds_bytes(T.t2, T.t3, P.r1max, P.r2max, T.nwg);
  if (lds > 160 * 1024)
    return set_error(TV_ERR_NOT_SUPPORTED, "ranks too large for the LDS tile");
  hipError_t e = hipFuncSetAttribute((const void*)fn,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_error(e, "hipFuncSetAttribute");
  const int64_t grid = (P.nitems + 7) / 8 * 8;
  hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(256), lds, st, P);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "fused kernel launch");
  return TV_OK;
}

tv_status launch_forward_f32(const tv_plan_s* p, const float2* x, float2* out, int split,
                             const int32_t* d_split, int64_t out_stride, hipStream_t st) {
  return launch_fused(p, false, x, out, split, d_split, out_stride, st);
}

tv_status launch_adjoint_f32(const tv_plan_s* p, const float2* y, float2* partial, int split,
                             const int32_t* d_split, hipStream_t st) {
  return launch_fused(p, true, y, partial, split, d_split, 0, st);
}

tv_status launch_sum_partials(const float2* ws, int split, int64_t n, float2* y,
                              hipStream_t st) {
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)blocks), dim3(256), 0, st, ws, split,
                     n, y);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TV_OK : hip_error(e, "sum_partials launch");
}

tv_status launch_reduce_adjoint(const float2* partial, int q, int64_t tiles, int64_t m,
                                float2* x, hipStream_t st) {
  const int64_t blocks = (m + 255) / 256;
  hipLaunchKernelGGL(reduce_adjoint_kernel, dim3((unsigned)blocks), dim3(256), 0, st, partial,
                     (int64_t)q * tiles, m, x);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TV_OK : hip_error(e, "reduce_adjoint launch");
}

}  // namespace tv
