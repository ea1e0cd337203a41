// Decompress-then-GEMM form of Algorithm 1 (gfx950), for large voxel grids.
//
// Per slab of i3 values, every tensor of every component is decompressed in
// modes 3 and 2 into the stacked operand B_k = [x_1 M_1; ...; x_m M_m]
// (M_j = G_j x2 U2_j x3 U3_j unfolded along mode 1, r1 x (n2 n3)), written
// to HBM, and the mode-1 product of the whole component is then one complex
// GEMM Y^k_(1)[:, slab] = A_k B_k with A_k = [U1_1 ... U1_m] (eq. 6/7,
// Sec. III.B).  Against the fused kernels this spends the HBM traffic of B
// (written once, read once per 256-row tile) to run the dominant product as
// a plain, well-fed MFMA GEMM with long K loops.
//
// Operand layouts (real embedding of the complex product, as in the fused
// kernels; 32x32x2 f32 MFMA: A lane l = A[l%32][l/32], B lane l =
// B[l/32][l%32], accumulator register r of lane l = D[8(r/4) + 4(l/32) +
// r%4][l%32]):
//   A (apack4): per component, k-steps a (stacked rows of A_k, padded to a
//     multiple of 16) grouped by four: float index
//     ((a/4 * nbtp + blk) * 64 + lane) * 4 + a%4 holds
//     A_emb[32 blk + lane%32][(a, lane/32)], A_emb = [[Ar, -Ai], [Ai, Ar]]
//     with output rows interleaved (Re, Im), so a lane reads four k-steps of
//     one row block with one 16-byte load;
//   B: per component, row a (stacked) then 32-column blocks of the slab,
//     each block 64 floats: Re of the 32 columns, then Im.
// The GEMM stages 16 k-steps of A (8 row blocks) and B (4 column blocks)
// through LDS per step, double-buffered, one barrier per step.
#include <algorithm>
#include <cstring>

#include "tv_internal.h"

namespace tv {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int DTG_KC = 16;     // k-steps per LDS stage
constexpr int DTG_MAXQ = 12;

struct DecompParams {
  const TensorMeta* meta;
  const float2* cores;
  const float2* u2t;
  const float2* u3t;
  const float2* x;   // x_j scaling (forward) or null
  const int32_t* drow;  // first stacked row of each tensor [k * m + j]
  float* B;
  int64_t ldb;       // floats per stacked row of B
  int64_t brow[DTG_MAXQ];
  int64_t m;
  int n2, n3, i30, s3, nsub;
  int t3w;           // i3 values per decompression workgroup
  int layout;        // 0: FP32 planar (forward), 1: FP32 accumulator order
                     // (adjoint), 2: BF16 hi/lo operand order (forward, BF16X3)
  int64_t nitems;
};

// Adjoint layout of B: stacked rows in blocks of 16 (a row block of the
// adjoint GEMM's 32x32 accumulator), float offset
// ((R/16 * nbl + n/32) * 4 + g) * 256 + lane * 4 + 2 e + (Re, Im) for row R
// with R%16 = 4 g + 2 h + e and lane = 32 h + n%32: a lane of the GEMM's
// epilogue finds the values matching its accumulator registers 4g..4g+3 in
// one 16-byte load.
__host__ __device__ inline int64_t adj_b_index(int64_t R, int64_t n, int64_t nbl) {
  const int al = (int)(R & 15);
  const int g = al >> 2, h = (al >> 1) & 1, e = al & 1;
  return (((R >> 4) * nbl + (n >> 5)) * 4 + g) * 256 + (32 * h + (n & 31)) * 4 + 2 * e;
}

// BF16X3 layout of B: stacked rows in chunks of 8, per (chunk, 32-column
// block) the hi then the lo halves as 64 lanes x 8 bf16, lane 32 h + n%32
// holding rows 8c + 4h + 0..3 as (Re, Im) pairs: the B operand of
// v_mfma_f32_32x32x16_bf16 for eight k-steps.  Index of the 32-bit (Re, Im)
// word of row R, column n, hi half (the lo half is 256 words further).
__host__ __device__ inline int64_t bf_b_index(int64_t R, int64_t n, int64_t nbl) {
  const int rl = (int)(R & 7);
  return (((R >> 3) * nbl + (n >> 5)) * 2) * 256 + (32 * (rl >> 2) + (n & 31)) * 4 + (rl & 3);
}

__host__ __device__ inline uint32_t bf16_rne(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__host__ __device__ inline float bf16_float(uint32_t h) {
  const uint32_t u = h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// B rows of one tensor for t3w values of i3: H3[a][i3][b] = x_j sum_c
// G[a,b,c] U3[i3,c] in LDS, then B[a][(i2, i3)] = sum_b H3[a][i3][b] U2[i2,b]
// with each thread on one i2 and its U2 row in registers (R2MAX >= r2).
template <int R2MAX>
__global__ __launch_bounds__(256) void dtg_decomp_kernel(DecompParams P) {
  extern __shared__ float2 h3[];
  const int64_t item = blockIdx.x;
  if (item >= P.nitems) return;
  const int64_t kt = item / P.nsub;           // k * m + j
  const int sub = (int)(item - kt * P.nsub);
  const int k = (int)(kt / P.m);
  const int64_t j = kt - (int64_t)k * P.m;
  const TensorMeta t = P.meta[kt];
  const int r1 = t.r1, r2 = t.r2, r3 = t.r3;
  const int T3 = P.t3w;
  const int i3a = P.i30 + sub * T3;
  const int cnt = min(T3, P.i30 + P.s3 - i3a);
  const float2 xj = P.x ? P.x[j] : make_float2(1.f, 0.f);
  const float2* G = P.cores + t.g_off;
  const float2* U3 = P.u3t + t.u3_off;
  const int nh = r1 * cnt * r2;
  for (int e = threadIdx.x; e < nh; e += 256) {
    const int b = e % r2;
    const int rest = e / r2;
    const int i3l = rest % cnt;
    const int a = rest / cnt;
    float2 s = make_float2(0.f, 0.f);
    const float2* g = G + a + (int64_t)r1 * b;
    const float2* u = U3 + (int64_t)(i3a + i3l) * r3;
    for (int c = 0; c < r3; ++c) {
      const float2 gv = g[(int64_t)r1 * r2 * c], uv = u[c];
      s.x = fmaf(gv.x, uv.x, fmaf(-gv.y, uv.y, s.x));
      s.y = fmaf(gv.x, uv.y, fmaf(gv.y, uv.x, s.y));
    }
    h3[(a * T3 + i3l) * r2 + b] = cmul(xj, s);
  }
  __syncthreads();
  const int64_t row0 = P.brow[k] + P.drow[kt];
  float* Bk = P.B + row0 * P.ldb;
  const int64_t nbl = P.ldb / 64;
  for (int i2 = threadIdx.x; i2 < P.n2; i2 += 256) {
    float2 u[R2MAX];
    const float2* u2 = P.u2t + t.u2_off + (int64_t)i2 * r2;
#pragma unroll
    for (int b = 0; b < R2MAX; ++b) u[b] = b < r2 ? u2[b] : make_float2(0.f, 0.f);
    for (int a = 0; a < r1; ++a) {
      float* row = Bk + (int64_t)a * P.ldb;
      for (int i3l = 0; i3l < cnt; ++i3l) {
        const float2* hv = h3 + (a * T3 + i3l) * r2;
        float sr = 0.f, si = 0.f;
#pragma unroll
        for (int b = 0; b < R2MAX; ++b) {
          if (b < r2) {
            const float2 h = hv[b];
            sr = fmaf(h.x, u[b].x, fmaf(-h.y, u[b].y, sr));
            si = fmaf(h.x, u[b].y, fmaf(h.y, u[b].x, si));
          }
        }
        const int64_t n = i2 + (int64_t)P.n2 * (i3a + i3l - P.i30);
        if (P.layout == 1) {
          *(float2*)(P.B + adj_b_index(row0 + a, n, nbl)) = make_float2(sr, si);
        } else if (P.layout == 2) {
          const uint32_t hr = bf16_rne(sr), hi_ = bf16_rne(si);
          const uint32_t lr = bf16_rne(sr - bf16_float(hr)), li = bf16_rne(si - bf16_float(hi_));
          uint32_t* dst = (uint32_t*)P.B + bf_b_index(row0 + a, n, nbl);
          dst[0] = hr | (hi_ << 16);
          dst[256] = lr | (li << 16);
        } else {
          float* dst = row + (n >> 5) * 64 + (n & 31);
          dst[0] = sr;
          dst[32] = si;
        }
      }
    }
  }
}

// zero rows [from_k, to_k) of B for every component k (k-steps past the
// stacked rows: A is zero there and B must be finite)
struct ZeroParams {
  float* B;
  int64_t ldb;
  int64_t from[DTG_MAXQ], to[DTG_MAXQ];
  int q;
};
__global__ void dtg_zero_rows_kernel(ZeroParams Z) {
  for (int k = 0; k < Z.q; ++k) {
    const int64_t n = (Z.to[k] - Z.from[k]) * Z.ldb;
    float* p = Z.B + Z.from[k] * Z.ldb;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
      p[i] = 0.f;
  }
}

struct GemmParams {
  const float* apack4;
  const float* B;
  float2* out;
  int64_t out_stride;      // per split (partial buffers)
  int64_t a4off[DTG_MAXQ];
  int64_t brow[DTG_MAXQ];
  int kst[DTG_MAXQ];       // LDS stages (16 k-steps) per component
  int q, nbtp, mtiles, ntiles, S;
  int64_t nitems;
  int64_t ldb;
  int64_t nv;
  int n1;
  int64_t col0, ncols;     // first column of the slab in Y^k_(1), its width
  int vec4;
};

// One workgroup: MT = 2 MBW row blocks x NT = 64 NBW columns of Y^k_(1)
// over a range of k-steps; 4 waves in 2 x 2, each MBW x NBW 32x32 blocks.
template <int MBW, int NBW>
__global__ __launch_bounds__(256) void dtg_gemm_kernel(GemmParams P) {
  constexpr int MT = 2 * MBW, NBT = 2 * NBW;
  constexpr int A_ST = 4 * MT * 64 * 4;      // floats per A stage
  constexpr int B_ST = DTG_KC * NBT * 64;    // floats per B stage
  extern __shared__ float lds[];
  // consecutive logical tiles on one XCD (workgroups go round-robin over 8)
  const int64_t nwg = gridDim.x;
  const int64_t L = (int64_t)(blockIdx.x % 8) * (nwg / 8) + blockIdx.x / 8;
  if (L >= P.nitems) return;
  const int mt = (int)(L % P.mtiles);
  int64_t rest = L / P.mtiles;
  const int nt = (int)(rest % P.ntiles);
  rest /= P.ntiles;
  const int k = (int)(rest % P.q);
  const int s = (int)(rest / P.q);
  const int nst = P.kst[k];
  const int st0 = (int)((int64_t)nst * s / P.S), st1 = (int)((int64_t)nst * (s + 1) / P.S);

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const float* Ag = P.apack4 + P.a4off[k];
  const float* Bg = P.B + P.brow[k] * P.ldb;

  v4f ra[MT], rb[NBT];
  auto gload = [&](int st) {
#pragma unroll
    for (int c = 0; c < MT; ++c) {
      const int u = c * 256 + tid;
      const int kg = u / (MT * 64), rem = u % (MT * 64);
      ra[c] = *(const v4f*)(Ag + ((((int64_t)st * 4 + kg) * P.nbtp + mt * MT + rem / 64) * 64 +
                                  rem % 64) * 4);
    }
#pragma unroll
    for (int c = 0; c < NBT; ++c) {
      const int u = c * 256 + tid;
      const int kk = u / (NBT * 16), rem = u % (NBT * 16);
      rb[c] = *(const v4f*)(Bg + ((int64_t)st * DTG_KC + kk) * P.ldb +
                            ((int64_t)nt * NBT + rem / 16) * 64 + (rem % 16) * 4);
    }
  };
  auto lstore = [&](int buf) {
    float* As = lds + buf * (A_ST + B_ST);
    float* Bs = As + A_ST;
#pragma unroll
    for (int c = 0; c < MT; ++c) *(v4f*)(As + (c * 256 + tid) * 4) = ra[c];
#pragma unroll
    for (int c = 0; c < NBT; ++c) *(v4f*)(Bs + (c * 256 + tid) * 4) = rb[c];
  };

  v16f acc[MBW][NBW];
#pragma unroll
  for (int i = 0; i < MBW; ++i)
#pragma unroll
    for (int jn = 0; jn < NBW; ++jn) acc[i][jn] = v16f{0.f};

  if (st0 < st1) {
    gload(st0);
    lstore(0);
  }
  __syncthreads();
  for (int st = st0; st < st1; ++st) {
    const int buf = (st - st0) & 1;
    if (st + 1 < st1) gload(st + 1);
    const float* As = lds + buf * (A_ST + B_ST);
    const float* Bs = As + A_ST;
#pragma unroll
    for (int kg = 0; kg < 4; ++kg) {
      v4f a[MBW];
#pragma unroll
      for (int i = 0; i < MBW; ++i)
        a[i] = *(const v4f*)(As + ((kg * MT + wm * MBW + i) * 64 + lane) * 4);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        float b[NBW];
#pragma unroll
        for (int jn = 0; jn < NBW; ++jn)
          b[jn] = Bs[((kg * 4 + kk) * NBT + wn * NBW + jn) * 64 + lane];
#pragma unroll
        for (int i = 0; i < MBW; ++i)
#pragma unroll
          for (int jn = 0; jn < NBW; ++jn)
            acc[i][jn] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][kk], b[jn], acc[i][jn], 0, 0, 0);
      }
    }
    if (st + 1 < st1) lstore(buf ^ 1);
    __syncthreads();
  }

  // rows (i1, Re/Im) pairs: registers 4g..4g+3 are (Re, Im) of i1, i1 + 1
  float2* out = P.out + (int64_t)s * P.out_stride + (int64_t)k * P.nv;
#pragma unroll
  for (int jn = 0; jn < NBW; ++jn) {
    const int64_t n = ((int64_t)nt * NBT + wn * NBW + jn) * 32 + (lane & 31);
    if (n >= P.ncols) continue;
    float2* col = out + (int64_t)P.n1 * (P.col0 + n);
#pragma unroll
    for (int i = 0; i < MBW; ++i) {
      const int blk = mt * MT + wm * MBW + i;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int i1 = blk * 16 + 4 * g + 2 * (lane >> 5);
        const v16f& d = acc[i][jn];
        if (i1 + 1 < P.n1) {
          if (P.vec4) {
            *(v4f*)(col + i1) = v4f{d[4 * g], d[4 * g + 1], d[4 * g + 2], d[4 * g + 3]};
          } else {
            col[i1] = make_float2(d[4 * g], d[4 * g + 1]);
            col[i1 + 1] = make_float2(d[4 * g + 2], d[4 * g + 3]);
          }
        } else if (i1 < P.n1) {
          col[i1] = make_float2(d[4 * g], d[4 * g + 1]);
        }
      }
    }
  }
}

// zero rows [from_k, to_k) of the BF16 layout (both halves, every column)
__global__ void dtg_zero_rows_bf_kernel(ZeroParams Z) {
  const int64_t nbl = Z.ldb / 64;
  for (int k = 0; k < Z.q; ++k) {
    const int64_t n = (Z.to[k] - Z.from[k]) * nbl * 32;
    uint32_t* B = (uint32_t*)Z.B;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
      const int64_t R = Z.from[k] + i / (nbl * 32), c = i % (nbl * 32);
      const int64_t w = bf_b_index(R, c, nbl);
      B[w] = 0u;
      B[w + 256] = 0u;
    }
  }
}

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
__device__ __forceinline__ v8bf as_v8bf(uint4 v) { return __builtin_bit_cast(v8bf, v); }

// The stacked mode-1 GEMM with BF16 hi/lo operands: per 16 k-steps (two
// chunks of 8), Y += Ah Bh + Ah Bl + Al Bh on v_mfma_f32_32x32x16_bf16 (the
// lo x lo term is dropped), FP32 accumulation.  Tiles, waves, XCD grouping
// and epilogue as dtg_gemm_kernel; A (abf) per component as
// ((chunk * nbtp + blk) * 2 + hl) * 64 + lane uint4, lane l holding
// A_emb[32 blk + l%32][(8 chunk + 4 (l/32) + e/2, e%2)], e < 8.
template <int MBW, int NBW, int CPS>
__global__ __launch_bounds__(256, CPS == 1 ? 2 : 1) void dtg_gemm_bf_kernel(GemmParams P) {
  // CPS chunks of 8 k-steps per LDS stage; with one chunk per stage two
  // workgroups share a CU, which hides the loads behind the other's MFMAs
  constexpr int MT = 2 * MBW, NBT = 2 * NBW;
  constexpr int A_ST = CPS * MT * 128;      // uint4 per A stage
  constexpr int B_ST = CPS * NBT * 128;     // uint4 per B stage
  extern __shared__ uint4 ldsq[];
  const int64_t nwg = gridDim.x;
  const int64_t L = (int64_t)(blockIdx.x % 8) * (nwg / 8) + blockIdx.x / 8;
  if (L >= P.nitems) return;
  const int mt = (int)(L % P.mtiles);
  int64_t rest = L / P.mtiles;
  const int nt = (int)(rest % P.ntiles);
  rest /= P.ntiles;
  const int k = (int)(rest % P.q);
  const int s = (int)(rest / P.q);
  const int nst = P.kst[k] * (2 / CPS);
  const int st0 = (int)((int64_t)nst * s / P.S), st1 = (int)((int64_t)nst * (s + 1) / P.S);

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const uint4* Ag = (const uint4*)P.apack4 + P.a4off[k];
  const int64_t nbl = P.ldb / 64;
  const uint4* Bg = (const uint4*)P.B + (P.brow[k] >> 3) * nbl * 128;

  constexpr int NA = CPS * MT / 2, NB = CPS * NBT / 2;   // uint4 loads per thread
  uint4 ra[NA], rb[NB];
  auto gload = [&](int st) {
#pragma unroll
    for (int c = 0; c < NA; ++c) {
      const int u = c * 256 + tid;
      const int ch = u / (MT * 128), rem = u % (MT * 128);
      ra[c] = Ag[(((int64_t)st * CPS + ch) * P.nbtp + mt * MT + rem / 128) * 128 + rem % 128];
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const int u = c * 256 + tid;
      const int ch = u / (NBT * 128), rem = u % (NBT * 128);
      rb[c] = Bg[(((int64_t)st * CPS + ch) * nbl + (int64_t)nt * NBT + rem / 128) * 128 +
                 rem % 128];
    }
  };
  auto lstore = [&](int buf) {
    uint4* As = ldsq + buf * (A_ST + B_ST);
    uint4* Bs = As + A_ST;
#pragma unroll
    for (int c = 0; c < NA; ++c) As[c * 256 + tid] = ra[c];
#pragma unroll
    for (int c = 0; c < NB; ++c) Bs[c * 256 + tid] = rb[c];
  };

  v16f acc[MBW][NBW];
#pragma unroll
  for (int i = 0; i < MBW; ++i)
#pragma unroll
    for (int jn = 0; jn < NBW; ++jn) acc[i][jn] = v16f{0.f};

  if (st0 < st1) {
    gload(st0);
    lstore(0);
  }
  __syncthreads();
  for (int st = st0; st < st1; ++st) {
    const int buf = (st - st0) & 1;
    if (st + 1 < st1) gload(st + 1);
    const uint4* As = ldsq + buf * (A_ST + B_ST);
    const uint4* Bs = As + A_ST;
#pragma unroll
    for (int ch = 0; ch < CPS; ++ch) {
      v8bf ah[MBW], al[MBW], bh[NBW], bl[NBW];
#pragma unroll
      for (int i = 0; i < MBW; ++i) {
        const int b = ch * MT + wm * MBW + i;
        ah[i] = as_v8bf(As[(b * 2) * 64 + lane]);
        al[i] = as_v8bf(As[(b * 2 + 1) * 64 + lane]);
      }
#pragma unroll
      for (int jn = 0; jn < NBW; ++jn) {
        const int b = ch * NBT + wn * NBW + jn;
        bh[jn] = as_v8bf(Bs[(b * 2) * 64 + lane]);
        bl[jn] = as_v8bf(Bs[(b * 2 + 1) * 64 + lane]);
      }
#pragma unroll
      for (int i = 0; i < MBW; ++i)
#pragma unroll
        for (int jn = 0; jn < NBW; ++jn) {
          acc[i][jn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[jn], acc[i][jn], 0, 0, 0);
          acc[i][jn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[jn], acc[i][jn], 0, 0, 0);
          acc[i][jn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[jn], acc[i][jn], 0, 0, 0);
        }
    }
    if (st + 1 < st1) lstore(buf ^ 1);
    __syncthreads();
  }

  float2* out = P.out + (int64_t)s * P.out_stride + (int64_t)k * P.nv;
#pragma unroll
  for (int jn = 0; jn < NBW; ++jn) {
    const int64_t n = ((int64_t)nt * NBT + wn * NBW + jn) * 32 + (lane & 31);
    if (n >= P.ncols) continue;
    float2* col = out + (int64_t)P.n1 * (P.col0 + n);
#pragma unroll
    for (int i = 0; i < MBW; ++i) {
      const int blk = mt * MT + wm * MBW + i;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int i1 = blk * 16 + 4 * g + 2 * (lane >> 5);
        const v16f& d = acc[i][jn];
        if (i1 + 1 < P.n1) {
          if (P.vec4) {
            *(v4f*)(col + i1) = v4f{d[4 * g], d[4 * g + 1], d[4 * g + 2], d[4 * g + 3]};
          } else {
            col[i1] = make_float2(d[4 * g], d[4 * g + 1]);
            col[i1 + 1] = make_float2(d[4 * g + 2], d[4 * g + 3]);
          }
        } else if (i1 < P.n1) {
          col[i1] = make_float2(d[4 * g], d[4 * g + 1]);
        }
      }
    }
  }
}

typedef void (*gemm_fn)(GemmParams);

// ---- adjoint: W_k = A_k^* Y^k_(1) on MFMA, then the conjugated dot with the
// unscaled decompression B_k (Algorithm 2's inner products at the mode-1
// output), summed per stacked row -------------------------------------------
//
// A^* operand (apackh): per component, M = (a, s) rows (a stacked row of A_k,
// s = Re/Im), K = (i1, t) (t = Re/Im of y); float index
// ((i1/4 * mbh + blk) * 64 + lane) * 4 + i1%4 holds Ah_emb[32 blk + lane%32]
// [(i1, lane/32)], Ah_emb[(a,s)][(i1,t)] = Ur if s == t, Ui if s = 0, t = 1,
// -Ui if s = 1, t = 0 (U = U1[i1][a]): rows (a, Re), (a, Im) of U1^* y.
struct AdjParams {
  const float* apackh;
  const float* B;
  const float2* y;
  float2* partial;          // [chunk][prow] complex: sum over the chunk's columns
  int64_t ahoff[DTG_MAXQ];
  int64_t brow[DTG_MAXQ];
  int64_t rk[DTG_MAXQ];     // stacked rows of A_k
  int mbh[DTG_MAXQ];        // 32-row blocks of the A^* operand per component
  int mtb[DTG_MAXQ + 1];    // prefix sum of row tiles over components
  int q, kst, ntiles, ntw, nchunks;
  int order;                // 0: row tiles fastest, 1: column chunks fastest
  int64_t prow, nbl, nv;
  int n1;
  int64_t col0, ncols;
  int vec;                  // n1 even: y read two complex at a time
  int64_t nitems;
};

constexpr int ADJ_MBW = 4, ADJ_NBW = 2;
constexpr int ADJ_MT = 2 * ADJ_MBW, ADJ_NBT = 2 * ADJ_NBW;
constexpr int ADJ_YS = ADJ_NBT * 64 + 4;     // LDS row stride of the y stage (floats)
constexpr int ADJ_A_ST = 4 * ADJ_MT * 64 * 4;
constexpr int ADJ_Y_ST = DTG_KC * ADJ_YS;

__global__ __launch_bounds__(256) void dtg_adjoint_kernel(AdjParams P) {
  extern __shared__ float lds[];
  const int64_t nwg = gridDim.x;
  const int64_t L = (int64_t)(blockIdx.x % 8) * (nwg / 8) + blockIdx.x / 8;
  if (L >= P.nitems) return;
  const int mtot = P.mtb[P.q];
  // consecutive workgroups on an XCD share either their y columns (row tiles
  // fastest) or their U1^* rows (column chunks fastest)
  const int chunk = P.order ? (int)(L % P.nchunks) : (int)(L / mtot);
  const int mtg = P.order ? (int)(L / P.nchunks) : (int)(L - (int64_t)chunk * mtot);
  int k = 0;
  while (mtg >= P.mtb[k + 1]) ++k;
  const int mt = mtg - P.mtb[k];
  const int nt0 = chunk * P.ntw, nt1 = min(P.ntiles, nt0 + P.ntw);
  const int total = (nt1 - nt0) * P.kst;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1, h = lane >> 5;
  const float* Ag = P.apackh + P.ahoff[k];
  const float2* yk = P.y + (int64_t)k * P.nv;
  const int mbh = P.mbh[k];

  v4f ra[ADJ_MT], ry[4];
  auto gload = [&](int g) {
    const int nt = nt0 + g / P.kst, st = g % P.kst;
#pragma unroll
    for (int c = 0; c < ADJ_MT; ++c) {
      const int u = c * 256 + tid;
      const int kg = u / (ADJ_MT * 64), rem = u % (ADJ_MT * 64);
      ra[c] = *(const v4f*)(Ag + ((((int64_t)st * 4 + kg) * mbh + mt * ADJ_MT + rem / 64) * 64 +
                                  rem % 64) * 4);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int u = c * 256 + tid;
      const int col = u / 8, i1 = st * DTG_KC + 2 * (u % 8);
      const int64_t n = (int64_t)nt * (ADJ_NBT * 32) + col;
      v4f v = v4f{0.f, 0.f, 0.f, 0.f};
      if (n < P.ncols) {
        const float2* src = yk + (int64_t)P.n1 * (P.col0 + n) + i1;
        if (P.vec) {
          if (i1 < P.n1) v = *(const v4f*)src;
        } else {
          if (i1 < P.n1) { const float2 a = src[0]; v[0] = a.x; v[1] = a.y; }
          if (i1 + 1 < P.n1) { const float2 b = src[1]; v[2] = b.x; v[3] = b.y; }
        }
      }
      ry[c] = v;
    }
  };
  auto lstore = [&](int buf) {
    float* As = lds + buf * (ADJ_A_ST + ADJ_Y_ST);
    float* Ys = As + ADJ_A_ST;
#pragma unroll
    for (int c = 0; c < ADJ_MT; ++c) *(v4f*)(As + (c * 256 + tid) * 4) = ra[c];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int u = c * 256 + tid;
      const int col = u / 8, r = 2 * (u % 8);
      float* d = Ys + r * ADJ_YS + (col / 32) * 64 + (col & 31);
      d[0] = ry[c][0];
      d[32] = ry[c][1];
      d[ADJ_YS] = ry[c][2];
      d[ADJ_YS + 32] = ry[c][3];
    }
  };

  v16f acc[ADJ_MBW][ADJ_NBW];
  float dr[ADJ_MBW][8], di[ADJ_MBW][8];   // per lane: rows 4g + 2h + e of each block
#pragma unroll
  for (int i = 0; i < ADJ_MBW; ++i) {
#pragma unroll
    for (int jn = 0; jn < ADJ_NBW; ++jn) acc[i][jn] = v16f{0.f};
#pragma unroll
    for (int e = 0; e < 8; ++e) dr[i][e] = di[i][e] = 0.f;
  }

  if (total > 0) {
    gload(0);
    lstore(0);
  }
  __syncthreads();
  for (int g = 0; g < total; ++g) {
    const int buf = g & 1;
    if (g + 1 < total) gload(g + 1);
    const float* As = lds + buf * (ADJ_A_ST + ADJ_Y_ST);
    const float* Ys = As + ADJ_A_ST;
#pragma unroll
    for (int kg = 0; kg < 4; ++kg) {
      v4f a[ADJ_MBW];
#pragma unroll
      for (int i = 0; i < ADJ_MBW; ++i)
        a[i] = *(const v4f*)(As + ((kg * ADJ_MT + wm * ADJ_MBW + i) * 64 + lane) * 4);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        float b[ADJ_NBW];
#pragma unroll
        for (int jn = 0; jn < ADJ_NBW; ++jn)
          b[jn] = Ys[(kg * 4 + kk) * ADJ_YS + (wn * ADJ_NBW + jn) * 64 + lane];
#pragma unroll
        for (int i = 0; i < ADJ_MBW; ++i)
#pragma unroll
          for (int jn = 0; jn < ADJ_NBW; ++jn)
            acc[i][jn] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][kk], b[jn], acc[i][jn], 0, 0, 0);
      }
    }
    if (g % P.kst == P.kst - 1) {
      // the tile's W is complete: conjugated dot with B over its columns
      const int nt = nt0 + g / P.kst;
#pragma unroll
      for (int jn = 0; jn < ADJ_NBW; ++jn) {
        const int nblk = nt * ADJ_NBT + wn * ADJ_NBW + jn;
        const int64_t n = (int64_t)nblk * 32 + (lane & 31);
        const bool okn = n < P.ncols;
#pragma unroll
        for (int i = 0; i < ADJ_MBW; ++i) {
          const int64_t blk = mt * ADJ_MT + wm * ADJ_MBW + i;
          const int64_t a0 = blk * 16 + 2 * h;
          const float* bp = P.B + ((((P.brow[k] >> 4) + blk) * P.nbl + nblk) * 4) * 256 + lane * 4;
#pragma unroll
          for (int g4 = 0; g4 < 4; ++g4) {
            const int64_t a = a0 + 4 * g4;
            if (okn && a < P.rk[k]) {
              const v4f bv = *(const v4f*)(bp + g4 * 256);
#pragma unroll
              for (int e2 = 0; e2 < 2; ++e2) {
                const int e = 2 * g4 + e2;
                const float br = bv[2 * e2], bi = bv[2 * e2 + 1];
                const float wr = acc[i][jn][2 * e], wi = acc[i][jn][2 * e + 1];
                dr[i][e] = fmaf(br, wr, fmaf(bi, wi, dr[i][e]));
                di[i][e] = fmaf(br, wi, fmaf(-bi, wr, di[i][e]));
              }
            }
          }
        }
        // next tile starts from zero
#pragma unroll
        for (int i = 0; i < ADJ_MBW; ++i) acc[i][jn] = v16f{0.f};
      }
    }
    if (g + 1 < total) lstore(buf ^ 1);
    __syncthreads();
  }

  // sum over the 32 columns of each half-wave, then over the two waves along N
#pragma unroll
  for (int i = 0; i < ADJ_MBW; ++i)
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
      for (int off = 16; off >= 1; off >>= 1) {
        dr[i][e] += __shfl_xor(dr[i][e], off, 64);
        di[i][e] += __shfl_xor(di[i][e], off, 64);
      }
  float2* red = (float2*)lds;   // [wn][rows of the tile: 128 a]
  if ((lane & 31) == 0) {
#pragma unroll
    for (int i = 0; i < ADJ_MBW; ++i)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int al = (wm * ADJ_MBW + i) * 16 + 2 * h + 4 * (e / 2) + (e & 1);
        red[wn * (ADJ_MT * 16) + al] = make_float2(dr[i][e], di[i][e]);
      }
  }
  __syncthreads();
  if (tid < ADJ_MT * 16) {
    const int64_t a = (int64_t)mt * ADJ_MT * 16 + tid;
    if (a < P.rk[k]) {
      const float2 u = red[tid], v = red[ADJ_MT * 16 + tid];
      P.partial[(int64_t)chunk * P.prow + P.brow[k] + a] = make_float2(u.x + v.x, u.y + v.y);
    }
  }
}

// x'_j = sum over components, chunks and the tensor's stacked rows of the
// partial dots, in a fixed order (FP64)
struct AdjReduceParams {
  const TensorMeta* meta;
  const int32_t* drow;
  const float2* partial;
  float2* x;
  int64_t brow[DTG_MAXQ];
  int64_t prow, m;
  int q, nchunks;
};
__global__ void dtg_adjoint_reduce_kernel(AdjReduceParams P) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= P.m) return;
  double sr = 0.0, si = 0.0;
  for (int k = 0; k < P.q; ++k) {
    const TensorMeta t = P.meta[(int64_t)k * P.m + j];
    for (int c = 0; c < P.nchunks; ++c) {
      const float2* src = P.partial + (int64_t)c * P.prow + P.brow[k] + P.drow[(int64_t)k * P.m + j];
      for (int a = 0; a < t.r1; ++a) {
        sr += src[a].x;
        si += src[a].y;
      }
    }
  }
  P.x[j] = make_float2((float)sr, (float)si);
}

typedef void (*decomp_fn)(DecompParams);

decomp_fn decomp_pick(int r2max) {
  if (r2max <= 16) return dtg_decomp_kernel<16>;
  if (r2max <= 32) return dtg_decomp_kernel<32>;
  return dtg_decomp_kernel<64>;
}

// BF16X3 GEMM instances: nbw 2 and 4 with two chunks per stage (one
// workgroup per CU), nbw 1 stands for 2 column blocks per wave with one chunk
// per stage (two workgroups per CU)
gemm_fn gemm_pick_bf(int mbw, int nbw) {
  if (mbw == 4 && nbw == 1) return dtg_gemm_bf_kernel<4, 2, 1>;
  if (mbw == 4 && nbw == 2) return dtg_gemm_bf_kernel<4, 2, 2>;
  if (mbw == 4 && nbw == 4) return dtg_gemm_bf_kernel<4, 4, 2>;
  if (mbw == 2 && nbw == 1) return dtg_gemm_bf_kernel<2, 2, 1>;
  if (mbw == 2 && nbw == 2) return dtg_gemm_bf_kernel<2, 2, 2>;
  if (mbw == 2 && nbw == 4) return dtg_gemm_bf_kernel<2, 4, 2>;
  return nullptr;
}

gemm_fn gemm_pick(int mbw, int nbw) {
  if (mbw == 4 && nbw == 2) return dtg_gemm_kernel<4, 2>;
  if (mbw == 4 && nbw == 4) return dtg_gemm_kernel<4, 4>;
  if (mbw == 2 && nbw == 2) return dtg_gemm_kernel<2, 2>;
  if (mbw == 2 && nbw == 4) return dtg_gemm_kernel<2, 4>;
  return nullptr;
}

}  // namespace

// ---- host side -----------------------------------------------------------

// row blocks per workgroup tile of the GEMM for a plan (8 for n1 > 64, else 4)
int dtg_mt(const tv_plan_s* p) { return p->nbt_pack > 4 ? 8 : 4; }

size_t dtg_gemm_lds(int mbw, int nbw) {
  return 2 * sizeof(float) * (size_t)(4 * 2 * mbw * 64 * 4 + DTG_KC * 2 * nbw * 64);
}

// Pack A_k for the forward GEMM and A_k^* for the adjoint's (called at plan
// finalisation, FP32 plans).
tv_status dtg_pack(tv_plan_s* p, const std::vector<TensorMeta>& meta) {
  const tv_grid& g = p->grid;
  if (g.q > DTG_MAXQ) return TV_OK;
  const int MT = dtg_mt(p);
  const int nbtp = (p->nbt_pack + MT - 1) / MT * MT;
  p->dtg_nbtp = nbtp;
  p->dtg_rpad.assign(g.q, 0);
  p->dtg_a4off.assign(g.q + 1, 0);
  for (int k = 0; k < g.q; ++k) {
    p->dtg_rpad[k] = (p->sum_r1_k[k] + DTG_KC - 1) / DTG_KC * DTG_KC;
    p->dtg_a4off[k + 1] = p->dtg_a4off[k] + p->dtg_rpad[k] * nbtp * 64;
  }
  // stacked row of each tensor's first U1 column in A_k (the fused BF16X3
  // kernels pad tensors to 8-row chunks in their own packing; this one does not)
  std::vector<int32_t> drow((size_t)g.q * g.m);
  std::vector<std::vector<int64_t>> owner(g.q);
  for (int k = 0; k < g.q; ++k) {
    owner[k].assign(p->dtg_rpad[k], 0);
    int64_t r = 0;
    for (int64_t j = 0; j < g.m; ++j) {
      const TensorMeta& M = meta[(size_t)k * g.m + j];
      drow[(size_t)k * g.m + j] = (int32_t)r;
      for (int a = 0; a < M.r1; ++a) owner[k][r + a] = j;
      r += M.r1;
    }
  }
  // value of the real-embedded stacked U1 of component k at real row mrow
  // and k-step (stacked row a, part pp), from the tensor owning a
  auto emb = [&](const std::vector<int64_t>& own, int k, int64_t a, int mrow, int pp) -> double {
    const int i1 = mrow >> 1, s = mrow & 1;
    if (i1 >= g.n1 || a >= p->sum_r1_k[k]) return 0.0;
    const int64_t j = own[a];
    const int64_t t = k + (int64_t)g.q * j;
    const int al = (int)(a - drow[(size_t)k * g.m + j]);
    const size_t src = p->u1_off[t] + i1 + (size_t)g.n1 * al;
    const double ar = p->u1[2 * src], ai = p->u1[2 * src + 1];
    return s == pp ? ar : (s == 0 ? -ai : ai);
  };
  if (p->precision == TV_PREC_BF16X3) {
    // hi/lo bf16 in the A-operand order of v_mfma_f32_32x32x16_bf16
    p->dtg_abfoff.assign(g.q + 1, 0);
    for (int k = 0; k < g.q; ++k)
      p->dtg_abfoff[k + 1] = p->dtg_abfoff[k] + p->dtg_rpad[k] / 8 * nbtp * 128;
    std::vector<uint4> abf((size_t)p->dtg_abfoff[g.q], make_uint4(0, 0, 0, 0));
    for (int k = 0; k < g.q; ++k)
      for (int64_t c = 0; c < p->dtg_rpad[k] / 8; ++c)
        for (int blk = 0; blk < nbtp; ++blk)
          for (int lane = 0; lane < 64; ++lane) {
            uint32_t hi[8], lo[8];
            for (int e = 0; e < 8; ++e) {
              const int64_t a = 8 * c + 4 * (lane >> 5) + e / 2;
              const float v = (float)emb(owner[k], k, a, 32 * blk + (lane & 31), e % 2);
              hi[e] = bf16_rne(v);
              lo[e] = bf16_rne(v - bf16_float(hi[e]));
            }
            uint4* dst = &abf[p->dtg_abfoff[k] + ((c * nbtp + blk) * 2) * 64 + lane];
            dst[0] = make_uint4(hi[0] | (hi[1] << 16), hi[2] | (hi[3] << 16),
                                hi[4] | (hi[5] << 16), hi[6] | (hi[7] << 16));
            dst[64] = make_uint4(lo[0] | (lo[1] << 16), lo[2] | (lo[3] << 16),
                                 lo[4] | (lo[5] << 16), lo[6] | (lo[7] << 16));
          }
    p->hp.abf = std::move(abf);
  } else {
    std::vector<float> a4((size_t)p->dtg_a4off[g.q], 0.f);
    for (int k = 0; k < g.q; ++k)
      for (int64_t a = 0; a < p->sum_r1_k[k]; ++a) {
        float* base = &a4[p->dtg_a4off[k] + (a / 4) * nbtp * 256 + a % 4];
        for (int blk = 0; blk < nbtp; ++blk)
          for (int lane = 0; lane < 64; ++lane)
            base[((int64_t)blk * 64 + lane) * 4] =
                (float)emb(owner[k], k, a, 32 * blk + (lane & 31), lane >> 5);
      }
    p->hp.a4 = std::move(a4);
  }
  int64_t rp = 0;
  for (int k = 0; k < g.q; ++k) rp += p->dtg_rpad[k];
  p->dtg_rows = rp;

  // A^* operand of the adjoint: 256-row tiles (128 stacked rows), K = n1
  // padded to 16 voxel rows
  const int n1p = (g.n1 + DTG_KC - 1) / DTG_KC * DTG_KC;
  p->dtg_mbh.assign(g.q, 0);
  p->dtg_ahoff.assign(g.q + 1, 0);
  for (int k = 0; k < g.q; ++k) {
    p->dtg_mbh[k] = (int)((2 * p->sum_r1_k[k] + 255) / 256 * 8);
    p->dtg_ahoff[k + 1] = p->dtg_ahoff[k] + (int64_t)n1p * p->dtg_mbh[k] * 64;
  }
  std::vector<float> ah((size_t)p->dtg_ahoff[g.q], 0.f);
  for (int64_t j = 0; j < g.m; ++j)
    for (int k = 0; k < g.q; ++k) {
      const int64_t t = k + (int64_t)g.q * j;
      const TensorMeta& M = meta[(size_t)k * g.m + j];
      const int mbh = p->dtg_mbh[k];
      for (int al = 0; al < M.r1; ++al) {
        const int64_t a = drow[(size_t)k * g.m + j] + al;   // stacked row
        const int blk = (int)(a / 16), rl = (int)(a % 16);
        for (int i1 = 0; i1 < g.n1; ++i1) {
          const size_t src = p->u1_off[t] + i1 + (size_t)g.n1 * al;
          const float ur = (float)p->u1[2 * src], ui = (float)p->u1[2 * src + 1];
          float* base = &ah[p->dtg_ahoff[k] + (((int64_t)(i1 / 4) * mbh + blk) * 64) * 4 + i1 % 4];
          for (int sidx = 0; sidx < 2; ++sidx)
            for (int tt = 0; tt < 2; ++tt) {
              const int lane = 32 * tt + 2 * rl + sidx;
              base[lane * 4] = sidx == tt ? ur : (sidx == 0 ? ui : -ui);
            }
        }
      }
    }
  p->hp.ah = std::move(ah);
  p->hp.drow = std::move(drow);
  p->dtg_packed = true;
  return TV_OK;
}

bool dtg_supported(const tv_plan_s* p) { return p->dtg_packed && p->grid.q <= DTG_MAXQ; }

// 32-column blocks of one slab's B rows (a multiple of the widest tile)
static int64_t dtg_nblocks(const tv_plan_s* p, int s3) {
  const int64_t cols = (int64_t)p->grid.n2 * s3;
  return (cols + 255) / 256 * 8;
}

// i3 values per decompression workgroup: H3 (r1 x t3w x r2 complex) within
// 64 KB of LDS
static int dtg_t3w(const tv_plan_s* p) {
  const int64_t r12 = (int64_t)p->max_r[0] * p->max_r[1];
  int t = 8;
  while (t > 1 && r12 * t * 8 > 64 * 1024) t /= 2;
  return t;
}

int64_t dtg_launch_tiles(const tv_plan_s* p, int s3, int nbw) {
  const int64_t cols = (int64_t)p->grid.n2 * std::min(s3, p->grid.n3);
  const int w = nbw == 1 ? 2 : nbw;  // BF16X3's one-chunk stages keep 2 blocks per wave
  return (int64_t)p->grid.q * (p->dtg_nbtp / dtg_mt(p)) * ((cols + 64 * w - 1) / (64 * w));
}

// adjoint: row tiles over all components, N tiles per workgroup and chunks
// per slab (about 2048 workgroups per launch)
struct AdjGeom {
  int mtot, ntiles, ntw, nchunks, nslabs;
};
static AdjGeom adj_geom(const tv_plan_s* p, int s3) {
  AdjGeom G;
  G.mtot = 0;
  for (int k = 0; k < p->grid.q; ++k) G.mtot += p->dtg_mbh[k] / ADJ_MT;
  const int64_t cols = (int64_t)p->grid.n2 * s3;
  G.ntiles = (int)((cols + ADJ_NBT * 32 - 1) / (ADJ_NBT * 32));
  const int64_t want = std::max<int64_t>(1, ((int64_t)G.ntiles * G.mtot + 2047) / 2048);
  G.ntw = (int)std::min<int64_t>(want, G.ntiles);
  G.nchunks = (G.ntiles + G.ntw - 1) / G.ntw;
  G.nslabs = (p->grid.n3 + s3 - 1) / s3;
  return G;
}

size_t dtg_workspace_bytes(const tv_plan_s* p, int op) {
  if (!dtg_supported(p)) return 0;
  const int s3 = std::min(op == 0 ? p->dtg_s3 : p->dtg_s3_a, p->grid.n3);
  const size_t b = (size_t)p->dtg_rows * dtg_nblocks(p, s3) * 64 * sizeof(float);
  if (op == 1) {
    const AdjGeom G = adj_geom(p, s3);
    return b + (size_t)8 * G.nslabs * G.nchunks * p->dtg_rows;
  }
  const int64_t rows = (int64_t)p->grid.q * p->grid.n1 * p->grid.n2 * p->grid.n3;
  const size_t part = p->dtg_split > 1 ? (size_t)8 * p->dtg_split * rows : 0;
  return b + part;
}

tv_status launch_dtg_forward(const tv_plan_s* p, const float2* x, float2* y, void* ws,
                             hipStream_t st) {
  if (!dtg_supported(p)) return set_error(TV_ERR_NOT_SUPPORTED, "decompress-then-GEMM not packed");
  const tv_grid& g = p->grid;
  const int s3 = std::min(p->dtg_s3, g.n3);
  const int64_t nbl = dtg_nblocks(p, s3);
  const int64_t ldb = nbl * 64;
  float* B = (float*)ws;
  const int64_t rows = (int64_t)g.q * g.n1 * g.n2 * g.n3;
  const size_t bbytes = (size_t)p->dtg_rows * ldb * sizeof(float);
  const int S = std::max(1, p->dtg_split);
  float2* out = S > 1 ? (float2*)((char*)ws + bbytes) : y;

  DecompParams D;
  D.meta = p->d_meta;
  D.cores = p->d_cores;
  D.u2t = p->d_u2t;
  D.u3t = p->d_u3t;
  D.x = x;
  D.drow = p->d_drow;
  D.B = B;
  D.ldb = ldb;
  int64_t acc = 0;
  for (int k = 0; k < g.q; ++k) {
    D.brow[k] = acc;
    acc += p->dtg_rpad[k];
  }
  D.m = g.m;
  D.n2 = g.n2;
  D.n3 = g.n3;

  GemmParams G;
  G.apack4 = p->d_apack4;
  G.B = B;
  G.out = out;
  G.out_stride = rows;
  for (int k = 0; k < g.q; ++k) {
    G.a4off[k] = p->dtg_a4off[k];
    G.brow[k] = D.brow[k];
    G.kst[k] = (int)(p->dtg_rpad[k] / DTG_KC);
  }
  const int MT = dtg_mt(p);
  const bool bf = p->precision == TV_PREC_BF16X3;
  const int mbw = MT / 2, nbw = (bf && p->dtg_nbw == 1) ? 2 : p->dtg_nbw;
  const int cps = (bf && p->dtg_nbw == 1) ? 1 : 2;
  gemm_fn fn = bf ? gemm_pick_bf(mbw, p->dtg_nbw) : gemm_pick(mbw, nbw);
  if (!fn) return set_error(TV_ERR_NOT_SUPPORTED, "no GEMM instance for this tile");
  if (bf) {
    G.apack4 = (const float*)p->d_abf;
    for (int k = 0; k < g.q; ++k) G.a4off[k] = p->dtg_abfoff[k];
  }
  G.q = g.q;
  G.nbtp = p->dtg_nbtp;
  G.mtiles = p->dtg_nbtp / MT;
  G.S = S;
  G.ldb = ldb;
  G.nv = (int64_t)g.n1 * g.n2 * g.n3;
  G.n1 = g.n1;
  G.vec4 = (g.n1 % 2 == 0) && ((uintptr_t)out % 16 == 0);
  const size_t lds = bf ? 2 * sizeof(uint4) * (size_t)(cps * 2 * mbw * 128 + cps * 2 * nbw * 128)
                       : dtg_gemm_lds(mbw, nbw);
  hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return hip_error(e, "hipFuncSetAttribute");
  const int t3w = dtg_t3w(p);
  D.t3w = t3w;
  D.layout = p->precision == TV_PREC_BF16X3 ? 2 : 0;
  const size_t hl = sizeof(float2) * (size_t)p->max_r[0] * t3w * p->max_r[1];
  decomp_fn dfn = decomp_pick(p->max_r[1]);
  e = hipFuncSetAttribute((const void*)dfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)hl);
  if (e != hipSuccess) return hip_error(e, "hipFuncSetAttribute");

  // k-steps past the stacked rows: zeroed once per call by a kernel (the
  // decompression writes only the tensors' rows)
  ZeroParams Z;
  Z.B = B;
  Z.ldb = ldb;
  Z.q = g.q;
  for (int k = 0; k < g.q; ++k) {
    Z.from[k] = D.brow[k] + p->sum_r1_k[k];
    Z.to[k] = D.brow[k] + p->dtg_rpad[k];
  }
  if (bf)
    hipLaunchKernelGGL(dtg_zero_rows_bf_kernel, dim3(64), dim3(256), 0, st, Z);
  else
    hipLaunchKernelGGL(dtg_zero_rows_kernel, dim3(64), dim3(256), 0, st, Z);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "padding rows");
  for (int i30 = 0; i30 < g.n3; i30 += s3) {
    const int s3a = std::min(s3, g.n3 - i30);
    D.i30 = i30;
    D.s3 = s3a;
    D.nsub = (s3a + t3w - 1) / t3w;
    D.nitems = (int64_t)g.q * g.m * D.nsub;
    hipLaunchKernelGGL(dfn, dim3((unsigned)D.nitems), dim3(256), hl, st, D);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "slab decompression launch");
    G.col0 = (int64_t)g.n2 * i30;
    G.ncols = (int64_t)g.n2 * s3a;
    G.ntiles = (int)((G.ncols + 64 * nbw - 1) / (64 * nbw));
    G.nitems = (int64_t)G.mtiles * G.ntiles * g.q * S;
    const int64_t grid = (G.nitems + 7) / 8 * 8;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(256), lds, st, G);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "stacked GEMM launch");
  }
  if (S > 1) return launch_sum_partials(out, S, rows, y, st);
  return TV_OK;
}

tv_status launch_dtg_adjoint(const tv_plan_s* p, const float2* y, float2* x, void* ws,
                             hipStream_t st) {
  if (!dtg_supported(p)) return set_error(TV_ERR_NOT_SUPPORTED, "decompress-then-GEMM not packed");
  const tv_grid& g = p->grid;
  const int s3 = std::min(p->dtg_s3_a, g.n3);
  const int64_t nbl = dtg_nblocks(p, s3);
  const int64_t ldb = nbl * 64;
  float* B = (float*)ws;
  const size_t bbytes = (size_t)p->dtg_rows * ldb * sizeof(float);
  float2* partial = (float2*)((char*)ws + bbytes);
  const AdjGeom AG = adj_geom(p, s3);

  DecompParams D;
  D.meta = p->d_meta;
  D.cores = p->d_cores;
  D.u2t = p->d_u2t;
  D.u3t = p->d_u3t;
  D.x = nullptr;
  D.drow = p->d_drow;
  D.B = B;
  D.ldb = ldb;
  int64_t acc = 0;
  for (int k = 0; k < g.q; ++k) {
    D.brow[k] = acc;
    acc += p->dtg_rpad[k];
  }
  D.m = g.m;
  D.n2 = g.n2;
  D.n3 = g.n3;
  const int t3w = dtg_t3w(p);
  D.t3w = t3w;
  const size_t hl = sizeof(float2) * (size_t)p->max_r[0] * t3w * p->max_r[1];
  decomp_fn dfn = decomp_pick(p->max_r[1]);
  hipError_t e = hipFuncSetAttribute((const void*)dfn,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)hl);
  if (e != hipSuccess) return hip_error(e, "hipFuncSetAttribute");

  AdjParams A;
  A.apackh = p->d_apackh;
  A.B = B;
  A.y = y;
  A.q = g.q;
  A.mtb[0] = 0;
  for (int k = 0; k < g.q; ++k) {
    A.ahoff[k] = p->dtg_ahoff[k];
    A.brow[k] = D.brow[k];
    A.rk[k] = p->sum_r1_k[k];
    A.mbh[k] = p->dtg_mbh[k];
    A.mtb[k + 1] = A.mtb[k] + p->dtg_mbh[k] / ADJ_MT;
  }
  A.kst = (g.n1 + DTG_KC - 1) / DTG_KC;
  A.ntiles = AG.ntiles;
  A.ntw = AG.ntw;
  A.nchunks = AG.nchunks;
  A.prow = p->dtg_rows;
  A.nbl = nbl;
  A.order = p->dtg_order_a;
  A.nv = (int64_t)g.n1 * g.n2 * g.n3;
  A.n1 = g.n1;
  A.vec = (g.n1 % 2 == 0) && ((uintptr_t)y % 16 == 0);
  A.nitems = (int64_t)AG.mtot * AG.nchunks;
  const size_t lds = 2 * sizeof(float) * (size_t)(ADJ_A_ST + ADJ_Y_ST);
  e = hipFuncSetAttribute((const void*)dtg_adjoint_kernel,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_error(e, "hipFuncSetAttribute");

  // rows past the stacked rows and columns past the slab are masked in the
  // epilogue: no padding to clear
  D.layout = 1;
  int slab = 0;
  for (int i30 = 0; i30 < g.n3; i30 += s3, ++slab) {
    const int s3a = std::min(s3, g.n3 - i30);
    D.i30 = i30;
    D.s3 = s3a;
    D.nsub = (s3a + t3w - 1) / t3w;
    D.nitems = (int64_t)g.q * g.m * D.nsub;
    hipLaunchKernelGGL(dfn, dim3((unsigned)D.nitems), dim3(256), hl, st, D);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "slab decompression launch");
    A.col0 = (int64_t)g.n2 * i30;
    A.ncols = (int64_t)g.n2 * s3a;
    A.partial = partial + (int64_t)slab * AG.nchunks * p->dtg_rows;
    const int64_t grid = (A.nitems + 7) / 8 * 8;
    hipLaunchKernelGGL(dtg_adjoint_kernel, dim3((unsigned)grid), dim3(256), lds, st, A);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "adjoint GEMM launch");
  }
  AdjReduceParams R;
  R.meta = p->d_meta;
  R.drow = p->d_drow;
  R.partial = partial;
  R.x = x;
  for (int k = 0; k < g.q; ++k) R.brow[k] = D.brow[k];
  R.prow = p->dtg_rows;
  R.m = g.m;
  R.q = g.q;
  R.nchunks = AG.nslabs * AG.nchunks;
  hipLaunchKernelGGL(dtg_adjoint_reduce_kernel, dim3((unsigned)((g.m + 255) / 256)), dim3(256), 0,
                     st, R);
  e = hipGetLastError();
  return e == hipSuccess ? TV_OK : hip_error(e, "adjoint reduction launch");
}

}  // namespace tv
