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
typedef float v2f __attribute__((ext_vector_type(2)));

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
  int64_t nitems;
};

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
  // B is written once and read back by the GEMM after this kernel, and is far
  // larger than L2 and the MALL: non-temporal stores.  With n2 even (and U2
  // rows that fit the registers twice) each thread takes two adjacent i2,
  // whose entries are adjacent in both the Re and the Im 32-runs (n even),
  // and stores each pair as one 8-byte store; the threads' second index then
  // strides over i3.
  if (R2MAX <= 32 && (P.n2 & 1) == 0) {
    const int np2 = P.n2 >> 1;
    const int li3 = max(1, 256 / np2);
    for (int e = threadIdx.x; e < np2 * li3; e += 256) {
      const int i2 = 2 * (e % np2), i3s = e / np2;
      float2 u0[R2MAX], u1[R2MAX];
      const float2* u2 = P.u2t + t.u2_off + (int64_t)i2 * r2;
#pragma unroll
      for (int b = 0; b < R2MAX; ++b) {
        u0[b] = b < r2 ? u2[b] : make_float2(0.f, 0.f);
        u1[b] = b < r2 ? u2[r2 + b] : make_float2(0.f, 0.f);
      }
      for (int a = 0; a < r1; ++a) {
        float* row = Bk + (int64_t)a * P.ldb;
        for (int i3l = i3s; i3l < cnt; i3l += li3) {
          const float2* hv = h3 + (a * T3 + i3l) * r2;
          float sr0 = 0.f, si0 = 0.f, sr1 = 0.f, si1 = 0.f;
#pragma unroll
          for (int b = 0; b < R2MAX; ++b) {
            if (b < r2) {
              const float2 h = hv[b];
              sr0 = fmaf(h.x, u0[b].x, fmaf(-h.y, u0[b].y, sr0));
              si0 = fmaf(h.x, u0[b].y, fmaf(h.y, u0[b].x, si0));
              sr1 = fmaf(h.x, u1[b].x, fmaf(-h.y, u1[b].y, sr1));
              si1 = fmaf(h.x, u1[b].y, fmaf(h.y, u1[b].x, si1));
            }
          }
          const int64_t n = i2 + (int64_t)P.n2 * (i3a + i3l - P.i30);
          float* dst = row + (n >> 5) * 64 + (n & 31);
          __builtin_nontemporal_store(v2f{sr0, sr1}, reinterpret_cast<v2f*>(dst));
          __builtin_nontemporal_store(v2f{si0, si1}, reinterpret_cast<v2f*>(dst + 32));
        }
      }
    }
    return;
  }
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
        float* dst = row + (n >> 5) * 64 + (n & 31);
        __builtin_nontemporal_store(sr, dst);
        __builtin_nontemporal_store(si, dst + 32);
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
  // Per stage: the LDS operands of k-step q + 1 are read while the MFMAs of
  // q run, and the next stage's operands (loaded from global memory at the
  // top) are stored to the other buffer three quarters of the way through,
  // so that only the barrier separates two stages' MFMAs.  The last stage
  // reloads and stores its own operands (in bounds, never read), which keeps
  // the body free of branches.
  for (int st = st0; st < st1; ++st) {
    const int buf = (st - st0) & 1;
    gload(st + 1 < st1 ? st + 1 : st);
    // keep the global loads at the top of the stage (the scheduler would
    // otherwise sink them next to their LDS stores)
    __builtin_amdgcn_sched_barrier(0);
    const float* As = lds + buf * (A_ST + B_ST);
    const float* Bs = As + A_ST;
    v4f a[2][MBW];
    float b[2][NBW];
#pragma unroll
    for (int i = 0; i < MBW; ++i) a[0][i] = *(const v4f*)(As + ((wm * MBW + i) * 64 + lane) * 4);
#pragma unroll
    for (int jn = 0; jn < NBW; ++jn) b[0][jn] = Bs[(wn * NBW + jn) * 64 + lane];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int kg = q >> 2, kk = q & 3, cur = q & 1;
      if (q + 1 < 16) {
        const int kg1 = (q + 1) >> 2;
        if (((q + 1) & 3) == 0) {
#pragma unroll
          for (int i = 0; i < MBW; ++i)
            a[(kg1 & 1)][i] = *(const v4f*)(As + ((kg1 * MT + wm * MBW + i) * 64 + lane) * 4);
        }
#pragma unroll
        for (int jn = 0; jn < NBW; ++jn)
          b[cur ^ 1][jn] = Bs[((q + 1) * NBT + wn * NBW + jn) * 64 + lane];
      }
#pragma unroll
      for (int i = 0; i < MBW; ++i)
#pragma unroll
        for (int jn = 0; jn < NBW; ++jn)
          acc[i][jn] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[kg & 1][i][kk], b[cur][jn],
                                                            acc[i][jn], 0, 0, 0);
      if (q == 11) {
        __builtin_amdgcn_sched_barrier(0);
        lstore(buf ^ 1);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
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

// ---- BF16X3 GEMM on the FP32 stacked operand ------------------------------
// The forward GEMM of BF16X3 plans: A_k hi/lo from the plan (8-k-step chunks
// in the A-operand order of v_mfma_f32_32x32x16_bf16), B_k FP32 as the
// decompression writes it for FP32 plans, split into bf16 hi/lo while the
// MFMA operands are built (hi = rn(b), lo = rn(b - hi)); Ah Bh + Ah Bl + Al Bh
// with FP32 accumulation.  One LDS stage is one chunk (8 stacked rows, 16
// real k-steps).  Loads are staged through two register sets: the global
// loads of chunk c + 2 are in flight while chunk c is multiplied from LDS and
// chunk c + 1 (loaded one step earlier) is stored to the other LDS buffer,
// one barrier per chunk.  B rows are padded by 8 floats in LDS so that the
// operand reads of the two half-waves (rows 4 apart) fall on disjoint banks.
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v8bf as_v8bf(uint4 v) { return __builtin_bit_cast(v8bf, v); }
constexpr int BF2_RPAD = 8;        // floats of padding per B row in LDS

__device__ __forceinline__ uint32_t bf2_pack(float a, float b) {
  const v2bf h = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, h);
}

// one chunk (16 real k-steps) of the BF16X3 GEMM from LDS buffer `buf`
template <int MBW, int NBW>
__device__ __forceinline__ void bf2_compute(const float* lds, int buf, int lane, int wm, int wn,
                                            v16f (&acc)[MBW][NBW]) {
  constexpr int MT = 2 * MBW, NBT = 2 * NBW;
  constexpr int RS = NBT * 64 + BF2_RPAD;
  constexpr int A_ST = MT * 2 * 64 * 4;
  constexpr int ST = A_ST + 8 * RS;
  const int h = lane >> 5, ln = lane & 31;
  const float* As = lds + buf * ST;
  const float* Bs = As + A_ST;
  v8bf ah[MBW], al[MBW], bh[NBW], bl[NBW];
#pragma unroll
  for (int ii = 0; ii < MBW; ++ii) {
    const int b = wm * MBW + ii;
    ah[ii] = as_v8bf(*(const uint4*)(As + ((b * 2) * 64 + lane) * 4));
    al[ii] = as_v8bf(*(const uint4*)(As + ((b * 2 + 1) * 64 + lane) * 4));
  }
#pragma unroll
  for (int jn = 0; jn < NBW; ++jn) {
    const float* bp = Bs + (4 * h) * RS + (wn * NBW + jn) * 64 + ln;
    uint32_t hw[4], lw[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float re = bp[r * RS], im = bp[r * RS + 32];
      hw[r] = bf2_pack(re, im);
      const float hre = __builtin_bit_cast(float, hw[r] << 16);
      const float him = __builtin_bit_cast(float, hw[r] & 0xFFFF0000u);
      lw[r] = bf2_pack(re - hre, im - him);
    }
    bh[jn] = as_v8bf(make_uint4(hw[0], hw[1], hw[2], hw[3]));
    bl[jn] = as_v8bf(make_uint4(lw[0], lw[1], lw[2], lw[3]));
  }
#pragma unroll
  for (int ii = 0; ii < MBW; ++ii)
#pragma unroll
    for (int jn = 0; jn < NBW; ++jn) {
      acc[ii][jn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ii], bh[jn], acc[ii][jn], 0, 0, 0);
      acc[ii][jn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ii], bl[jn], acc[ii][jn], 0, 0, 0);
      acc[ii][jn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[ii], bh[jn], acc[ii][jn], 0, 0, 0);
    }
}

template <int MBW, int NBW>
__global__ __launch_bounds__(256, (NBW == 2 && MBW < 8) ? 2 : 1) void dtg_gemm_bf2_kernel(GemmParams P) {
  constexpr int MT = 2 * MBW, NBT = 2 * NBW;
  constexpr int RS = NBT * 64 + BF2_RPAD;          // floats per LDS row of B
  constexpr int A_ST = MT * 2 * 64 * 4;            // floats per A stage (hi, lo)
  constexpr int B_ST = 8 * RS;                     // floats per B stage
  constexpr int ST = A_ST + B_ST;
  constexpr int NA = MT * 2 * 64 / 256;            // uint4 of A per thread and chunk
  constexpr int NBQ = 8 * NBT * 16 / 256;          // float4 of B per thread and chunk
  extern __shared__ float lds[];
  const int64_t nwg = gridDim.x;
  const int64_t L = (int64_t)(blockIdx.x % 8) * (nwg / 8) + blockIdx.x / 8;
  if (L >= P.nitems) return;
  const int mt = (int)(L % P.mtiles);
  int64_t rest = L / P.mtiles;
  const int nt = (int)(rest % P.ntiles);
  rest /= P.ntiles;
  const int k = (int)(rest % P.q);
  const int s = (int)(rest / P.q);
  // chunk ranges of the splits start and end on even chunks (stacked rows
  // are padded to 16, so every component has an even number of chunks)
  const int c0 = 2 * (int)((int64_t)P.kst[k] * s / P.S);
  const int c1 = 2 * (int)((int64_t)P.kst[k] * (s + 1) / P.S);

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1, h = lane >> 5, ln = lane & 31;
  const uint4* Ag = (const uint4*)P.apack4 + P.a4off[k] + (int64_t)mt * MT * 128;
  const float* Bg = P.B + P.brow[k] * P.ldb + (int64_t)nt * NBT * 64;

  v4u ra0[NA], ra1[NA];
  v4f rb0[NBQ], rb1[NBQ];
  // global loads of chunk c (clamped to the last chunk, so the tail repeats
  // a load instead of branching) into a register set, and the set's store
  // into an LDS buffer
#define TV_BF2_GLOAD(c, RA, RB)                                                  \
  {                                                                             \
    const int cc = min((c), c1 - 1);                                            \
    const v4u* ac = (const v4u*)(Ag + (int64_t)cc * P.nbtp * 128);              \
    _Pragma("unroll") for (int j = 0; j < NA; ++j) RA[j] = ac[j * 256 + tid];   \
    const float* bc = Bg + (int64_t)cc * 8 * P.ldb;                             \
    _Pragma("unroll") for (int j = 0; j < NBQ; ++j) {                           \
      const int u = j * 256 + tid, r = u / (NBT * 16), q = u % (NBT * 16);      \
      RB[j] = *(const v4f*)(bc + r * P.ldb + q * 4);                            \
    }                                                                           \
  }
#define TV_BF2_LSTORE(buf, RA, RB)                                               \
  {                                                                             \
    float* As = lds + (buf) * ST;                                               \
    float* Bs = As + A_ST;                                                      \
    _Pragma("unroll") for (int j = 0; j < NA; ++j)                              \
      *(v4u*)(As + (j * 256 + tid) * 4) = RA[j];                                \
    _Pragma("unroll") for (int j = 0; j < NBQ; ++j) {                           \
      const int u = j * 256 + tid, r = u / (NBT * 16), q = u % (NBT * 16);      \
      *(v4f*)(Bs + r * RS + q * 4) = RB[j];                                     \
    }                                                                           \
  }

  v16f acc[MBW][NBW];
#pragma unroll
  for (int i = 0; i < MBW; ++i)
#pragma unroll
    for (int jn = 0; jn < NBW; ++jn) acc[i][jn] = v16f{0.f};

  // register set (c - c0) % 2 carries chunk c from global memory to LDS
  if (c0 < c1) {
    TV_BF2_GLOAD(c0, ra0, rb0);
    TV_BF2_GLOAD(c0 + 1, ra1, rb1);
    TV_BF2_LSTORE(0, ra0, rb0);
  }
  __syncthreads();
  for (int c = c0; c < c1; c += 2) {
    // even step: chunk c in LDS buffer 0, chunk c + 1 in set 1
    TV_BF2_GLOAD(c + 2, ra0, rb0);
    bf2_compute<MBW, NBW>(lds, 0, lane, wm, wn, acc);
    TV_BF2_LSTORE(1, ra1, rb1);
    __syncthreads();
    // odd step: chunk c + 1 in LDS buffer 1, chunk c + 2 in set 0
    TV_BF2_GLOAD(c + 3, ra1, rb1);
    bf2_compute<MBW, NBW>(lds, 1, lane, wm, wn, acc);
    TV_BF2_LSTORE(0, ra0, rb0);
    __syncthreads();
  }
#undef TV_BF2_GLOAD
#undef TV_BF2_LSTORE

  float2* out = P.out + (int64_t)s * P.out_stride + (int64_t)k * P.nv;
#pragma unroll
  for (int jn = 0; jn < NBW; ++jn) {
    const int64_t n = ((int64_t)nt * NBT + wn * NBW + jn) * 32 + ln;
    if (n >= P.ncols) continue;
    float2* col = out + (int64_t)P.n1 * (P.col0 + n);
#pragma unroll
    for (int ii = 0; ii < MBW; ++ii) {
      const int blk = mt * MT + wm * MBW + ii;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int i1 = blk * 16 + 4 * g + 2 * h;
        const v16f& d = acc[ii][jn];
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

// ---- adjoint as a GEMM over voxel columns ---------------------------------
// Algorithm 2's inner products with the sum over the columns (i2, i3) taken
// first: Z_k = Y^k_(1) B_k^* (n1 x stacked rows, contraction over the slab's
// columns, one partial per slab and column split), then x'_j = sum_k
// sum_{a of j} sum_i1 conj(U1_j[i1][a]) Z_k[i1][row of a] with the partials
// summed in FP64.  Z is a plain GEMM with the forward kernel's tile and stage
// structure; the final sum is a small pass.
//
// A operand (ypack, per slab): y^k real-embedded, M = (i1, s) rows
// interleaved as in the forward, K = (column n, t = Re/Im):
// [(i1,Re)][(n,Re)] = Re y, [(i1,Re)][(n,Im)] = Im y, [(i1,Im)][(n,Re)] =
// Im y, [(i1,Im)][(n,Im)] = -Re y (so the accumulator holds Re and Im of
// y conj(b)); float index ((n/4 * nbtp + blk) * 64 + lane) * 4 + n%4 per
// component, the layout of the forward's A operand.
// B operand: B_k as the forward writes it (row R, 32-column blocks of Re then
// Im); lane 32 t + R%32 of an MFMA reads four consecutive columns of one row
// with one 16-byte load, staged in LDS with a 32-float pad between k-step
// groups (the global-to-LDS copy is then free of bank conflicts).
struct YPackParams {
  const float2* y;
  float* yp;
  int64_t ystride;          // floats per component
  int64_t nv;
  int64_t col0, ncols, ngrp;  // slab's first column, width, 4-column groups packed
  int n1, nbtp, q;
};
__global__ void dtg_ypack_kernel(YPackParams P) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)P.q * P.ngrp * P.nbtp * 64;
  if (idx >= total) return;
  const int lane = (int)(idx & 63);
  int64_t rest = idx >> 6;
  const int blk = (int)(rest % P.nbtp);
  rest /= P.nbtp;
  const int64_t gq = rest % P.ngrp;
  const int k = (int)(rest / P.ngrp);
  const int mrow = 32 * blk + (lane & 31), i1 = mrow >> 1, s = mrow & 1, t = lane >> 5;
  v4f v;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t n = 4 * gq + e;
    float val = 0.f;
    if (n < P.ncols && i1 < P.n1) {
      const float2 c = P.y[(int64_t)k * P.nv + (P.col0 + n) * P.n1 + i1];
      val = s == 0 ? (t == 0 ? c.x : c.y) : (t == 0 ? c.y : -c.x);
    }
    v[e] = val;
  }
  *(v4f*)(P.yp + (int64_t)k * P.ystride + ((gq * P.nbtp + blk) * 64 + lane) * 4) = v;
}

struct ColGemmParams {
  const float* ypack;
  const float* B;
  float2* z;                // this slab's [split][stacked row][i1] complex
  int64_t ystride;          // floats per component of ypack
  int64_t zsplit;           // complex per split of z
  int64_t brow[DTG_MAXQ];
  int64_t rk[DTG_MAXQ];
  int ntb[DTG_MAXQ + 1];    // prefix sum over components of the N tiles
  int q, nbtp, mtiles, S;
  int order;                // 0: row tiles fastest, 1: N tiles fastest
  int64_t ldb;
  int n1;
  int64_t ncols;            // columns of the slab
  int vec4;
  int64_t nitems;
};
constexpr int COL_BPAD = 32;

template <int MBW, int NBW>
__global__ __launch_bounds__(256) void dtg_colgemm_kernel(ColGemmParams P) {
  constexpr int MT = 2 * MBW, NBT = 2 * NBW;
  constexpr int A_ST = 4 * MT * 64 * 4;
  constexpr int KGS = NBT * 64 * 4 + COL_BPAD;   // floats per k-step group of B
  constexpr int B_ST = 4 * KGS;
  extern __shared__ float lds[];
  const int64_t nwg = gridDim.x;
  const int64_t L = (int64_t)(blockIdx.x % 8) * (nwg / 8) + blockIdx.x / 8;
  if (L >= P.nitems) return;
  const int ntot = P.ntb[P.q];
  int mt, ntg;
  int64_t rest;
  if (P.order == 0) {
    mt = (int)(L % P.mtiles);
    rest = L / P.mtiles;
    ntg = (int)(rest % ntot);
    rest /= ntot;
  } else {
    ntg = (int)(L % ntot);
    rest = L / ntot;
    mt = (int)(rest % P.mtiles);
    rest /= P.mtiles;
  }
  const int s = (int)rest;
  int k = 0;
  while (ntg >= P.ntb[k + 1]) ++k;
  const int nt = ntg - P.ntb[k];
  const int nst = (int)((P.ncols + DTG_KC - 1) / DTG_KC);
  const int st0 = (int)((int64_t)nst * s / P.S), st1 = (int)((int64_t)nst * (s + 1) / P.S);

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const float* Ag = P.ypack + (int64_t)k * P.ystride;
  const float* Bg = P.B + P.brow[k] * P.ldb;
  const int64_t rk = P.rk[k];

  v4f ra[MT], rb[NBT];
  auto gload = [&](int st) {
#pragma unroll
    for (int c = 0; c < MT; ++c) {
      const int u = c * 256 + tid;
      const int kg = u / (MT * 64), rem = u % (MT * 64);
      ra[c] = *(const v4f*)(Ag + ((((int64_t)st * 4 + kg) * P.nbtp + mt * MT + rem / 64) * 64 +
                                  rem % 64) * 4);
    }
    // u = row-in-8 | kg | t | row-of-8: one instruction reads 8 rows x (Re,
    // Im) x 16 columns, 64-byte runs
#pragma unroll
    for (int c = 0; c < NBT; ++c) {
      const int u = c * 256 + tid;
      const int r8 = u & 7, kg = (u >> 3) & 3, t = (u >> 5) & 1;
      const int64_t R = (int64_t)nt * (NBT * 32) + (u >> 6) * 8 + r8;
      const int64_t n = (int64_t)st * DTG_KC + kg * 4;
      v4f v = v4f{0.f, 0.f, 0.f, 0.f};
      if (R < rk) {
        const float* src = Bg + R * P.ldb + (n >> 5) * 64 + t * 32 + (n & 31);
        if (n + 4 <= P.ncols) {
          v = *(const v4f*)src;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (n + e < P.ncols) v[e] = src[e];
        }
      }
      rb[c] = v;
    }
  };
  auto lstore = [&](int buf) {
    float* As = lds + buf * (A_ST + B_ST);
    float* Bs = As + A_ST;
#pragma unroll
    for (int c = 0; c < MT; ++c) *(v4f*)(As + (c * 256 + tid) * 4) = ra[c];
#pragma unroll
    for (int c = 0; c < NBT; ++c) {
      const int u = c * 256 + tid;
      const int r8 = u & 7, kg = (u >> 3) & 3, t = (u >> 5) & 1;
      const int R = (u >> 6) * 8 + r8;
      *(v4f*)(Bs + kg * KGS + ((R >> 5) * 64 + 32 * t + (R & 31)) * 4) = rb[c];
    }
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
  // as in dtg_gemm_kernel: the next k-step group's operands are read while
  // the current group's MFMAs run, the next stage is stored three quarters
  // of the way through, and the last stage reloads its own (in bounds)
  for (int st = st0; st < st1; ++st) {
    const int buf = (st - st0) & 1;
    gload(st + 1 < st1 ? st + 1 : st);
    __builtin_amdgcn_sched_barrier(0);
    const float* As = lds + buf * (A_ST + B_ST);
    const float* Bs = As + A_ST;
    v4f a[2][MBW], b[2][NBW];
#pragma unroll
    for (int i = 0; i < MBW; ++i) a[0][i] = *(const v4f*)(As + ((wm * MBW + i) * 64 + lane) * 4);
#pragma unroll
    for (int jn = 0; jn < NBW; ++jn)
      b[0][jn] = *(const v4f*)(Bs + ((wn * NBW + jn) * 64 + lane) * 4);
#pragma unroll
    for (int kg = 0; kg < 4; ++kg) {
      const int cur = kg & 1;
      if (kg + 1 < 4) {
#pragma unroll
        for (int i = 0; i < MBW; ++i)
          a[cur ^ 1][i] = *(const v4f*)(As + (((kg + 1) * MT + wm * MBW + i) * 64 + lane) * 4);
#pragma unroll
        for (int jn = 0; jn < NBW; ++jn)
          b[cur ^ 1][jn] = *(const v4f*)(Bs + (kg + 1) * KGS + ((wn * NBW + jn) * 64 + lane) * 4);
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int i = 0; i < MBW; ++i)
#pragma unroll
          for (int jn = 0; jn < NBW; ++jn)
            acc[i][jn] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[cur][i][kk], b[cur][jn][kk],
                                                              acc[i][jn], 0, 0, 0);
      if (kg == 2) {
        __builtin_amdgcn_sched_barrier(0);
        lstore(buf ^ 1);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    __syncthreads();
  }

  // accumulator rows (i1, Re/Im) pairs: registers 4g..4g+3 are (Re, Im) of
  // i1, i1 + 1; column = stacked row R of component k
  float2* zs = P.z + (int64_t)s * P.zsplit;
#pragma unroll
  for (int jn = 0; jn < NBW; ++jn) {
    const int64_t R = ((int64_t)nt * NBT + wn * NBW + jn) * 32 + (lane & 31);
    if (R >= rk) continue;
    float2* col = zs + (P.brow[k] + R) * P.n1;
#pragma unroll
    for (int i = 0; i < MBW; ++i) {
      const int blk = mt * MT + wm * MBW + i;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int i1 = blk * 16 + 4 * g + 2 * (lane >> 5);
        const v16f& d = acc[i][jn];
        if (i1 + 1 < P.n1 && P.vec4) {
          *(v4f*)(col + i1) = v4f{d[4 * g], d[4 * g + 1], d[4 * g + 2], d[4 * g + 3]};
        } else {
          if (i1 < P.n1) col[i1] = make_float2(d[4 * g], d[4 * g + 1]);
          if (i1 + 1 < P.n1) col[i1 + 1] = make_float2(d[4 * g + 2], d[4 * g + 3]);
        }
      }
    }
  }
}

// x'_j = sum_k sum_{a < r1} sum_i1 conj(U1_j[i1][a]) sum_s Z_s[row a][i1]
// over the partials s of every slab and split, in FP64, one workgroup per
// column j, fixed order
struct ColReduceParams {
  const TensorMeta* meta;
  const int32_t* drow;
  const float2* u1t;
  const float2* z;
  float2* x;
  int64_t brow[DTG_MAXQ];
  int64_t zsplit, m;
  int q, S, n1;
};
__global__ __launch_bounds__(256) void dtg_colgemm_reduce_kernel(ColReduceParams P) {
  __shared__ double red[2][256];
  const int64_t j = blockIdx.x;
  double sr = 0.0, si = 0.0;
  for (int k = 0; k < P.q; ++k) {
    const TensorMeta t = P.meta[(int64_t)k * P.m + j];
    const int64_t r0 = P.brow[k] + P.drow[(int64_t)k * P.m + j];
    for (int i1 = threadIdx.x; i1 < P.n1; i1 += 256) {
      const float2* u = P.u1t + t.u1_off + (int64_t)i1 * t.r1;
      for (int a = 0; a < t.r1; ++a) {
        double zr = 0.0, zi = 0.0;
        for (int s = 0; s < P.S; ++s) {
          const float2 z = P.z[(int64_t)s * P.zsplit + (r0 + a) * P.n1 + i1];
          zr += z.x;
          zi += z.y;
        }
        const double ur = u[a].x, ui = u[a].y;
        sr += ur * zr + ui * zi;
        si += ur * zi - ui * zr;
      }
    }
  }
  red[0][threadIdx.x] = sr;
  red[1][threadIdx.x] = si;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) P.x[j] = make_float2((float)red[0][0], (float)red[1][0]);
}

// BF16X3 plans: the packed y as hi/lo bf16 in the A-operand order of
// v_mfma_f32_32x32x16_bf16, 8-column chunks (k = 2 (column) + Re/Im):
// uint4 index ((c * nbtp + blk) * 2 + hl) * 64 + lane per component, lane
// 32 h + m%32 holding columns 8c + 4h .. 8c + 4h + 3 of row m, the real
// embedding as in dtg_ypack_kernel.
__global__ void dtg_ypack_bf_kernel(YPackParams P) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nchk = P.ngrp / 2;                 // 8-column chunks
  const int64_t total = (int64_t)P.q * nchk * P.nbtp * 64;
  if (idx >= total) return;
  const int lane = (int)(idx & 63);
  int64_t rest = idx >> 6;
  const int blk = (int)(rest % P.nbtp);
  rest /= P.nbtp;
  const int64_t c = rest % nchk;
  const int k = (int)(rest / nchk);
  const int mrow = 32 * blk + (lane & 31), i1 = mrow >> 1, sr = mrow & 1, h = lane >> 5;
  uint32_t hw[4], lw[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t n = 8 * c + 4 * h + j;
    float v0 = 0.f, v1 = 0.f;                      // k = 2j (Re part), 2j + 1 (Im part)
    if (n < P.ncols && i1 < P.n1) {
      const float2 y = P.y[(int64_t)k * P.nv + (P.col0 + n) * P.n1 + i1];
      v0 = sr == 0 ? y.x : y.y;
      v1 = sr == 0 ? y.y : -y.x;
    }
    hw[j] = bf2_pack(v0, v1);
    const float h0 = __builtin_bit_cast(float, hw[j] << 16);
    const float h1 = __builtin_bit_cast(float, hw[j] & 0xFFFF0000u);
    lw[j] = bf2_pack(v0 - h0, v1 - h1);
  }
  uint4* dst = (uint4*)(P.yp + (int64_t)k * P.ystride) + ((c * P.nbtp + blk) * 2) * 64 + lane;
  dst[0] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
  dst[64] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
}

// The adjoint's column GEMM for BF16X3 plans: A = the packed y (hi/lo), B =
// the unscaled FP32 slab split into hi/lo while the operands are built; one
// LDS stage is one 8-column chunk, staged through two register sets as in
// dtg_gemm_bf2_kernel.  A B row of a stage (8 Re then 8 Im values of one
// stacked row) sits in LDS at a stride of 20 floats, free of bank conflicts
// for the 16-byte operand reads.
constexpr int CBF_RS = 20;

template <int MBW, int NBW>
__device__ __forceinline__ void colbf2_compute(const float* lds, int buf, int lane, int wm, int wn,
                                               v16f (&acc)[MBW][NBW]) {
  constexpr int MT = 2 * MBW, NBT = 2 * NBW;
  constexpr int A_ST = MT * 2 * 64 * 4;
  constexpr int ST = A_ST + NBT * 32 * CBF_RS;
  const int h = lane >> 5, ln = lane & 31;
  const float* As = lds + buf * ST;
  const float* Bs = As + A_ST;
  v8bf ah[MBW], al[MBW], bh[NBW], bl[NBW];
#pragma unroll
  for (int ii = 0; ii < MBW; ++ii) {
    const int b = wm * MBW + ii;
    ah[ii] = as_v8bf(*(const uint4*)(As + ((b * 2) * 64 + lane) * 4));
    al[ii] = as_v8bf(*(const uint4*)(As + ((b * 2 + 1) * 64 + lane) * 4));
  }
#pragma unroll
  for (int jn = 0; jn < NBW; ++jn) {
    const float* bp = Bs + ((wn * NBW + jn) * 32 + ln) * CBF_RS + 4 * h;
    const v4f re = *(const v4f*)bp, im = *(const v4f*)(bp + 8);
    uint32_t hw[4], lw[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      hw[j] = bf2_pack(re[j], im[j]);
      const float hre = __builtin_bit_cast(float, hw[j] << 16);
      const float him = __builtin_bit_cast(float, hw[j] & 0xFFFF0000u);
      lw[j] = bf2_pack(re[j] - hre, im[j] - him);
    }
    bh[jn] = as_v8bf(make_uint4(hw[0], hw[1], hw[2], hw[3]));
    bl[jn] = as_v8bf(make_uint4(lw[0], lw[1], lw[2], lw[3]));
  }
#pragma unroll
  for (int ii = 0; ii < MBW; ++ii)
#pragma unroll
    for (int jn = 0; jn < NBW; ++jn) {
      acc[ii][jn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ii], bh[jn], acc[ii][jn], 0, 0, 0);
      acc[ii][jn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ii], bl[jn], acc[ii][jn], 0, 0, 0);
      acc[ii][jn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[ii], bh[jn], acc[ii][jn], 0, 0, 0);
    }
}

template <int MBW, int NBW>
__global__ __launch_bounds__(256, (NBW == 2 && MBW < 8) ? 2 : 1) void dtg_colgemm_bf2_kernel(ColGemmParams P) {
  constexpr int MT = 2 * MBW, NBT = 2 * NBW;
  constexpr int A_ST = MT * 2 * 64 * 4;
  constexpr int ST = A_ST + NBT * 32 * CBF_RS;
  constexpr int NA = MT * 2 * 64 / 256;            // uint4 of A per thread and chunk
  constexpr int NBQ = NBT * 32 * 4 / 256;          // float4 of B per thread and chunk
  extern __shared__ float lds[];
  const int64_t nwg = gridDim.x;
  const int64_t L = (int64_t)(blockIdx.x % 8) * (nwg / 8) + blockIdx.x / 8;
  if (L >= P.nitems) return;
  const int ntot = P.ntb[P.q];
  int mt, ntg;
  int64_t rest;
  if (P.order == 0) {
    mt = (int)(L % P.mtiles);
    rest = L / P.mtiles;
    ntg = (int)(rest % ntot);
    rest /= ntot;
  } else {
    ntg = (int)(L % ntot);
    rest = L / ntot;
    mt = (int)(rest % P.mtiles);
    rest /= P.mtiles;
  }
  const int s = (int)rest;
  int k = 0;
  while (ntg >= P.ntb[k + 1]) ++k;
  const int nt = ntg - P.ntb[k];
  // 16-column stages split as in the FP32 kernel, two chunks each
  const int nst = (int)((P.ncols + DTG_KC - 1) / DTG_KC);
  const int c0 = 2 * (int)((int64_t)nst * s / P.S), c1 = 2 * (int)((int64_t)nst * (s + 1) / P.S);

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const v4u* Ag = (const v4u*)((const uint4*)(P.ypack + (int64_t)k * P.ystride) +
                               (int64_t)mt * MT * 128);
  const float* Bg = P.B + P.brow[k] * P.ldb;
  const int64_t rk = P.rk[k];

  v4u ra0[NA], ra1[NA];
  v4f rb0[NBQ], rb1[NBQ];
  // thread u of a chunk's B: stacked row R = u / 4, q = u % 4: Re (q < 2) or
  // Im of columns 8c + 4 (q & 1) .. + 3
#define TV_CBF_GLOAD(c, RA, RB)                                                  \
  {                                                                             \
    const int cc = min((c), c1 - 1);                                            \
    const v4u* ac = Ag + (int64_t)cc * P.nbtp * 128;                            \
    _Pragma("unroll") for (int j = 0; j < NA; ++j) RA[j] = ac[j * 256 + tid];   \
    _Pragma("unroll") for (int j = 0; j < NBQ; ++j) {                           \
      const int u = j * 256 + tid, q = u & 3;                                   \
      const int64_t R = (int64_t)nt * (NBT * 32) + (u >> 2);                    \
      const int64_t n = (int64_t)cc * 8 + (q & 1) * 4;                          \
      v4f v = v4f{0.f, 0.f, 0.f, 0.f};                                          \
      if (R < rk) {                                                             \
        const float* src = Bg + R * P.ldb + (n >> 5) * 64 + (q >> 1) * 32 + (n & 31); \
        if (n + 4 <= P.ncols) {                                                 \
          v = *(const v4f*)src;                                                 \
        } else {                                                                \
          _Pragma("unroll") for (int e = 0; e < 4; ++e)                          \
            if (n + e < P.ncols) v[e] = src[e];                                 \
        }                                                                       \
      }                                                                         \
      RB[j] = v;                                                                \
    }                                                                           \
  }
#define TV_CBF_LSTORE(buf, RA, RB)                                               \
  {                                                                             \
    float* As = lds + (buf) * ST;                                               \
    float* Bs = As + A_ST;                                                      \
    _Pragma("unroll") for (int j = 0; j < NA; ++j)                              \
      *(v4u*)(As + (j * 256 + tid) * 4) = RA[j];                                \
    _Pragma("unroll") for (int j = 0; j < NBQ; ++j) {                           \
      const int u = j * 256 + tid, q = u & 3;                                   \
      *(v4f*)(Bs + (u >> 2) * CBF_RS + (q >> 1) * 8 + (q & 1) * 4) = RB[j];     \
    }                                                                           \
  }

  v16f acc[MBW][NBW];
#pragma unroll
  for (int i = 0; i < MBW; ++i)
#pragma unroll
    for (int jn = 0; jn < NBW; ++jn) acc[i][jn] = v16f{0.f};

  if (c0 < c1) {
    TV_CBF_GLOAD(c0, ra0, rb0);
    TV_CBF_GLOAD(c0 + 1, ra1, rb1);
    TV_CBF_LSTORE(0, ra0, rb0);
  }
  __syncthreads();
  for (int c = c0; c < c1; c += 2) {
    TV_CBF_GLOAD(c + 2, ra0, rb0);
    colbf2_compute<MBW, NBW>(lds, 0, lane, wm, wn, acc);
    TV_CBF_LSTORE(1, ra1, rb1);
    __syncthreads();
    TV_CBF_GLOAD(c + 3, ra1, rb1);
    colbf2_compute<MBW, NBW>(lds, 1, lane, wm, wn, acc);
    TV_CBF_LSTORE(0, ra0, rb0);
    __syncthreads();
  }
#undef TV_CBF_GLOAD
#undef TV_CBF_LSTORE

  float2* zs = P.z + (int64_t)s * P.zsplit;
#pragma unroll
  for (int jn = 0; jn < NBW; ++jn) {
    const int64_t R = ((int64_t)nt * NBT + wn * NBW + jn) * 32 + (lane & 31);
    if (R >= rk) continue;
    float2* col = zs + (P.brow[k] + R) * P.n1;
#pragma unroll
    for (int i = 0; i < MBW; ++i) {
      const int blk = mt * MT + wm * MBW + i;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int i1 = blk * 16 + 4 * g + 2 * (lane >> 5);
        const v16f& d = acc[i][jn];
        if (i1 + 1 < P.n1 && P.vec4) {
          *(v4f*)(col + i1) = v4f{d[4 * g], d[4 * g + 1], d[4 * g + 2], d[4 * g + 3]};
        } else {
          if (i1 < P.n1) col[i1] = make_float2(d[4 * g], d[4 * g + 1]);
          if (i1 + 1 < P.n1) col[i1 + 1] = make_float2(d[4 * g + 2], d[4 * g + 3]);
        }
      }
    }
  }
}

typedef void (*colgemm_fn)(ColGemmParams);
colgemm_fn colgemm_pick_bf2(int mbw, int nbw) {
  if (mbw == 4 && nbw == 2) return dtg_colgemm_bf2_kernel<4, 2>;
  if (mbw == 8 && nbw == 2) return dtg_colgemm_bf2_kernel<8, 2>;
  if (mbw == 4 && nbw == 4) return dtg_colgemm_bf2_kernel<4, 4>;
  if (mbw == 2 && nbw == 2) return dtg_colgemm_bf2_kernel<2, 2>;
  if (mbw == 2 && nbw == 4) return dtg_colgemm_bf2_kernel<2, 4>;
  return nullptr;
}
size_t colgemm_bf2_lds(int mbw, int nbw) {
  return 2 * sizeof(float) * (size_t)(2 * mbw * 2 * 64 * 4 + 2 * nbw * 32 * CBF_RS);
}
colgemm_fn colgemm_pick(int mbw, int nbw) {
  if (mbw == 4 && nbw == 2) return dtg_colgemm_kernel<4, 2>;
  if (mbw == 4 && nbw == 4) return dtg_colgemm_kernel<4, 4>;
  if (mbw == 2 && nbw == 2) return dtg_colgemm_kernel<2, 2>;
  if (mbw == 2 && nbw == 4) return dtg_colgemm_kernel<2, 4>;
  return nullptr;
}
size_t colgemm_lds(int mbw, int nbw) {
  return 2 * sizeof(float) * (size_t)(4 * 2 * mbw * 64 * 4 + 4 * (2 * nbw * 64 * 4 + COL_BPAD));
}

typedef void (*decomp_fn)(DecompParams);

decomp_fn decomp_pick(int r2max) {
  if (r2max <= 16) return dtg_decomp_kernel<16>;
  if (r2max <= 32) return dtg_decomp_kernel<32>;
  return dtg_decomp_kernel<64>;
}

typedef void (*gemm_fn)(GemmParams);

gemm_fn gemm_pick_bf2(int mbw, int nbw) {
  if (mbw == 4 && nbw == 4) return dtg_gemm_bf2_kernel<4, 4>;
  if (mbw == 8 && nbw == 2) return dtg_gemm_bf2_kernel<8, 2>;
  if (mbw == 4 && nbw == 2) return dtg_gemm_bf2_kernel<4, 2>;
  if (mbw == 2 && nbw == 4) return dtg_gemm_bf2_kernel<2, 4>;
  if (mbw == 2 && nbw == 2) return dtg_gemm_bf2_kernel<2, 2>;
  return nullptr;
}
size_t bf2_lds(int mbw, int nbw) {
  return sizeof(float) * 2 * ((size_t)2 * mbw * 2 * 64 * 4 + 8 * ((size_t)2 * nbw * 64 + BF2_RPAD));
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

// 32-row blocks of a GEMM workgroup tile along the voxel rows for op 0 / 1:
// the plan's default, or all 16 blocks of 2 n1 = 512 rows when the launch
// configuration asks for 8 blocks per wave (BF16X3 plans; the packed rows
// come in tiles of 16 blocks when dtg_nbtp is a multiple of 16)
int dtg_mt_op(const tv_plan_s* p, int op) {
  return p->dtg_mbw[op] == 8 ? 16 : dtg_mt(p);
}

size_t dtg_gemm_lds(int mbw, int nbw) {
  return 2 * sizeof(float) * (size_t)(4 * 2 * mbw * 64 * 4 + DTG_KC * 2 * nbw * 64);
}

// Pack A_k for the forward GEMM (called at plan finalisation).
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
  for (int k = 0; k < g.q; ++k) {
    int64_t r = 0;
    for (int64_t j = 0; j < g.m; ++j) {
      drow[(size_t)k * g.m + j] = (int32_t)r;
      r += meta[(size_t)k * g.m + j].r1;
    }
  }
  // every stacked row a (column al of tensor j's U1) fills, for each voxel row
  // i1, the real-embedded rows 2 i1 (Re) and 2 i1 + 1 (Im) of its two k-steps
  // (a, Re part) and (a, Im part): A_emb = [[Ur, -Ui], [Ui, Ur]]; rows past n1
  // stay zero
  const int n1e = std::min(g.n1, nbtp * 16);
  auto for_rows = [&](auto&& put) {
    for (int64_t j = 0; j < g.m; ++j)
      for (int k = 0; k < g.q; ++k) {
        const int64_t t = k + (int64_t)g.q * j;
        const int r1 = meta[(size_t)k * g.m + j].r1;
        for (int al = 0; al < r1; ++al) {
          const int64_t a = drow[(size_t)k * g.m + j] + al;
          const double* u = &p->u1[2 * (p->u1_off[t] + (size_t)g.n1 * al)];
          for (int i1 = 0; i1 < n1e; ++i1) {
            const float ur = (float)u[2 * i1], ui = (float)u[2 * i1 + 1];
            const int mrow = 2 * i1, blk = mrow >> 5, l = mrow & 31;
            put(k, a, blk, l, 0, ur);        // (Re row, Re part)
            put(k, a, blk, l, 1, -ui);       // (Re row, Im part)
            put(k, a, blk, l + 1, 0, ui);    // (Im row, Re part)
            put(k, a, blk, l + 1, 1, ur);    // (Im row, Im part)
          }
        }
      }
  };
  if (p->precision == TV_PREC_BF16X3) {
    // hi/lo bf16 in the A-operand order of v_mfma_f32_32x32x16_bf16: chunk c
    // = 8 stacked rows, lane 32 h + row%32 holds k-slots e = 0..7 of rows
    // 8c + 4h + e/2, part e%2
    p->dtg_abfoff.assign(g.q + 1, 0);
    for (int k = 0; k < g.q; ++k)
      p->dtg_abfoff[k + 1] = p->dtg_abfoff[k] + p->dtg_rpad[k] / 8 * nbtp * 128;
    std::vector<uint4> abf((size_t)p->dtg_abfoff[g.q], make_uint4(0, 0, 0, 0));
    uint16_t* h16 = reinterpret_cast<uint16_t*>(abf.data());
    for_rows([&](int k, int64_t a, int blk, int l, int pp, float v) {
      const int64_t c = a >> 3;
      const int h = (int)((a >> 2) & 1), e = (int)(2 * (a & 3) + pp);
      const int64_t q4 = p->dtg_abfoff[k] + ((c * nbtp + blk) * 2) * 64 + 32 * h + l;
      const uint32_t hi = bf16_rne(v);
      h16[q4 * 8 + e] = (uint16_t)hi;
      h16[(q4 + 64) * 8 + e] = (uint16_t)bf16_rne(v - bf16_float(hi));
    });
    p->hp.abf = std::move(abf);
  } else {
    std::vector<float> a4((size_t)p->dtg_a4off[g.q], 0.f);
    for_rows([&](int k, int64_t a, int blk, int l, int pp, float v) {
      a4[p->dtg_a4off[k] + (a / 4) * nbtp * 256 + ((int64_t)blk * 64 + 32 * pp + l) * 4 + a % 4] = v;
    });
    p->hp.a4 = std::move(a4);
  }
  int64_t rp = 0;
  for (int k = 0; k < g.q; ++k) rp += p->dtg_rpad[k];
  p->dtg_rows = rp;

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
  return (int64_t)p->grid.q * (p->dtg_nbtp / dtg_mt(p)) * ((cols + 64 * nbw - 1) / (64 * nbw));
}

int64_t dtg_colgemm_tiles(const tv_plan_s* p, int nbw) {
  int64_t nt = 0;
  for (int k = 0; k < p->grid.q; ++k) nt += (p->sum_r1_k[k] + 64 * nbw - 1) / (64 * nbw);
  return nt * (p->dtg_nbtp / dtg_mt(p));
}

// the column-contraction adjoint: ypack floats per component, z complex per split
static int64_t col_ystride(const tv_plan_s* p, int s3) {
  const int64_t cols = (int64_t)p->grid.n2 * s3;
  return (cols + DTG_KC - 1) / DTG_KC * DTG_KC / 4 * p->dtg_nbtp * 256;
}
static int64_t col_zsplit(const tv_plan_s* p) { return p->dtg_rows * p->grid.n1; }

// column splits of the adjoint GEMM per slab of s3 values of i3: the
// configured count, raised so that no FP32 accumulation chain spans more than
// COL_CHAIN_STAGES LDS stages (2048 columns; the partials meet in FP64)
constexpr int COL_CHAIN_STAGES = 128;
int dtg_colgemm_splits(const tv_plan_s* p, int s3) {
  const int64_t nst = ((int64_t)p->grid.n2 * s3 + DTG_KC - 1) / DTG_KC;
  return (int)std::max<int64_t>(std::max(1, p->dtg_split_a),
                                (nst + COL_CHAIN_STAGES - 1) / COL_CHAIN_STAGES);
}

size_t dtg_workspace_bytes(const tv_plan_s* p, int op) {
  if (!dtg_supported(p)) return 0;
  const int s3 = std::min(op == 0 ? p->dtg_s3 : p->dtg_s3_a, p->grid.n3);
  const size_t b = (size_t)p->dtg_rows * dtg_nblocks(p, s3) * 64 * sizeof(float);
  if (op == 1) {
    const int64_t nslabs = (p->grid.n3 + s3 - 1) / s3;
    return b + (size_t)p->grid.q * col_ystride(p, s3) * sizeof(float) +
           (size_t)nslabs * dtg_colgemm_splits(p, s3) * col_zsplit(p) * sizeof(float2);
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
  const int MT = dtg_mt_op(p, 0);
  const bool bf16 = p->precision == TV_PREC_BF16X3;
  const int mbw = MT / 2, nbw = p->dtg_nbw;
  gemm_fn fn = bf16 ? gemm_pick_bf2(mbw, nbw) : gemm_pick(mbw, nbw);
  if (!fn) return set_error(TV_ERR_NOT_SUPPORTED, "no GEMM instance for this tile");
  if (bf16) {
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
  const size_t lds = bf16 ? bf2_lds(mbw, nbw) : dtg_gemm_lds(mbw, nbw);
  hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return hip_error(e, "hipFuncSetAttribute");
  const int t3w = dtg_t3w(p);
  D.t3w = t3w;
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

// Adjoint by the column contraction: per slab, the unscaled B_k (forward
// layout), y packed as the GEMM's A operand, the slab's partials of Y B^*;
// then the FP64 sum of all partials against conj(U1) per column.
static tv_status launch_dtg_colgemm_adjoint(const tv_plan_s* p, const float2* y, float2* x,
                                            void* ws, hipStream_t st) {
  const tv_grid& g = p->grid;
  const int s3 = std::min(p->dtg_s3_a, g.n3);
  const int64_t nbl = dtg_nblocks(p, s3);
  const int64_t ldb = nbl * 64;
  float* B = (float*)ws;
  const size_t bbytes = (size_t)p->dtg_rows * ldb * sizeof(float);
  const int64_t ystride = col_ystride(p, s3);
  float* yp = (float*)((char*)ws + bbytes);
  float2* z = (float2*)((char*)yp + (size_t)g.q * ystride * sizeof(float));
  const int S = dtg_colgemm_splits(p, s3);
  const int MT = dtg_mt_op(p, 1);
  const int mbw = MT / 2, nbw = p->dtg_nbw_a;
  const bool bf16 = p->precision == TV_PREC_BF16X3;
  colgemm_fn fn = bf16 ? colgemm_pick_bf2(mbw, nbw) : colgemm_pick(mbw, nbw);
  if (!fn) return set_error(TV_ERR_NOT_SUPPORTED, "no adjoint GEMM instance for this tile");

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

  YPackParams Y;
  Y.y = y;
  Y.yp = yp;
  Y.ystride = ystride;
  Y.nv = (int64_t)g.n1 * g.n2 * g.n3;
  Y.n1 = g.n1;
  Y.nbtp = p->dtg_nbtp;
  Y.q = g.q;

  ColGemmParams C;
  C.ypack = yp;
  C.B = B;
  C.z = z;
  C.ystride = ystride;
  C.zsplit = col_zsplit(p);
  C.ntb[0] = 0;
  const int ntile_rows = 64 * nbw;
  for (int k = 0; k < g.q; ++k) {
    C.brow[k] = D.brow[k];
    C.rk[k] = p->sum_r1_k[k];
    C.ntb[k + 1] = C.ntb[k] + (int)((p->sum_r1_k[k] + ntile_rows - 1) / ntile_rows);
  }
  C.q = g.q;
  C.nbtp = p->dtg_nbtp;
  C.mtiles = p->dtg_nbtp / MT;
  C.S = S;
  C.order = p->dtg_order_a;
  C.ldb = ldb;
  C.n1 = g.n1;
  C.vec4 = (g.n1 % 2 == 0) && ((uintptr_t)z % 16 == 0);
  C.nitems = (int64_t)C.mtiles * C.ntb[g.q] * S;
  const size_t lds = bf16 ? colgemm_bf2_lds(mbw, nbw) : colgemm_lds(mbw, nbw);
  e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_error(e, "hipFuncSetAttribute");

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
    const int64_t ncols = (int64_t)g.n2 * s3a;
    Y.col0 = (int64_t)g.n2 * i30;
    Y.ncols = ncols;
    Y.ngrp = (ncols + DTG_KC - 1) / DTG_KC * DTG_KC / 4;
    const int64_t yth = (int64_t)g.q * (bf16 ? Y.ngrp / 2 : Y.ngrp) * Y.nbtp * 64;
    hipLaunchKernelGGL(bf16 ? dtg_ypack_bf_kernel : dtg_ypack_kernel,
                       dim3((unsigned)((yth + 255) / 256)), dim3(256), 0, st, Y);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "adjoint operand packing launch");
    C.ncols = ncols;
    C.z = z + (int64_t)slab * S * C.zsplit;
    const int64_t grid = (C.nitems + 7) / 8 * 8;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(256), lds, st, C);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "adjoint column GEMM launch");
  }
  ColReduceParams R;
  R.meta = p->d_meta;
  R.drow = p->d_drow;
  R.u1t = p->d_u1t;
  R.z = z;
  R.x = x;
  for (int k = 0; k < g.q; ++k) R.brow[k] = D.brow[k];
  R.zsplit = C.zsplit;
  R.m = g.m;
  R.q = g.q;
  R.S = slab * S;
  R.n1 = g.n1;
  hipLaunchKernelGGL(dtg_colgemm_reduce_kernel, dim3((unsigned)g.m), dim3(256), 0, st, R);
  e = hipGetLastError();
  return e == hipSuccess ? TV_OK : hip_error(e, "adjoint reduction launch");
}

tv_status launch_dtg_adjoint(const tv_plan_s* p, const float2* y, float2* x, void* ws,
                             hipStream_t st) {
  if (!dtg_supported(p)) return set_error(TV_ERR_NOT_SUPPORTED, "decompress-then-GEMM not packed");
  return launch_dtg_colgemm_adjoint(p, y, x, ws, st);
}

}  // namespace tv
