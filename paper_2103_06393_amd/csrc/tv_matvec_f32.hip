// Fused Tucker-decompress-and-multiply kernels, FP32 on MFMA (gfx950).
//
// For component k the product Y^k = sum_j x_j Z^{kj}(:) (Algorithm 1) is the
// stacked GEMM Y^k_(1) = [U1_1 ... U1_m] [x_1 M_1; ...; x_m M_m], where
// Y^k_(1) is the n1 x (n2 n3) mode-1 unfolding and M_j = G_j x2 U2_j x3 U3_j
// unfolded along mode 1 (r1 x n2 n3), from eq. (6)/(7).  Each workgroup owns
// all n1 rows of a tile of t2 x t3 columns (i2, i3) and a contiguous range of
// columns j; per tensor it
//   S) stages the tile's U2 and U3 rows and the core into LDS as one batch of
//      independent loads, issued while the previous tensor's MFMAs run,
//   A) contracts the core with the tile's U3 rows (mode 3, eq. 7), scaling by
//      x_j: H[t3][a][b] = x_j sum_c G[a,b,c] U3[i3,c]            -> LDS
//   B) applies U2 per column (mode 2): B[a][(i2,i3)] = sum_b H U2[i2,b] -> LDS
//   C) accumulates the mode-1 product on v_mfma_f32_32x32x2f32 with the
//      complex product in real form: rows 2*i1 + {0,1} hold (Re, Im) of
//      output row i1, K step {0,1} carries (Re, Im) of B's row a, and the
//      A operand is [[Ar, -Ai], [Ai, Ar]] pre-packed in lane order; the next
//      four rows' A operands are in flight while four rows' MFMAs run.
// The adjoint (Algorithm 2) reuses A-C without the x_j scaling: it forms the
// tile of Z^{kj} = U1_j M_j, takes its conjugated dot product with the
// matching tile of y (held in registers) and writes one partial per
// (component, tile, column); a second kernel sums them in a fixed order.
//
// MFMA 32x32x2 f32 lane layout: A operand lane l = A[l%32][l/32], B operand
// lane l = B[l/32][l%32], accumulator register i of lane l =
// D[8*(i/4) + 4*(l/32) + i%4][l%32].
//
// BF16X3 form: every FP32 operand x is split into bf16 hi = rn(x) and
// lo = rn(x - hi) (round to nearest even) and the product is accumulated as
// hi*hi + hi*lo + lo*hi in FP32 on v_mfma_f32_32x32x16_bf16 (A operand lane l
// holds A[l%32][8(l/32) .. 8(l/32)+7], B operand lane l holds
// B[8(l/32) .. 8(l/32)+7][l%32]).  One MFMA K step of 16 carries 8 complex
// rows of B as (Re, Im) pairs; each tensor's rows are padded to a multiple
// of 8 with zeros.
#include "tv_internal.h"

namespace tv {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// float -> bf16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint32_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_to_float(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ v8bf as_v8bf(uint4 v) { return __builtin_bit_cast(v8bf, v); }

struct KParams {
  const TensorMeta* meta;
  const float2* cores;
  const float2* u2t;
  const float2* u3t;
  const float* apack;      // FP32 plans
  const uint4* apack_bf;   // BF16X3 plans: [chunk][blk][hi|lo][lane] 8 x bf16
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
  int r1max, r2max, r3max;
  int core_lds;          // core elements staged in LDS per pass
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

// LDS carve-up shared by host sizing and the kernel (float2 units, each
// region a multiple of 16 bytes).  r1 is padded to a multiple of 4 in H so
// that four consecutive rows are one 32-byte load.
__host__ __device__ inline int pad4(int r) { return (r + 3) & ~3; }
__host__ __device__ inline int pad8(int r) { return (r + 7) & ~7; }
__host__ __device__ inline int even(int n) { return (n + 1) & ~1; }
__host__ __device__ inline int lds_hs_elems(int t3, int r1, int r2) { return t3 * pad8(r1) * r2; }
__host__ __device__ inline int lds_u2_elems(int t2, int r2) { return even(t2 * r2); }
__host__ __device__ inline int lds_u3_elems(int t3, int r3) { return even(t3 * r3); }
__host__ __device__ inline int lds_gs_elems(int cb) { return even(cb + 8); }
__host__ __device__ inline int lds_bs_elems(int r1, int nwg) {
  return pad8(r1) * 2 * nwg;  // float (FP32) or 2 x bf16 (hi, lo)
}
constexpr int DOT_RING = 8;  // adjoint: tensors whose dots are reduced together
constexpr int CORE_LDS_MAX = 4096;  // complex core elements staged at a time

// Core elements staged per pass: every tensor's core if it fits, else
// whole mode-3 slices of at most CORE_LDS_MAX elements.
int core_lds_elems(const tv_plan_s* p) {
  const int64_t r12 = (int64_t)p->max_r12;
  return (int)std::max<int64_t>(r12, std::min<int64_t>(p->max_core, CORE_LDS_MAX));
}
size_t fused_lds_bytes(const tv_plan_s* p, const Tiling& T, bool adj) {
  const int r1 = p->max_r[0], r2 = p->max_r[1], r3 = p->max_r[2];
  size_t e = (size_t)lds_hs_elems(T.t3, r1, r2) + lds_u2_elems(T.t2, r2) +
             lds_u3_elems(T.t3, r3) + lds_gs_elems(core_lds_elems(p));
  size_t bytes = 8 * e + 4 * (size_t)lds_bs_elems(r1, T.nwg);
  if (adj) bytes += 8 * DOT_RING * 4 * 64;
  return bytes;
}

// Staging of one tensor's tile inputs as a single index space: the tile's U2
// rows (t2 x r2, contiguous in U2^T), its U3 rows (t3 x r3) and the first
// cc mode-3 slices of the core (r1 r2 cc), so that each thread keeps up to
// PF independent loads in flight (fewer in the adjoint, whose registers
// also hold the y tile).  Rows outside the grid are staged as zeros.
template <bool ADJ>
struct Prefetch {
  static constexpr int PF = ADJ ? 4 : 8;
};
struct StageSrc {
  const float2* u2;
  const float2* u3;
  const float2* g;
  int n2e, n3e, n0;   // U2 elements, U2 + U3 elements, total
  int lim2, lim3;     // valid U2 / U3 elements (rows inside the grid)
  int r2, cc;
};

__device__ __forceinline__ TensorMeta load_meta(const TensorMeta* m) {
  TensorMeta t = *m;
  t.r1 = __builtin_amdgcn_readfirstlane(t.r1);
  t.r2 = __builtin_amdgcn_readfirstlane(t.r2);
  t.r3 = __builtin_amdgcn_readfirstlane(t.r3);
  t.arow = __builtin_amdgcn_readfirstlane(t.arow);
  return t;
}

__device__ __forceinline__ StageSrc stage_src(const KParams& P, const TensorMeta& t, int T2,
                                              int t3, int i2_0, int i3_0) {
  StageSrc s;
  s.u2 = P.u2t + t.u2_off + (int64_t)i2_0 * t.r2;
  s.u3 = P.u3t + t.u3_off + (int64_t)i3_0 * t.r3;
  s.g = P.cores + t.g_off;
  const int r12 = t.r1 * t.r2;
  s.cc = max(1, min(t.r3, P.core_lds / r12));
  s.n2e = T2 * t.r2;
  s.n3e = s.n2e + t3 * t.r3;
  s.n0 = s.n3e + r12 * s.cc;
  s.lim2 = min(T2, P.n2 - i2_0) * t.r2;
  s.lim3 = s.n2e + min(t3, P.n3 - i3_0) * t.r3;
  s.r2 = t.r2;
  return s;
}

// Element e of the staging space: its address (elements past the end or
// outside the grid point at the core's first element) and whether it is
// live.  The address is formed with bit masks so that the loads of a batch
// issue back to back; dead elements are zeroed when they are stored.
__device__ __forceinline__ bool stage_ok(const StageSrc& s, int e) {
  // bitwise selection (a ternary chain here becomes an indexed stack load)
  const int m2 = -(int)(e < s.n2e), m3 = -(int)(e >= s.n2e && e < s.n3e);
  const int lim = (s.lim2 & m2) | (s.lim3 & m3) | (s.n0 & ~(m2 | m3));
  return e < lim;
}
__device__ __forceinline__ const float2* stage_addr(const StageSrc& s, int e) {
  const bool in2 = e < s.n2e, in3 = !in2 && e < s.n3e, ok = stage_ok(s, e);
  const uint64_t m2 = 0ull - (uint64_t)(in2 && ok);
  const uint64_t m3 = 0ull - (uint64_t)(in3 && ok);
  const uint64_t mg = 0ull - (uint64_t)(!in2 && !in3 && ok);
  const uint64_t a2 = (uint64_t)(s.u2 + e), a3 = (uint64_t)(s.u3 + (e - s.n2e));
  const uint64_t ag = (uint64_t)(s.g + (e - s.n3e)), a0 = (uint64_t)s.g;
  return reinterpret_cast<const float2*>((a2 & m2) | (a3 & m3) | (ag & mg) |
                                         (a0 & ~(m2 | m3 | mg)));
}
// a global-memory load (not a flat one, which would also count against the
// LDS wait counter)
__device__ __forceinline__ float2 stage_load(const StageSrc& s, int e) {
  typedef const __attribute__((address_space(1))) uint64_t* gptr;
  const uint64_t v = *(gptr)(uint64_t)stage_addr(s, e);
  return make_float2(__uint_as_float((uint32_t)v), __uint_as_float((uint32_t)(v >> 32)));
}

// U2 is stored b-major in LDS (U2s[b * t2 + i]) so that phase B reads
// consecutive i2 for one b
__device__ __forceinline__ void stage_store(const StageSrc& s, int e, float2 v, float2* U2s,
                                            float2* U3s, float2* Gs, int T2) {
  if (!stage_ok(s, e)) v = make_float2(0.f, 0.f);
  if (e < s.n2e) {
    const int i = e / s.r2, b = e - i * s.r2;
    U2s[b * T2 + i] = v;
  } else if (e < s.n3e) {
    U3s[e - s.n2e] = v;
  } else if (e < s.n0) {
    Gs[e - s.n3e] = v;
  }
}

// FP32 A operand rows a .. a+3 of a tensor (first stacked row arow); rows
// past r1 repeat row r1 - 1 (their MFMAs are skipped)
template <int NB>
__device__ __forceinline__ void load_arows(float (&dst)[4][NB], const float* apack, int64_t koff,
                                           int arow, int a, int r1, int nbt, int wm,
                                           int64_t rstride, int lane) {
  const float* base = apack + koff + ((int64_t)arow * nbt + wm * NB) * 64 + lane;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int aa = min(a + e, r1 - 1);
#pragma unroll
    for (int b = 0; b < NB; ++b) dst[e][b] = base[aa * rstride + b * 64];
  }
}

// Adjoint: sum the per-lane dot products of tensors [j0, j0 + cnt) (ring
// slots (j - jb) % DOT_RING) over the 4 waves and 64 lanes in a fixed order
// and write one partial per tensor.
__device__ __forceinline__ void flush_dots(const float2* dots, int cnt, int jb, int j0,
                                           float2* out, int64_t base) {
  const int tid = threadIdx.x;
  const int slot_i = tid >> 5, part = tid & 31;
  float sr = 0.f, si = 0.f;
  if (slot_i < cnt) {
    const int slot = (j0 + slot_i - jb) % DOT_RING;
    const float2* d = dots + slot * 256;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const float2 a = d[w * 64 + part], b = d[w * 64 + 32 + part];
      sr += a.x;
      si += a.y;
      sr += b.x;
      si += b.y;
    }
  }
#pragma unroll
  for (int off = 16; off >= 1; off >>= 1) {
    sr += __shfl_xor(sr, off);
    si += __shfl_xor(si, off);
  }
  if (slot_i < cnt && part == 0) out[base + j0 + slot_i] = make_float2(sr, si);
}

template <int NB, int WN, bool ADJ, bool BF>
__global__ __launch_bounds__(256) void fused_f32(KParams P) {
  extern __shared__ float4 smem4[];
  constexpr int NWG = 32 * WN;
  constexpr int NP = NWG / 2;  // column pairs per tile
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
  float2* U3s = U2s + lds_u2_elems(T2, P.r2max);
  float2* Gs = U3s + lds_u3_elems(P.t3, P.r3max);
  float* Bs = reinterpret_cast<float*>(Gs + lds_gs_elems(P.core_lds));
  float2* dots = reinterpret_cast<float2*>(Bs + lds_bs_elems(P.r1max, NWG));

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
  const int64_t pbase = ((int64_t)k * P.tiles + tile) * P.m;
  const int64_t koff = P.apack_koff[k];
  const int64_t rstride = (int64_t)P.nbt * 64;
  int flushed = jb;
  TensorMeta tn;
  if (jb < je) tn = load_meta(meta + jb);

  // staging of tensor jb, then in every iteration of tensor j + 1 while
  // tensor j's mode-1 product runs
  constexpr int PF = Prefetch<ADJ>::PF;
  float2 pf[PF];
  StageSrc ss;
  if (jb < je) {
    ss = stage_src(P, tn, T2, P.t3, i2_0, i3_0);
#pragma unroll
    for (int u = 0; u < PF; ++u) pf[u] = stage_load(ss, tid + 256 * u);
  }
  // FP32: the first four A operand rows of the current tensor
  float an[4][NB];
  if (!BF && jb < je) load_arows<NB>(an, P.apack, koff, tn.arow, 0, tn.r1, P.nbt, wm, rstride, lane);

  for (int j = jb; j < je; ++j) {
    const TensorMeta t = tn;
    const StageSrc sc = ss;
    if (j + 1 < je) tn = load_meta(meta + j + 1);
    const int r1 = t.r1, r2 = t.r2, r3 = t.r3;
    const int r1p = BF ? pad8(r1) : pad4(r1), r1q = r1p >> 2;
    const int r12 = r1 * r2;
    const float2 xj = ADJ ? make_float2(1.f, 0.f) : P.vec[j];

    // U2 rows, U3 rows and the first core chunk: registers -> LDS, then any
    // elements past the prefetched PF * 256
#pragma unroll
    for (int u = 0; u < PF; ++u) stage_store(sc, tid + 256 * u, pf[u], U2s, U3s, Gs, T2);
    for (int e0 = PF * 256; e0 < sc.n0; e0 += 1024) {
      float2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = stage_load(sc, e0 + tid + 256 * u);
#pragma unroll
      for (int u = 0; u < 4; ++u) stage_store(sc, e0 + tid + 256 * u, v[u], U2s, U3s, Gs, T2);
    }
    __syncthreads();

    // A) mode-3 contraction of the core with the tile's U3 rows, four rows a
    //    per task: H[t3][b][a] = x_j sum_c G[a,b,c] U3[i3,c]; cores larger
    //    than the LDS chunk are swept in chunks of cc mode-3 slices
    const int nch = (r3 + sc.cc - 1) / sc.cc;
    for (int ch = 0; ch < nch; ++ch) {
      const int c0 = ch * sc.cc, c1 = min(r3, c0 + sc.cc);
      if (ch > 0) {
        __syncthreads();
        const float2* gsrc = P.cores + t.g_off + (int64_t)r12 * c0;
        const int ne = r12 * (c1 - c0);
        for (int e0 = 0; e0 < ne; e0 += 1024) {
          float2 v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e = e0 + tid + 256 * u;
            v[u] = gsrc[e < ne ? e : 0];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (e0 + tid + 256 * u < ne) Gs[e0 + tid + 256 * u] = v[u];
        }
        __syncthreads();
      }
      for (int task = tid; task < P.t3 * r2 * r1q; task += 256) {
        const int a4 = task % r1q, rest = task / r1q;
        const int b = rest % r2, t3 = rest / r2;
        const int ne = min(4, r1 - 4 * a4);
        float2* dst = Hs + (t3 * r2 + b) * r1p + 4 * a4;
        float2 h[4];
        if (ch == 0) {
#pragma unroll
          for (int e = 0; e < 4; ++e) h[e] = make_float2(0.f, 0.f);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) h[e] = dst[e];
        }
        const float2* g = Gs + 4 * a4 + r1 * b;
        const float2* u3 = U3s + t3 * r3;
        for (int c = c0; c < c1; ++c) {
          const float2 u = u3[c];
          const float2* gc = g + r12 * (c - c0);
#pragma unroll
          for (int e = 0; e < 4; ++e) h[e] = cfma(gc[e], u, h[e]);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (!ADJ && ch == nch - 1) h[e] = cmul(xj, h[e]);
          if (e >= ne) h[e] = make_float2(0.f, 0.f);  // rows past r1 read other data
        }
        *reinterpret_cast<float4*>(dst) = make_float4(h[0].x, h[0].y, h[1].x, h[1].y);
        *reinterpret_cast<float4*>(dst + 2) = make_float4(h[2].x, h[2].y, h[3].x, h[3].y);
      }
    }
    __syncthreads();

    // B) mode-2 product per column pair into the MFMA B tile, 4 rows a x 2
    //    columns per task: B[a][n] = sum_b H[t3(n)][b][a] U2[i2(n), b]
    for (int task = tid; task < r1q * NP; task += 256) {
      const int np = task % NP, a4 = task / NP;
      const int n = 2 * np;
      const int t2n = n % T2, t3n = n / T2;
      const float2* hb = Hs + (t3n * r2) * r1p + 4 * a4;
      const float2* ub = U2s + t2n;
      float2 v[4][2];
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e][0] = v[e][1] = make_float2(0.f, 0.f);
      for (int b = 0; b < r2; ++b) {
        const float4 h01 = *reinterpret_cast<const float4*>(hb + b * r1p);
        const float4 h23 = *reinterpret_cast<const float4*>(hb + b * r1p + 2);
        const float4 uu = *reinterpret_cast<const float4*>(ub + b * T2);
        const float2 u0 = make_float2(uu.x, uu.y), u1 = make_float2(uu.z, uu.w);
        const float2 hh[4] = {make_float2(h01.x, h01.y), make_float2(h01.z, h01.w),
                              make_float2(h23.x, h23.y), make_float2(h23.z, h23.w)};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          v[e][0] = cfma(hh[e], u0, v[e][0]);
          v[e][1] = cfma(hh[e], u1, v[e][1]);
        }
      }
      if (BF) {
        // rows 4 a4 .. 4 a4 + 3 are half (a4 & 1) of 8-row chunk a4 / 2: one
        // 16-byte vector of 8 bf16 (Re, Im of 4 rows) per column, hi and lo
        uint4* bh = reinterpret_cast<uint4*>(Bs);
        uint4* bl = bh + (size_t)(r1p / 8) * 2 * NWG;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          uint32_t h[8], l[8];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float re = c ? v[e][1].x : v[e][0].x, im = c ? v[e][1].y : v[e][0].y;
            h[2 * e] = bf16_rne(re);
            h[2 * e + 1] = bf16_rne(im);
            l[2 * e] = bf16_rne(re - bf16_to_float(h[2 * e]));
            l[2 * e + 1] = bf16_rne(im - bf16_to_float(h[2 * e + 1]));
          }
          const size_t at = (size_t)((a4 >> 1) * 2 + (a4 & 1)) * NWG + n + c;
          bh[at] = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16),
                              h[6] | (h[7] << 16));
          bl[at] = make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16),
                              l[6] | (l[7] << 16));
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int a = 4 * a4 + e;
          if (a < r1) {
            *reinterpret_cast<float2*>(Bs + (2 * a) * NWG + n) =
                make_float2(v[e][0].x, v[e][1].x);
            *reinterpret_cast<float2*>(Bs + (2 * a + 1) * NWG + n) =
                make_float2(v[e][0].y, v[e][1].y);
          }
        }
      }
    }
    // loads for the next tensor's staging, in flight during this tensor's
    // mode-1 product
    if (j + 1 < je) {
      ss = stage_src(P, tn, T2, P.t3, i2_0, i3_0);
#pragma unroll
      for (int u = 0; u < PF; ++u) pf[u] = stage_load(ss, tid + 256 * u);
    }
    __syncthreads();

    // adjoint: reduce the dots of the last DOT_RING tensors (their per-lane
    // values were written before the barrier above)
    if (ADJ && j - flushed == DOT_RING) {
      flush_dots(dots, DOT_RING, jb, flushed, P.out, pbase);
      flushed += DOT_RING;
      __syncthreads();  // the ring slots are rewritten below
    }

    // C) stacked mode-1 product on MFMA
    if (ADJ) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[b][i] = 0.f;
    }
    if (BF) {
      // t.arow counts 8-row chunks; A chunk layout [chunk][blk][hi|lo][lane]
      const uint4* Ach = P.apack_bf + P.apack_koff[k] +
                         ((int64_t)t.arow * P.nbt + wm * NB) * 128 + lane;
      const uint4* bh = reinterpret_cast<const uint4*>(Bs) + (lane >> 5) * NWG + wn * 32 +
                        (lane & 31);
      const uint4* bl = bh + (size_t)(r1p / 8) * 2 * NWG;
      for (int c = 0; c < r1p / 8; ++c) {
        const v8bf Bh = as_v8bf(bh[(size_t)c * 2 * NWG]);
        const v8bf Bl = as_v8bf(bl[(size_t)c * 2 * NWG]);
        const uint4* ap = Ach + (int64_t)c * P.nbt * 128;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const v8bf Ah = as_v8bf(ap[b * 128]);
          const v8bf Al = as_v8bf(ap[b * 128 + 64]);
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bh, acc[b], 0, 0, 0);
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bl, acc[b], 0, 0, 0);
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Al, Bh, acc[b], 0, 0, 0);
        }
      }
    } else {
      // rows in groups of four; the next group's A operand (or the next
      // tensor's first group) is loaded while the current group's MFMAs run
      const float* Brow = Bs + (lane >> 5) * NWG + wn * 32 + (lane & 31);
      for (int a0 = 0; a0 < r1; a0 += 4) {
        float ac[4][NB], bc[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          bc[e] = Brow[2 * min(a0 + e, r1 - 1) * NWG];
#pragma unroll
          for (int b = 0; b < NB; ++b) ac[e][b] = an[e][b];
        }
        if (a0 + 4 < r1)
          load_arows<NB>(an, P.apack, koff, t.arow, a0 + 4, r1, P.nbt, wm, rstride, lane);
        else if (j + 1 < je)
          load_arows<NB>(an, P.apack, koff, tn.arow, 0, tn.r1, P.nbt, wm, rstride, lane);
        const int ne = min(4, r1 - a0);
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (e < ne) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
              acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ac[e][b], bc[e], acc[b], 0, 0, 0);
          }
      }
    }

    if (ADJ) {
      // conjugated dot product of the Z^{kj} tile with the y tile, per lane
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
      dots[((j - jb) % DOT_RING) * 256 + wave * 64 + lane] = make_float2(dr, di);
    }
  }

  if (ADJ) {
    __syncthreads();
    if (je > flushed) flush_dots(dots, je - flushed, jb, flushed, P.out, pbase);
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

// x[j] = sum over r < rows of partial[r * m + j], in a fixed order: each of
// the 8 row groups of a block sums its strided rows in sequence (FP64), then
// the groups are added in index order.
__global__ __launch_bounds__(256) void reduce_adjoint_kernel(const float2* __restrict__ partial,
                                                             int64_t rows, int64_t m,
                                                             float2* __restrict__ x) {
  __shared__ double2 red[8][32];
  const int jl = threadIdx.x % 32, g = threadIdx.x / 32;
  const int64_t j = (int64_t)blockIdx.x * 32 + jl;
  double sr = 0.0, si = 0.0;
  if (j < m) {
    int64_t r = g;
    for (; r + 24 < rows; r += 32) {  // four independent loads in flight
      const float2 v0 = partial[r * m + j], v1 = partial[(r + 8) * m + j];
      const float2 v2 = partial[(r + 16) * m + j], v3 = partial[(r + 24) * m + j];
      sr += v0.x; si += v0.y;
      sr += v1.x; si += v1.y;
      sr += v2.x; si += v2.y;
      sr += v3.x; si += v3.y;
    }
    for (; r < rows; r += 8) {
      const float2 v = partial[r * m + j];
      sr += v.x;
      si += v.y;
    }
  }
  red[g][jl] = make_double2(sr, si);
  __syncthreads();
  if (g == 0 && j < m) {
    double2 t = red[0][jl];
    for (int q = 1; q < 8; ++q) {
      t.x += red[q][jl].x;
      t.y += red[q][jl].y;
    }
    x[j] = make_float2((float)t.x, (float)t.y);
  }
}

typedef void (*fused_fn)(KParams);

template <bool ADJ, bool BF>
static fused_fn pick(int nb, int wn) {
#define TV_CASE(NB)                                                          \
  case NB:                                                                   \
    return wn == 4 ? fused_f32<NB, 4, ADJ, BF>                               \
                   : (wn == 2 ? fused_f32<NB, 2, ADJ, BF> : fused_f32<NB, 1, ADJ, BF>);
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
  const Tiling& T = adj ? p->tiling_a : p->tiling;
  KParams P;
  P.meta = p->d_meta;
  P.cores = p->d_cores;
  P.u2t = p->d_u2t;
  P.u3t = p->d_u3t;
  P.apack = p->d_apack;
  P.apack_bf = p->d_apack_bf;
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
  P.nbt = p->nbt_pack;
  P.t2 = T.t2;
  P.t3 = T.t3;
  P.tiles2 = T.tiles2;
  P.tiles = T.tiles;
  P.S = split;
  P.nitems = (int64_t)p->grid.q * split * T.tiles;
  P.r1max = p->max_r[0];
  P.r2max = p->max_r[1];
  P.r3max = p->max_r[2];
  P.core_lds = core_lds_elems(p);
  P.vec4 = (p->grid.n1 % 2 == 0) && ((uintptr_t)out % 16 == 0) && (out_stride % 2 == 0);
  const bool bf = p->precision == TV_PREC_BF16X3;
  fused_fn fn = adj ? (bf ? pick<true, true>(T.nb, T.wn) : pick<true, false>(T.nb, T.wn))
                    : (bf ? pick<false, true>(T.nb, T.wn) : pick<false, false>(T.nb, T.wn));
  if (!fn) return set_error(TV_ERR_NOT_SUPPORTED, "no kernel instance for this tiling");
  const size_t lds = fused_lds_bytes(p, T, adj);
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
  if (p->kernel_ws[0] && ws_supported(p, p->tiling, false))
    return launch_fused_ws(p, false, x, out, split, d_split, out_stride, st);
  return launch_fused(p, false, x, out, split, d_split, out_stride, st);
}

tv_status launch_adjoint_f32(const tv_plan_s* p, const float2* y, float2* partial, int split,
                             const int32_t* d_split, hipStream_t st) {
  if (p->kernel_ws[1] && ws_supported(p, p->tiling_a, true))
    return launch_fused_ws(p, true, y, partial, split, d_split, 0, st);
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
  const int64_t blocks = (m + 31) / 32;
  hipLaunchKernelGGL(reduce_adjoint_kernel, dim3((unsigned)blocks), dim3(256), 0, st, partial,
                     (int64_t)q * tiles, m, x);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TV_OK : hip_error(e, "reduce_adjoint launch");
}

}  // namespace tv
