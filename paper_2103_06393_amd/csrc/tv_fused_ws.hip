// Warp-specialised fused Tucker-decompress-and-multiply kernels (gfx950).
//
// Same contraction as the phased kernels (the stacked mode-1 GEMM of
// Algorithm 1, Y^k_(1) = [U1_1 ... U1_m] [x_1 M_1; ...; x_m M_m], and the
// per-tensor inner products of Algorithm 2), as a three-stage pipeline over
// the workgroup's columns j with one workgroup barrier per step:
//
//   producer waves (4), step s: stage the tile's U2 / U3 rows and the core of
//     tensor s into LDS (loads in flight while they compute), and contract
//     the core of tensor s - 1 with the tile's U3 rows (mode 3, eq. 7, scaled
//     by x_j) into H;
//   consumer waves (4), step s: apply U2 to H for tensor s - 2 (mode 2, on
//     16x16x4 MFMAs, 16 columns per task) into the shared B tile of that
//     tensor, and run tensor s - 3's mode-1 product on MFMA from the B tile
//     built one step earlier, the A operand (stacked U1) streaming from L2
//     one group of rows ahead.
//
// A single wave issues VALU work at a fraction of a SIMD's rate, so the
// mode-2 work (the largest VALU term) sits with the consumers, whose MFMAs
// leave the VALU idle, and the producers keep the loads and the mode-3
// contraction.  Staging is triple-buffered for U2 and double-buffered for
// the core and U3; H and the B tile are double-buffered.  In the adjoint the consumers also
// form the conjugated dot of the decompressed tile with the y tile held in
// registers, and a producer wave reduces those per-lane dots one step later.
//
// MFMA lane layouts are those of the phased kernels: 32x32x2 f32 A operand
// lane l = A[l%32][l/32], B operand lane l = B[l/32][l%32], accumulator
// register i of lane l = D[8(i/4) + 4(l/32) + i%4][l%32]; the BF16X3 form
// accumulates hi*hi + hi*lo + lo*hi on v_mfma_f32_32x32x16_bf16.
#include <algorithm>

#include "tv_internal.h"

namespace tv {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

struct WsParams {
  const TensorMeta* meta;
  const float2* cores;
  const float2* u2t;
  const float2* u3t;
  const float* apack;
  const uint4* apack_bf;
  const int64_t* apack_koff;
  const int32_t* split;  // [q][S+1] first column of each split
  const float2* vec;     // x (forward) or one column of y (adjoint)
  float2* out;           // forward: y or its split partials; adjoint: partials
  int64_t out_stride;
  int64_t m;
  int64_t nv;
  int n1, n2, n3;
  int nbt, t2, t3, tiles2;
  int64_t tiles;
  int S;
  int64_t nitems;
  int r1max, r2max, r3max;
  int cb;    // largest core staged in LDS (complex elements); larger ones stream
  int vec4;  // forward output may use 16-byte stores
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
__device__ __forceinline__ uint32_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_to_float(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ v8bf as_v8bf(uint4 v) { return __builtin_bit_cast(v8bf, v); }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// the ranks and stacked row are wave-uniform: moved to scalar registers
__device__ __forceinline__ TensorMeta uniform_meta(TensorMeta t) {
  t.r1 = __builtin_amdgcn_readfirstlane(t.r1);
  t.r2 = __builtin_amdgcn_readfirstlane(t.r2);
  t.r3 = __builtin_amdgcn_readfirstlane(t.r3);
  t.arow = __builtin_amdgcn_readfirstlane(t.arow);
  return t;
}

// a 64-bit global-memory load of one complex value (not a flat load, which
// would also count against the LDS wait counter)
__device__ __forceinline__ float2 gload(const float2* p) {
  typedef const __attribute__((address_space(1))) uint64_t* gptr;
  const uint64_t v = *(gptr)(uint64_t)p;
  return make_float2(__uint_as_float((uint32_t)v), __uint_as_float((uint32_t)(v >> 32)));
}

}  // namespace

// ---- LDS carve-up (float2 units; every region a multiple of 16 bytes) ----
// Tensor metadata and x_j of the workgroup's columns pass through an LDS ring
// of WS_META_RING entries, refilled WS_META_RING / 2 at a time one step
// before use, so that no wave waits on a metadata load inside the loop.
constexpr int WS_META_RING = 128;
__host__ __device__ inline int ws_pad4(int r) { return (r + 3) & ~3; }
__host__ __device__ inline int ws_pad8(int r) { return (r + 7) & ~7; }
__host__ __device__ inline int ws_even(int n) { return (n + 1) & ~1; }
// one B tile: pad8(r1) rows x 2 (Re, Im) x nwg columns floats (BF16: hi and
// lo bf16)
__host__ __device__ inline int ws_b_elems(int r1max, int nwg) { return ws_pad8(r1max) * nwg; }
// staging: U2 tile rows (b-major), t2 x r2; U3 tile rows t3 x r3 then core
__host__ __device__ inline int ws_u2_elems(int t2, int r2max) { return ws_even(t2 * r2max); }
__host__ __device__ inline int ws_cu_elems(int t3, int r3max, int cb) {
  return ws_even(t3 * r3max) + ws_even(cb);
}
// H for the tile's t3 rows: [t3][b][a], a padded to a multiple of 8
__host__ __device__ inline int ws_h_elems(int t3, int r1max, int r2max) {
  return t3 * ws_pad8(r1max) * r2max;
}

size_t ws_lds_bytes(const tv_plan_s* p, const Tiling& T, bool adj, int cb) {
  const int r1 = p->max_r[0], r2 = p->max_r[1], r3 = p->max_r[2];
  size_t e = 2 * (size_t)ws_b_elems(r1, T.nwg) + 3 * (size_t)ws_u2_elems(T.t2, r2) +
             2 * (size_t)ws_cu_elems(T.t3, r3, cb) + 2 * (size_t)ws_h_elems(T.t3, r1, r2) +
             (adj ? 2 * 256 : 0);
  return 8 * e + WS_META_RING * (sizeof(TensorMeta) + sizeof(float2));
}

namespace {

// FP32 A operand rows a .. a+3 of a tensor (first stacked row arow); rows
// past r1 repeat row r1 - 1 (their MFMAs are skipped)
template <int NB>
__device__ __forceinline__ void load_arows(float (&dst)[4][NB], const float* base, int arow,
                                           int a, int r1, int nbt, int64_t rstride) {
  const float* p = base + (int64_t)arow * nbt * 64;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int aa = min(a + e, r1 - 1);
#pragma unroll
    for (int b = 0; b < NB; ++b) dst[e][b] = p[aa * rstride + b * 64];
  }
}

// Mode-3 contraction on the producer threads: H[t3][b][a] = x_j sum_c
// G[a,b,c] U3[i3,c], one row a per task so that all producer waves share
// the work (rows r1 <= a < r1p are zeros); the loads of four mode-3 slices
// are issued together.  G is the staged core in LDS or the core in global
// memory (two instances).
template <bool ADJ>
__device__ __forceinline__ void mode3(const float2* G, const float2* U3s, float2* H, int r1,
                                      int r1p, int r2, int r3, int t3n, float2 xj, int ptid) {
  const int r12 = r1 * r2;
  for (int task = ptid; task < t3n * r2 * r1p; task += 256) {
    const int row = task / r1p, a = task - row * r1p;  // row = t3 * r2 + b
    const int t3 = row / r2, b = row - t3 * r2;
    const float2* g = G + min(a, r1 - 1) + r1 * b;
    const float2* u3 = U3s + t3 * r3;
    float2 h = make_float2(0.f, 0.f);
    for (int c0 = 0; c0 < r3; c0 += 4) {
      float2 gv[4], uv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = min(c0 + q, r3 - 1);
        gv[q] = g[(int64_t)c * r12];
        uv[q] = c0 + q < r3 ? u3[c] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) h = cfma(gv[q], uv[q], h);
    }
    if (!ADJ) h = cmul(xj, h);
    H[task] = a < r1 ? h : make_float2(0.f, 0.f);
  }
}

// Staging of one tensor on a tile by the 256 producer threads: the tile's
// U2 rows (t2 x r2, contiguous in U2^T, stored b-major), its U3 rows
// (t3 x r3) and, if it fits, the core.  Rows outside the grid are clamped to
// the last valid row (finite values in columns that are never stored).
constexpr int SU2 = 4, SU3 = 1, SCO = 6;  // register slots per thread and segment
struct Stage {
  float2 u2[SU2], u3[SU3], co[SCO];
};

__device__ __forceinline__ void stage_issue(Stage& S, const WsParams& P, const TensorMeta& t,
                                            int i2_0, int i3_0, int ptid) {
  const float2* u2 = P.u2t + t.u2_off + (int64_t)i2_0 * t.r2;
  const float2* u3 = P.u3t + t.u3_off + (int64_t)i3_0 * t.r3;
  const float2* g = P.cores + t.g_off;
  const int lim2 = min(P.t2, P.n2 - i2_0) * t.r2 - 1;
  const int lim3 = min(P.t3, P.n3 - i3_0) * t.r3 - 1;
  const int core = t.r1 * t.r2 * t.r3;
  const int limg = (core <= P.cb ? core : 1) - 1;
#pragma unroll
  for (int u = 0; u < SU2; ++u) S.u2[u] = gload(u2 + min(ptid + 256 * u, lim2));
#pragma unroll
  for (int u = 0; u < SU3; ++u) S.u3[u] = gload(u3 + min(ptid + 256 * u, lim3));
#pragma unroll
  for (int u = 0; u < SCO; ++u) S.co[u] = gload(g + min(ptid + 256 * u, limg));
}

// stores the registers, then loads and stores whatever did not fit in them
__device__ __forceinline__ void stage_commit(const Stage& S, const WsParams& P,
                                             const TensorMeta& t, int i2_0, int i3_0, int ptid,
                                             float2* U2s, float2* U3s, float2* Gs) {
  const int r2 = t.r2, n2e = P.t2 * r2, n3e = P.t3 * t.r3;
  const int core = t.r1 * t.r2 * t.r3;
  const int nge = core <= P.cb ? core : 0;
  const int T2 = P.t2;
  // U2 element e = i * r2 + b lands at U2s[b * t2 + i]
  int si = ptid / r2, sb = ptid - si * r2;
  const int q256 = 256 / r2, m256 = 256 - q256 * r2;
#pragma unroll
  for (int u = 0; u < SU2; ++u) {
    if (ptid + 256 * u < n2e) U2s[sb * T2 + si] = S.u2[u];
    si += q256;
    sb += m256;
    if (sb >= r2) {
      sb -= r2;
      ++si;
    }
  }
#pragma unroll
  for (int u = 0; u < SU3; ++u)
    if (ptid + 256 * u < n3e) U3s[ptid + 256 * u] = S.u3[u];
#pragma unroll
  for (int u = 0; u < SCO; ++u)
    if (ptid + 256 * u < nge) Gs[ptid + 256 * u] = S.co[u];
  // overflow of the register slots (large tiles or cores)
  if (n2e > SU2 * 256 || n3e > SU3 * 256 || nge > SCO * 256) {
    const float2* u2 = P.u2t + t.u2_off + (int64_t)i2_0 * r2;
    const float2* u3 = P.u3t + t.u3_off + (int64_t)i3_0 * t.r3;
    const float2* g = P.cores + t.g_off;
    const int lim2 = min(P.t2, P.n2 - i2_0) * r2 - 1;
    const int lim3 = min(P.t3, P.n3 - i3_0) * t.r3 - 1;
    for (int e = SU2 * 256 + ptid; e < n2e; e += 256) {
      const int i = e / r2;
      U2s[(e - i * r2) * T2 + i] = gload(u2 + min(e, lim2));
    }
    for (int e = SU3 * 256 + ptid; e < n3e; e += 256) U3s[e] = gload(u3 + min(e, lim3));
    for (int e = SCO * 256 + ptid; e < nge; e += 256) Gs[e] = gload(g + e);
  }
}

// Two workgroups per CU (four waves per SIMD, 128 registers) where the
// accumulators allow it.
template <int NB, bool ADJ>
struct WsOccupancy {
  static constexpr int waves = (NB > 4 || (ADJ && NB > 2)) ? 2 : 4;
};

template <int NB, int WN, bool ADJ, bool BF>
__global__ __launch_bounds__(512)
__attribute__((amdgpu_waves_per_eu(WsOccupancy<NB, ADJ>::waves))) void ws_fused(WsParams P) {
  extern __shared__ float4 smem4[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool consumer = wave < 4;

  const int64_t G8 = gridDim.x / 8;
  const int64_t item = (int64_t)(blockIdx.x % 8) * G8 + blockIdx.x / 8;
  if (item >= P.nitems) return;
  const int64_t tile = item % P.tiles;
  const int64_t ks = item / P.tiles;
  const int s = (int)(ks % P.S);
  const int k = (int)(ks / P.S);
  const int T2 = P.t2;
  const int i2_0 = (int)(tile % P.tiles2) * T2;
  const int i3_0 = (int)(tile / P.tiles2) * P.t3;
  const int jb = P.split[k * (P.S + 1) + s];
  const int je = P.split[k * (P.S + 1) + s + 1];
  const int cnt = je - jb;
  const TensorMeta* meta = P.meta + (int64_t)k * P.m + jb;

  constexpr int NWG = 32 * WN;
  const int be = ws_b_elems(P.r1max, NWG);
  const int u2e = ws_u2_elems(T2, P.r2max);
  const int u3e = ws_even(P.t3 * P.r3max);
  const int cue = ws_cu_elems(P.t3, P.r3max, P.cb);
  const int he = ws_h_elems(P.t3, P.r1max, P.r2max);
  float2* Bbuf = reinterpret_cast<float2*>(smem4);
  float2* U2buf = Bbuf + 2 * be;
  float2* CUbuf = U2buf + 3 * u2e;
  float2* Hbuf = CUbuf + 2 * cue;
  float2* dots = Hbuf + 2 * he;
  float2* XL = dots + (ADJ ? 2 * 256 : 0);
  TensorMeta* ML = reinterpret_cast<TensorMeta*>(XL + WS_META_RING);
  constexpr int HALF = WS_META_RING / 2;

  // first refill of the metadata ring, by producer threads
  if (tid >= 256 && tid - 256 < min(cnt, HALF)) {
    const int e = tid - 256;
    ML[e] = meta[e];
    XL[e] = ADJ ? make_float2(1.f, 0.f) : P.vec[jb + e];
  }
  __syncthreads();

  if (consumer) {
    // ------------------------------------------------------------ consumer
    const int wm = wave / WN, wn = wave % WN;
    const int ncol = wn * 32 + (lane & 31);
    const int t2n = ncol % T2, t3n = ncol / T2;  // the wave's 32 columns share t3n
    const int i2 = i2_0 + t2n, i3 = i3_0 + t3n;
    const bool colok = (i2 < P.n2) && (i3 < P.n3);
    const int64_t fibre = (int64_t)k * P.nv + (int64_t)P.n1 * (i2 + (int64_t)P.n2 * i3);
    const int64_t rstride = (int64_t)P.nbt * 64;
    const float* abase = P.apack + P.apack_koff[k] + wm * NB * 64 + lane;

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
          const int i1 = ((wm * NB + b) * 32 + 8 * g + 4 * (lane >> 5)) >> 1;
          float2 v0 = make_float2(0.f, 0.f), v1 = v0;
          if (colok && i1 < P.n1) v0 = P.vec[fibre + i1];
          if (colok && i1 + 1 < P.n1) v1 = P.vec[fibre + i1 + 1];
          yv[ADJ ? b : 0][4 * g + 0] = v0.x;
          yv[ADJ ? b : 0][4 * g + 1] = v0.y;
          yv[ADJ ? b : 0][4 * g + 2] = v1.x;
          yv[ADJ ? b : 0][4 * g + 3] = v1.y;
        }
    }
    float an[4][NB];
    TensorMeta tc;
    if (cnt > 0) {
      tc = uniform_meta(ML[0]);
      if constexpr (!BF) load_arows<NB>(an, abase, tc.arow, 0, tc.r1, P.nbt, rstride);
    }
    const int half = lane >> 5, cl = lane & 31;
    for (int st = 0; st < cnt + 4; ++st) {
      // B) mode 2 of tensor tb = st - 2 into its B tile, 16 columns per
      //    task on v_mfma_f32_16x16x4f32 (A lane l = A[l%16][l/16], B lane
      //    l = B[l/16][l%16], D register r of lane l = D[4(l/16)+r][l%16]):
      //    B[2a+s][n] = sum_b Hemb[2a+s][2b+t] U2emb[2b+t][n], two b per
      //    instruction, Hemb = [[Re H, -Im H], [Im H, Re H]] per (a, b) and
      //    U2emb the real / imaginary parts of U2[i2(n), b]
      const int tb = st - 2;
      if (tb >= 0 && tb < cnt) {
        const TensorMeta mbt = uniform_meta(ML[tb % WS_META_RING]);
        const int r1 = mbt.r1, r2 = mbt.r2;
        const int r1p = BF ? ws_pad8(r1) : ws_pad4(r1);
        const float2* Hb = Hbuf + (tb & 1) * he;
        const float2* U2b = U2buf + (tb % 3) * u2e;
        float2* Bt = Bbuf + (tb & 1) * be;
        const int m16 = lane & 15, k4 = lane >> 4;  // A row / B column, K index
        const int sa = m16 & 1, ta = k4 & 1, bq = k4 >> 1;
        // Hemb entry as Re H * cx + Im H * cy with per-lane constants: a
        // select between the loaded parts is compiled into a branch with a
        // one-float LDS read and a full wait per operand
        const float cx = sa == ta ? 1.f : 0.f;
        const float cy = sa == ta ? 0.f : (sa ? 1.f : -1.f);
        const float ux = ta ? 0.f : 1.f, uy = ta ? 1.f : 0.f;
        // the wave's chunks ch = wave + 4 c (c < CH) are processed together:
        // operand loads of 2 QB values of b for all of them, then their MFMAs
        constexpr int CH = NWG >= 64 ? NWG / 64 : 1;
        constexpr int QB = CH > 1 ? 2 : 4;  // MFMAs (2 b each) per batch of loads
        const float2* U2c[CH];
        const float2* Hcc[CH];
        int nn[CH];
        bool live[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int ch = wave + 4 * c;
          live[c] = ch < NWG / 16;
          nn[c] = ch * 16 + m16;                              // this lane's B column
          U2c[c] = U2b + (live[c] ? nn[c] % T2 : 0);
          Hcc[c] = Hb + (live[c] ? (ch * 16) / T2 : 0) * r2 * r1p;  // the chunk's i3 row
        }
        for (int mb = 0; mb * 8 < r1; ++mb) {
          const int a = mb * 8 + (m16 >> 1);
          const int ac = min(a, r1 - 1);
          v4f d[CH];
#pragma unroll
          for (int c = 0; c < CH; ++c) d[c] = v4f{0.f, 0.f, 0.f, 0.f};
          for (int b0 = 0; b0 < r2; b0 += 2 * QB) {
            float av[CH][QB], bv[CH][QB];
#pragma unroll
            for (int q = 0; q < QB; ++q) {
              const int bb = b0 + 2 * q + bq;
              const bool ok = bb < r2 && a < r1;
              const int bc = min(bb, r2 - 1);
#pragma unroll
              for (int c = 0; c < CH; ++c) {
                // masks folded into the weights (the clamped reads are
                // finite), so that the loads are not sunk into branches
                const float wx = ok ? cx : 0.f, wy = ok ? cy : 0.f;
                const float vx = bb < r2 ? ux : 0.f, vy = bb < r2 ? uy : 0.f;
                const float2 h = Hcc[c][bc * r1p + ac];
                const float2 u = U2c[c][bc * T2];
                av[c][q] = fmaf(h.x, wx, h.y * wy);
                bv[c][q] = fmaf(u.x, vx, u.y * vy);
              }
            }
#pragma unroll
            for (int q = 0; q < QB; ++q)
              if (b0 + 2 * q < r2) {
#pragma unroll
                for (int c = 0; c < CH; ++c)
                  d[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[c][q], bv[c][q], d[c], 0, 0, 0);
              }
          }
          // lane holds real rows R0 .. R0 + 3 of its column, R0 = 16 mb + 4 k4
          const int R0 = 16 * mb + 4 * k4;
#pragma unroll
          for (int c = 0; c < CH; ++c) {
            if (!live[c]) continue;
            const int n = nn[c];
            if constexpr (BF) {
              if (R0 < 2 * r1p) {
                uint32_t hh[4], ll[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                  hh[e] = bf16_rne(d[c][e]);
                  ll[e] = bf16_rne(d[c][e] - bf16_to_float(hh[e]));
                }
                // uint4 (R0 / 8) * nwg + n holds real rows R0 & ~7 .. + 7
                uint2* bh = reinterpret_cast<uint2*>(Bt);
                uint2* bl = bh + (size_t)(r1p / 8) * 2 * NWG * 2;
                const int at = ((R0 >> 3) * NWG + n) * 2 + ((R0 >> 2) & 1);
                bh[at] = make_uint2(hh[0] | (hh[1] << 16), hh[2] | (hh[3] << 16));
                bl[at] = make_uint2(ll[0] | (ll[1] << 16), ll[2] | (ll[3] << 16));
              }
            } else {
              float* Bf = reinterpret_cast<float*>(Bt);
#pragma unroll
              for (int e = 0; e < 4; ++e)
                if (R0 + e < 2 * r1) Bf[(R0 + e) * NWG + n] = d[c][e];
            }
          }
        }
      }
      // C) mode 1 of tensor t = st - 3 on MFMA from its B tile
      const int t = st - 3;
      if (t >= 0 && t < cnt) {
        const int r1 = tc.r1;
        const int r1p = BF ? ws_pad8(r1) : ws_pad4(r1);
        const float2* Bt = Bbuf + (t & 1) * be;
        if (ADJ) {
#pragma unroll
          for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[b][i] = 0.f;
        }
        if constexpr (BF) {
          const uint4* Ach = P.apack_bf + P.apack_koff[k] +
                             ((int64_t)tc.arow * P.nbt + wm * NB) * 128 + lane;
          const uint4* bh = reinterpret_cast<const uint4*>(Bt) + half * NWG + wn * 32 + cl;
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
          // tensor's first group) is in flight while this group's MFMAs run
          const float* Brow = reinterpret_cast<const float*>(Bt) + half * NWG + wn * 32 + cl;
          for (int a0 = 0; a0 < r1; a0 += 4) {
            float ac[4][NB], bc[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              bc[e] = Brow[2 * min(a0 + e, r1 - 1) * NWG];
#pragma unroll
              for (int b = 0; b < NB; ++b) ac[e][b] = an[e][b];
            }
            if (a0 + 4 < r1) {
              load_arows<NB>(an, abase, tc.arow, a0 + 4, r1, P.nbt, rstride);
            } else if (t + 1 < cnt) {
              const TensorMeta tn = uniform_meta(ML[(t + 1) % WS_META_RING]);
              load_arows<NB>(an, abase, tn.arow, 0, tn.r1, P.nbt, rstride);
            }
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
          // conjugated dot of the Z^{kj} tile with the y tile, per lane
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
          dots[(t & 1) * 256 + wave * 64 + lane] = make_float2(dr, di);
        }
        if (t + 1 < cnt) tc = uniform_meta(ML[(t + 1) % WS_META_RING]);
      }
      __syncthreads();
    }
    if (ADJ) return;
    // forward epilogue: a lane's register quad holds (Re, Im) of voxels i1
    // and i1 + 1 of its fibre
    if (!colok) return;
    float2* dst = P.out + (int64_t)s * P.out_stride + fibre;
    const bool vec4 = P.vec4 != 0;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int i1 = ((wm * NB + b) * 32 + 8 * g + 4 * (lane >> 5)) >> 1;
        if (i1 >= P.n1) continue;
        if (vec4 && i1 + 1 < P.n1) {
          *reinterpret_cast<float4*>(dst + i1) = make_float4(acc[b][4 * g], acc[b][4 * g + 1],
                                                             acc[b][4 * g + 2], acc[b][4 * g + 3]);
        } else {
          dst[i1] = make_float2(acc[b][4 * g], acc[b][4 * g + 1]);
          if (i1 + 1 < P.n1) dst[i1 + 1] = make_float2(acc[b][4 * g + 2], acc[b][4 * g + 3]);
        }
      }
    return;
  }

  // -------------------------------------------------------------- producer
  const int pw = wave - 4, ptid = tid - 256;
  const int64_t pbase = ((int64_t)k * P.tiles + tile) * P.m;
  Stage SR;
  for (int st = 0; st < cnt + 4; ++st) {
    // stage(st): loads issued first, in flight during mode3(st - 1)
    const bool do_stage = st < cnt;
    TensorMeta ts;
    if (do_stage) {
      ts = uniform_meta(ML[st % WS_META_RING]);
      stage_issue(SR, P, ts, i2_0, i3_0, ptid);
    }
    const int ta = st - 1;
    if (ta >= 0 && ta < cnt) {
      const TensorMeta tb = uniform_meta(ML[ta % WS_META_RING]);
      const int r1p = BF ? ws_pad8(tb.r1) : ws_pad4(tb.r1);
      const float2* CU = CUbuf + (ta & 1) * cue;
      float2* H = Hbuf + (ta & 1) * he;
      const float2 xj = XL[ta % WS_META_RING];
      const bool staged = tb.r1 * tb.r2 * tb.r3 <= P.cb;
      if (staged)
        mode3<ADJ>(CU + u3e, CU, H, tb.r1, r1p, tb.r2, tb.r3, P.t3, xj, ptid);
      else
        mode3<ADJ>(P.cores + tb.g_off, CU, H, tb.r1, r1p, tb.r2, tb.r3, P.t3, xj, ptid);
    }
    // adjoint: reduce the per-lane dots of tensor st - 4 (written one step
    // earlier) in a fixed order: 4 waves x 64 lanes
    if (ADJ && pw == 0 && st >= 4 && st - 4 < cnt) {
      const float2* d = dots + ((st - 4) & 1) * 256;
      float sr = 0.f, si = 0.f;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const float2 a = d[w * 64 + lane];
        sr += a.x;
        si += a.y;
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        sr += __shfl_xor(sr, off);
        si += __shfl_xor(si, off);
      }
      if (lane == 0) P.out[pbase + jb + st - 4] = make_float2(sr, si);
    }
    if (do_stage) {
      float2* CU = CUbuf + (st & 1) * cue;
      stage_commit(SR, P, ts, i2_0, i3_0, ptid, U2buf + (st % 3) * u2e, CU, CU + u3e);
    }
    // refill of the metadata ring for the next HALF tensors, once every HALF
    // steps (its load latency is exposed once per refill)
    const int rf = st + 1;
    if (rf % HALF == 0 && rf < cnt && ptid < min(HALF, cnt - rf)) {
      ML[(rf + ptid) % WS_META_RING] = meta[rf + ptid];
      XL[(rf + ptid) % WS_META_RING] = ADJ ? make_float2(1.f, 0.f) : P.vec[jb + rf + ptid];
    }
    __syncthreads();
  }
}

typedef void (*ws_fn)(WsParams);

template <bool ADJ, bool BF>
ws_fn ws_pick(int nb, int wn) {
#define TV_WS_CASE(NB)                                                 \
  case NB:                                                             \
    return wn == 4 ? ws_fused<NB, 4, ADJ, BF>                          \
                   : (wn == 2 ? ws_fused<NB, 2, ADJ, BF> : ws_fused<NB, 1, ADJ, BF>);
  switch (nb) {
    TV_WS_CASE(1) TV_WS_CASE(2) TV_WS_CASE(3) TV_WS_CASE(4)
    TV_WS_CASE(5) TV_WS_CASE(6) TV_WS_CASE(7) TV_WS_CASE(8)
  }
#undef TV_WS_CASE
  return nullptr;
}

}  // namespace

// Largest core staged through LDS: all cores when the buffers stay within
// half the LDS (two workgroups per CU), else none (cores stream from L2).
int ws_core_elems(const tv_plan_s* p, const Tiling& T, bool adj) {
  const int cb = (int)std::min<int64_t>(p->max_core, 8192);
  if (ws_lds_bytes(p, T, adj, cb) <= 80 * 1024) return cb;
  return 0;
}

// The warp-specialised kernels need each consumer wave's 32 columns inside
// one i3 row of the tile.
bool ws_supported(const tv_plan_s* p, const Tiling& T, bool adj) {
  if (T.t2 % 32 != 0) return false;
  return ws_lds_bytes(p, T, adj, ws_core_elems(p, T, adj)) <= 160 * 1024;
}

tv_status launch_fused_ws(const tv_plan_s* p, bool adj, const float2* vec, float2* out, int split,
                          const int32_t* d_split, int64_t out_stride, hipStream_t st) {
  const Tiling& T = adj ? p->tiling_a : p->tiling;
  if (!ws_supported(p, T, adj))
    return set_error(TV_ERR_NOT_SUPPORTED, "tile not supported by the warp-specialised kernel");
  WsParams P;
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
  P.cb = ws_core_elems(p, T, adj);
  P.vec4 = (p->grid.n1 % 2 == 0) && ((uintptr_t)out % 16 == 0) && (out_stride % 2 == 0);
  const bool bf = p->precision == TV_PREC_BF16X3;
  ws_fn fn = adj ? (bf ? ws_pick<true, true>(T.nb, T.wn) : ws_pick<true, false>(T.nb, T.wn))
                 : (bf ? ws_pick<false, true>(T.nb, T.wn) : ws_pick<false, false>(T.nb, T.wn));
  if (!fn) return set_error(TV_ERR_NOT_SUPPORTED, "no kernel instance for this tiling");
  const size_t lds = ws_lds_bytes(p, T, adj, P.cb);
  hipError_t e = hipFuncSetAttribute((const void*)fn,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_error(e, "hipFuncSetAttribute");
  const int64_t grid = (P.nitems + 7) / 8 * 8;
  hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(512), lds, st, P);
  e = hipGetLastError();
  return e == hipSuccess ? TV_OK : hip_error(e, "warp-specialised kernel launch");
}

}  // namespace tv
