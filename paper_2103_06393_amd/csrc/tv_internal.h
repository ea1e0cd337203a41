// Internal structures shared by the host library and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/tuckvsie.h"

namespace tv {

// Per-tensor metadata on the device, indexed [k * m + j].
struct TensorMeta {
  int32_t r1, r2, r3;
  int32_t arow;    // first row of this tensor in component k's stacked A_k
  int64_t g_off;   // core G[a,b,c] (complex) at g_off + a + r1*(b + r2*c)
  int64_t u2_off;  // U2 row-major: U2[i2][b] at u2_off + i2*r2 + b
  int64_t u3_off;  // U3 row-major: U3[i3][c] at u3_off + i3*r3 + c
  int64_t u1_off;  // U1 row-major: U1[i1][a] at u1_off + i1*r1 + a
};

// Geometry of the fused FP32 / BF16 kernels for one plan.
struct Tiling {
  int wm, wn;      // waves along M (voxel rows) and N (columns of Y^k_(1))
  int nb;          // 32-row MFMA blocks per wave along M
  int nbt;         // total 32-row blocks (2*n1p/32), = wm*nb
  int n1p;         // n1 padded to 16*nbt
  int nwg;         // columns per workgroup, 32*wn
  int t2, t3;      // workgroup column tile: t2 values of i2 x t3 of i3
  int tiles2, tiles3;
  int64_t tiles;   // per component
};

// Host-side packed form of a plan, kept from packing until the plan is bound
// to its device arena.
struct HostPack {
  std::vector<TensorMeta> meta;
  std::vector<float2> cores, u1t, u2t, u3t;
  std::vector<float> apack, a4;
  std::vector<uint4> apack_bf, abf;
  std::vector<int32_t> drow;
};

// caller-provided host staging (pinned memory makes copies asynchronous)
struct HostStage {
  char* ptr = nullptr;
  size_t bytes = 0;
};

// column-split tables hold up to this many splits per component
constexpr int TV_SPLIT_MAX = 64;

// one group of Hermitian matrices for the batched Jacobi eigensolver
struct JacobiGroup {
  const double2* S;   // nmat matrices n x n at `stride`
  double* W;          // n eigenvalues per matrix at `wstride`
  double2* V;         // n x n eigenvectors per matrix at `vstride`
  int64_t stride, wstride, vstride;
  int n, nmat;
};
struct JacobiBatch {
  JacobiGroup g[3];
  int ng, max_sweeps;
};
// one group of n x l matrices for the batched CGS2 orthogonalization
struct Cgs2Group {
  double2* Z;
  int64_t stride;
  int n, nmat;
};
struct Cgs2Batch {
  Cgs2Group g[3];
  int ng, l;
};
// one mode's subspace iteration: nmat Gram matrices n x n at sS, traces,
// workspace (Q, Z, V: n x 64 each per matrix, then T: 64 x 64 per matrix)
struct SubspaceJob {
  const double2* S;
  int64_t sS;
  double* tr;
  double2* ws;
  int n;
};

}  // namespace tv

struct tv_plan_s {
  tv_grid grid{};
  tv_precision precision = TV_PREC_FP32;
  bool finalized = false;
  std::vector<int32_t> ranks;  // [q*m][3], tensor t = k + q*j

  // host FP64 factors (kept for export and for packing), tensor order t
  std::vector<int64_t> g_off, u1_off, u2_off, u3_off;  // complex offsets
  std::vector<double> cores, u1, u2, u3;               // interleaved re,im

  // compression parameters and per-tensor relative discarded energies
  double tol = 0.0;
  int32_t rank_min = 1, rank_cap = 0;
  int64_t appended = 0;               // columns whose factors are present
  std::vector<double> rel_discarded;  // [q*m][3]
  int64_t appended_or_all() const { return appended; }

  // device packed form
  tv::Tiling tiling{};    // forward kernel tiling
  tv::Tiling tiling_a{};  // adjoint kernel tiling (sizes its workspace)
  tv::TensorMeta* d_meta = nullptr;
  float2* d_cores = nullptr;
  float2* d_u1t = nullptr;         // U1 row-major [i1][a] (batched kernels)
  float2* d_u2t = nullptr;
  float2* d_u3t = nullptr;
  float* d_apack = nullptr;        // FP32 real-embedded U1, MFMA lane order
  uint4* d_apack_bf = nullptr;     // BF16X3: hi/lo bf16 of the same, 8-row chunks
  int64_t* d_apack_koff = nullptr;
  std::vector<int64_t> apack_koff;
  std::vector<int64_t> sum_r1_k;   // rows of A_k per component
  int split_f = 1, split_a = 1;    // column splits of the forward / adjoint
  int nbcap_a = 2;                 // row blocks per wave allowed in the adjoint tiling
  bool kernel_ws[2] = {true, true};  // warp-specialised kernel (when the tile allows)
  int32_t* d_split_f = nullptr;    // [q][split+1] first column per split
  int32_t* d_split_a = nullptr;
  size_t device_bytes = 0;          // bytes the plan needs in its device arena
  tv::HostPack hp;                   // packed data awaiting tv_plan_bind_arena
  bool bound = false;                // device pointers point into the caller's arena
  // decompress-then-GEMM form of the forward product (large grids)
  float* d_apack4 = nullptr;       // stacked U1 in 4-k-step groups (FP32 plans)
  int dtg_nbtp = 0;                // 32-row blocks per k-step, padded to the GEMM tile
  std::vector<int64_t> dtg_rpad;   // rows of A_k padded to 16, per component
  std::vector<int64_t> dtg_a4off;  // float offset of component k in d_apack4
  int64_t dtg_rows = 0;            // sum of dtg_rpad
  uint4* d_abf = nullptr;          // BF16X3 plans: stacked U1 hi/lo in 8-k-step chunks
  int32_t* d_drow = nullptr;       // first stacked row of each tensor in A_k, [k][j]
  std::vector<int64_t> dtg_abfoff; // uint4 offset of component k in d_abf
  bool with_dtg = true;             // pack the GEMM operands (FP32 plans)
  bool dtg_packed = false;          // the GEMM operands are part of the plan
  bool use_dtg[2] = {false, false};
  int dtg_s3 = 1 << 30;            // i3 values per slab of B (forward)
  int dtg_s3_a = 1 << 30;          // i3 values per slab of B (adjoint)
  int dtg_order_a = 0;             // adjoint GEMM workgroup order (tv_launch_config)
  int dtg_split_a = 1;             // column splits of the adjoint's column GEMM
  int dtg_nbw_a = 4;               // 32-row blocks per wave along N of that GEMM
  int dtg_nbw = 2;                 // 32-column blocks per wave of the GEMM tile
  int dtg_split = 1;               // k-step splits of the GEMM
  int dtg_mbw[2] = {0, 0};         // GEMM 32-row blocks per wave (0: default; 8: BF16X3 full-M tile)
  int max_r[3] = {0, 0, 0};
  int nbt_pack = 0;      // 32-row blocks per stacked A row in the packed layout
  int max_r12 = 0;       // largest r1 r2
  int64_t max_core = 0;  // largest r1 r2 r3
  int64_t sum_r1 = 0;
  // growable plans (grow_plan_create): column capacity, rank caps, BF16X3
  // chunks per component and the host staging of one append
  int64_t grow_mcap = 0;
  int grow_rcap[3] = {0, 0, 0};
  std::vector<int64_t> grow_chunks_k;
  tv::HostPack grow_stage;
  std::vector<int32_t> grow_split;
  std::vector<char> grow_buf;  // the pieces of one append, packed for one copy
  char* grow_pinned = nullptr; // or the caller's staging, when handed over
  size_t grow_pinned_bytes = 0;
  char* d_stage = nullptr;     // their device staging region in the arena
  size_t stage_bytes = 0;
  size_t grow_adj_ws = 0;      // adjoint workspace the caller provides
};

namespace tv {
tv_status set_error(tv_status s, const std::string& msg);
tv_status hip_error(hipError_t e, const char* what);
void clear_error();

// kernels (tv_matvec_f32.hip)
tv_status launch_forward_f32(const tv_plan_s* p, const float2* x, float2* out,
                             int split, const int32_t* d_split, int64_t out_stride,
                             hipStream_t st);
tv_status launch_adjoint_f32(const tv_plan_s* p, const float2* y, float2* partial,
                             int split, const int32_t* d_split, hipStream_t st);
tv_status launch_sum_partials(const float2* ws, int split, int64_t n, float2* y,
                              hipStream_t st);
tv_status launch_reduce_adjoint(const float2* partial, int q, int64_t tiles,
                                int64_t m, float2* x, hipStream_t st);
// warp-specialised kernels (tv_fused_ws.hip)
bool ws_supported(const tv_plan_s* p, const Tiling& T, bool adj);
tv_status launch_fused_ws(const tv_plan_s* p, bool adj, const float2* vec, float2* out,
                          int split, const int32_t* d_split, int64_t out_stride,
                          hipStream_t st);
// dynamic LDS of the fused kernels for a plan and tiling
size_t fused_lds_bytes(const tv_plan_s* p, const Tiling& T, bool adj);
// tiling with a given i2 extent t2 (0: the one covering the fewest columns)
// (at most nbcap MFMA row blocks per wave)
tv_status make_tiling(const tv_grid& g, int t2, int nbcap, Tiling* T);
// row-block cap of a plan's kernel for op 0 (forward) / 1 (adjoint)
int nb_cap(const tv_plan_s* p, int op);
// (re)build and upload the column split table of one direction
tv_status set_split(tv_plan_s* p, int op, int S);
// decompress-then-GEMM forward (tv_dtg.hip)
tv_status dtg_pack(tv_plan_s* p, const std::vector<TensorMeta>& meta);
bool dtg_supported(const tv_plan_s* p);
// 32-row blocks of one decompress-then-GEMM workgroup tile (tv_dtg.hip), and
// the most components that path takes (DTG_MAXQ there)
int dtg_mt(const tv_plan_s* p);
constexpr int DTG_MAXQ_HOST = 12;
size_t dtg_workspace_bytes(const tv_plan_s* p, int op);
int64_t dtg_launch_tiles(const tv_plan_s* p, int s3, int nbw);  // workgroups of one GEMM launch
int64_t dtg_colgemm_tiles(const tv_plan_s* p, int nbw);  // adjoint column GEMM tiles per split
int dtg_colgemm_splits(const tv_plan_s* p, int s3);     // its column splits as launched
tv_status launch_dtg_forward(const tv_plan_s* p, const float2* x, float2* y, void* ws,
                             hipStream_t st);
tv_status launch_dtg_adjoint(const tv_plan_s* p, const float2* y, float2* x, void* ws,
                             hipStream_t st);
// an upper bound of the device arena of a plan of grid g whose ranks are at
// most rmax, without the decompress-then-GEMM operands (the arena of a
// growable plan of g.m columns)
size_t plan_arena_bound(const tv_grid& g, const int rmax[3], tv_precision precision);
// Growable plan (Algorithm 3's U, which gains one column per step): created
// empty with its device arrays at fixed offsets of `arena`, each sized for
// g.m columns at ranks up to rmax; every append converts and uploads only
// the new column's factors (ranks [q][3], factors of its q tensors in tensor
// order, FP64 interleaved, laid out as tv_plan_from_factors takes them) and
// rewrites the small metadata and split tables, then waits for the copies.
// The plan keeps no FP64 factors (no export).
tv_status grow_plan_create(const tv_grid& g, const int rmax[3], tv_precision precision,
                           void* arena, size_t bytes, hipStream_t st, tv_plan* out);
// host staging an append of a growable plan of g.m columns at ranks up to
// rmax packs its pieces into (grow_plan_set_stage hands one over; without one
// the plan uses a host vector)
size_t grow_stage_bytes(const tv_grid& g, const int rmax[3], tv_precision precision);
// workspace of a growable plan's column-GEMM adjoint at its capacity; the
// plan takes that path from kGrowColGemmMin columns on while its workspace at
// the current ranks fits what grow_plan_set_stage was told the caller holds,
// the fused kernels otherwise
constexpr int kGrowColGemmMin = 8;
size_t grow_adjoint_ws_bytes(const tv_grid& g, const int rmax[3]);
void grow_plan_set_stage(tv_plan p, const HostStage& stage, size_t adj_ws_bytes);
tv_status grow_plan_append(tv_plan p, const int32_t* ranks, const double* cores,
                           const double* u1, const double* u2, const double* u3,
                           hipStream_t st);
// Copy of up to kMaxCopySegs byte ranges of one device staging buffer to
// their destinations (4-byte aligned, sizes multiples of 4), one launch.
struct CopySeg {
  void* dst;
  int64_t src_off, bytes;
};
constexpr int kMaxCopySegs = 24;
tv_status launch_segment_copy(const CopySeg* segs, int nseg, const void* src, hipStream_t st);
// compression scratch of one append call of T tensors (tv_compress.cpp)
size_t compress_scratch_bytes(const tv_plan_s* p, int T);
// Host staging of one append call's transfers (eigenpair readback, factor
// upload, core readback): with `bytes` >= compress_stage_bytes the call uses
// it instead of host vectors (pinned memory makes the copies asynchronous).
size_t compress_stage_bytes(const tv_plan_s* p, int T);
tv_status compress_append_staged(tv_plan p, const void* cols, int64_t ncols, void* ws,
                                 size_t ws_bytes, hipStream_t st, const HostStage& stage);
// the autotuners' JSON cache: key -> list of integers (tv_autotune.cpp)
std::map<std::string, std::vector<int>> read_tune_cache(const char* path);
void write_tune_cache(const char* path, const std::map<std::string, std::vector<int>>& m);
std::string device_arch();
// point-current fields (tv_columns.hip): sources as device [n][6]
tv_status stage_sources(int n1, int n2, int n3, double h, int64_t n, const double* pos,
                        const double* ori, std::vector<double>& src);
tv_status launch_dipole_columns(int n1, int n2, int n3, double h, double k0, int basis,
                                int64_t ncols, const double* d_src, double2* out, hipStream_t st);
tv_status launch_dipole_rows(int n1, int n2, int n3, double h, double k0, int basis,
                             int64_t nsrc, const double* d_src, int64_t nrows,
                             const int64_t* d_rows, double2* out, hipStream_t st);
}  // namespace tv
