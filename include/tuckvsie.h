/*
 * libtuckvsie -- matrix-vector products with a Tucker-compressed VSIE
 * coil-to-body coupling matrix on AMD Instinct MI355X (gfx950).
 *
 * The coupling matrix Z (q*nv rows, m columns) maps coil currents to voxel
 * fields (Sec. II.A.1 of Giannakopoulos et al., "Compression of volume-
 * surface integral equation matrices via Tucker decomposition for magnetic
 * resonance applications").  Column j is q stacked vectors, each reshaped to
 * an n1 x n2 x n3 voxel tensor Z^{kj} and held in Tucker form
 *     Z^{kj} = G x1 U1 x2 U2 x3 U3                       (eq. 6, Sec. III.A)
 * with per-tensor multilinear ranks (r1, r2, r3).  The library computes
 *     Y = Z X      (Algorithm 1, Sec. III.B)
 *     X = Z^* Y    (Algorithm 2, Sec. III.B; ^* = conjugate transpose)
 * without ever forming Z, and builds the Tucker form from dense columns with
 * the truncated HOSVD (Sec. II.B.1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Complex numbers are interleaved (re, im).  Host factor arrays are
 *   complex128 (double pairs); device vectors are complex64 (float pairs).
 * - Tensor t = k + q*j is component k (0-based) of column j.
 * - Row order of Y is [Y^1; ...; Y^q] (Algorithm 1's last step): row
 *   k*nv + i1 + n1*(i2 + n2*i3) holds voxel (i1, i2, i3) of component k,
 *   i.e. each block is the column-major vectorisation (:) of its tensor.
 * - Multi-vector operands are column-major with a leading dimension: entry
 *   (row, col) of X lives at X[row + ld*col].
 * - Streams are hipStream_t passed as void* (NULL = default stream).  Every
 *   hot-path call is asynchronous on its stream, never allocates and never
 *   synchronises.
 * - Ownership: the caller owns every buffer it passes (vectors, workspace);
 *   a plan owns the device copy of its factors until tv_plan_destroy.
 * - Errors: every call returns a tv_status.  Argument errors are detected on
 *   the host before any device work is queued; the detail of the last error
 *   on the calling thread is available from tv_last_error().  Device faults
 *   surface at the caller's next synchronisation.
 * - A plan is read-only after creation: concurrent calls on different
 *   streams are safe if each uses its own workspace.
 */
#ifndef TUCKVSIE_H
#define TUCKVSIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Enumerations are int32 in C and C++ alike; in C++ the fixed underlying
 * type makes every int32 value a valid enumerator value, so an unknown value
 * passed by a caller is refused instead of being undefined behaviour. */
#ifdef __cplusplus
#define TV_ENUM(tag) enum tag : int32_t
#else
#define TV_ENUM(tag) enum tag
#endif

typedef TV_ENUM(tv_status_e) {
  TV_OK = 0,
  TV_ERR_INVALID_ARG = -1,   /* null pointer, negative size, bad enum    */
  TV_ERR_SHAPE = -2,         /* grid / leading dimension inconsistent    */
  TV_ERR_RANK = -3,          /* rank < 1, > grid size or > TV_MAX_RANK   */
  TV_ERR_OOM = -4,           /* device or host allocation failed         */
  TV_ERR_HIP = -5,           /* a HIP runtime call failed                */
  TV_ERR_NOT_SUPPORTED = -6, /* valid request outside what is built      */
  TV_ERR_NUMERIC = -7,       /* non-finite factor values                 */
  TV_ERR_WORKSPACE = -8      /* workspace missing or too small           */
} tv_status;

/* Arithmetic of the products.  FP32: factors stored as float, products on
 * FP32 MFMA with FP32 accumulation.  BF16X3: every FP32 operand x is split
 * into bf16 hi = rn(x), lo = rn(x - hi) and a*b is formed as
 * hi*hi + hi*lo + lo*hi on BF16 MFMA with FP32 accumulation. */
typedef TV_ENUM(tv_precision_e) { TV_PREC_FP32 = 0, TV_PREC_BF16X3 = 1 } tv_precision;

/* Flag ORed into the `basis` argument of the field entry points
 * (tv_dipole_columns, tv_dipole_rows, tv_aca_assemble): the K operator of
 * eq. (5) (magnetic field) instead of the N operator of eq. (2). */
#define TV_FIELD_K 2

/* Largest multilinear rank a plan may hold in any mode. */
#define TV_MAX_RANK 64

typedef struct {
  int32_t n1, n2, n3; /* voxel grid (Sec. III.A: nv = n1*n2*n3)            */
  int32_t q;          /* tensors per column: 3 (PWC) or 12 (PWL), any >= 1 */
  int64_t m;          /* columns (coil basis functions)                    */
} tv_grid;

typedef struct tv_plan_s* tv_plan;

typedef struct {
  tv_grid grid;
  tv_precision precision;
  int32_t max_rank[3];     /* largest r1, r2, r3 over all tensors          */
  double mean_rank[3];     /* mean r1, r2, r3                              */
  int64_t sum_r1;          /* sum of r1 over all q*m tensors               */
  size_t factor_bytes;     /* Tucker entries x 8 B (complex64), Table II   */
  size_t device_bytes;     /* device memory the plan holds (packed forms)  */
  double flops_matvec;     /* algorithmic real flops of one Z x (p = 1)    */
  double flops_rmatvec;    /* algorithmic real flops of one Z^* y (p = 1)  */
  /* launch configuration of the fused kernels, [0] forward, [1] adjoint:
   * tile extent along i2 and i3, column splits, and the kernel family
   * (0: phased, 1: warp-specialised producer/consumer, 2: decompress-then-
   * GEMM, for which tile_t2 is the i3 values per slab, tile_t3 the GEMM's
   * column blocks per wave (adjoint: row blocks) and splits its k-step
   * (adjoint: column) split count)                                         */
  int32_t tile_t2[2], tile_t3[2], splits[2], kernel[2];
} tv_plan_info_t;

/* ------------------------------------------------------------------------
 * Plan creation from given Tucker factors (eq. 6).
 *
 * ranks : host int32[q*m][3], (r1, r2, r3) of tensor t = k + q*j.
 * cores : host complex128, the q*m cores concatenated in tensor order; core
 *         t is r1*r2*r3 values, G[a,b,c] at a + r1*(b + r2*c).
 * u1, u2, u3 : host complex128, the factors concatenated in tensor order;
 *         U_n of tensor t is n_n x r_n column-major, U[i,a] at i + n_n*a.
 * The library copies and repacks the factors (FP64 -> FP32 round to
 * nearest even) on the host; the host arrays may be freed on return.  The
 * plan holds no device memory until tv_plan_bind_arena.  Host-only.
 * Returns TV_ERR_RANK for a rank outside [1, min(n_n, TV_MAX_RANK)],
 * TV_ERR_NUMERIC for non-finite values.
 * ---------------------------------------------------------------------- */
tv_status tv_plan_from_factors(const tv_grid* grid, const int32_t* ranks,
                               const double* cores, const double* u1,
                               const double* u2, const double* u3,
                               tv_precision precision, tv_plan* out);

/* Device memory of a plan (Table II's Tucker entries in the packed layouts
 * of the kernels: FP32 cores and factors, the stacked U1 operands, split
 * tables) is owned by the caller: tv_plan_required_bytes gives the size of
 * the arena a finalized plan needs, tv_plan_bind_arena copies the packed
 * plan into the caller's device buffer [arena, arena + bytes) (256-byte
 * aligned) on `stream` and waits for the copies (set-up call), after which
 * the plan's products and autotuning may run.  The arena must stay
 * allocated and unmodified while the plan is used; a plan binds once.
 * TV_ERR_WORKSPACE (before any device work) if bytes is short. */
tv_status tv_plan_required_bytes(tv_plan plan, size_t* bytes);
tv_status tv_plan_bind_arena(tv_plan plan, void* arena, size_t bytes, void* stream);

/* Release a plan (host memory only; its arena belongs to the caller).
 * NULL is accepted. */
tv_status tv_plan_destroy(tv_plan plan);

/* Sizes, ranks and operation counts of a plan. */
tv_status tv_plan_info(tv_plan plan, tv_plan_info_t* info);

/* Copy the ranks (int32[q*m][3]) and, if the pointers are non-NULL, the
 * complex128 factors of a plan back to host arrays in the layout of
 * tv_plan_from_factors (sizes from tv_plan_info / the ranks).  Synchronous.
 * Factors are returned in FP64 as the plan keeps them on the host (the
 * values given to tv_plan_from_factors, or the compression's FP64 factors);
 * the products use their FP32 rounding. */
tv_status tv_plan_export_factors(tv_plan plan, int32_t* ranks, double* cores,
                                 double* u1, double* u2, double* u3);

/* ------------------------------------------------------------------------
 * Workspace needed by tv_matvec (op = 0) or tv_rmatvec (op = 1) for nrhs
 * right-hand sides.  May be 0; a larger workspace is always accepted.
 * ---------------------------------------------------------------------- */
tv_status tv_workspace_bytes(tv_plan plan, int32_t op, int32_t nrhs,
                             size_t* bytes);

/* Y = Z X (Algorithm 1).  x: device complex64, m x nrhs, leading dim ldx
 * >= m.  y: device complex64, q*nv x nrhs, leading dim ldy >= q*nv,
 * overwritten.  ws: device workspace of at least tv_workspace_bytes(op=0)
 * bytes (may be NULL if that is 0).  x and y must not overlap.  The result
 * is deterministic: fixed reduction order, no atomics. */
tv_status tv_matvec(tv_plan plan, const void* x, int64_t ldx, int32_t nrhs,
                    void* y, int64_t ldy, void* ws, size_t ws_bytes,
                    void* stream);

/* X = Z^* Y (Algorithm 2).  y: device complex64, q*nv x nrhs, leading dim
 * ldy >= q*nv.  x: device complex64, m x nrhs, leading dim ldx >= m,
 * overwritten.  ws as for tv_matvec with op = 1.  Deterministic. */
tv_status tv_rmatvec(tv_plan plan, const void* y, int64_t ldy, int32_t nrhs,
                     void* x, int64_t ldx, void* ws, size_t ws_bytes,
                     void* stream);

/* Launch configuration of one direction of a plan's products (what the
 * autotuner chooses; set-up call, not thread-safe against concurrent
 * products on the same plan).
 *   path 0: the fused kernels (Algorithms 1/2 with decompression inside the
 *     mode-1 product): tile_t2 = i2 extent of a workgroup tile (0: the tile
 *     covering the fewest columns), splits = column-range splits (split-K
 *     over j), row_cap = row blocks per consumer wave (forward 8; adjoint 2
 *     or 3).
 *   path 1 (FP32 plans): decompress-then-GEMM: per slab of slab_i3 values
 *     of i3 (0: all), modes 3 and 2 of every tensor are decompressed into
 *     the stacked operand B_k = [x_1 M_1; ...] (unscaled for the adjoint) in
 *     the workspace, then the forward runs Y^k_(1) = A_k B_k as one MFMA
 *     GEMM per component (gemm_nbw = 2 or 4 column blocks per wave; splits
 *     k-step splits; BF16X3 plans split the FP32 slab into bf16 hi/lo
 *     inside the GEMM); the adjoint takes
 *     Algorithm 2's sum over voxel columns first: Z_k = Y^k_(1) B_k^* as one
 *     GEMM per slab over the slab's columns (gemm_nbw 2 or 4 blocks of 32
 *     stacked rows per wave, splits 1..64 column splits, gemm_order 0:
 *     workgroups sharing B rows adjacent, 1: sharing y columns adjacent),
 *     one FP32 partial per slab and split, then x'_j = sum conj(U1_j) Z_k
 *     with the partials summed in FP64 (Algorithms 1 and 2, Sec. III.B).
 *     row_cap on path 1: 0 (the plan's GEMM tile along the voxel rows) or
 *     8 (BF16X3 plans whose 2 n1 real rows pack into 16 blocks of 32, with
 *     gemm_nbw 2: one workgroup over all voxel rows, 8 row blocks per wave,
 *     so the slab is read once per column tile).
 * TV_ERR_INVALID_ARG / TV_ERR_NOT_SUPPORTED for a configuration the plan
 * cannot run; the previous configuration is then kept.  Afterwards
 * tv_workspace_bytes reflects the configuration. */
typedef struct {
  int32_t path;
  int32_t tile_t2, splits, row_cap;
  int32_t slab_i3, gemm_nbw, gemm_order;
} tv_launch_config;
tv_status tv_plan_configure(tv_plan plan, int32_t op, const tv_launch_config* cfg);

/* Z^* y exactly as tv_rmatvec, with no workspace argument and no device
 * allocation: for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * adjoint's scratch is a static device array of TV_STATIC_SCRATCH_BYTES per
 * GPU, held until the process ends; a plan configuration needing more
 * (tv_workspace_bytes(plan, 1, nrhs)) returns TV_ERR_WORKSPACE before any
 * device work.  All calls on one GPU share the array: calls that overlap in
 * time on one GPU (different streams or threads) race and must be
 * serialised by the caller.  Every scratch entry a call reads is written
 * earlier in the same call, so nothing carries over between calls. */
#define TV_STATIC_SCRATCH_BYTES (32u << 20)
tv_status tv_rmatvec_noalloc(tv_plan plan, const void* y, int64_t ldy, int32_t nrhs,
                             void* x, int64_t ldx, void* stream);

/* Pick the fastest launch configuration (tv_launch_config: fused-kernel
 * tiles, splits and row caps, and for the forward also the
 * decompress-then-GEMM path with its slab and tile) for this plan by timing
 * every candidate on the device (HIP events, `stream`), for op 0
 * (tv_matvec), 1 (tv_rmatvec) or 2 (both).
 * Results are cached in the JSON file cache_path (NULL: no cache), keyed by
 * device architecture, grid, q, m, precision and a hash of the ranks; a
 * cached entry is applied without timing.  Allocates and synchronises (a
 * set-up call); afterwards tv_workspace_bytes reflects the chosen
 * configuration.  Results do not depend on the configuration beyond
 * floating-point summation order. */
tv_status tv_autotune(tv_plan plan, int32_t op, const char* cache_path,
                      void* stream);

/* ------------------------------------------------------------------------
 * Synthetic coil columns on the device (stand-in for the MoM assembly of
 * Sec. II.A.1): column j is the E-field operator of eq. (2), with the
 * Green's function of eq. (3), applied to a unit point current at pos[j]
 * with unit orientation ori[j] (host double[ncols][3] arrays), evaluated on
 * the centred grid of voxel edge h at wavenumber k0.
 * basis 0 (PWC, q = 3): the field at each voxel centre.
 * basis 1 (PWL, q = 12): tensor 4c + l is (1/h^3) * integral over the voxel
 *   of field component c times phi_l, phi_0 = 1, phi_l = (x_l - centre_l)/h,
 *   by the 2x2x2 Gauss-Legendre rule.
 * basis | TV_FIELD_K: the magnetic-field operator of eq. (5) instead (the
 *   coupling matrix Z_bc): curl(g p) = g (-i k0 - 1/R) Rhat x p, same bases.
 * out: device complex128, ncols*q*nv values, column j's tensor k at
 *   out + 2*((j*q + k)*nv + v), v = i1 + n1*(i2 + n2*i3).  Runs on
 *   `stream` and synchronises it before returning; the sources reach the
 *   kernels through their launch arguments (no device allocation).
 * ---------------------------------------------------------------------- */
tv_status tv_dipole_columns(int32_t n1, int32_t n2, int32_t n3, double h,
                            double k0, int32_t basis, int64_t ncols,
                            const double* pos, const double* ori, void* out,
                            void* stream);

/* ------------------------------------------------------------------------
 * Compression (truncated HOSVD, Sec. II.B.1) of dense columns on the device.
 *
 * tv_compress_begin creates an empty plan for grid->m columns.  Each mode
 * keeps the smallest rank whose discarded squared singular values sum to at
 * most tol^2 * ||Z^{kj}||_F^2 / 3, extended over near-equal singular
 * values and clamped to [rank_min, min(rank_cap, n_n, TV_MAX_RANK)]
 * (rank_cap <= 0 means no cap).
 * tv_compress_append compresses the next ncols columns, given as device
 * complex128 in the layout written by tv_dipole_columns, with the caller's
 * device workspace ws (256-byte aligned, at least
 * tv_compress_workspace_bytes(plan, ncols) bytes: Gram matrices (and, for
 * calls of few tensors, whose Gram products are split over the unfoldings'
 * columns, their partial tiles), eigenpairs, factors and partial
 * projections of the call; TV_ERR_WORKSPACE
 * before any device work if short); work happens on `stream`, and the call
 * synchronises it before returning.  The factors are kept on the host.
 * tv_plan_finalize packs the plan for the products once all m columns are
 * in; after tv_plan_bind_arena it may be used with tv_matvec / tv_rmatvec.
 * ---------------------------------------------------------------------- */
tv_status tv_compress_begin(const tv_grid* grid, double tol, int32_t rank_min,
                            int32_t rank_cap, tv_precision precision,
                            tv_plan* out);
tv_status tv_compress_workspace_bytes(tv_plan plan, int64_t ncols, size_t* bytes);
tv_status tv_compress_append(tv_plan plan, const void* cols, int64_t ncols,
                             void* ws, size_t ws_bytes, void* stream);
tv_status tv_plan_finalize(tv_plan plan, void* stream);

/* Largest singular-value tail discarded per mode for every tensor appended
 * so far: host double[q*m][3] of sum_{i > r_n} sigma_i^2 / ||Z^{kj}||^2
 * (the HOSVD bound's terms, relative).  Synchronous. */
tv_status tv_compress_discarded(tv_plan plan, double* rel_discarded);

/* ------------------------------------------------------------------------
 * Batched products with many right-hand sides (Table III's multi-vector
 * form): nplans plans on one voxel grid (same n1, n2, n3, q), plan c with
 * nrhs[c] right-hand sides, in one persistent launch.
 *   op 0:  Y_c = Z_c X_c,    in[c] = X_c (m_c x nrhs[c]), out[c] = Y_c
 *   op 1:  X_c = Z_c^* Y_c,  in[c] = Y_c (q nv x nrhs[c]), out[c] = X_c
 * Every tensor is decompressed once per voxel tile and applied to all
 * right-hand sides on MFMA, in FP32; when every plan is TV_PREC_BF16X3 both
 * directions apply with the BF16 hi/lo split (FP32 accumulation).  With all
 * ranks <= 32 (and, forward, n1 <= 96) the decompression runs on MFMA too,
 * from G x3 U3 precomputed per (tensor, i3) into the workspace.
 * tv_batch_create builds the work queue (longest job first) and the packed
 * operands on the host (host-only; the plans must be bound to their arenas
 * and outlive the batch); tv_batch_required_bytes gives the device arena
 * the batch needs and tv_batch_bind_arena copies the queue and operands
 * into the caller's buffer (256-byte aligned; set-up call, synchronous;
 * TV_ERR_WORKSPACE before any device work if short).  A batch binds once
 * and its arena must stay allocated while it is used.
 * tv_batch_run queues a counter-reset kernel, (MFMA path) the mode-3
 * kernel, the persistent kernel and (op 1) a reduction kernel on `stream`:
 * no allocation, no synchronisation and no memset, so it may be captured
 * into a hipGraph.  Pointer arrays are host arrays of nplans device
 * pointers (column-major, leading dimensions ld_in/ld_out); outputs are
 * overwritten.  ws: at least tv_batch_workspace_bytes bytes (on the MFMA
 * path this includes sum over tensors of r1 r2 n3 complex64), 16-byte
 * aligned; concurrent runs need distinct workspaces.
 * Deterministic: fixed summation order, no floating-point atomics.
 * ---------------------------------------------------------------------- */
#define TV_BATCH_MAX_PLANS 32
typedef struct tv_batch_s* tv_batch;
/* Launch configuration of a batch (what tv_batch_autotune chooses):
 * tsplit = adjoint work items per (plan, component, 32-column chunk,
 * right-hand-side group), each a slice of the voxel tiles (0: automatic,
 * about 4096 items; ignored by the forward); blocks_per_cu = persistent
 * workgroups per compute unit (0: as many as fit).  cfg NULL: automatic. */
typedef struct {
  int32_t tsplit, blocks_per_cu;
} tv_batch_config;
tv_status tv_batch_create(int32_t nplans, const tv_plan* plans, int32_t op,
                          const int32_t* nrhs, const tv_batch_config* cfg, tv_batch* out);
/* The configuration a batch uses (tsplit reported as 0 for the forward). */
tv_status tv_batch_info(tv_batch batch, tv_batch_config* cfg);
/* Time the batch configurations for these plans, direction and right-hand
 * sides (set-up call: allocates its own timing buffers and synchronises)
 * and return the fastest in *best; cached in the JSON file cache_path
 * (shared with tv_autotune; NULL: no cache) keyed by device, grid, q, the
 * plans' ranks and nrhs. */
tv_status tv_batch_autotune(int32_t nplans, const tv_plan* plans, int32_t op,
                            const int32_t* nrhs, const char* cache_path, void* stream,
                            tv_batch_config* best);
tv_status tv_batch_required_bytes(tv_batch batch, size_t* bytes);
tv_status tv_batch_bind_arena(tv_batch batch, void* arena, size_t bytes, void* stream);
tv_status tv_batch_workspace_bytes(tv_batch batch, size_t* bytes);
tv_status tv_batch_run(tv_batch batch, const void* const* in,
                       const int64_t* ld_in, void* const* out,
                       const int64_t* ld_out, void* ws, size_t ws_bytes,
                       void* stream);
tv_status tv_batch_destroy(tv_batch batch);

/* ------------------------------------------------------------------------
 * ACA + Tucker products (Sec. III.B, the substitution stated after
 * Algorithms 1 and 2; Table III, row ACA+Tucker).  The coupling matrix is
 * held as Z ~= U V^* (cross approximation, Sec. II.B.2; Algorithm 3 builds
 * it with U compressed column by column):
 *   plan : the r_c columns of U as Tucker tensors (grid->m = r_c);
 *   v    : V, m x r_c, device complex64, column-major, V[j, l] at
 *          v[j + ldv*l], ldv >= m (m = coil basis functions).
 *   tv_aca_matvec:   Y = U (V^* X)   x: m x nrhs (ldx >= m),
 *                                    y: q nv x nrhs (ldy >= q nv)
 *   tv_aca_rmatvec:  X = V (U^* Y)   y: q nv x nrhs, x: m x nrhs
 * Outputs are overwritten.  V^* X and V W accumulate in FP64 in a fixed
 * order; the Tucker products are those of tv_matvec / tv_rmatvec, so the
 * result is deterministic.  nrhs <= 65535.
 * ws: device workspace of at least tv_aca_workspace_bytes(op) bytes
 * (op 0 forward, 1 adjoint), 16-byte aligned, not overlapping any operand:
 * the r_c x nrhs intermediate followed by the Tucker product's workspace.
 * Asynchronous on `stream`; no allocation, no synchronisation.  Argument
 * errors (NULL pointers, ldv < m, overlaps, small workspace) are reported
 * before any work is queued.
 * ---------------------------------------------------------------------- */
tv_status tv_aca_workspace_bytes(tv_plan plan, int32_t op, int32_t nrhs,
                                 size_t* bytes);
tv_status tv_aca_matvec(tv_plan plan, const void* v, int64_t m, int64_t ldv,
                        const void* x, int64_t ldx, int32_t nrhs, void* y,
                        int64_t ldy, void* ws, size_t ws_bytes, void* stream);
tv_status tv_aca_rmatvec(tv_plan plan, const void* v, int64_t m, int64_t ldv,
                         const void* y, int64_t ldy, int32_t nrhs, void* x,
                         int64_t ldx, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Rows of the synthetic coupling matrix (the same point-current fields and
 * `basis` codes as tv_dipole_columns): out[r*nsrc + j] = Z[rows[r], j],
 * device complex128,
 * row = k nv + i1 + n1 (i2 + n2 i3) (Algorithm 1's row order), nrows <=
 * 65535, rows in [0, q nv).  Synchronous; sources and row indices reach
 * the kernels through their launch arguments (no device allocation).
 * ---------------------------------------------------------------------- */
tv_status tv_dipole_rows(int32_t n1, int32_t n2, int32_t n3, double h,
                         double k0, int32_t basis, int64_t nsrc,
                         const double* pos, const double* ori, int64_t nrows,
                         const int64_t* rows, void* out, void* stream);

/* ------------------------------------------------------------------------
 * Tucker-based ACA assembly (Algorithm 3, Sec. III.C) of the point-current
 * coupling matrix Z (q nv x m, grid->m coil elements at pos/ori, host
 * double[m][3]) on the device: adaptive cross approximation with partial
 * pivoting in which each new column of U is compressed at once by the
 * truncated HOSVD (tolerance hosvd_tol, <= 0 for Algorithm 3's 3 tol; rank
 * rule and clamps as tv_compress_begin), rows of U come from single-element
 * decompression, U V_j^* from the fused forward and U^* x from the
 * decompress-then-GEMM adjoint once U has 8 columns (the fused adjoint
 * before, or when that path's workspace at the current ranks would pass
 * 16 GiB), in the given precision.
 * The loop stops when |x||y| <= tol sqrt(s) (s the running estimate of
 * ||U V^*||_F^2, with the cross term 2 Re sum conj(V^* y) (U^* x)), when a
 * residual row is exactly zero, or after max_terms steps.
 * Outputs: *u_out a finalized plan of the r_c columns of U (grid m = r_c;
 * not bound: bind it with tv_plan_bind_arena before its products; release
 * with tv_plan_destroy); v_out host complex128 m x max_terms,
 * column-major, first r_c columns written; *rc_out = r_c; *converged_out =
 * 1 if the stopping test was met; pivots (optional, host int64
 * [max_terms][2]) the pivot row i and column j of each step; s_out
 * (optional, host double[max_terms]) the estimate after each step.
 * basis as for tv_dipole_columns (bit 0 PWL, TV_FIELD_K for the magnetic
 * coupling matrix Z_bc); PWC needs grid->q = 3, PWL q = 12.  Synchronous.
 * ws: the caller's device workspace (256-byte aligned) of at least
 * tv_aca_assemble_workspace_bytes(grid, max_terms, tol, hosvd_tol,
 * rank_min, rank_cap, precision) bytes: the row, column and V buffers, one
 * column's compression scratch, U's device arena at max_terms columns of the
 * largest ranks the HOSVD clamps allow (rank_cap bounds it) and the products'
 * workspace (the adjoint's slab of U at those ranks, at most 16 GiB);
 * TV_ERR_WORKSPACE before any device work if short.
 * TV_ERR_NUMERIC if the first pivot row of Z is zero.
 * ---------------------------------------------------------------------- */
tv_status tv_aca_assemble_workspace_bytes(const tv_grid* grid, int32_t max_terms,
                                          double tol, double hosvd_tol,
                                          int32_t rank_min, int32_t rank_cap,
                                          tv_precision precision, size_t* bytes);
tv_status tv_aca_assemble(const tv_grid* grid, double h, double k0,
                          int32_t basis, const double* pos, const double* ori,
                          double tol, double hosvd_tol, int32_t rank_min,
                          int32_t rank_cap, int32_t max_terms,
                          tv_precision precision, void* ws, size_t ws_bytes,
                          tv_plan* u_out, double* v_out, int32_t* rc_out,
                          int32_t* converged_out, int64_t* pivots,
                          double* s_out, void* stream);

/* Human-readable name of a status code (static storage). */
const char* tv_status_string(tv_status status);

/* Detail of the last failing call on this thread ("" if none). */
const char* tv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TUCKVSIE_H */
