"""ctypes binding of libtuckvsie (include/tuckvsie.h), same names as the C ABI.

Argument marshalling only: every arithmetic step runs in the library's HIP
kernels.  Device buffers are passed as raw pointers (``tensor.data_ptr()``)
and streams as ``torch.cuda.current_stream().cuda_stream``.  Importing this
module fails loudly if the shared library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtuckvsie.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                      "(or python -m paper_2103_06393_amd.build)")
_L = ctypes.CDLL(LIB_PATH)

c_i32, c_i64, c_dbl, c_vp, c_sz = (ctypes.c_int32, ctypes.c_int64,
                                   ctypes.c_double, ctypes.c_void_p,
                                   ctypes.c_size_t)

TV_OK = 0
STATUS = {0: "TV_OK", -1: "TV_ERR_INVALID_ARG", -2: "TV_ERR_SHAPE",
          -3: "TV_ERR_RANK", -4: "TV_ERR_OOM", -5: "TV_ERR_HIP",
          -6: "TV_ERR_NOT_SUPPORTED", -7: "TV_ERR_NUMERIC",
          -8: "TV_ERR_WORKSPACE"}
TV_PREC_FP32 = 0
TV_PREC_BF16X3 = 1
TV_MAX_RANK = 64
TV_STATIC_SCRATCH_BYTES = 32 << 20
TV_FIELD_K = 2              # OR into `basis`: the H-field operator of eq. (5)


def field_code(basis: str, operator: str = "N") -> int:
    """`basis` argument of the field entry points: bit 0 PWL, bit 1 K."""
    return (1 if basis == "pwl" else 0) | (TV_FIELD_K if operator == "K" else 0)


class tv_grid(ctypes.Structure):
    _fields_ = [("n1", c_i32), ("n2", c_i32), ("n3", c_i32), ("q", c_i32),
                ("m", c_i64)]


class tv_plan_info_t(ctypes.Structure):
    _fields_ = [("grid", tv_grid), ("precision", ctypes.c_int),
                ("max_rank", c_i32 * 3), ("mean_rank", c_dbl * 3),
                ("sum_r1", c_i64), ("factor_bytes", c_sz),
                ("device_bytes", c_sz), ("flops_matvec", c_dbl),
                ("flops_rmatvec", c_dbl), ("tile_t2", c_i32 * 2),
                ("tile_t3", c_i32 * 2), ("splits", c_i32 * 2), ("kernel", c_i32 * 2)]


class tv_launch_config(ctypes.Structure):
    _fields_ = [("path", c_i32), ("tile_t2", c_i32), ("splits", c_i32),
                ("row_cap", c_i32), ("slab_i3", c_i32), ("gemm_nbw", c_i32),
                ("gemm_order", c_i32)]


class TuckVsieError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {tv_last_error() or STATUS.get(status, status)}")


def _sig(name, args, res=ctypes.c_int):
    f = getattr(_L, name)
    f.argtypes = args
    f.restype = res
    return f


_dp = ctypes.POINTER(c_dbl)
_ip = ctypes.POINTER(c_i32)
_tv_plan_from_factors = _sig("tv_plan_from_factors",
                             [ctypes.POINTER(tv_grid), _ip, _dp, _dp, _dp, _dp,
                              ctypes.c_int, ctypes.POINTER(c_vp)])
_tv_plan_destroy = _sig("tv_plan_destroy", [c_vp])
_tv_plan_info = _sig("tv_plan_info", [c_vp, ctypes.POINTER(tv_plan_info_t)])
_tv_plan_export_factors = _sig("tv_plan_export_factors",
                               [c_vp, _ip, _dp, _dp, _dp, _dp])
_tv_workspace_bytes = _sig("tv_workspace_bytes",
                           [c_vp, c_i32, c_i32, ctypes.POINTER(c_sz)])
_tv_matvec = _sig("tv_matvec", [c_vp, c_vp, c_i64, c_i32, c_vp, c_i64, c_vp,
                                c_sz, c_vp])
_tv_rmatvec = _sig("tv_rmatvec", [c_vp, c_vp, c_i64, c_i32, c_vp, c_i64, c_vp,
                                  c_sz, c_vp])
_tv_dipole_columns = _sig("tv_dipole_columns",
                          [c_i32, c_i32, c_i32, c_dbl, c_dbl, c_i32, c_i64,
                           _dp, _dp, c_vp, c_vp])
_tv_compress_begin = _sig("tv_compress_begin",
                          [ctypes.POINTER(tv_grid), c_dbl, c_i32, c_i32,
                           ctypes.c_int, ctypes.POINTER(c_vp)])
_tv_compress_append = _sig("tv_compress_append", [c_vp, c_vp, c_i64, c_vp, c_sz, c_vp])
_tv_compress_workspace_bytes = _sig("tv_compress_workspace_bytes",
                                    [c_vp, c_i64, ctypes.POINTER(c_sz)])
_tv_plan_required_bytes = _sig("tv_plan_required_bytes", [c_vp, ctypes.POINTER(c_sz)])
_tv_plan_bind_arena = _sig("tv_plan_bind_arena", [c_vp, c_vp, c_sz, c_vp])
_tv_batch_required_bytes = _sig("tv_batch_required_bytes", [c_vp, ctypes.POINTER(c_sz)])
_tv_batch_bind_arena = _sig("tv_batch_bind_arena", [c_vp, c_vp, c_sz, c_vp])
_tv_plan_finalize = _sig("tv_plan_finalize", [c_vp, c_vp])
_tv_compress_discarded = _sig("tv_compress_discarded", [c_vp, _dp])
_tv_autotune = _sig("tv_autotune", [c_vp, c_i32, ctypes.c_char_p, c_vp])
_tv_rmatvec_noalloc = _sig("tv_rmatvec_noalloc", [c_vp, c_vp, c_i64, c_i32, c_vp, c_i64,
                                                   c_vp])
_tv_plan_configure = _sig("tv_plan_configure",
                          [c_vp, c_i32, ctypes.POINTER(tv_launch_config)])
class tv_batch_config(ctypes.Structure):
    _fields_ = [("tsplit", c_i32), ("blocks_per_cu", c_i32)]


_tv_batch_create = _sig("tv_batch_create", [c_i32, ctypes.POINTER(c_vp), c_i32, _ip,
                                            ctypes.POINTER(tv_batch_config),
                                            ctypes.POINTER(c_vp)])
_tv_batch_info = _sig("tv_batch_info", [c_vp, ctypes.POINTER(tv_batch_config)])
_tv_batch_autotune = _sig("tv_batch_autotune", [c_i32, ctypes.POINTER(c_vp), c_i32, _ip,
                                                ctypes.c_char_p, c_vp,
                                                ctypes.POINTER(tv_batch_config)])
_tv_batch_workspace_bytes = _sig("tv_batch_workspace_bytes",
                                 [c_vp, ctypes.POINTER(c_sz)])
_tv_batch_run = _sig("tv_batch_run", [c_vp, ctypes.POINTER(c_vp),
                                      ctypes.POINTER(c_i64), ctypes.POINTER(c_vp),
                                      ctypes.POINTER(c_i64), c_vp, c_sz, c_vp])
_tv_batch_destroy = _sig("tv_batch_destroy", [c_vp])
_tv_aca_workspace_bytes = _sig("tv_aca_workspace_bytes",
                               [c_vp, c_i32, c_i32, ctypes.POINTER(c_sz)])
_tv_aca_matvec = _sig("tv_aca_matvec", [c_vp, c_vp, c_i64, c_i64, c_vp, c_i64,
                                        c_i32, c_vp, c_i64, c_vp, c_sz, c_vp])
_tv_aca_rmatvec = _sig("tv_aca_rmatvec", [c_vp, c_vp, c_i64, c_i64, c_vp,
                                          c_i64, c_i32, c_vp, c_i64, c_vp,
                                          c_sz, c_vp])
_tv_dipole_rows = _sig("tv_dipole_rows", [c_i32, c_i32, c_i32, c_dbl, c_dbl, c_i32,
                                          c_i64, _dp, _dp, c_i64,
                                          ctypes.POINTER(c_i64), c_vp, c_vp])
_tv_aca_assemble = _sig("tv_aca_assemble",
                        [ctypes.POINTER(tv_grid), c_dbl, c_dbl, c_i32, _dp, _dp,
                         c_dbl, c_dbl, c_i32, c_i32, c_i32, ctypes.c_int, c_vp, c_sz,
                         ctypes.POINTER(c_vp), _dp, _ip, _ip,
                         ctypes.POINTER(c_i64), _dp, c_vp])
_tv_aca_assemble_workspace_bytes = _sig("tv_aca_assemble_workspace_bytes",
                                        [ctypes.POINTER(tv_grid), c_i32, c_dbl, c_dbl, c_i32,
                                         c_i32, ctypes.c_int, ctypes.POINTER(c_sz)])
_tv_status_string = _sig("tv_status_string", [ctypes.c_int], ctypes.c_char_p)
_tv_last_error = _sig("tv_last_error", [], ctypes.c_char_p)

EXPORTED = ("tv_plan_from_factors", "tv_plan_required_bytes", "tv_plan_bind_arena",
            "tv_plan_destroy", "tv_plan_info",
            "tv_plan_export_factors", "tv_workspace_bytes", "tv_matvec",
            "tv_rmatvec", "tv_rmatvec_noalloc", "tv_dipole_columns", "tv_compress_begin",
            "tv_compress_workspace_bytes", "tv_compress_append", "tv_plan_finalize",
            "tv_compress_discarded",
            "tv_autotune", "tv_plan_configure", "tv_batch_create", "tv_batch_info", "tv_batch_autotune",
            "tv_batch_required_bytes", "tv_batch_bind_arena",
            "tv_batch_workspace_bytes", "tv_batch_run",
            "tv_batch_destroy", "tv_aca_workspace_bytes", "tv_aca_matvec",
            "tv_aca_rmatvec", "tv_dipole_rows", "tv_aca_assemble_workspace_bytes",
            "tv_aca_assemble",
            "tv_status_string", "tv_last_error")
TV_BATCH_MAX_PLANS = 32


def _check(status: int, where: str):
    if status != TV_OK:
        raise TuckVsieError(status, where)


def _f64(a) -> np.ndarray:
    """Complex or real array -> contiguous float64 view (interleaved)."""
    a = np.ascontiguousarray(a)
    if np.iscomplexobj(a):
        a = np.ascontiguousarray(a.astype(np.complex128)).view(np.float64)
    return np.ascontiguousarray(a, dtype=np.float64)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def make_grid(n1, n2, n3, q, m) -> tv_grid:
    return tv_grid(int(n1), int(n2), int(n3), int(q), int(m))


def tv_status_string(status: int) -> str:
    return _tv_status_string(int(status)).decode()


def tv_last_error() -> str:
    return _tv_last_error().decode()


def tv_plan_from_factors(grid: tv_grid, ranks, cores, u1, u2, u3,
                         precision: int = TV_PREC_FP32) -> int:
    """Returns the plan handle.  ``ranks`` int32 (q*m, 3); the factor arrays
    are complex (or interleaved float64), concatenated in tensor order."""
    r = np.ascontiguousarray(ranks, dtype=np.int32)
    arrs = [_f64(a) for a in (cores, u1, u2, u3)]
    h = c_vp()
    _check(_tv_plan_from_factors(ctypes.byref(grid), r.ctypes.data_as(_ip),
                                 *[_dptr(a) for a in arrs], int(precision),
                                 ctypes.byref(h)), "tv_plan_from_factors")
    return h.value


def tv_plan_destroy(plan: int) -> None:
    _check(_tv_plan_destroy(plan), "tv_plan_destroy")


def tv_plan_info(plan: int) -> tv_plan_info_t:
    info = tv_plan_info_t()
    _check(_tv_plan_info(plan, ctypes.byref(info)), "tv_plan_info")
    return info


def tv_plan_export_factors(plan: int):
    """Returns (ranks int32 (q*m,3), cores, u1, u2, u3) as complex128."""
    info = tv_plan_info(plan)
    g = info.grid
    K = g.q * g.m
    ranks = np.zeros((K, 3), np.int32)
    _check(_tv_plan_export_factors(plan, ranks.ctypes.data_as(_ip), None,
                                   None, None, None), "tv_plan_export_factors")
    r = ranks.astype(np.int64)
    sizes = [int(np.sum(r[:, 0] * r[:, 1] * r[:, 2])), int(np.sum(g.n1 * r[:, 0])),
             int(np.sum(g.n2 * r[:, 1])), int(np.sum(g.n3 * r[:, 2]))]
    bufs = [np.zeros(2 * s, np.float64) for s in sizes]
    _check(_tv_plan_export_factors(plan, ranks.ctypes.data_as(_ip),
                                   *[_dptr(b) for b in bufs]),
           "tv_plan_export_factors")
    return (ranks,) + tuple(b.view(np.complex128) for b in bufs)


def tv_workspace_bytes(plan: int, op: int, nrhs: int) -> int:
    n = c_sz()
    _check(_tv_workspace_bytes(plan, int(op), int(nrhs), ctypes.byref(n)),
           "tv_workspace_bytes")
    return n.value


def tv_matvec(plan, x_ptr, ldx, nrhs, y_ptr, ldy, ws_ptr, ws_bytes, stream):
    _check(_tv_matvec(plan, x_ptr, int(ldx), int(nrhs), y_ptr, int(ldy),
                      ws_ptr, int(ws_bytes), stream), "tv_matvec")


def tv_rmatvec(plan, y_ptr, ldy, nrhs, x_ptr, ldx, ws_ptr, ws_bytes, stream):
    _check(_tv_rmatvec(plan, y_ptr, int(ldy), int(nrhs), x_ptr, int(ldx),
                       ws_ptr, int(ws_bytes), stream), "tv_rmatvec")


def tv_rmatvec_noalloc(plan, y_ptr, ldy, nrhs, x_ptr, ldx, stream):
    _check(_tv_rmatvec_noalloc(plan, y_ptr, int(ldy), int(nrhs), x_ptr, int(ldx), stream),
           "tv_rmatvec_noalloc")


def tv_dipole_columns(n1, n2, n3, h, k0, basis, pos, ori, out_ptr, stream):
    pos = np.ascontiguousarray(pos, np.float64)
    ori = np.ascontiguousarray(ori, np.float64)
    _check(_tv_dipole_columns(int(n1), int(n2), int(n3), float(h), float(k0),
                              int(basis), int(pos.shape[0]), _dptr(pos),
                              _dptr(ori), out_ptr, stream), "tv_dipole_columns")


def tv_compress_begin(grid: tv_grid, tol: float, rank_min: int, rank_cap: int,
                      precision: int = TV_PREC_FP32) -> int:
    h = c_vp()
    _check(_tv_compress_begin(ctypes.byref(grid), float(tol), int(rank_min),
                              int(rank_cap), int(precision), ctypes.byref(h)),
           "tv_compress_begin")
    return h.value


def tv_compress_workspace_bytes(plan, ncols) -> int:
    n = c_sz()
    _check(_tv_compress_workspace_bytes(plan, int(ncols), ctypes.byref(n)),
           "tv_compress_workspace_bytes")
    return n.value


def tv_compress_append(plan, cols_ptr, ncols, ws_ptr, ws_bytes, stream):
    _check(_tv_compress_append(plan, cols_ptr, int(ncols), ws_ptr, int(ws_bytes), stream),
           "tv_compress_append")


def tv_plan_required_bytes(plan) -> int:
    n = c_sz()
    _check(_tv_plan_required_bytes(plan, ctypes.byref(n)), "tv_plan_required_bytes")
    return n.value


def tv_plan_bind_arena(plan, arena_ptr, nbytes, stream):
    _check(_tv_plan_bind_arena(plan, arena_ptr, int(nbytes), stream), "tv_plan_bind_arena")


def tv_batch_required_bytes(batch) -> int:
    n = c_sz()
    _check(_tv_batch_required_bytes(batch, ctypes.byref(n)), "tv_batch_required_bytes")
    return n.value


def tv_batch_bind_arena(batch, arena_ptr, nbytes, stream):
    _check(_tv_batch_bind_arena(batch, arena_ptr, int(nbytes), stream), "tv_batch_bind_arena")


def tv_plan_finalize(plan, stream):
    _check(_tv_plan_finalize(plan, stream), "tv_plan_finalize")


def tv_compress_discarded(plan) -> np.ndarray:
    info = tv_plan_info(plan)
    out = np.zeros((info.grid.q * info.grid.m, 3), np.float64)
    _check(_tv_compress_discarded(plan, _dptr(out)), "tv_compress_discarded")
    return out


def tv_batch_create(plans, op: int, nrhs, tsplit: int = 0, blocks_per_cu: int = 0) -> int:
    n = len(plans)
    parr = (c_vp * n)(*plans)
    r = np.ascontiguousarray(nrhs, dtype=np.int32)
    cfg = tv_batch_config(int(tsplit), int(blocks_per_cu))
    h = c_vp()
    _check(_tv_batch_create(n, parr, int(op), r.ctypes.data_as(_ip), ctypes.byref(cfg),
                            ctypes.byref(h)), "tv_batch_create")
    return h.value


def tv_batch_info(batch) -> tuple:
    cfg = tv_batch_config()
    _check(_tv_batch_info(batch, ctypes.byref(cfg)), "tv_batch_info")
    return cfg.tsplit, cfg.blocks_per_cu


def tv_batch_autotune(plans, op: int, nrhs, cache_path=None, stream=None) -> tuple:
    """Returns the fastest (tsplit, blocks_per_cu)."""
    n = len(plans)
    parr = (c_vp * n)(*plans)
    r = np.ascontiguousarray(nrhs, dtype=np.int32)
    cp = None if cache_path is None else str(cache_path).encode()
    cfg = tv_batch_config()
    _check(_tv_batch_autotune(n, parr, int(op), r.ctypes.data_as(_ip), cp, stream,
                              ctypes.byref(cfg)), "tv_batch_autotune")
    return cfg.tsplit, cfg.blocks_per_cu


def tv_batch_workspace_bytes(batch: int) -> int:
    n = c_sz()
    _check(_tv_batch_workspace_bytes(batch, ctypes.byref(n)),
           "tv_batch_workspace_bytes")
    return n.value


def tv_batch_run(batch, in_ptrs, ld_in, out_ptrs, ld_out, ws_ptr, ws_bytes,
                 stream):
    n = len(in_ptrs)
    _check(_tv_batch_run(batch, (c_vp * n)(*in_ptrs), (c_i64 * n)(*ld_in),
                         (c_vp * n)(*out_ptrs), (c_i64 * n)(*ld_out), ws_ptr,
                         int(ws_bytes), stream), "tv_batch_run")


def tv_batch_destroy(batch: int) -> None:
    _check(_tv_batch_destroy(batch), "tv_batch_destroy")


def tv_plan_configure(plan: int, op: int, path: int = 0, tile_t2: int = 0,
                      splits: int = 1, row_cap: int = 0, slab_i3: int = 0,
                      gemm_nbw: int = 2, gemm_order: int = 0) -> None:
    cfg = tv_launch_config(int(path), int(tile_t2), int(splits), int(row_cap),
                           int(slab_i3), int(gemm_nbw), int(gemm_order))
    _check(_tv_plan_configure(plan, int(op), ctypes.byref(cfg)), "tv_plan_configure")


def tv_autotune(plan: int, op: int = 2, cache_path=None, stream=None) -> None:
    cp = None if cache_path is None else str(cache_path).encode()
    _check(_tv_autotune(plan, int(op), cp, stream), "tv_autotune")


def tv_aca_workspace_bytes(plan: int, op: int, nrhs: int) -> int:
    n = c_sz()
    _check(_tv_aca_workspace_bytes(plan, int(op), int(nrhs), ctypes.byref(n)),
           "tv_aca_workspace_bytes")
    return n.value


def tv_aca_matvec(plan, v_ptr, m, ldv, x_ptr, ldx, nrhs, y_ptr, ldy, ws_ptr,
                  ws_bytes, stream):
    _check(_tv_aca_matvec(plan, v_ptr, int(m), int(ldv), x_ptr, int(ldx),
                          int(nrhs), y_ptr, int(ldy), ws_ptr, int(ws_bytes),
                          stream), "tv_aca_matvec")


def tv_aca_rmatvec(plan, v_ptr, m, ldv, y_ptr, ldy, nrhs, x_ptr, ldx, ws_ptr,
                   ws_bytes, stream):
    _check(_tv_aca_rmatvec(plan, v_ptr, int(m), int(ldv), y_ptr, int(ldy),
                           int(nrhs), x_ptr, int(ldx), ws_ptr, int(ws_bytes),
                           stream), "tv_aca_rmatvec")


def tv_dipole_rows(n1, n2, n3, h, k0, basis, pos, ori, rows, out_ptr, stream):
    pos = np.ascontiguousarray(pos, np.float64)
    ori = np.ascontiguousarray(ori, np.float64)
    r = np.ascontiguousarray(rows, np.int64)
    _check(_tv_dipole_rows(int(n1), int(n2), int(n3), float(h), float(k0),
                           int(basis), int(pos.shape[0]), _dptr(pos), _dptr(ori),
                           int(r.shape[0]), r.ctypes.data_as(ctypes.POINTER(c_i64)),
                           out_ptr, stream), "tv_dipole_rows")


def tv_aca_assemble_workspace_bytes(grid: tv_grid, max_terms, tol, hosvd_tol=0.0,
                                    rank_min=1, rank_cap=0,
                                    precision=TV_PREC_FP32) -> int:
    n = c_sz()
    _check(_tv_aca_assemble_workspace_bytes(ctypes.byref(grid), int(max_terms), float(tol),
                                            float(hosvd_tol), int(rank_min), int(rank_cap),
                                            int(precision), ctypes.byref(n)),
           "tv_aca_assemble_workspace_bytes")
    return n.value


def tv_aca_assemble(grid: tv_grid, h, k0, basis, pos, ori, tol, hosvd_tol=0.0,
                    rank_min=1, rank_cap=0, max_terms=64,
                    precision=TV_PREC_FP32, stream=None, ws_ptr=None, ws_bytes=0):
    """Algorithm 3 on the device, with the caller's device workspace
    (tv_aca_assemble_workspace_bytes).  Returns (plan handle (unbound),
    V complex128 (m x r_c), r_c, converged, pivots int64 (r_c x 2),
    s float64 (r_c,))."""
    pos = np.ascontiguousarray(pos, np.float64)
    ori = np.ascontiguousarray(ori, np.float64)
    m, K = int(grid.m), int(max_terms)
    V = np.zeros(2 * m * K, np.float64)
    piv = np.zeros(2 * K, np.int64)
    sv = np.zeros(K, np.float64)
    h_plan = c_vp()
    rc = c_i32()
    conv = c_i32()
    _check(_tv_aca_assemble(ctypes.byref(grid), float(h), float(k0), int(basis),
                            _dptr(pos), _dptr(ori), float(tol), float(hosvd_tol),
                            int(rank_min), int(rank_cap), K, int(precision),
                            ws_ptr, int(ws_bytes),
                            ctypes.byref(h_plan), _dptr(V), ctypes.byref(rc),
                            ctypes.byref(conv),
                            piv.ctypes.data_as(ctypes.POINTER(c_i64)), _dptr(sv),
                            stream), "tv_aca_assemble")
    n = rc.value
    Vc = V.view(np.complex128).reshape(K, m).T[:, :n].copy()
    return (h_plan.value, Vc, n, bool(conv.value), piv.reshape(K, 2)[:n].copy(),
            sv[:n].copy())
