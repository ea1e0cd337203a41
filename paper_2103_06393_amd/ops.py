"""Torch-facing wrappers over the C ABI.

``TuckerPlan`` holds a plan and runs Y = Z X / X = Z^* Y on torch complex64
CUDA tensors through ``tv_matvec`` / ``tv_rmatvec``; the plan's device arena,
compression scratch, outputs and workspaces all come from torch's caching
allocator: the library itself never allocates device memory for them.  ``TuckerMatvec`` is the autograd Function whose
backward is the adjoint kernel: for the linear map y = Z x the
vector-Jacobian product is Z^* g (the conjugate transpose needed by the GMT
cost gradient, Sec. II.A.2).
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import lib


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _check_operand(t: torch.Tensor, rows: int, name: str) -> int:
    """Validate a product operand before its pointer reaches the C ABI:
    complex64, on the current CUDA device, shaped (rows,) or (rows, p).
    Returns p.  Raises ValueError otherwise (no kernel is launched)."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != torch.complex64:
        raise ValueError(f"{name} must be complex64, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor, got {t.device}")
    if t.device.index != torch.cuda.current_device():
        raise ValueError(f"{name} must be on the current CUDA device "
                         f"(cuda:{torch.cuda.current_device()}), got {t.device}")
    if t.dim() not in (1, 2) or t.shape[0] != rows or (t.dim() == 2 and t.shape[1] < 1):
        raise ValueError(f"{name} must be shaped ({rows},) or ({rows}, p), "
                         f"got {tuple(t.shape)}")
    return 1 if t.dim() == 1 else int(t.shape[1])


def _check_out(out: torch.Tensor, p: int, rows: int, device) -> torch.Tensor:
    """The output buffer of a product, returned as the (p, rows) view the
    C ABI writes (column-major rows x p): complex64 on the operand's device,
    either contiguous with p * rows elements or a (rows, p) column-major view."""
    if not isinstance(out, torch.Tensor) or out.dtype != torch.complex64:
        raise ValueError("out must be a complex64 tensor")
    if out.device != device:
        raise ValueError(f"out must be on {device}, got {out.device}")
    buf = out
    if out.dim() == 2 and tuple(out.shape) == (rows, p) and out.stride() == (1, rows):
        buf = out.t()
    shape_ok = (buf.dim() == 1 and p == 1) or tuple(buf.shape) == (p, rows)
    if not shape_ok or not buf.is_contiguous() or buf.numel() != p * rows:
        raise ValueError(f"out must be contiguous with {p * rows} elements or a "
                         f"({rows}, {p}) column-major view, got shape "
                         f"{tuple(out.shape)} strides {out.stride()}")
    return buf.view(p, rows)


def _device_bytes(n: int) -> torch.Tensor:
    """A device buffer of at least n bytes (torch's allocator aligns to 512)."""
    return torch.empty(max(int(n), 256), dtype=torch.uint8, device="cuda")


def batch_create(handles, op: int, nrhs, config=(0, 0)):
    """tv_batch_create (config = (tsplit, blocks_per_cu), zeros: automatic)
    plus its device arena: returns (batch handle, arena); the arena tensor
    must outlive the batch."""
    b = lib.tv_batch_create(handles, op, nrhs, *config)
    try:
        nb = lib.tv_batch_required_bytes(b)
        arena = _device_bytes(nb)
        lib.tv_batch_bind_arena(b, arena.data_ptr(), arena.numel(), _stream())
    except Exception:
        lib.tv_batch_destroy(b)
        raise
    return b, arena


class TuckerPlan:
    def __init__(self, handle: int):
        self.handle = handle
        # the plan's packed factors live in a device arena from torch
        try:
            nb = lib.tv_plan_required_bytes(handle)
            self._arena = _device_bytes(nb)
            lib.tv_plan_bind_arena(handle, self._arena.data_ptr(), self._arena.numel(),
                                   _stream())
        except Exception:
            lib.tv_plan_destroy(handle)
            self.handle = 0
            raise
        g = self.info.grid
        self.dims = (g.n1, g.n2, g.n3)
        self.q = g.q
        self.m = g.m
        self.nv = g.n1 * g.n2 * g.n3
        self.rows = self.q * self.nv
        self._ws = {}

    @property
    def info(self) -> lib.tv_plan_info_t:
        """Plan summary queried now (the launch configuration changes with
        autotuning)."""
        return lib.tv_plan_info(self.handle)

    # -- construction ---------------------------------------------------
    @classmethod
    def from_factors(cls, dims, q, m, ranks, cores, u1, u2, u3,
                     precision: int = lib.TV_PREC_FP32) -> "TuckerPlan":
        grid = lib.make_grid(*dims, q, m)
        return cls(lib.tv_plan_from_factors(grid, ranks, cores, u1, u2, u3,
                                            precision))

    @classmethod
    def compress_dipoles(cls, dims, h, k0, basis, pos, ori, tol, rank_min=1,
                         rank_cap=0, precision: int = lib.TV_PREC_FP32,
                         chunk: Optional[int] = None) -> "TuckerPlan":
        """Generate point-current columns on the device and compress them
        with the library's truncated HOSVD, a chunk of columns at a time."""
        q = 12 if basis & 1 else 3
        m = int(pos.shape[0])
        nv = int(np.prod(dims))
        grid = lib.make_grid(*dims, q, m)
        h_plan = lib.tv_compress_begin(grid, tol, rank_min, rank_cap, precision)
        try:
            if chunk is None:       # about 24 GiB of complex128 columns (of 288 GB)
                chunk = max(1, min(m, (24 << 30) // (16 * q * nv), 65535 // q))
            buf = torch.empty(chunk * q * nv * 2, dtype=torch.float64,
                              device="cuda")
            ws = _device_bytes(lib.tv_compress_workspace_bytes(h_plan, chunk))
            st = _stream()
            for j0 in range(0, m, chunk):
                n = min(chunk, m - j0)
                lib.tv_dipole_columns(*dims, h, k0, basis, pos[j0:j0 + n],
                                      ori[j0:j0 + n], buf.data_ptr(), st)
                lib.tv_compress_append(h_plan, buf.data_ptr(), n, ws.data_ptr(),
                                       ws.numel(), st)
            del buf, ws
            lib.tv_plan_finalize(h_plan, st)
        except Exception:
            lib.tv_plan_destroy(h_plan)
            raise
        return cls(h_plan)

    def close(self):
        if self.handle:
            lib.tv_plan_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- products ---------------------------------------------------------
    def workspace(self, op: int, nrhs: int) -> torch.Tensor:
        key = (op, nrhs)
        if key not in self._ws:
            n = lib.tv_workspace_bytes(self.handle, op, nrhs)
            self._ws[key] = torch.empty(max(n, 16), dtype=torch.uint8,
                                        device="cuda")
        return self._ws[key]

    def matvec(self, x: torch.Tensor, out: Optional[torch.Tensor] = None):
        """Y = Z X for x of shape (m,) or (m, p), complex64 on the GPU."""
        p = _check_operand(x, self.m, "x")
        vec = x.dim() == 1
        X = x.reshape(self.m, -1)
        Xc = X.t().contiguous()                  # column-major m x p
        Y = _check_out(out, p, self.rows, x.device) if out is not None else torch.empty(
            (p, self.rows), dtype=torch.complex64, device=x.device)
        ws = self.workspace(0, p)
        lib.tv_matvec(self.handle, Xc.data_ptr(), self.m, p, Y.data_ptr(),
                      self.rows, ws.data_ptr(), ws.numel(), _stream())
        return Y.reshape(-1) if vec else Y.t()

    def rmatvec(self, y: torch.Tensor, out: Optional[torch.Tensor] = None):
        """X = Z^* Y for y of shape (q nv,) or (q nv, p), complex64."""
        p = _check_operand(y, self.rows, "y")
        vec = y.dim() == 1
        Yv = y.reshape(self.rows, -1)
        Yc = Yv.t().contiguous()
        X = _check_out(out, p, self.m, y.device) if out is not None else torch.empty(
            (p, self.m), dtype=torch.complex64, device=y.device)
        ws = self.workspace(1, p)
        lib.tv_rmatvec(self.handle, Yc.data_ptr(), self.rows, p, X.data_ptr(),
                       self.m, ws.data_ptr(), ws.numel(), _stream())
        return X.reshape(-1) if vec else X.t()

    def autotune(self, op: int = 2, cache_path: Optional[str] = None):
        """Time the kernel configurations and keep the fastest (set-up call)."""
        lib.tv_autotune(self.handle, op, cache_path, _stream())
        self._ws.clear()

    def export_factors(self):
        return lib.tv_plan_export_factors(self.handle)


class AcaTuckerOperator:
    """Z ~= U V^* with U's r_c columns in a Tucker plan (Algorithm 3's
    output) and V (m x r_c, complex64 on the GPU): Z X = U (V^* X) and
    Z^* Y = V (U^* Y) through tv_aca_matvec / tv_aca_rmatvec (Sec. III.B)."""

    def __init__(self, plan: TuckerPlan, V: torch.Tensor):
        if not isinstance(V, torch.Tensor) or V.dim() != 2 or V.shape[1] != plan.m:
            raise ValueError("V must be m x r_c with r_c = the plan's columns")
        if not V.is_cuda:
            raise ValueError("V must be on the GPU")
        self.plan = plan
        self.m = int(V.shape[0])
        self.rows = plan.rows
        # column-major m x r_c: the transpose of a contiguous (r_c, m) tensor
        self.Vc = V.to(torch.complex64).t().contiguous()
        self._ws = {}

    def workspace(self, op: int, nrhs: int) -> torch.Tensor:
        key = (op, nrhs)
        if key not in self._ws:
            n = lib.tv_aca_workspace_bytes(self.plan.handle, op, nrhs)
            self._ws[key] = torch.empty(max(n, 16), dtype=torch.uint8,
                                        device="cuda")
        return self._ws[key]

    def matvec(self, x: torch.Tensor) -> torch.Tensor:
        """Y = U (V^* X) for x of shape (m,) or (m, p)."""
        p = _check_operand(x, self.m, "x")
        vec = x.dim() == 1
        X = x.reshape(self.m, -1)
        Xc = X.t().contiguous()
        Y = torch.empty((p, self.rows), dtype=torch.complex64, device=x.device)
        ws = self.workspace(0, p)
        lib.tv_aca_matvec(self.plan.handle, self.Vc.data_ptr(), self.m, self.m,
                          Xc.data_ptr(), self.m, p, Y.data_ptr(), self.rows,
                          ws.data_ptr(), ws.numel(), _stream())
        return Y.reshape(-1) if vec else Y.t()

    def rmatvec(self, y: torch.Tensor) -> torch.Tensor:
        """X = V (U^* Y) for y of shape (q nv,) or (q nv, p)."""
        p = _check_operand(y, self.rows, "y")
        vec = y.dim() == 1
        Yv = y.reshape(self.rows, -1)
        Yc = Yv.t().contiguous()
        X = torch.empty((p, self.m), dtype=torch.complex64, device=y.device)
        ws = self.workspace(1, p)
        lib.tv_aca_rmatvec(self.plan.handle, self.Vc.data_ptr(), self.m,
                           self.m, Yc.data_ptr(), self.rows, p, X.data_ptr(),
                           self.m, ws.data_ptr(), ws.numel(), _stream())
        return X.reshape(-1) if vec else X.t()


def aca_assemble(wl_dims, h, k0, basis, pos, ori, tol, hosvd_tol=0.0,
                 rank_min=1, rank_cap=0, max_terms=64,
                 precision: int = lib.TV_PREC_FP32):
    """Algorithm 3 (Tucker-based ACA) on the device for point-current coil
    elements: returns an AcaTuckerOperator (U as a Tucker plan, V on the GPU)
    and a dict with r_c, convergence, the pivots and the norm estimates."""
    q = 12 if basis & 1 else 3
    grid = lib.make_grid(*wl_dims, q, int(pos.shape[0]))
    ws = _device_bytes(lib.tv_aca_assemble_workspace_bytes(
        grid, max_terms, tol, hosvd_tol, rank_min, rank_cap, precision))
    h_plan, V, rc, conv, piv, s = lib.tv_aca_assemble(
        grid, h, k0, basis, pos, ori, tol, hosvd_tol, rank_min, rank_cap,
        max_terms, precision, _stream(), ws.data_ptr(), ws.numel())
    del ws
    plan = TuckerPlan(h_plan)
    op = AcaTuckerOperator(plan, torch.from_numpy(V.astype(np.complex64)).cuda())
    return op, {"rc": rc, "converged": conv, "pivots": piv, "s": s, "V": V}


class TuckerMatvec(torch.autograd.Function):
    """y = Z x with the hand-written Z^* kernel as the backward."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, plan: TuckerPlan):
        ctx.plan = plan
        return plan.matvec(x)

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        return ctx.plan.rmatvec(g.contiguous()), None
