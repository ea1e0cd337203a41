"""Matrix-vector products with the Tucker-compressed coupling matrix (oracle).

Sec. III.B: the coupling matrix Z (q nv x m) is held as a q x m struct of
Tucker tensors Z^{kj}.  Algorithm 1 forms Y = Z X by decompressing each
Z^{kj} and adding Z^{kj}(:) X_{j,:} into block Y^k; Algorithm 2 forms
Y = Z^* X (conjugate transpose, Table I) by decompressing the q tensors of
column j and taking their conjugated inner product with X.  (:) is the
column-major vectorisation, so row k nv + i1 + n1 (i2 + n2 i3) of Z holds
voxel (i1, i2, i3) of component k.

Everything is complex128.  The products are computed from their definition
(decompressed columns times the vectors, a library matrix product per block
of columns); nothing is fused or reordered beyond that blocking.
"""
from __future__ import annotations

import dataclasses
from typing import Iterable, List, Optional, Sequence

import numpy as np

from . import fields
from .hosvd import Tucker, hosvd, tucker_full


def vec(T: np.ndarray) -> np.ndarray:
    """Column-major vectorisation T(:)."""
    return T.reshape(-1, order="F")


@dataclasses.dataclass
class TuckerStruct:
    """The struct of Tucker tensors, q x m (Sec. III.C, Table I).

    ``t[j][k]`` is the Tucker tensor of component k of column j.
    """
    dims: tuple
    q: int
    t: List[List[Tucker]]

    @property
    def m(self) -> int:
        return len(self.t)

    @property
    def nv(self) -> int:
        return int(np.prod(self.dims))

    def ranks(self) -> np.ndarray:
        """(m, q, 3) int array of multilinear ranks."""
        return np.array([[tk.ranks for tk in col] for col in self.t])


def from_factors(dims, q, cores, factors) -> TuckerStruct:
    """Struct from raw factors: ``cores[j][k]`` and ``factors[j][k] = (U1,U2,U3)``."""
    cols = []
    for j in range(len(cores)):
        col = []
        for k in range(q):
            U = [np.asarray(u, np.complex128) for u in factors[j][k]]
            col.append(Tucker(np.asarray(cores[j][k], np.complex128), U,
                              [None] * 3, np.zeros(3), float("nan")))
        cols.append(col)
    return TuckerStruct(tuple(dims), q, cols)


def compress_columns(wl, cols: Optional[Iterable[int]] = None) -> TuckerStruct:
    """Compress columns of a workload tensor by tensor with the HOSVD
    (Sec. III.A, Fig. 2), tolerance per tensor (Algorithm 3 applies its
    HOSVD per reshaped tensor)."""
    js = range(wl.m) if cols is None else list(cols)
    out = []
    for j in js:
        T = fields.column_tensors(wl, j)
        out.append([hosvd(T[k], wl.tol, wl.rank_min, wl.rank_cap)
                    for k in range(wl.q)])
    return TuckerStruct(wl.grid.dims, wl.q, out)


def _block(S: TuckerStruct, entries: int = 1 << 22) -> int:
    """Columns of Z formed at once: about ``entries`` complex entries
    (default 2^22, 64 MiB)."""
    return max(1, entries // (S.q * S.nv))


def alg1(S: TuckerStruct, X: np.ndarray, block_entries: int = 1 << 22) -> np.ndarray:
    """Y = Z X, the product Algorithm 1 computes, from its definition: the
    columns of Z are the decompressed tensors (eq. 6) stacked in component
    order, and Y is the matrix product Z X, taken over blocks of columns so
    that only a block of Z (about ``block_entries`` entries) exists at a time.
    X is m x p; returns q nv x p."""
    X = np.asarray(X, np.complex128).reshape(S.m, -1)
    Y = np.zeros((S.q * S.nv, X.shape[1]), np.complex128)
    b = _block(S, block_entries)
    for j0 in range(0, S.m, b):
        js = range(j0, min(S.m, j0 + b))
        Y += np.stack([column(S, j) for j in js], axis=1) @ X[j0:j0 + len(js)]
    return Y


def alg2(S: TuckerStruct, X: np.ndarray, block_entries: int = 1 << 22) -> np.ndarray:
    """Y = Z^* X (conjugate transpose, Table I), the product Algorithm 2
    computes, from its definition over blocks of decompressed columns as in
    alg1.  X is q nv x p; returns m x p."""
    X = np.asarray(X, np.complex128).reshape(S.q * S.nv, -1)
    Y = np.zeros((S.m, X.shape[1]), np.complex128)
    b = _block(S, block_entries)
    for j0 in range(0, S.m, b):
        js = range(j0, min(S.m, j0 + b))
        Y[j0:j0 + len(js)] = np.stack([column(S, j) for j in js], axis=1).conj().T @ X
    return Y


def column(S: TuckerStruct, j: int) -> np.ndarray:
    """Decompressed column j of Z."""
    return np.concatenate([vec(S.t[j][k].full()) for k in range(S.q)])


def entries(S: TuckerStruct, x: np.ndarray, rows: Sequence[int]) -> np.ndarray:
    """Selected entries of y = Z x without forming any tensor.

    Each row is split into its component and voxel indices (f1, f2, f3) and
    each tensor is decompressed at that single element,
    t = G x1 U1[f1,:] x2 U2[f2,:] x3 U3[f3,:] (Sec. III.C).
    """
    n1, n2, _ = S.dims
    x = np.asarray(x, np.complex128).reshape(-1)
    out = np.zeros(len(rows), np.complex128)
    for i, row in enumerate(rows):
        k, v = divmod(int(row), S.nv)
        f1 = v % n1
        f2 = (v // n1) % n2
        f3 = v // (n1 * n2)
        acc = 0.0 + 0.0j
        for j in range(S.m):
            tk = S.t[j][k]
            U1, U2, U3 = tk.U
            t = np.einsum("abc,a,b,c->", tk.G, U1[f1], U2[f2], U3[f3])
            acc += x[j] * t
        out[i] = acc
    return out


def fibre(S: TuckerStruct, X: np.ndarray, k: int, i2: int, i3: int) -> np.ndarray:
    """The n1 entries of Y = Z X along the mode-1 fibre (k, :, i2, i3): the
    single-element decompression of Sec. III.C kept open in mode 1, i.e.
    U1 (G x2 U2[i2,:] x3 U3[i3,:]) for every column j, weighted by X_{j,:}.
    X is m x p (or length m); returns n1 x p (or n1)."""
    x = np.asarray(X, np.complex128)
    Xm = x.reshape(S.m, -1)
    out = np.zeros((S.dims[0], Xm.shape[1]), np.complex128)
    for j in range(S.m):
        t = S.t[j][k]
        g = np.einsum("abc,b,c->a", t.G, t.U[1][i2], t.U[2][i3])
        out += np.outer(t.U[0] @ g, Xm[j])
    return out[:, 0] if x.ndim == 1 else out


def adjoint_entries(S: TuckerStruct, y: np.ndarray,
                    cols: Sequence[int]) -> np.ndarray:
    """Selected entries of Z^* Y: Algorithm 2's inner step for chosen j.
    Y is a vector (returns len(cols)) or q nv x p (returns len(cols) x p)."""
    Y = np.asarray(y, np.complex128)
    if Y.ndim == 1:
        return np.array([np.vdot(column(S, j), Y) for j in cols])
    return np.stack([column(S, j).conj() @ Y for j in cols])


def dense(wl, cols: Optional[Iterable[int]] = None) -> np.ndarray:
    """Uncompressed coupling matrix (q nv x m) from the closed-form columns."""
    js = range(wl.m) if cols is None else list(cols)
    return np.stack([fields.column_vector(wl, j) for j in js], axis=1)


def loss(S: TuckerStruct, x: np.ndarray, b: np.ndarray) -> float:
    """L(x) = ||Z x - b||^2."""
    r = alg1(S, x).reshape(-1) - np.asarray(b).reshape(-1)
    return float(np.vdot(r, r).real)


def loss_grad(S: TuckerStruct, x: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Gradient of L as dL/dRe x + i dL/dIm x = 2 Z^* (Z x - b).

    Z^* is applied with Algorithm 2, as the gradient of the GMT cost needs
    products with the conjugate transpose (Sec. II.A.2).
    """
    r = alg1(S, x).reshape(-1) - np.asarray(b).reshape(-1)
    return 2.0 * alg2(S, r[:, None]).reshape(-1)


def truncation_bound(S: TuckerStruct) -> np.ndarray:
    """Per-column bound e_j = (sum_k discarded_kj)^(1/2) on ||Z_j - Zhat_j||.

    From the HOSVD bound ||A - A_hat||^2 <= sum_n discarded_n per tensor.
    """
    return np.array([np.sqrt(sum(float(np.sum(t.discarded)) for t in col))
                     for col in S.t])
