"""Adaptive cross approximation and the ACA + Tucker products (oracle, FP64).

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.

Sec. II.B.2: a matrix A (m1 x m2) is approximated as U V^* (U: m1 x r_c,
V: m2 x r_c) from a few of its rows and columns by the adaptive cross
approximation (ACA) with partial pivoting.  Algorithm 3 (Sec. III.C) runs
that loop with U held compressed: each new column of U is split into its q
voxel tensors and compressed at once by a truncated HOSVD of tolerance
3 eps; a row of U is read by decompressing single elements (eq. 6), and
products with U are Algorithms 1 and 2.

``aca`` below is the residual-cross iteration of the ACA for either storage
of U: ``DenseU`` (the traditional ACA that Algorithm 3 extends) or
``TuckerU`` (Algorithm 3 proper: compressed columns, single-element rows,
products by Algorithms 1 and 2).

Readings where the paper is silent or its printed formula is off:
* the norm estimate's cross term is 2 Re sum_l conj((V^* y)_l) (U^* x)_l,
  the exact expansion of ||U V^* + x y^*||_F^2; the printed Hadamard
  product carries no conjugate, which is not a norm for complex data;
* indices are 0-based and the first pivot row is row 0;
* a row residual that is exactly zero ends the loop (its pivot division is
  undefined);
* the HOSVD tolerance 3 eps is relative to each tensor's own norm, as for
  the plain compression.

Products with Z = U V^* (Sec. III.B, the substitution stated after
Algorithms 1 and 2; Table III, row ACA+Tucker): Z X = U (V^* X), i.e.
Algorithm 1 on U with X replaced by V^* X, and Z^* Y = V (U^* Y), i.e.
Algorithm 2 on U followed by a product with V.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

from . import fields
from .hosvd import hosvd
from .matvec import TuckerStruct, alg1, alg2, column, entries


class DenseU:
    """U kept as dense columns: the traditional ACA."""

    def __init__(self):
        self.cols: List[np.ndarray] = []

    @property
    def k(self) -> int:
        return len(self.cols)

    def row(self, i: int) -> np.ndarray:
        """Row i of U (length k)."""
        return np.array([c[i] for c in self.cols], np.complex128)

    def times(self, w: np.ndarray) -> np.ndarray:
        """U w."""
        return self.dense() @ np.asarray(w, np.complex128)

    def adjoint_times(self, x: np.ndarray) -> np.ndarray:
        """U^* x."""
        return self.dense().conj().T @ np.asarray(x, np.complex128)

    def append(self, x: np.ndarray) -> None:
        self.cols.append(np.array(x, np.complex128))

    def dense(self) -> np.ndarray:
        return np.stack(self.cols, axis=1)


class TuckerU:
    """U kept as a q x r_c struct of Tucker tensors (Algorithm 3)."""

    def __init__(self, dims, q: int, tol: float, rank_min: int = 1,
                 rank_cap: Optional[int] = None):
        self.S = TuckerStruct(tuple(dims), q, [])
        self.tol, self.rank_min, self.rank_cap = tol, rank_min, rank_cap

    @property
    def k(self) -> int:
        return self.S.m

    def row(self, i: int) -> np.ndarray:
        """Row i of U by single-element decompression: split i into the
        component p and voxel (f1, f2, f3), then for every column l
        t_l = G x1 U1[f1,:] x2 U2[f2,:] x3 U3[f3,:] of tensor U_{pl}."""
        n1, n2, _ = self.S.dims
        p, v = divmod(int(i), self.S.nv)
        f1, f2, f3 = v % n1, (v // n1) % n2, v // (n1 * n2)
        t = np.zeros(self.k, np.complex128)
        for l in range(self.k):
            tk = self.S.t[l][p]
            U1, U2, U3 = tk.U
            t[l] = np.einsum("abc,a,b,c->", tk.G, U1[f1], U2[f2], U3[f3])
        return t

    def times(self, w: np.ndarray) -> np.ndarray:
        """U w (the product of Algorithm 1 with U's struct)."""
        return alg1(self.S, np.asarray(w).reshape(-1, 1))[:, 0]

    def adjoint_times(self, x: np.ndarray) -> np.ndarray:
        """U^* x (the product of Algorithm 2 with U's struct)."""
        return alg2(self.S, np.asarray(x).reshape(-1, 1))[:, 0]

    def append(self, x: np.ndarray) -> None:
        """Reshape x to q voxel tensors (column-major, as (:) vectorises)
        and compress each with the truncated HOSVD."""
        nv = self.S.nv
        col = []
        for p in range(self.S.q):
            T = np.asarray(x[p * nv:(p + 1) * nv]).reshape(self.S.dims,
                                                           order="F")
            col.append(hosvd(T, self.tol, self.rank_min, self.rank_cap))
        self.S.t.append(col)

    def dense(self) -> np.ndarray:
        return np.stack([column(self.S, l) for l in range(self.k)], axis=1)


@dataclasses.dataclass
class ACAResult:
    U: object                  # DenseU or TuckerU, r_c columns
    V: np.ndarray              # m2 x r_c
    rows: List[int]            # pivot row of each step
    cols: List[int]            # pivot column of each step
    s: List[float]             # norm estimate s_{k+1} after each step
    converged: bool

    @property
    def rc(self) -> int:
        return self.V.shape[1]


def _residual_row(row, U, V, i: int) -> np.ndarray:
    """Row i of the residual Z - U V^*: Z's row minus (row i of U) V^*."""
    r = np.array(row(i), np.complex128)
    return r if U.k == 0 else r - V.conj() @ U.row(i)


def _residual_col(col, U, V, j: int) -> np.ndarray:
    """Column j of the residual Z - U V^*: Z's column minus U conj(V[j, :])."""
    x = np.array(col(j), np.complex128)
    return x if U.k == 0 else x - U.times(V[j, :].conj())


def _norm2_with_cross(s: float, u: np.ndarray, v: np.ndarray, U, V) -> float:
    """||U V^* + u v^*||_F^2 from s = ||U V^*||_F^2, by expanding the square:
    ||A + u v^*||^2 = ||A||^2 + ||u||^2 ||v||^2 + 2 Re <A, u v^*>, where
    <U V^*, u v^*> = trace(V U^* u v^*) = sum_l conj((V^* v)_l) (U^* u)_l."""
    out = s + float(np.linalg.norm(u) * np.linalg.norm(v)) ** 2
    if U.k:
        out += 2.0 * float(np.real(np.vdot(V.conj().T @ v, U.adjoint_times(u))))
    return out


def aca(row: Callable[[int], np.ndarray], col: Callable[[int], np.ndarray],
        m1: int, m2: int, tol: float, U, max_rank: Optional[int] = None
        ) -> ACAResult:
    """Adaptive cross approximation with partial pivoting (Sec. II.B.2) of
    Z (m1 x m2), given by its rows and columns; U is a DenseU or a TuckerU
    (Algorithm 3 runs this loop with U compressed, Sec. III.C).

    Z ~= U V^* grows by one rank-1 cross u v^* per step, chosen on the
    residual R = Z - U V^*: from the current pivot row i of R, the pivot
    column j is its entry of largest modulus, and u = R[:, j],
    v = conj(R[i, :] / R[i, j]), so that u v^* reproduces row i and column j
    of R exactly.  The estimate s of ||U V^*||_F^2 follows the expansion in
    _norm2_with_cross; the loop ends once ||u|| ||v|| <= tol sqrt(s), or at a
    residual row that is exactly zero; otherwise the next pivot row is the
    entry of u of largest modulus other than row i.
    """
    kmax = min(m1, m2) if max_rank is None else min(m1, m2, max_rank)
    V = np.zeros((m2, 0), np.complex128)
    rows, cols, hist = [], [], []
    s = 0.0
    converged = False
    i = 0
    while U.k < kmax:
        r = _residual_row(row, U, V, i)
        j = int(np.argmax(np.abs(r)))
        if r[j] == 0:
            converged = True
            break
        v = np.conj(r / r[j])
        u = _residual_col(col, U, V, j)
        s = _norm2_with_cross(s, u, v, U, V)
        size = float(np.linalg.norm(u) * np.linalg.norm(v))
        U.append(u)
        V = np.column_stack([V, v])
        rows.append(i)
        cols.append(j)
        hist.append(s)
        if size <= tol * math.sqrt(s):
            converged = True
            break
        mod = np.abs(u)
        mod[i] = 0.0
        i = int(np.argmax(mod))
    return ACAResult(U, V, rows, cols, hist, converged)


def aca_dense(A: np.ndarray, tol: float, max_rank: Optional[int] = None
              ) -> ACAResult:
    """Traditional ACA of an explicit matrix (rows and columns read from A)."""
    A = np.asarray(A, np.complex128)
    return aca(lambda i: A[i, :], lambda j: A[:, j], A.shape[0], A.shape[1],
               tol, DenseU(), max_rank)


def aca_tucker(wl, tol: float, hosvd_tol: Optional[float] = None,
               rank_min: int = 1, rank_cap: Optional[int] = None,
               max_rank: Optional[int] = None) -> ACAResult:
    """Algorithm 3 on a workload's coupling matrix: rows and columns from
    the closed-form point-current fields, U compressed with HOSVD(3 eps)."""
    U = TuckerU(wl.grid.dims, wl.q, 3.0 * tol if hosvd_tol is None
                else hosvd_tol, rank_min, rank_cap)
    return aca(lambda i: fields.row_vector(wl, i),
               lambda j: fields.column_vector(wl, j),
               wl.rows, wl.m, tol, U, max_rank)


def aca_matvec(S: TuckerStruct, V: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Z X = U (V^* X): Algorithm 1 on U with X replaced by V^* X."""
    V = np.asarray(V, np.complex128)
    X = np.asarray(X, np.complex128).reshape(V.shape[0], -1)
    return alg1(S, V.conj().T @ X)


def aca_rmatvec(S: TuckerStruct, V: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Z^* Y = V (U^* Y): Algorithm 2 on U, then V."""
    V = np.asarray(V, np.complex128)
    return V @ alg2(S, Y)


def aca_entries(S: TuckerStruct, V: np.ndarray, x: np.ndarray,
                rows) -> np.ndarray:
    """Selected entries of U (V^* x) by single-element decompression."""
    w = np.asarray(V, np.complex128).conj().T @ np.asarray(x, np.complex128)
    return entries(S, w, rows)
