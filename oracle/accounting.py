"""Memory and operation counts of Tables II and III (oracle).

Table II lists the memory of the full coupling matrix (q nv m entries), of its
adaptive cross approximation U V^* (q nv r_c + m r_c) and of the Tucker form
(q (r^3 + 3 n r) m for equal ranks r and sizes n).  Entries are complex128,
16 bytes each, and the tables quote GiB (2^30 bytes).
"""
from __future__ import annotations

import numpy as np

BYTES_C128 = 16
GIB = float(2**30)
MIB = float(2**20)


def full_bytes(q: int, nv: int, m: int) -> int:
    """Full assembly, Table II: q nv m complex entries."""
    return BYTES_C128 * q * nv * m


def aca_bytes(q: int, nv: int, m: int, rc: int) -> int:
    """ACA assembly, Table II: q nv r_c + m r_c complex entries."""
    return BYTES_C128 * (q * nv * rc + m * rc)


def tucker_entries(ranks, dims) -> int:
    """Entries of one Tucker tensor: r1 r2 r3 + n1 r1 + n2 r2 + n3 r3.

    Table II's q (r^3 + 3 n r) m per matrix is this with equal r and n.
    """
    r1, r2, r3 = (int(r) for r in ranks)
    n1, n2, n3 = dims
    return r1 * r2 * r3 + n1 * r1 + n2 * r2 + n3 * r3


def tucker_bytes(rank_array, dims) -> int:
    """Tucker memory of a whole struct; rank_array is (..., 3)."""
    ra = np.asarray(rank_array).reshape(-1, 3)
    return BYTES_C128 * sum(tucker_entries(r, dims) for r in ra)


def matvec_flops(rank_array, dims, p: int = 1) -> float:
    """Real flops of one product with p right-hand sides, decompressing each
    tensor mode by mode (modes 2, 3, then 1) and applying it to p vectors.

    Table III: O(r q nv m) decompression + O(q nv m p) application; one
    complex multiply-add is 8 real flops.
    """
    n1, n2, n3 = dims
    nv = n1 * n2 * n3
    tot = 0.0
    for r1, r2, r3 in np.asarray(rank_array).reshape(-1, 3):
        dec = r1 * r2 * r3 * n2 + r1 * r3 * n2 * n3 + r1 * nv
        tot += 8.0 * (dec + (nv * p if p > 1 else 0))
    return tot


def rmatvec_flops(rank_array, dims) -> float:
    """Real flops of one adjoint product Z^* y (p = 1): each tensor is
    decompressed in modes 2 and 3 as for Z x, y's block is contracted with
    U1^* (mode 1, r1 nv multiply-adds) and the result is dotted with the
    conjugated mode-2/3 decompression (r1 n2 n3 multiply-adds): Algorithm 2's
    inner product of the decompressed column with y, taken at the mode-1
    output (Table III: the adjoint costs as much as the forward)."""
    n1, n2, n3 = dims
    tot = matvec_flops(rank_array, dims)
    for r1, _, _ in np.asarray(rank_array).reshape(-1, 3):
        tot += 8.0 * r1 * n2 * n3
    return tot


def aca_tucker_bytes(rank_array, dims, m: int, rc: int) -> int:
    """ACA+Tucker assembly, Table II: the q r_c Tucker tensors of U's
    columns plus V (m r_c entries)."""
    return tucker_bytes(rank_array, dims) + BYTES_C128 * m * rc


def aca_matvec_flops(rank_array, dims, m: int, p: int = 1) -> float:
    """Real flops of one ACA+Tucker product, Table III: the Tucker product
    over U's r_c columns plus the coil-side product with V, O(r_c m p)
    (8 real flops per complex multiply-add)."""
    ra = np.asarray(rank_array).reshape(-1, 3)
    return matvec_flops(ra, dims, p) + 8.0 * m * p * _columns(ra, rank_array)


def _columns(ra, rank_array) -> int:
    """r_c from a rank array shaped (r_c, q, 3)."""
    shape = np.asarray(rank_array).shape
    if len(shape) != 3:
        raise ValueError("rank_array must be shaped (r_c, q, 3)")
    return int(shape[0])
