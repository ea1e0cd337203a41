"""Pins of the ACA oracle (Sec. II.B.2, Algorithm 3) and of the ACA + Tucker
products (Sec. III.B, the substitution after Algorithms 1 and 2).

Each check rests on something other than the oracle itself: exact recovery
of matrices of known rank, the cross (interpolation) property of partial-
pivot ACA, the Frobenius-norm identity behind the stopping estimate, the
agreement of the compressed and dense storages when the HOSVD keeps
everything, the product's error bound against the dense matrix, and the
adjoint identity.
"""
import numpy as np
import pytest

from oracle import aca, fields, matvec
from workloads import configs as wc


def _lowrank(m1, m2, r, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((m1, r)) + 1j * rng.standard_normal((m1, r))
    C = rng.standard_normal((m2, r)) + 1j * rng.standard_normal((m2, r))
    return B @ C.conj().T


@pytest.mark.parametrize("m1,m2,r", [(60, 40, 5), (30, 70, 1), (50, 50, 12)])
def test_exact_rank_recovered(m1, m2, r):
    A = _lowrank(m1, m2, r, 7 + r)
    R = aca.aca_dense(A, 1e-12)
    assert R.rc <= r + 1
    E = A - R.U.dense() @ R.V.conj().T
    assert np.linalg.norm(E) <= 1e-11 * np.linalg.norm(A)


def _smooth(m1=80, m2=60):
    """A smooth kernel matrix: 1 / |s_i - t_j| for separated point sets."""
    rng = np.random.default_rng(3)
    s = rng.uniform(0, 1, (m1, 3))
    t = rng.uniform(0, 1, (m2, 3)) + np.array([3.0, 0, 0])
    D = np.linalg.norm(s[:, None, :] - t[None, :, :], axis=-1)
    return np.exp(-1j * 2.0 * D) / D


def test_cross_property():
    """After any number of steps, U V^* reproduces Z exactly on every pivot
    row and pivot column (partial-pivot ACA interpolates its crosses)."""
    A = _smooth()
    R = aca.aca_dense(A, 1e-9, max_rank=9)
    Ap = R.U.dense() @ R.V.conj().T
    scale = np.max(np.abs(A))
    for i in R.rows:
        assert np.max(np.abs(Ap[i, :] - A[i, :])) <= 1e-12 * scale
    for j in R.cols:
        assert np.max(np.abs(Ap[:, j] - A[:, j])) <= 1e-12 * scale
    assert len(set(R.rows)) == len(R.rows)
    assert len(set(R.cols)) == len(R.cols)


def test_norm_estimate_is_frobenius_norm():
    """s_{k+1} is ||U_k V_k^*||_F^2 at every step: the update adds the new
    term's norm and twice the real inner product with the previous sum."""
    A = _smooth()
    R = aca.aca_dense(A, 1e-10, max_rank=20)
    U, V = R.U.dense(), R.V
    for k, s in enumerate(R.s):
        M = U[:, :k + 1] @ V[:, :k + 1].conj().T
        ref = np.linalg.norm(M) ** 2
        assert abs(s - ref) <= 1e-10 * ref


def test_stopping_rule_and_error():
    A = _smooth()
    for tol in (1e-3, 1e-6):
        R = aca.aca_dense(A, tol)
        assert R.converged
        k = R.rc - 1
        u, v = R.U.dense()[:, k], R.V[:, k]
        assert np.linalg.norm(u) * np.linalg.norm(v) <= tol * np.sqrt(R.s[-1])
        E = A - R.U.dense() @ R.V.conj().T
        assert np.linalg.norm(E) <= 50 * tol * np.linalg.norm(A)
        # Eckart-Young: no rank-r_c matrix beats the SVD tail at r_c
        sig = np.linalg.svd(A, compute_uv=False)
        tail = np.sqrt(np.concatenate([np.cumsum(sig[::-1] ** 2)[::-1], [0]]))
        assert tail[R.rc] <= np.linalg.norm(E) * (1 + 1e-12)
        assert R.rc <= A.shape[1]


def _tiny_bodycoil():
    wl = wc.make_bodycoil("aca_s")
    # a 4 x 3 x 5 sub-box of the stand-in keeps the dense matrix small
    g = wc.Grid(4, 3, 5, 0.1)
    return wc.Workload("aca_t", g, "pwc", wl.freq, wl.pos[::10], wl.ori[::10],
                       1e-3)


def test_tucker_storage_matches_dense_when_lossless():
    """With an HOSVD tolerance of zero the compressed U is U itself, so
    Algorithm 3 makes the same pivots and the same V as the dense loop; this
    pins the single-element row decompression, the reshape order of a new
    column and the Algorithm 1/2 products inside the loop."""
    wl = _tiny_bodycoil()
    Z = matvec.dense(wl)
    Rd = aca.aca_dense(Z, 1e-6, max_rank=12)
    Rt = aca.aca_tucker(wl, 1e-6, hosvd_tol=0.0, max_rank=12)
    assert Rt.rows == Rd.rows and Rt.cols == Rd.cols
    assert np.allclose(Rt.V, Rd.V, rtol=1e-9, atol=1e-12)
    assert np.allclose(Rt.U.dense(), Rd.U.dense(), rtol=1e-9,
                       atol=1e-12 * np.max(np.abs(Z)))
    assert np.allclose(Rt.s, Rd.s, rtol=1e-9)


def test_rows_and_columns_agree():
    wl = _tiny_bodycoil()
    Z = matvec.dense(wl)
    for i in (0, 7, wl.rows - 1):
        assert np.allclose(fields.row_vector(wl, i), Z[i, :], rtol=0, atol=0)


def test_products_error_bound_and_adjoint():
    """||U(V^*x) - Zx|| <= ||Z - U V^*||_F ||x|| with U decompressed
    independently of Algorithm 1, and <Zx, y> = <x, Z^* y>."""
    wl = _tiny_bodycoil()
    Z = matvec.dense(wl)
    R = aca.aca_tucker(wl, 1e-3, max_rank=16)
    S, V = R.U.S, R.V
    Ud = np.stack([np.concatenate([t.full().reshape(-1, order="F")
                                   for t in col]) for col in S.t], axis=1)
    E = np.linalg.norm(Z - Ud @ V.conj().T)
    x = wc.complex_normal((wl.m, 2), 5)
    y = wc.complex_normal((wl.rows, 2), 6)
    Yx = aca.aca_matvec(S, V, x)
    assert np.linalg.norm(Yx - Z @ x) <= E * np.linalg.norm(x) * (1 + 1e-12)
    assert np.allclose(Yx, Ud @ (V.conj().T @ x), rtol=1e-12, atol=0)
    Xy = aca.aca_rmatvec(S, V, y)
    lhs = np.vdot(y, Yx)
    rhs = np.vdot(Xy, x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    rows = [0, 5, wl.rows // 2, wl.rows - 1]
    assert np.allclose(aca.aca_entries(S, V, x[:, 0], rows), Yx[rows, 0],
                       rtol=1e-12, atol=0)


def test_compressed_columns_have_low_ranks():
    """The Tucker ranks of U's columns stay small (Sec. II.B.2: cross
    approximation is well conditioned, so U's reshaped columns compress like
    the coupling matrix's)."""
    wl = _tiny_bodycoil()
    R = aca.aca_tucker(wl, 1e-3, max_rank=6)
    r = R.U.S.ranks().reshape(-1, 3)
    assert r.max() <= 5
    S = matvec.compress_columns(
        wc.Workload("c", wl.grid, "pwc", wl.freq, wl.pos, wl.ori, 3e-3), range(6))
    assert r.mean() <= S.ranks().reshape(-1, 3).mean() + 1.0


def test_table2_table3_counts():
    """Table II: ACA+Tucker memory is q (r^3 + 3 n r) r_c + m r_c entries for
    equal ranks and sizes."""
    from oracle import accounting as acc
    q, n, r, rc, m = 3, 20, 4, 7, 50
    ranks = np.full((rc, q, 3), r)
    assert acc.aca_tucker_bytes(ranks, (n, n, n), m, rc) == \
        16 * (q * (r ** 3 + 3 * n * r) * rc + m * rc)
    # the operation count is pinned against a literal count of multiply-adds
    # in tests/test_oracle_accounting.py
