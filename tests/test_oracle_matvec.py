"""Pins for the oracle's Algorithm 1, Algorithm 2, entries and gradient.

Brute force on tiny structs (the matrix built entry by entry from eq. 6),
the adjoint identity, unit vectors recovering columns, the truncation bound
against the uncompressed closed-form matrix, and the exactness of central
differences on a quadratic loss.
"""
import itertools

import numpy as np
import pytest

import workloads
from oracle import hosvd, matvec

RNG = np.random.default_rng(5)
DIMS = (4, 5, 6)                 # unequal sizes catch transposed indices


def crandn(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def random_struct(dims=DIMS, q=3, m=5):
    cores, facs = [], []
    for j in range(m):
        cj, fj = [], []
        for k in range(q):
            r = RNG.integers(1, 4, size=3)
            cj.append(crandn(*r))
            fj.append(tuple(crandn(n, rr) for n, rr in zip(dims, r)))
        cores.append(cj)
        facs.append(fj)
    return matvec.from_factors(dims, q, cores, facs)


def brute_dense(S):
    n1, n2, n3 = S.dims
    nv = n1 * n2 * n3
    Z = np.zeros((S.q * nv, S.m), complex)
    for j, k in itertools.product(range(S.m), range(S.q)):
        t = S.t[j][k]
        U1, U2, U3 = t.U
        r1, r2, r3 = t.ranks
        for i1, i2, i3 in itertools.product(range(n1), range(n2), range(n3)):
            s = 0
            for a, b, c in itertools.product(range(r1), range(r2), range(r3)):
                s += t.G[a, b, c] * U1[i1, a] * U2[i2, b] * U3[i3, c]
            Z[k * nv + i1 + n1 * (i2 + n2 * i3), j] = s
    return Z


@pytest.fixture(scope="module")
def struct_and_dense():
    S = random_struct()
    return S, brute_dense(S)


def test_alg1_matches_brute_force(struct_and_dense):
    S, Z = struct_and_dense
    X = crandn(S.m, 3)
    assert np.allclose(matvec.alg1(S, X), Z @ X, atol=1e-11, rtol=0)


def test_alg2_matches_brute_force(struct_and_dense):
    S, Z = struct_and_dense
    Y = crandn(Z.shape[0], 2)
    assert np.allclose(matvec.alg2(S, Y), Z.conj().T @ Y, atol=1e-11, rtol=0)


def test_adjoint_identity(struct_and_dense):
    S, _ = struct_and_dense
    x = crandn(S.m, 1)
    y = crandn(S.q * S.nv, 1)
    lhs = np.vdot(matvec.alg1(S, x), y)
    rhs = np.vdot(x, matvec.alg2(S, y))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_unit_vector_recovers_column(struct_and_dense):
    S, Z = struct_and_dense
    e = np.zeros((S.m, 1), complex)
    e[3] = 1
    y = matvec.alg1(S, e)[:, 0]
    assert np.allclose(y, Z[:, 3], atol=1e-12, rtol=0)
    assert np.allclose(matvec.column(S, 3), Z[:, 3], atol=1e-12, rtol=0)


def test_single_entries(struct_and_dense):
    S, Z = struct_and_dense
    x = crandn(S.m)
    rows = [0, 7, S.nv - 1, S.nv, 2 * S.nv + 31, 3 * S.nv - 1]
    assert np.allclose(matvec.entries(S, x, rows), (Z @ x)[rows],
                       atol=1e-12, rtol=0)
    y = crandn(Z.shape[0])
    assert np.allclose(matvec.adjoint_entries(S, y, [1, 4]),
                       (Z.conj().T @ y)[[1, 4]], atol=1e-11, rtol=0)


def test_fibres(struct_and_dense):
    S, Z = struct_and_dense
    n1, n2, n3 = S.dims
    X = crandn(S.m, 2)
    Y = Z @ X
    for k, i2, i3 in [(0, 0, 0), (1, n2 - 1, 2), (2, 3, n3 - 1)]:
        rows = [k * S.nv + i1 + n1 * (i2 + n2 * i3) for i1 in range(n1)]
        assert np.allclose(matvec.fibre(S, X, k, i2, i3), Y[rows], atol=1e-11, rtol=0)
        assert np.allclose(matvec.fibre(S, X[:, 0], k, i2, i3), Y[rows, 0],
                           atol=1e-11, rtol=0)
    W = crandn(Z.shape[0], 3)
    assert np.allclose(matvec.adjoint_entries(S, W, [0, 2]),
                       (Z.conj().T @ W)[[0, 2]], atol=1e-11, rtol=0)


def test_compressed_matvec_within_truncation_bound():
    wl = workloads.make("tiny")
    Zd = matvec.dense(wl)
    S = matvec.compress_columns(wl)
    x = wl.x()[:, 0]
    err = np.linalg.norm(matvec.alg1(S, x)[:, 0] - Zd @ x)
    bound = np.sum(np.abs(x) * matvec.truncation_bound(S))
    assert err <= bound * (1 + 1e-9) + 1e-12 * np.linalg.norm(Zd @ x)
    # per tensor the relative error is at most the tolerance
    for j in range(wl.m):
        rel = np.linalg.norm(matvec.column(S, j) - Zd[:, j]) / np.linalg.norm(Zd[:, j])
        assert rel <= wl.tol


def test_exact_compression_reproduces_dense_matvec():
    wl = workloads.make("tiny")
    wl.tol = 0.0
    Zd = matvec.dense(wl)
    S = matvec.compress_columns(wl)
    X = wl.x(2)
    assert np.allclose(matvec.alg1(S, X), Zd @ X,
                       rtol=0, atol=1e-12 * np.abs(Zd @ X).max())
    Y = wl.y(2)
    assert np.allclose(matvec.alg2(S, Y), Zd.conj().T @ Y,
                       rtol=0, atol=1e-12 * np.abs(Zd.conj().T @ Y).max())


def test_pwl_struct_dimensions():
    wl = workloads.make("tiny_pwl")
    S = matvec.compress_columns(wl, cols=[0, 1])
    assert S.q == 12 and S.m == 2
    Zd = matvec.dense(wl, cols=[0, 1])
    x = np.array([1.0 + 0.5j, -0.25j])
    err = np.linalg.norm(matvec.alg1(S, x)[:, 0] - Zd @ x)
    assert err <= np.sum(np.abs(x) * matvec.truncation_bound(S)) * (1 + 1e-9)


def test_loss_central_difference_is_exact(struct_and_dense):
    S, _ = struct_and_dense
    x = crandn(S.m)
    b = crandn(S.q * S.nv)
    g = matvec.loss_grad(S, x, b)
    for _ in range(4):
        d = crandn(S.m)
        t = np.linalg.norm(x) / np.linalg.norm(d)
        fd = (matvec.loss(S, x + t * d, b) - matvec.loss(S, x - t * d, b)) / (2 * t)
        assert abs(fd - np.vdot(g, d).real) <= 1e-11 * matvec.loss(S, x, b)


@pytest.mark.parametrize("dims", [(6, 3, 2), (2, 6, 3), (3, 2, 6)])
def test_truncation_bound_is_attained_with_one_truncated_mode(dims):
    """When the rank cap truncates a single mode (the other two keep their
    full size), the HOSVD reconstruction is an orthogonal projection in that
    mode alone, so its squared error equals that mode's discarded energy
    exactly: truncation_bound must equal (sum_k ||Z^kj - Zhat^kj||^2)^(1/2)
    to rounding.  A bound without the square root, or one that drops a mode's
    term, fails here."""
    from oracle.hosvd import hosvd
    rng = np.random.default_rng(sum(dims))
    q, m = 2, 3
    cols, errs = [], []
    for _ in range(m):
        col, e2 = [], 0.0
        for _ in range(q):
            A = rng.standard_normal(dims) + 1j * rng.standard_normal(dims)
            t = hosvd(A, 0.0, 1, 3)          # cap 3: only the mode of length 6 is cut
            assert sorted(t.ranks) == sorted(min(3, n) for n in dims)
            e2 += float(np.linalg.norm(A - t.full()) ** 2)
            col.append(t)
        cols.append(col)
        errs.append(np.sqrt(e2))
    S = matvec.TuckerStruct(dims, q, cols)
    bound = matvec.truncation_bound(S)
    assert np.all(bound > 0)
    assert np.allclose(bound, errs, rtol=1e-12, atol=0)
