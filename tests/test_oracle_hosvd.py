"""Pins for the oracle's Tucker model and truncated HOSVD (Sec. II.B.1).

Checked against brute force (eq. 6 and eq. 7 as explicit loops), planted
Tucker tensors of known multilinear rank, and the HOSVD theorems: orthonormal
factors, the discarded-energy error bound, and the Pythagoras identity of an
orthogonal projection.
"""
import itertools

import numpy as np
import pytest

from oracle import hosvd

RNG = np.random.default_rng(3)


def crandn(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def orth(n, r):
    q, _ = np.linalg.qr(crandn(n, r))
    return q


def test_mode_product_brute_force():
    T = crandn(3, 4, 5)
    U = crandn(6, 4)
    got = hosvd.mode_product(T, U, 1)
    ref = np.zeros((3, 6, 5), complex)
    for i, a, c, b in itertools.product(range(6), range(3), range(5), range(4)):
        ref[a, i, c] += T[a, b, c] * U[i, b]                 # eq. (7)
    assert np.allclose(got, ref, atol=1e-13, rtol=0)


def test_tucker_full_brute_force():
    G = crandn(2, 3, 2)
    U1, U2, U3 = crandn(4, 2), crandn(5, 3), crandn(3, 2)
    got = hosvd.tucker_full(G, U1, U2, U3)
    ref = np.zeros((4, 5, 3), complex)
    for i, j, k in itertools.product(range(4), range(5), range(3)):
        s = 0
        for a, b, c in itertools.product(range(2), range(3), range(2)):
            s += G[a, b, c] * U1[i, a] * U2[j, b] * U3[k, c]    # eq. (6)
        ref[i, j, k] = s
    assert np.allclose(got, ref, atol=1e-13, rtol=0)


def test_unfolding_columns_are_mode_fibres():
    T = crandn(3, 4, 5)
    A1 = hosvd.unfold(T, 1)
    assert A1.shape == (4, 15)
    fibres = {tuple(np.round(T[a, :, c], 12)) for a in range(3) for c in range(5)}
    cols = {tuple(np.round(A1[:, i], 12)) for i in range(15)}
    assert fibres == cols


def test_planted_ranks_are_recovered_exactly():
    G = crandn(3, 4, 5)
    U = [orth(10, 3), orth(12, 4), orth(14, 5)]
    A = hosvd.tucker_full(G, *U)
    t = hosvd.hosvd(A, 1e-12)
    assert t.ranks == (3, 4, 5)
    assert np.linalg.norm(t.full() - A) <= 1e-12 * np.linalg.norm(A)
    for u, ref in zip(t.U, U):          # same subspace (factors not unique)
        assert np.allclose(u @ u.conj().T, ref @ ref.conj().T, atol=1e-12)


def test_separable_tensor_has_rank_one():
    a, b, c = crandn(7), crandn(6), crandn(5)
    A = np.einsum("i,j,k->ijk", a, b, c)
    t = hosvd.hosvd(A, 1e-10)
    assert t.ranks == (1, 1, 1)
    assert np.linalg.norm(t.full() - A) <= 1e-13 * np.linalg.norm(A)


@pytest.mark.parametrize("tol", [0.05, 0.3, 0.8])
def test_orthonormality_bound_and_pythagoras(tol):
    # a tensor with decaying spectrum in every mode
    A = hosvd.tucker_full(crandn(9, 8, 7) * np.exp(-np.arange(9))[:, None, None],
                          orth(9, 9), orth(8, 8), orth(7, 7))
    A = A + 1e-3 * crandn(9, 8, 7)
    t = hosvd.hosvd(A, tol)
    for u in t.U:
        assert np.allclose(u.conj().T @ u, np.eye(u.shape[1]), atol=1e-13)
    err2 = np.linalg.norm(t.full() - A) ** 2
    norm2 = np.linalg.norm(A) ** 2
    # De Lathauwer's bound: error energy <= discarded energy of all modes
    assert err2 <= np.sum(t.discarded) * (1 + 1e-10) + 1e-24
    # the truncation rule keeps the relative error below tol
    assert err2 <= tol * tol * norm2 * (1 + 1e-10)
    # orthogonal projection: ||A||^2 = ||G||^2 + ||A - A_hat||^2
    assert abs(norm2 - (np.linalg.norm(t.G) ** 2 + err2)) <= 1e-12 * norm2


def test_zero_tolerance_is_exact():
    A = crandn(5, 6, 4)
    t = hosvd.hosvd(A, 0.0)
    assert t.ranks == (5, 6, 4)
    assert np.linalg.norm(t.full() - A) <= 1e-13 * np.linalg.norm(A)


def test_truncation_rank_rule():
    s = np.array([10.0, 5.0, 1.0, 0.1, 0.01])
    norm2 = float(np.sum(s ** 2))
    # budget tol^2 norm2 / 3 with tol chosen so the tail {0.1, 0.01} fits
    tol = np.sqrt(3 * (0.1**2 + 0.01**2) / norm2) * 1.0001
    assert hosvd.truncation_rank(s, tol, norm2) == 3
    assert hosvd.truncation_rank(s, tol * 0.999, norm2) == 4
    assert hosvd.truncation_rank(s, tol, norm2, rank_cap=2) == 2
    assert hosvd.truncation_rank(s, 10.0, norm2) == 1       # rank_min = 1
    assert hosvd.truncation_rank(s, tol, norm2, rank_min=5) == 5
    # near-tie at the cut is kept together
    s2 = np.array([3.0, 2.0, 2.0, 0.001])
    tol2 = np.sqrt(3 * (4.0 + 1e-6) / float(np.sum(s2 ** 2))) * 1.0001
    assert hosvd.truncation_rank(s2, tol2, float(np.sum(s2 ** 2))) == 3
