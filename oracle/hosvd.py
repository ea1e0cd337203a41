"""Tucker model, n-mode products and truncated HOSVD (oracle, FP64).

Sec. II.B.1: a tensor A (n1 x n2 x n3) is written A = G x1 U1 x2 U2 x3 U3
(eq. 6) with factors U_n (n_n x r_n) having orthonormal columns and a core G
(r1 x r2 x r3).  The n-mode product contracts a tensor's n-th index with the
second index of a matrix (eq. 7).  The HOSVD takes U_n from the SVD of the
mode-n unfolding A_(n) and the core as A x1 U1^* x2 U2^* x3 U3^*
(De Lathauwer et al. 2000, cited in Sec. II.B.1).

Truncation to a tolerance (Sec. II.B.1) is not spelled out in the paper.
Reading used here: per mode keep the smallest r_n whose discarded squared
singular values sum to at most tol^2 ||A||_F^2 / 3, so that the HOSVD bound
||A - A_hat||^2 <= sum_n sum_{i > r_n} sigma_i^(n)^2 gives a relative error
of at most tol.  Then extend r_n across (near-)equal singular values and clamp
it to [rank_min, min(rank_cap, n_n)].
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np


def unfold(T: np.ndarray, mode: int) -> np.ndarray:
    """Mode-n unfolding A_(n): the mode-n fibres as columns (n_n x rest)."""
    return np.moveaxis(T, mode, 0).reshape(T.shape[mode], -1)


def mode_product(T: np.ndarray, U: np.ndarray, mode: int) -> np.ndarray:
    """n-mode product T x_n U, eq. (7): sum_chi T[..chi..] U[i, chi]."""
    out = np.tensordot(U, T, axes=([1], [mode]))      # new axis first
    return np.moveaxis(out, 0, mode)


def tucker_full(G, U1, U2, U3) -> np.ndarray:
    """A = G x1 U1 x2 U2 x3 U3, eq. (6)."""
    return mode_product(mode_product(mode_product(G, U1, 0), U2, 1), U3, 2)


@dataclasses.dataclass
class Tucker:
    G: np.ndarray
    U: List[np.ndarray]                 # [U1, U2, U3]
    sigma: List[np.ndarray]             # mode-n singular values (all)
    discarded: np.ndarray               # (3,) discarded squared energy
    norm2: float                        # ||A||_F^2

    @property
    def ranks(self):
        return tuple(int(u.shape[1]) for u in self.U)

    def full(self) -> np.ndarray:
        return tucker_full(self.G, *self.U)


def truncation_rank(sigma: np.ndarray, tol: float, norm2: float,
                    rank_min: int = 1, rank_cap: Optional[int] = None) -> int:
    """Smallest r with sum_{i >= r} sigma_i^2 <= tol^2 norm2 / 3 (0-based),
    extended over near-ties, clamped to [rank_min, min(rank_cap, len)]."""
    s2 = np.asarray(sigma, dtype=np.float64) ** 2
    n = len(s2)
    # tail[r] = sum of s2[r:]
    tail = np.concatenate([np.cumsum(s2[::-1])[::-1], [0.0]])
    budget = tol * tol * norm2 / 3.0
    r = n
    for cand in range(n + 1):
        if tail[cand] <= budget:
            r = cand
            break
    cap = n if rank_cap is None else min(rank_cap, n)
    while 0 < r < cap and sigma[r] >= (1.0 - 1e-10) * sigma[r - 1]:
        r += 1
    r = max(r, rank_min)
    return int(min(r, cap))


def hosvd(T: np.ndarray, tol: float, rank_min: int = 1,
          rank_cap: Optional[int] = None) -> Tucker:
    """Truncated HOSVD of a 3-D complex tensor (Sec. II.B.1)."""
    T = np.asarray(T, dtype=np.complex128)
    norm2 = float(np.vdot(T, T).real)
    Us, sig, disc = [], [], []
    for mode in range(3):
        u, s, _ = np.linalg.svd(unfold(T, mode), full_matrices=False)
        r = truncation_rank(s, tol, norm2, rank_min, rank_cap)
        Us.append(u[:, :r].copy())
        sig.append(s)
        disc.append(float(np.sum(s[r:] ** 2)))
    G = T
    for mode in range(3):
        G = mode_product(G, Us[mode].conj().T, mode)
    return Tucker(G, Us, sig, np.asarray(disc), norm2)
