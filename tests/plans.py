"""Test helpers: oracle Tucker structs <-> the library's factor layout.

Layout of the C ABI (tv_plan_from_factors): tensor t = k + q*j, cores
G[a,b,c] at a + r1*(b + r2*c), factors U_n column-major n_n x r_n, all
complex128 and concatenated in tensor order.
"""
import numpy as np

from oracle import matvec as om


def struct_to_abi(S):
    ranks, cores, u1, u2, u3 = [], [], [], [], []
    for j in range(S.m):
        for k in range(S.q):
            t = S.t[j][k]
            ranks.append(t.ranks)
            cores.append(t.G.reshape(-1, order="F"))
            u1.append(t.U[0].reshape(-1, order="F"))
            u2.append(t.U[1].reshape(-1, order="F"))
            u3.append(t.U[2].reshape(-1, order="F"))
    cat = lambda xs: np.concatenate(xs).astype(np.complex128)  # noqa: E731
    return (np.asarray(ranks, np.int32), cat(cores), cat(u1), cat(u2),
            cat(u3))


def abi_to_struct(dims, q, ranks, cores, u1, u2, u3):
    """Inverse of struct_to_abi (for factors exported by the library)."""
    ranks = np.asarray(ranks).reshape(-1, 3)
    m = ranks.shape[0] // q
    n1, n2, n3 = dims
    og = o1 = o2 = o3 = 0
    cs, fs = [], []
    for j in range(m):
        cj, fj = [], []
        for k in range(q):
            r1, r2, r3 = (int(v) for v in ranks[k + q * j])
            cj.append(cores[og:og + r1 * r2 * r3].reshape((r1, r2, r3), order="F"))
            fj.append((u1[o1:o1 + n1 * r1].reshape((n1, r1), order="F"),
                       u2[o2:o2 + n2 * r2].reshape((n2, r2), order="F"),
                       u3[o3:o3 + n3 * r3].reshape((n3, r3), order="F")))
            og += r1 * r2 * r3
            o1 += n1 * r1
            o2 += n2 * r2
            o3 += n3 * r3
        cs.append(cj)
        fs.append(fj)
    return om.from_factors(dims, q, cs, fs)


def random_struct(dims, q, m, rmax, seed):
    """Random Tucker struct with ranks in [1, rmax] (orthonormal factors)."""
    rng = np.random.default_rng(seed)
    cores, facs = [], []
    for j in range(m):
        cj, fj = [], []
        for k in range(q):
            r = [int(rng.integers(1, min(rmax, n) + 1)) for n in dims]
            G = rng.standard_normal(r) + 1j * rng.standard_normal(r)
            us = []
            for n, rr in zip(dims, r):
                a = rng.standard_normal((n, rr)) + 1j * rng.standard_normal((n, rr))
                us.append(np.linalg.qr(a)[0])
            cj.append(G)
            fj.append(tuple(us))
        cores.append(cj)
        facs.append(fj)
    return om.from_factors(dims, q, cores, facs)


def rel_err(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
