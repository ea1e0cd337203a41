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


def abs_struct(S):
    """The struct with every core and factor replaced by its entrywise
    modulus: its products with |x| bound the sum of the moduli of the terms
    that make each entry of Z x (and likewise for Z^* y)."""
    cols = []
    for col in S.t:
        cols.append([om.Tucker(np.abs(t.G).astype(np.complex128),
                               [np.abs(u).astype(np.complex128) for u in t.U],
                               [None] * 3, np.zeros(3), float("nan")) for t in col])
    return om.TuckerStruct(S.dims, S.q, cols)


def fwd_terms(S, x):
    """Per entry of Z x: sum over j and (a, b, c) of |x_j G U1 U2 U3|."""
    r = np.abs(om.alg1(abs_struct(S), np.abs(np.asarray(x))))
    return r.reshape(-1) if np.ndim(x) == 1 else r


def adj_terms(S, y):
    """Per entry of Z^* y: sum over rows and (a, b, c) of the moduli of the terms."""
    r = np.abs(om.alg2(abs_struct(S), np.abs(np.asarray(y))))
    return r.reshape(-1) if np.ndim(y) == 1 else r


def assert_close(got, ref, tol, terms=None, elem=None, blocks=1, what=""):
    """Parity of a GPU result with the oracle, entry by entry.

    * relative 2-norm error over all entries <= tol;
    * every entry: |got_i - ref_i| <= elem * terms_i when ``terms`` (the sum of
      the moduli of the terms that make entry i) is given, else
      <= elem * max|ref| within each of ``blocks`` equal slices (the field
      components of a voxel vector); elem defaults to tol.
    """
    g = np.asarray(got).reshape(-1).astype(np.complex128)
    r = np.asarray(ref).reshape(-1).astype(np.complex128)
    assert g.shape == r.shape, (what, g.shape, r.shape)
    elem = tol if elem is None else elem
    nr = np.linalg.norm(r)
    e2 = np.linalg.norm(g - r) / nr if nr > 0 else np.linalg.norm(g - r)
    assert e2 <= tol, f"{what}: relative 2-norm error {e2:.3e} > {tol:.1e}"
    d = np.abs(g - r)
    if terms is not None:
        t = np.asarray(terms).reshape(-1).astype(np.float64)
        assert t.shape == d.shape
        bad = d > elem * t + 1e-300
        i = int(np.argmax(d / np.maximum(t, 1e-300)))
        assert not bad.any(), (f"{what}: {int(bad.sum())} entries off by more than "
                               f"{elem:.1e} x their terms' moduli (worst index {i}: "
                               f"{d[i]:.3e} vs {t[i]:.3e})")
    else:
        for b, (db, rb) in enumerate(zip(np.array_split(d, blocks), np.array_split(r, blocks))):
            scale = np.max(np.abs(rb)) if rb.size else 0.0
            worst = float(np.max(db)) if db.size else 0.0
            assert worst <= elem * scale, (f"{what}: block {b}: max entry error "
                                           f"{worst:.3e} > {elem:.1e} x max|ref| {scale:.3e}")
    return e2


def boundary_fibres(dims, t2, t3):
    """(i2, i3) of mode-1 fibres on the edges of the first and last column
    tiles of a t2 x t3 tiling: first/last fibre of the first tile, the first
    fibre of the second tile, and the last fibre of the grid (ragged tile)."""
    _, n2, n3 = dims
    i2s = sorted({0, min(t2 - 1, n2 - 1), min(t2, n2 - 1), n2 - 1})
    i3s = sorted({0, min(t3 - 1, n3 - 1), min(t3, n3 - 1), n3 - 1})
    return [(a, b) for a in i2s for b in i3s]


def split_boundary_columns(ranks, q, m, nsplit):
    """Columns on both sides of every boundary of the balanced column splits
    (equal shares of sum r1 per component, the split-K ranges of the fused
    kernels), plus the first and last column."""
    r = np.asarray(ranks).reshape(m, q, 3)
    cols = {0, m - 1}
    for k in range(q):
        c = np.cumsum(r[:, k, 0])
        total = int(c[-1])
        for s in range(1, nsplit):
            j = int(np.searchsorted(c * nsplit >= total * s, True))   # first j with acc*S >= total*s
            cols.update({max(0, j), min(m - 1, j + 1)})
    return sorted(cols)


def fibre_check(S, P_out, X, k, i2, i3, tol, what=""):
    """Compare one mode-1 fibre of a GPU product (the q nv x p result) with the
    oracle's, entry by entry against the moduli of the terms."""
    n1, n2, _ = S.dims
    rows = [k * S.nv + i1 + n1 * (i2 + n2 * i3) for i1 in range(n1)]
    ref = om.fibre(S, X, k, i2, i3)
    terms = np.abs(om.fibre(abs_struct(S), np.abs(np.asarray(X)), k, i2, i3))
    return assert_close(np.asarray(P_out)[rows], ref, tol, terms=terms,
                        what=f"{what} fibre (k={k}, i2={i2}, i3={i3})")
