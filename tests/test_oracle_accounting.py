"""Pin the memory accounting (Table II) to the numbers the paper prints.

The fixture lists every "Full" entry of Tables IV and VIII, the "ACA-CPU"
entries of Table VIII and the 5848 MB of Sec. IV.A.1; each must come out of
the Table II formulas with 16-byte complex entries within one unit of its last
printed digit.  This fixes rows = q nv, columns = m and the byte size.
"""
import os

import numpy as np

from oracle import accounting

HERE = os.path.dirname(os.path.abspath(__file__))


def _rows():
    with open(os.path.join(HERE, "golden", "memory_tables.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line.split()


def test_paper_memory_tables():
    n = 0
    for kind, q, n1, n2, n3, m, rc, printed, unit in _rows():
        q, n1, n2, n3, m, rc = map(int, (q, n1, n2, n3, m, rc))
        nv = n1 * n2 * n3
        if kind == "full":
            b = accounting.full_bytes(q, nv, m)
        else:
            b = accounting.aca_bytes(q, nv, m, rc)
        val = b / (accounting.GIB if unit == "GiB" else accounting.MIB)
        ulp = 10.0 ** -(len(printed.split(".")[1]) if "." in printed else 0)
        assert abs(val - float(printed)) <= ulp, (kind, q, n1, m, val, printed)
        n += 1
    assert n == 25


def test_tucker_entries_match_table_ii_form():
    # equal ranks and sizes: r^3 + 3 n r per tensor, q m tensors
    q, m, n, r = 3, 7, 20, 4
    ranks = np.full((m, q, 3), r)
    assert accounting.tucker_bytes(ranks, (n, n, n)) == 16 * q * (r**3 + 3 * n * r) * m


# ---- operation counts (Table III) against a literal count -----------------
# The decompression of one tensor is carried out with explicit loops in the
# order modes 2, 3, 1 (Algorithm 1's decompress-then-add with x_j folded into
# the core), and every complex multiply-add is counted as it is executed; the
# loops' result is checked against the tensor, so the count is of real work.

def _counted_forward(G, U1, U2, U3, xj, y, p=1):
    r1, r2, r3 = G.shape
    n1, n2, n3 = U1.shape[0], U2.shape[0], U3.shape[0]
    cm = 0
    H = np.zeros((r1, n2, r3), complex)              # mode 2
    for a in range(r1):
        for i2 in range(n2):
            for c in range(r3):
                for b in range(r2):
                    H[a, i2, c] += G[a, b, c] * U2[i2, b]
                    cm += 1
    B = np.zeros((r1, n2, n3), complex)              # mode 3
    for a in range(r1):
        for i2 in range(n2):
            for i3 in range(n3):
                for c in range(r3):
                    B[a, i2, i3] += H[a, i2, c] * U3[i3, c]
                    cm += 1
    T = np.zeros((n1, n2, n3), complex)              # mode 1
    for i1 in range(n1):
        for i2 in range(n2):
            for i3 in range(n3):
                for a in range(r1):
                    T[i1, i2, i3] += U1[i1, a] * B[a, i2, i3]
                    cm += 1
    if p == 1:
        y += xj[0] * T                               # folded into the core: free
    else:
        for col in range(p):                         # apply to p vectors
            for v in np.ndindex(T.shape):
                y[col][v] += xj[col] * T[v]
                cm += 1
    return cm, B, T


def _counted_adjoint(G, U1, U2, U3, Y):
    r1 = G.shape[0]
    n1, n2, n3 = U1.shape[0], U2.shape[0], U3.shape[0]
    cm, B, _ = _counted_forward(G, np.zeros((0, r1)), U2, U3, [0.0],
                                np.zeros((0, n2, n3), complex))
    W = np.zeros((r1, n2, n3), complex)              # mode 1 of y: U1^* Y
    for a in range(r1):
        for i2 in range(n2):
            for i3 in range(n3):
                for i1 in range(n1):
                    W[a, i2, i3] += np.conj(U1[i1, a]) * Y[i1, i2, i3]
                    cm += 1
    acc = 0j
    for v in np.ndindex(W.shape):                    # <B, W>
        acc += np.conj(B[v]) * W[v]
        cm += 1
    return cm, acc


def _random_tucker(rng, dims, ranks):
    G = rng.standard_normal(ranks) + 1j * rng.standard_normal(ranks)
    Us = [rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))
          for n, r in zip(dims, ranks)]
    return G, Us


UNEQUAL = [((5, 4, 3), (2, 3, 2)), ((3, 6, 4), (3, 2, 4)), ((4, 3, 7), (1, 2, 3))]


def test_matvec_flops_equal_a_literal_count():
    from oracle.hosvd import tucker_full
    rng = np.random.default_rng(7)
    for dims, ranks in UNEQUAL:
        G, (U1, U2, U3) = _random_tucker(rng, dims, ranks)
        for p in (1, 3):
            y = [np.zeros(dims, complex) for _ in range(p)] if p > 1 else np.zeros(dims, complex)
            cm, _, T = _counted_forward(G, U1, U2, U3, [1.0] * p, y, p)
            assert np.allclose(T, tucker_full(G, U1, U2, U3))
            assert accounting.matvec_flops([ranks], dims, p) == 8 * cm, (dims, ranks, p)


def test_rmatvec_flops_equal_a_literal_count():
    from oracle.hosvd import tucker_full
    rng = np.random.default_rng(8)
    for dims, ranks in UNEQUAL:
        G, (U1, U2, U3) = _random_tucker(rng, dims, ranks)
        Y = rng.standard_normal(dims) + 1j * rng.standard_normal(dims)
        cm, acc = _counted_adjoint(G, U1, U2, U3, Y)
        assert np.isclose(acc, np.vdot(tucker_full(G, U1, U2, U3), Y))
        assert accounting.rmatvec_flops([ranks], dims) == 8 * cm, (dims, ranks)


def test_aca_matvec_flops_equal_a_literal_count():
    # Z X = U (V^* X): the Tucker product over U's r_c columns with the
    # r_c x p weights V^* X, plus m r_c p multiply-adds for V^* X
    rng = np.random.default_rng(9)
    dims, q, rc, m = (4, 3, 5), 2, 3, 7
    ranks = np.array([[[2, 1, 3], [1, 2, 2]], [[3, 3, 1], [2, 2, 2]], [[1, 1, 1], [2, 3, 4]]])
    for p in (1, 2):
        cm = m * rc * p                              # V^* X
        for l in range(rc):
            for k in range(q):
                G, (U1, U2, U3) = _random_tucker(rng, dims, tuple(ranks[l, k]))
                y = [np.zeros(dims, complex) for _ in range(p)] if p > 1 else np.zeros(dims, complex)
                c, _, _ = _counted_forward(G, U1, U2, U3, [1.0] * p, y, p)
                cm += c
        assert accounting.aca_matvec_flops(ranks, dims, m, p) == 8 * cm


def test_flop_pins_catch_a_wrong_term():
    """A mode-3 term typed as r1 r2 n2 n3, or a mode-2 term missing r3,
    disagrees with the literal count on unequal ranks."""
    rng = np.random.default_rng(10)
    dims, ranks = UNEQUAL[0]
    G, (U1, U2, U3) = _random_tucker(rng, dims, ranks)
    cm, _, _ = _counted_forward(G, U1, U2, U3, [1.0], np.zeros(dims, complex))
    r1, r2, r3 = ranks
    n1, n2, n3 = dims
    wrong = [8 * (r1 * r2 * r3 * n2 + r1 * r2 * n2 * n3 + r1 * n1 * n2 * n3),
             8 * (r1 * r2 * n2 + r1 * r3 * n2 * n3 + r1 * n1 * n2 * n3),
             8 * (r1 * r2 * r3 * n2 + r1 * r3 * n2 * n3 + r2 * n1 * n2 * n3)]
    for w in wrong:
        assert w != 8 * cm
