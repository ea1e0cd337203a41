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


def test_matvec_flops_terms():
    # one tensor, ranks (2, 3, 4), dims (5, 6, 7), one vector
    f = accounting.matvec_flops([[2, 3, 4]], (5, 6, 7))
    assert f == 8 * (2 * 3 * 4 * 6 + 2 * 4 * 6 * 7 + 2 * 210)
    f8 = accounting.matvec_flops([[2, 3, 4]], (5, 6, 7), p=8)
    assert f8 == f + 8 * 210 * 8
