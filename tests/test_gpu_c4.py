"""The batching workload at full size against the FP64 oracle: 16 coils
(64..1024 point currents each) on the 96x128x112 grid, 32 right-hand sides
per coil, both directions in one persistent launch each.

The oracle runs on the plans' own factors (exported from the library): the
two coils with the fewest columns are compared in full (every entry of
Y = Z X and X' = Z^* Y, all 32 right-hand sides), every coil on whole mode-1
fibres on the edges of the first and last voxel tiles and on its first,
middle and last columns, entry by entry against the moduli of the terms.
"""
import numpy as np
import pytest

import workloads
from oracle import matvec as om
from tests.plans import (abi_to_struct, abs_struct, assert_close, boundary_fibres,
                         fibre_check)

pytestmark = pytest.mark.gpu
TOL = 1e-5
P_RHS = 32


@pytest.fixture(scope="module")
def c4_run():
    import torch
    from paper_2103_06393_amd import lib
    from paper_2103_06393_amd.ops import TuckerPlan, batch_create
    wls = workloads.make_batch("c4")
    plans = [TuckerPlan.compress_dipoles(w.grid.dims, w.grid.h, w.k0, 0, w.pos, w.ori,
                                         w.tol, w.rank_min, w.rank_cap) for w in wls]
    X = [w.x(P_RHS) for w in wls]
    Y = [w.y(P_RHS) for w in wls]
    outs = {}
    for op, ins in ((0, X), (1, Y)):
        b, b_arena = batch_create([P.handle for P in plans], op, [P_RHS] * len(plans))
        try:
            # column-major (rows x 32) device operands
            dev_in = [torch.from_numpy(np.ascontiguousarray(a.T.astype(np.complex64)))
                      .cuda().t() for a in ins]
            dev_out = [torch.empty((P_RHS, P.rows if op == 0 else P.m), dtype=torch.complex64,
                                   device="cuda").t() for P in plans]
            ws = torch.empty(lib.tv_batch_workspace_bytes(b), dtype=torch.uint8, device="cuda")
            lib.tv_batch_run(b, [a.data_ptr() for a in dev_in], [a.stride(1) for a in dev_in],
                             [a.data_ptr() for a in dev_out], [a.stride(1) for a in dev_out],
                             ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
            torch.cuda.synchronize()
            del ws, dev_in
            outs[op] = dev_out
        finally:
            lib.tv_batch_destroy(b)
    structs = [abi_to_struct(w.grid.dims, w.q, *P.export_factors()) for w, P in zip(wls, plans)]
    print(f"c4: columns per coil {[w.m for w in wls]}", flush=True)
    return wls, plans, structs, X, Y, outs


def test_c4_two_coils_in_full(gpu_lib, c4_run):
    wls, plans, structs, X, Y, outs = c4_run
    for c in np.argsort([w.m for w in wls])[:2]:
        S = structs[c]
        # (32, rows) and (32, m): blocks are one component of one right-hand side
        got_f = outs[0][c].t().cpu().numpy()
        got_a = outs[1][c].t().cpu().numpy()
        ef = assert_close(got_f, om.alg1(S, X[c], block_entries=1 << 28).T, TOL,
                          blocks=S.q * P_RHS, what=f"coil {c} Z X")
        ea = assert_close(got_a, om.alg2(S, Y[c], block_entries=1 << 28).T, TOL,
                          blocks=P_RHS, what=f"coil {c} Z^* Y")
        print(f"c4 coil {c} (m = {S.m}) in full: rel err {ef:.2e} / {ea:.2e}", flush=True)


def test_c4_every_coil_sampled(gpu_lib, c4_run):
    wls, plans, structs, X, Y, outs = c4_run
    for c, S in enumerate(structs):
        n1, n2, n3 = S.dims
        fib = boundary_fibres(S.dims, 8, 1)
        rows = []
        for n, (i2, i3) in enumerate(fib[::3] + [fib[-1]]):
            k = n % S.q
            rows.append((k, i2, i3))
        idx = [k * S.nv + i1 + n1 * (i2 + n2 * i3) for k, i2, i3 in rows for i1 in range(n1)]
        got_f = outs[0][c][idx].cpu().numpy()          # (len(idx), 32)
        for n, (k, i2, i3) in enumerate(rows):
            part = got_f[n * n1:(n + 1) * n1]
            ref = om.fibre(S, X[c], k, i2, i3)
            terms = np.abs(om.fibre(abs_struct(S), np.abs(X[c]), k, i2, i3))
            assert_close(part, ref, TOL, terms=terms, what=f"coil {c} fibre {(k, i2, i3)}")
        cols = sorted({0, S.m // 2, S.m - 1})
        got_a = outs[1][c].cpu().numpy()[cols]
        ref_a = om.adjoint_entries(S, Y[c], cols)
        terms = np.abs(om.adjoint_entries(abs_struct(S), np.abs(Y[c]), cols))
        assert_close(got_a, ref_a, TOL, terms=terms, what=f"coil {c} Z^* Y columns {cols}")
