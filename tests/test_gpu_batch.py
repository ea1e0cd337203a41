"""Batched multi-right-hand-side products (tv_batch_*) against the oracle.

Several coil configurations on one grid, each with its own number of
right-hand sides, in one persistent launch; then the same launch captured
into a graph and replayed, each replay checked against the eager result.
"""
import numpy as np
import pytest

import workloads
from oracle import matvec as om
from tests.plans import assert_close, rel_err, struct_to_abi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c4s():
    from paper_2103_06393_amd.ops import TuckerPlan
    wls = workloads.make_batch("c4s")
    structs = [om.compress_columns(w) for w in wls]
    plans = [TuckerPlan.from_factors(S.dims, S.q, S.m, *struct_to_abi(S))
             for S in structs]
    return wls, structs, plans


def _ld(t):
    """Leading dimension of a column-major (rows x cols) tensor; a single
    column reports stride 1, its leading dimension is the row count."""
    return t.shape[0] if t.shape[1] == 1 else t.stride(1)


def _run(plans, op, inputs, nrhs):
    import torch
    from paper_2103_06393_amd import lib
    from paper_2103_06393_amd.ops import batch_create
    b, b_arena = batch_create([p.handle for p in plans], op, nrhs)
    try:
        rows = [p.rows for p in plans]
        outs = [torch.zeros((r if op == 0 else p.m, n), dtype=torch.complex64,
                            device="cuda").t().contiguous().t()
                for p, r, n in zip(plans, rows, nrhs)]
        ws = torch.empty(lib.tv_batch_workspace_bytes(b), dtype=torch.uint8, device="cuda")
        ins = [x.t().contiguous().t() for x in inputs]
        lib.tv_batch_run(b, [x.data_ptr() for x in ins], [_ld(x) for x in ins],
                         [y.data_ptr() for y in outs], [_ld(y) for y in outs],
                         ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        return [y.cpu().numpy() for y in outs]
    finally:
        lib.tv_batch_destroy(b)


def test_batch_forward_and_adjoint(gpu_lib, c4s):
    import torch
    wls, structs, plans = c4s
    nrhs = [8, 3, 40, 1][:len(plans)]
    X = [workloads.complex_normal((S.m, n), 200 + c) for c, (S, n) in enumerate(zip(structs, nrhs))]
    Y = [workloads.complex_normal((S.q * S.nv, n), 300 + c) for c, (S, n) in enumerate(zip(structs, nrhs))]
    cx = lambda a: torch.from_numpy(a.astype(np.complex64)).cuda()  # noqa: E731
    got_f = _run(plans, 0, [cx(x) for x in X], nrhs)
    got_a = _run(plans, 1, [cx(y) for y in Y], nrhs)
    for c, S in enumerate(structs):
        assert_close(got_f[c], om.alg1(S, X[c]), 1e-5)
        assert_close(got_a[c], om.alg2(S, Y[c]), 1e-5)


def test_batch_graph_replay(gpu_lib, c4s):
    import torch
    from paper_2103_06393_amd import lib
    wls, structs, plans = c4s
    nrhs = [8] * len(plans)
    X = [torch.from_numpy(workloads.complex_normal((S.m, 8), 210 + c).astype(np.complex64))
         .cuda().t().contiguous().t() for c, S in enumerate(structs)]
    outs = [torch.zeros((8, p.rows), dtype=torch.complex64, device="cuda").t() for p in plans]
    from paper_2103_06393_amd.ops import batch_create
    b, b_arena = batch_create([p.handle for p in plans], 0, nrhs)
    ws = torch.empty(lib.tv_batch_workspace_bytes(b), dtype=torch.uint8, device="cuda")
    args = ([x.data_ptr() for x in X], [_ld(x) for x in X],
            [y.data_ptr() for y in outs], [_ld(y) for y in outs], ws.data_ptr(), ws.numel())
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        lib.tv_batch_run(b, *args, s.cuda_stream)
    torch.cuda.synchronize()
    eager = [y.cpu().numpy().copy() for y in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        lib.tv_batch_run(b, *args, s.cuda_stream)
    for rep in range(3):
        for y in outs:
            y.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for y, e in zip(outs, eager):
            assert np.array_equal(y.cpu().numpy(), e), rep
    lib.tv_batch_destroy(b)
    for c, S in enumerate(structs):
        assert_close(eager[c], om.alg1(S, X[c].cpu().numpy()), 1e-5)


# Shapes chosen to reach every batched kernel: forward with n1p32 / 32 = 3,
# 2, 1 (MFMA decompression) and n1 = 128 (wave-local decompression), adjoint
# with 48-, 48-, 16- and 48-row i1 chunks; ragged column groups (n2 not a
# multiple of 8), counts of tensors off the 4- and 32-multiples, ranks above
# 16 (two 16-row a-blocks) and odd ranks; the fifth case has ranks above 32
# and runs the VALU decompression in both directions; the last has q = 12
# (the piecewise-linear basis: 3 field components x 4 basis functions).
MFMA_CASES = [
    ((96, 20, 7), 3, (37, 9), 32, 41),
    ((40, 9, 5), 1, (6, 3), 20, 42),
    ((13, 17, 3), 2, (70, 5), 13, 43),
    ((128, 6, 4), 1, (5, 4), 8, 44),
    ((24, 20, 36), 1, (4, 2), 36, 45),
    ((20, 12, 6), 12, (10, 3), 12, 46),
]


@pytest.mark.parametrize("dims,q,ms,rmax,seed", MFMA_CASES)
def test_batch_kernels_against_oracle(gpu_lib, dims, q, ms, rmax, seed):
    import torch
    from paper_2103_06393_amd.ops import TuckerPlan
    from tests.plans import random_struct
    structs = [random_struct(dims, q, m, rmax, seed + 10 * c) for c, m in enumerate(ms)]
    plans = [TuckerPlan.from_factors(S.dims, S.q, S.m, *struct_to_abi(S)) for S in structs]
    nrhs = [33, 1][:len(plans)]
    X = [workloads.complex_normal((S.m, n), 500 + c) for c, (S, n) in enumerate(zip(structs, nrhs))]
    Y = [workloads.complex_normal((S.q * S.nv, n), 600 + c) for c, (S, n) in enumerate(zip(structs, nrhs))]
    cx = lambda a: torch.from_numpy(a.astype(np.complex64)).cuda()  # noqa: E731
    print(f"batched kernels dims={dims} q={q} m={ms} rmax={rmax}", flush=True)
    got_f = _run(plans, 0, [cx(x) for x in X], nrhs)
    got_a = _run(plans, 1, [cx(y) for y in Y], nrhs)
    for c, S in enumerate(structs):
        assert_close(got_f[c], om.alg1(S, X[c]), 1e-5, what=("forward", c))
        assert_close(got_a[c], om.alg2(S, Y[c]), 1e-5, what=("adjoint", c))


def test_batch_adjoint_items_span_tiles(gpu_lib):
    """Enough work that each adjoint item sweeps several voxel tiles, with
    partial 32-column chunks (waves owning 0, 1 or 4 columns), so that the
    operand prefetch across tiles is exercised; forward checked too."""
    import torch
    from paper_2103_06393_amd.ops import TuckerPlan
    from tests.plans import random_struct
    dims, q = (40, 16, 120), 3
    ms, nrhs = (40, 33, 9, 64), [40, 33, 7, 64]
    structs = [random_struct(dims, q, m, 24, 70 + c) for c, m in enumerate(ms)]
    plans = [TuckerPlan.from_factors(S.dims, S.q, S.m, *struct_to_abi(S)) for S in structs]
    X = [workloads.complex_normal((S.m, n), 700 + c) for c, (S, n) in enumerate(zip(structs, nrhs))]
    Y = [workloads.complex_normal((S.q * S.nv, n), 800 + c) for c, (S, n) in enumerate(zip(structs, nrhs))]
    cx = lambda a: torch.from_numpy(a.astype(np.complex64)).cuda()  # noqa: E731
    got_f = _run(plans, 0, [cx(x) for x in X], nrhs)
    got_a = _run(plans, 1, [cx(y) for y in Y], nrhs)
    for c, S in enumerate(structs):
        assert_close(got_f[c], om.alg1(S, X[c]), 1e-5, what=("forward", c))
        assert_close(got_a[c], om.alg2(S, Y[c]), 1e-5, what=("adjoint", c))


def test_batch_bf16x3(gpu_lib):
    """Plans in BF16X3 form: both batched directions apply the decompressed
    tensors with the hi/lo split on v_mfma_f32_32x32x16_bf16 (three of the
    four hi/lo products, FP32 accumulation); checked against the FP64 oracle
    below the 1e-3 bar of the split form (and far inside it)."""
    import torch
    from paper_2103_06393_amd import lib
    from paper_2103_06393_amd.ops import TuckerPlan
    from tests.plans import random_struct
    dims, q = (96, 20, 7), 3
    ms, nrhs = (37, 9), [33, 5]
    structs = [random_struct(dims, q, m, 32, 90 + c) for c, m in enumerate(ms)]
    plans = [TuckerPlan.from_factors(S.dims, S.q, S.m, *struct_to_abi(S),
                                     precision=lib.TV_PREC_BF16X3) for S in structs]
    X = [workloads.complex_normal((S.m, n), 910 + c) for c, (S, n) in enumerate(zip(structs, nrhs))]
    Y = [workloads.complex_normal((S.q * S.nv, n), 920 + c) for c, (S, n) in enumerate(zip(structs, nrhs))]
    cx = lambda a: torch.from_numpy(a.astype(np.complex64)).cuda()  # noqa: E731
    got_f = _run(plans, 0, [cx(x) for x in X], nrhs)
    got_a = _run(plans, 1, [cx(y) for y in Y], nrhs)
    for c, S in enumerate(structs):
        ef = rel_err(got_f[c], om.alg1(S, X[c]))
        print(f"bf16x3 batched forward, plan {c}: rel err {ef:.2e}", flush=True)
        assert ef <= 1e-4, ("forward", c, ef)
        ea = rel_err(got_a[c], om.alg2(S, Y[c]))
        print(f"bf16x3 batched adjoint, plan {c}: rel err {ea:.2e}", flush=True)
        assert ea <= 1e-4, ("adjoint", c, ea)


def test_batch_autotune_and_forced_configurations(gpu_lib, c4s, tmp_path):
    """tv_batch_autotune picks (tsplit, workgroups per CU) by timing, caches
    the choice, and every configuration it may choose gives the oracle's
    products (adjoint voxel-tile slices change only the summation order)."""
    import json
    import torch
    from paper_2103_06393_amd import lib
    from paper_2103_06393_amd.ops import batch_create
    wls, structs, plans = c4s
    nrhs = [5, 2, 9, 3][:len(plans)]
    hs = [p.handle for p in plans]
    cache = tmp_path / "tune.json"
    st = torch.cuda.current_stream().cuda_stream
    cfg_f = lib.tv_batch_autotune(hs, 0, nrhs, str(cache), st)
    cfg_a = lib.tv_batch_autotune(hs, 1, nrhs, str(cache), st)
    entries = json.loads(cache.read_text())
    assert len([k for k in entries if k.startswith("b1|")]) == 2
    assert lib.tv_batch_autotune(hs, 1, nrhs, str(cache), st) == cfg_a   # from the cache
    X = [workloads.complex_normal((S.m, n), 400 + c) for c, (S, n) in enumerate(zip(structs, nrhs))]
    Y = [workloads.complex_normal((S.q * S.nv, n), 500 + c) for c, (S, n) in enumerate(zip(structs, nrhs))]
    cx = lambda a: torch.from_numpy(a.astype(np.complex64)).cuda()  # noqa: E731
    for op, cfgs in ((0, [cfg_f, (0, 1)]), (1, [cfg_a, (1, 1), (3, 2)])):
        for cfg in cfgs:
            b, arena = batch_create(hs, op, nrhs, cfg)
            try:
                assert lib.tv_batch_info(b)[1] >= 1
                ins = [cx(a).t().contiguous().t() for a in (X if op == 0 else Y)]
                outs = [torch.zeros((p.rows if op == 0 else p.m, n), dtype=torch.complex64,
                                    device="cuda").t().contiguous().t()
                        for p, n in zip(plans, nrhs)]
                ws = torch.empty(lib.tv_batch_workspace_bytes(b), dtype=torch.uint8,
                                 device="cuda")
                lib.tv_batch_run(b, [x.data_ptr() for x in ins], [_ld(x) for x in ins],
                                 [y.data_ptr() for y in outs], [_ld(y) for y in outs],
                                 ws.data_ptr(), ws.numel(), st)
                torch.cuda.synchronize()
                for c, S in enumerate(structs):
                    ref = om.alg1(S, X[c]) if op == 0 else om.alg2(S, Y[c])
                    assert_close(outs[c].cpu().numpy(), ref, 1e-5,
                                 what=f"op {op} config {cfg} coil {c}")
            finally:
                lib.tv_batch_destroy(b)
