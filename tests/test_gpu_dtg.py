"""The decompress-then-GEMM form of Algorithms 1 and 2 (slabs of the stacked
operand B written by the decompression kernel, then one MFMA GEMM per
component; the adjoint's contraction over voxel columns as its own GEMM
followed by the FP64 sum against conj(U1)) against the
FP64 oracle, in every configuration the autotuner may choose: slab sizes
(ragged last slab), GEMM tiles, k-step splits, ragged voxel rows and columns,
ranks up to 32 and single-column plans."""
import numpy as np
import pytest

from oracle import matvec as om
from tests.plans import adj_terms, assert_close, fwd_terms, random_struct, struct_to_abi

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _plan(S):
    from paper_2103_06393_amd.ops import TuckerPlan
    return TuckerPlan.from_factors(S.dims, S.q, S.m, *struct_to_abi(S))


@pytest.mark.parametrize("dims,q,m,rmax,seed,slab,nbw,splits", [
    ((20, 13, 7), 2, 5, 5, 1, 0, 2, 1),       # n1 = 20: one 4-block row tile, ragged
    ((64, 32, 24), 3, 9, 12, 2, 8, 2, 1),     # three slabs
    ((64, 32, 24), 3, 9, 12, 2, 5, 4, 3),     # ragged last slab, wide tile, 3 splits
    ((96, 40, 33), 3, 6, 20, 4, 16, 4, 1),    # 6 blocks padded to 8, i2 ragged
    ((130, 24, 10), 1, 7, 32, 5, 0, 2, 2),    # n1 > 128: 2 row tiles, ranks to 32
    ((256, 16, 9), 3, 4, 10, 6, 3, 2, 1),     # 16 row blocks
    ((17, 9, 5), 12, 1, 4, 7, 2, 4, 1),       # q = 12, one column, odd n1
])
def test_dtg_forward_matches_oracle(gpu_lib, dims, q, m, rmax, seed, slab, nbw, splits):
    import torch
    from paper_2103_06393_amd import lib
    S = random_struct(dims, q, m, rmax, seed)
    P = _plan(S)
    lib.tv_plan_configure(P.handle, 0, path=1, splits=splits, slab_i3=slab, gemm_nbw=nbw)
    P._ws.clear()
    info = P.info
    assert info.kernel[0] == 2 and info.splits[0] == splits and info.tile_t3[0] == nbw
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    got = P.matvec(torch.from_numpy(x.astype(np.complex64)).cuda()).cpu().numpy()
    assert_close(got, om.alg1(S, x)[:, 0], TOL, terms=fwd_terms(S, x), what="GEMM path Z x")
    # a second call reuses the workspace (stale B rows must not leak in)
    x2 = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    got2 = P.matvec(torch.from_numpy(x2.astype(np.complex64)).cuda()).cpu().numpy()
    assert_close(got2, om.alg1(S, x2)[:, 0], TOL, terms=fwd_terms(S, x2), what="second call")
    # the adjoint on the same path and slab, tile and splits, both workgroup orders
    lib.tv_plan_configure(P.handle, 1, path=1, splits=splits, slab_i3=slab, gemm_nbw=nbw,
                          gemm_order=seed % 2)
    P._ws.clear()
    assert P.info.kernel[1] == 2
    for rep in range(2):
        y = rng.standard_normal(S.q * S.nv) + 1j * rng.standard_normal(S.q * S.nv)
        gx = P.rmatvec(torch.from_numpy(y.astype(np.complex64)).cuda()).cpu().numpy()
        assert_close(gx, om.alg2(S, y)[:, 0], TOL, terms=adj_terms(S, y),
                     what=f"GEMM path Z^* y, call {rep}")


@pytest.mark.parametrize("dims,q,m,rmax,seed,slab,nbw,splits,order", [
    ((20, 13, 7), 2, 5, 5, 31, 0, 2, 1, 0),     # 91 columns: a ragged 4-column group
    ((64, 32, 24), 3, 9, 12, 32, 5, 4, 3, 1),   # five slabs (ragged last), 3 splits each
    ((96, 40, 33), 3, 6, 20, 33, 16, 4, 2, 0),  # last slab of 40 columns, 6 blocks padded to 8
    ((130, 24, 10), 1, 7, 32, 34, 0, 2, 5, 1),  # n1 > 128: 2 row tiles, ranks to 32
    ((256, 16, 9), 3, 4, 10, 35, 3, 4, 1, 0),   # 16 row blocks
    ((17, 9, 5), 12, 1, 4, 36, 2, 2, 64, 1),    # q = 12, one column, splits past the stages
    ((33, 9, 7), 2, 4, 7, 37, 0, 4, 2, 0),      # odd n1: element-wise partial stores
])
def test_dtg_column_adjoint_matches_oracle(gpu_lib, dims, q, m, rmax, seed, slab, nbw, splits,
                                           order):
    """The adjoint with the sum over voxel columns first (Z_k = Y B_k^* as a
    GEMM over the slab's columns, one partial per slab and split, then the
    FP64 sum against conj(U1)) in every tile, split and order the autotuner
    may choose, two calls on one workspace."""
    import torch
    from paper_2103_06393_amd import lib
    S = random_struct(dims, q, m, rmax, seed)
    P = _plan(S)
    lib.tv_plan_configure(P.handle, 1, path=1, splits=splits, slab_i3=slab, gemm_nbw=nbw,
                          gemm_order=order)
    P._ws.clear()
    info = P.info
    assert info.kernel[1] == 2 and info.splits[1] == splits and info.tile_t3[1] == nbw
    rng = np.random.default_rng(seed)
    for rep in range(2):
        y = rng.standard_normal(S.q * S.nv) + 1j * rng.standard_normal(S.q * S.nv)
        gx = P.rmatvec(torch.from_numpy(y.astype(np.complex64)).cuda()).cpu().numpy()
        assert_close(gx, om.alg2(S, y)[:, 0], TOL, terms=adj_terms(S, y),
                     what=f"column-GEMM adjoint Z^* y, call {rep}")


def test_dtg_workspace_poisoned_and_multi_rhs(gpu_lib):
    """NaN-filled workspace (the decompression must overwrite or zero every
    element the GEMM reads) and several right-hand sides with leading dims."""
    import torch
    from paper_2103_06393_amd import lib
    S = random_struct((48, 20, 12), 3, 6, 9, 11)
    P = _plan(S)
    lib.tv_plan_configure(P.handle, 0, path=1, splits=1, slab_i3=5, gemm_nbw=2)
    p = 3
    rng = np.random.default_rng(4)
    X = rng.standard_normal((S.m, p)) + 1j * rng.standard_normal((S.m, p))
    nb = lib.tv_workspace_bytes(P.handle, 0, p)
    ws = torch.full((nb // 4,), float("nan"), dtype=torch.float32, device="cuda")
    ldx, ldy = S.m + 2, S.q * S.nv + 4
    xb = np.zeros((p, ldx), np.complex64)
    xb[:, :S.m] = X.T
    xd = torch.from_numpy(xb).cuda()
    yd = torch.zeros((p, ldy), dtype=torch.complex64, device="cuda")
    lib.tv_matvec(P.handle, xd.data_ptr(), ldx, p, yd.data_ptr(), ldy, ws.data_ptr(), nb,
                  torch.cuda.current_stream().cuda_stream)
    got = yd.cpu().numpy()[:, :S.q * S.nv].T
    assert_close(got, om.alg1(S, X), TOL, terms=fwd_terms(S, X), what="GEMM path, 3 RHS")


@pytest.mark.parametrize("dims,q,m,rmax,seed,slab,nbw,splits", [
    ((20, 13, 7), 2, 5, 5, 21, 0, 2, 1),
    ((64, 32, 24), 3, 9, 12, 22, 5, 4, 3),
    ((96, 40, 33), 3, 6, 20, 23, 16, 4, 1),
    ((130, 24, 10), 1, 7, 32, 24, 0, 2, 2),
    ((17, 9, 5), 12, 1, 4, 25, 2, 2, 1),
    ((64, 32, 24), 3, 9, 12, 26, 5, 2, 1),    # 2 workgroups per CU
    ((160, 20, 9), 2, 5, 10, 27, 0, 2, 2),
])
def test_dtg_bf16x3_forward_matches_oracle(gpu_lib, dims, q, m, rmax, seed, slab, nbw, splits):
    """BF16X3 plans: the stacked GEMM on v_mfma_f32_32x32x16_bf16 with hi/lo
    operands (hi hi + hi lo + lo hi, FP32 accumulation), the FP32 slab split
    into bf16 hi/lo inside the GEMM; every entry within 1e-4 of the moduli of
    its terms (each product carries a relative error of about 2^-17)."""
    import torch
    from paper_2103_06393_amd import lib
    from paper_2103_06393_amd.ops import TuckerPlan
    S = random_struct(dims, q, m, rmax, seed)
    P = TuckerPlan.from_factors(S.dims, S.q, S.m, *struct_to_abi(S),
                                precision=lib.TV_PREC_BF16X3)
    lib.tv_plan_configure(P.handle, 0, path=1, splits=splits, slab_i3=slab, gemm_nbw=nbw)
    P._ws.clear()
    assert P.info.kernel[0] == 2
    rng = np.random.default_rng(seed)
    for rep in range(2):
        x = rng.standard_normal(m) + 1j * rng.standard_normal(m)
        got = P.matvec(torch.from_numpy(x.astype(np.complex64)).cuda()).cpu().numpy()
        e = assert_close(got, om.alg1(S, x)[:, 0], 1e-4, terms=fwd_terms(S, x),
                         what=f"BF16X3 GEMM path Z x, call {rep}")
        print(f"bf16x3 dtg {dims}: rel err {e:.2e}")


@pytest.mark.parametrize("dims,q,m,rmax,seed,slab,nbw,splits,order", [
    ((20, 13, 7), 2, 5, 5, 41, 0, 2, 1, 0),     # ragged 8-column chunk, n1 = 20
    ((64, 32, 24), 3, 9, 12, 42, 5, 4, 3, 1),   # five slabs, 3 splits
    ((130, 24, 10), 1, 7, 32, 43, 0, 4, 5, 0),  # n1 > 128, ranks to 32
    ((33, 9, 7), 2, 4, 7, 44, 0, 2, 2, 1),      # odd n1
    ((17, 9, 5), 12, 1, 4, 45, 2, 4, 64, 0),    # q = 12, splits past the stages
])
def test_dtg_bf16x3_column_adjoint_matches_oracle(gpu_lib, dims, q, m, rmax, seed, slab, nbw,
                                                  splits, order):
    """BF16X3 plans: y packed as bf16 hi/lo, the FP32 slab split into hi/lo
    in the column GEMM (hi hi + hi lo + lo hi, FP32 accumulation); within
    1e-4 of the moduli of the terms, two calls on one workspace."""
    import torch
    from paper_2103_06393_amd import lib
    from paper_2103_06393_amd.ops import TuckerPlan
    S = random_struct(dims, q, m, rmax, seed)
    P = TuckerPlan.from_factors(S.dims, S.q, S.m, *struct_to_abi(S),
                                precision=lib.TV_PREC_BF16X3)
    lib.tv_plan_configure(P.handle, 1, path=1, splits=splits, slab_i3=slab, gemm_nbw=nbw,
                          gemm_order=order)
    P._ws.clear()
    assert P.info.kernel[1] == 2
    rng = np.random.default_rng(seed)
    for rep in range(2):
        y = rng.standard_normal(S.q * S.nv) + 1j * rng.standard_normal(S.q * S.nv)
        gx = P.rmatvec(torch.from_numpy(y.astype(np.complex64)).cuda()).cpu().numpy()
        e = assert_close(gx, om.alg2(S, y)[:, 0], 1e-4, terms=adj_terms(S, y),
                         what=f"BF16X3 column adjoint, call {rep}")
        print(f"bf16x3 column adjoint {dims}: rel err {e:.2e}")


@pytest.mark.parametrize("dims,q,m,rmax,seed,slab,splits", [
    ((256, 16, 9), 3, 4, 10, 51, 3, 1),     # 2 n1 = 512: one workgroup over all rows
    ((256, 20, 11), 2, 6, 14, 52, 0, 2),    # ragged columns, 2 splits
    ((250, 12, 7), 1, 5, 9, 53, 0, 1),      # n1 = 250: the last 6 rows are padding
])
def test_dtg_bf16x3_full_row_tile_matches_oracle(gpu_lib, dims, q, m, rmax, seed, slab, splits):
    """BF16X3 plans with 2 n1 = 512 (the packed rows come in 16 blocks of
    32): the GEMMs' workgroup tile over all voxel rows (row_cap 8, 8 blocks
    per wave, one workgroup per CU, accumulators in AGPRs), forward and
    column adjoint, within 1e-4 of the moduli of the terms, two calls each."""
    import torch
    from paper_2103_06393_amd import lib
    from paper_2103_06393_amd.ops import TuckerPlan
    S = random_struct(dims, q, m, rmax, seed)
    P = TuckerPlan.from_factors(S.dims, S.q, S.m, *struct_to_abi(S),
                                precision=lib.TV_PREC_BF16X3)
    lib.tv_plan_configure(P.handle, 0, path=1, splits=splits, slab_i3=slab, gemm_nbw=2,
                          row_cap=8)
    lib.tv_plan_configure(P.handle, 1, path=1, splits=splits, slab_i3=slab, gemm_nbw=2,
                          gemm_order=seed % 2, row_cap=8)
    P._ws.clear()
    assert P.info.kernel[0] == 2 and P.info.kernel[1] == 2
    rng = np.random.default_rng(seed)
    for rep in range(2):
        x = rng.standard_normal(m) + 1j * rng.standard_normal(m)
        got = P.matvec(torch.from_numpy(x.astype(np.complex64)).cuda()).cpu().numpy()
        assert_close(got, om.alg1(S, x)[:, 0], 1e-4, terms=fwd_terms(S, x),
                     what=f"BF16X3 full-row tile Z x, call {rep}")
        y = rng.standard_normal(S.q * S.nv) + 1j * rng.standard_normal(S.q * S.nv)
        gx = P.rmatvec(torch.from_numpy(y.astype(np.complex64)).cuda()).cpu().numpy()
        assert_close(gx, om.alg2(S, y)[:, 0], 1e-4, terms=adj_terms(S, y),
                     what=f"BF16X3 full-row tile Z^* y, call {rep}")


def test_dtg_adjoint_poisoned_workspace_and_multi_rhs(gpu_lib):
    import torch
    from paper_2103_06393_amd import lib
    S = random_struct((50, 20, 12), 3, 6, 9, 12)       # even n1: paired y loads
    T = random_struct((33, 9, 7), 2, 4, 7, 13)          # odd n1: single loads
    for R, slab, order, nbw, splits in ((S, 5, 0, 2, 1), (T, 0, 1, 2, 1), (S, 0, 1, 2, 1),
                                        (S, 5, 0, 4, 3), (T, 0, 1, 4, 2)):
        P = _plan(R)
        lib.tv_plan_configure(P.handle, 1, path=1, splits=splits, slab_i3=slab, gemm_nbw=nbw,
                              gemm_order=order)
        p = 2
        rng = np.random.default_rng(5)
        Y = rng.standard_normal((R.q * R.nv, p)) + 1j * rng.standard_normal((R.q * R.nv, p))
        nb = lib.tv_workspace_bytes(P.handle, 1, p)
        ws = torch.full((nb // 4,), float("nan"), dtype=torch.float32, device="cuda")
        ldy, ldx = R.q * R.nv + 2, R.m + 3
        yb = np.zeros((p, ldy), np.complex64)
        yb[:, :R.q * R.nv] = Y.T
        yd = torch.from_numpy(yb).cuda()
        xd = torch.zeros((p, ldx), dtype=torch.complex64, device="cuda")
        lib.tv_rmatvec(P.handle, yd.data_ptr(), ldy, p, xd.data_ptr(), ldx, ws.data_ptr(), nb,
                       torch.cuda.current_stream().cuda_stream)
        got = xd.cpu().numpy()[:, :R.m].T
        assert_close(got, om.alg2(R, Y), TOL, terms=adj_terms(R, Y), what="GEMM adjoint, 2 RHS")


def test_dtg_refused_configurations(gpu_lib):
    from paper_2103_06393_amd import lib
    from paper_2103_06393_amd.ops import TuckerPlan
    S = random_struct((20, 13, 7), 2, 3, 5, 1)
    P = _plan(S)
    with pytest.raises(lib.TuckVsieError):
        lib.tv_plan_configure(P.handle, 1, path=1, splits=1, gemm_nbw=2, gemm_order=2)
    with pytest.raises(lib.TuckVsieError):
        lib.tv_plan_configure(P.handle, 1, path=1, splits=1, gemm_nbw=3, gemm_order=0)
    with pytest.raises(lib.TuckVsieError):
        lib.tv_plan_configure(P.handle, 1, path=1, splits=65, gemm_nbw=4, gemm_order=1)
    with pytest.raises(lib.TuckVsieError):
        lib.tv_plan_configure(P.handle, 0, path=1, splits=1, gemm_nbw=3)
    with pytest.raises(lib.TuckVsieError):
        lib.tv_plan_configure(P.handle, 0, path=1, splits=1, gemm_nbw=1)
    # the full-row tile: BF16X3 plans with 2 n1 = 512 and gemm_nbw 2 only
    with pytest.raises(lib.TuckVsieError):
        lib.tv_plan_configure(P.handle, 0, path=1, splits=1, gemm_nbw=2, row_cap=8)
    with pytest.raises(lib.TuckVsieError):
        lib.tv_plan_configure(P.handle, 1, path=1, splits=1, gemm_nbw=2, row_cap=4)
    assert P.info.kernel[0] != 2 and P.info.kernel[1] != 2   # refusals left no trace
    B = TuckerPlan.from_factors(S.dims, S.q, S.m, *struct_to_abi(S),
                                precision=lib.TV_PREC_BF16X3)
    with pytest.raises(lib.TuckVsieError):                   # 2 n1 = 40, not 512
        lib.tv_plan_configure(B.handle, 0, path=1, splits=1, gemm_nbw=2, row_cap=8)
    W = TuckerPlan.from_factors((256, 8, 5), 1, 2, *struct_to_abi(random_struct((256, 8, 5), 1, 2,
                                                                                4, 2)),
                                precision=lib.TV_PREC_BF16X3)
    with pytest.raises(lib.TuckVsieError):                   # full-row tile needs gemm_nbw 2
        lib.tv_plan_configure(W.handle, 1, path=1, splits=1, gemm_nbw=4, row_cap=8)


def test_dtg_several_slabs_in_a_graph(gpu_lib):
    """Several slabs per call (one workspace reused slab after slab): both
    products match the oracle, and a captured graph of them replays
    bit-identical to eager calls with fresh inputs and eager work between
    the replays."""
    import torch
    from paper_2103_06393_amd import lib
    S = random_struct((48, 20, 12), 3, 6, 9, 81)
    P = _plan(S)
    lib.tv_plan_configure(P.handle, 0, path=1, splits=1, slab_i3=3, gemm_nbw=2)
    lib.tv_plan_configure(P.handle, 1, path=1, splits=2, slab_i3=5, gemm_nbw=4, gemm_order=0)
    rows = S.q * S.nv
    x = torch.zeros(S.m, dtype=torch.complex64, device="cuda")
    y = torch.zeros(rows, dtype=torch.complex64, device="cuda")
    yo = torch.empty(rows, dtype=torch.complex64, device="cuda")
    xo = torch.empty(S.m, dtype=torch.complex64, device="cuda")
    ws0, ws1 = P.workspace(0, 1), P.workspace(1, 1)

    def fill(seed):
        r = np.random.default_rng(seed)
        xv = r.standard_normal(S.m) + 1j * r.standard_normal(S.m)
        yv = r.standard_normal(rows) + 1j * r.standard_normal(rows)
        x.copy_(torch.from_numpy(xv.astype(np.complex64)))
        y.copy_(torch.from_numpy(yv.astype(np.complex64)))
        return xv.astype(np.complex64).astype(np.complex128), \
            yv.astype(np.complex64).astype(np.complex128)

    def run(stream):
        lib.tv_matvec(P.handle, x.data_ptr(), S.m, 1, yo.data_ptr(), rows, ws0.data_ptr(),
                      ws0.numel(), stream)
        lib.tv_rmatvec(P.handle, y.data_ptr(), rows, 1, xo.data_ptr(), S.m, ws1.data_ptr(),
                       ws1.numel(), stream)

    xv, yv = fill(83)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run(s.cuda_stream)
    torch.cuda.synchronize()
    assert_close(yo.cpu().numpy(), om.alg1(S, xv)[:, 0], TOL, terms=fwd_terms(S, xv),
                 what="several slabs, Z x")
    assert_close(xo.cpu().numpy(), om.alg2(S, yv)[:, 0], TOL, terms=adj_terms(S, yv),
                 what="several slabs, Z^* y")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        run(s.cuda_stream)
    torch.cuda.synchronize()
    for rep in range(3):
        fill(90 + rep)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        gy, gx = yo.clone(), xo.clone()
        yo.zero_()
        xo.zero_()
        run(torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        assert torch.equal(gy, yo) and torch.equal(gx, xo), rep
