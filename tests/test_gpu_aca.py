"""GPU parity of the ACA + Tucker products, tv_aca_matvec (Y = U (V^* X)) and
tv_aca_rmatvec (X = V (U^* Y)), against the FP64 oracle (Sec. III.B, the
substitution after Algorithms 1 and 2; U from Algorithm 3).

The library runs on the oracle's factors, imported through the C ABI, and on
V and the vectors rounded to complex64 (both sides take those same values).
Bar: relative 2-norm error <= 1e-5 per right-hand side for FP32 plans (FP32
Tucker products, FP64 coil-side sums), 1e-3 for BF16X3 plans.
"""
import numpy as np
import pytest

import workloads
from oracle import aca as oaca
from oracle import matvec as om
from tests.plans import abs_struct, assert_close, random_struct, rel_err, struct_to_abi

pytestmark = pytest.mark.gpu
TOL_FP32 = 1e-5
TOL_BF16X3 = 1e-3


def _plan(S, precision=0):
    from paper_2103_06393_amd.ops import TuckerPlan
    ranks, G, U1, U2, U3 = struct_to_abi(S)
    return TuckerPlan.from_factors(S.dims, S.q, S.m, ranks, G, U1, U2, U3,
                                   precision)


def _c64(a):
    return np.ascontiguousarray(a, np.complex64)


def _cuda(a):
    import torch
    return torch.from_numpy(_c64(a)).cuda()


def _up(a):
    """Values as the GPU sees them (complex64), widened for the oracle."""
    return _c64(a).astype(np.complex128)


@pytest.fixture(scope="module")
def alg3():
    """Algorithm 3 on the body-coil stand-in (2.5 cm voxels, 400 elements),
    stopped after 24 cross steps: U compressed with HOSVD(3 eps)."""
    wl = workloads.make_bodycoil("aca_s")
    R = oaca.aca_tucker(wl, wl.tol, max_rank=24)
    return wl, R


def test_algorithm3_factors(gpu_lib, alg3):
    import torch
    from paper_2103_06393_amd.ops import AcaTuckerOperator
    wl, R = alg3
    S, V = R.U.S, _up(R.V)
    op = AcaTuckerOperator(_plan(S), _cuda(V))
    X = _up(wl.x(3))
    Y = _up(wl.y(2))
    got_y = op.matvec(_cuda(X)).cpu().numpy()
    got_x = op.rmatvec(_cuda(Y)).cpu().numpy()
    torch.cuda.synchronize()
    ref_y = oaca.aca_matvec(S, V, X)
    ref_x = oaca.aca_rmatvec(S, V, Y)
    for c in range(3):
        assert_close(got_y[:, c], ref_y[:, c], TOL_FP32)
    for c in range(2):
        assert_close(got_x[:, c], ref_x[:, c], TOL_FP32)
    # one right-hand side through the vector form
    g1 = op.matvec(_cuda(X[:, 0])).cpu().numpy()
    assert_close(g1, ref_y[:, 0], TOL_FP32)


@pytest.mark.parametrize("dims,q,rc,m,rmax,nrhs,seed", [
    ((37, 20, 9), 3, 7, 1000, 8, 2, 1),     # m ragged against 256-row blocks
    ((16, 8, 8), 1, 1, 1, 4, 1, 2),         # r_c = 1 and m = 1
    ((24, 10, 12), 12, 3, 257, 6, 3, 3),    # q = 12, m one past a block
    ((40, 9, 5), 3, 40, 300, 5, 1, 4),      # r_c > workgroup count per row
])
def test_shapes_and_leading_dimensions(gpu_lib, dims, q, rc, m, rmax, nrhs,
                                       seed):
    import torch
    lib = gpu_lib
    S = random_struct(dims, q, rc, rmax, seed)
    P = _plan(S)
    rows = S.q * S.nv
    V = _up(workloads.complex_normal((m, rc), 100 + seed))
    X = _up(workloads.complex_normal((m, nrhs), 200 + seed))
    Y = _up(workloads.complex_normal((rows, nrhs), 300 + seed))
    ldv, ldx, ldy = m + 5, m + 3, rows + 11
    Vb = np.zeros((rc, ldv), np.complex64)
    Vb[:, :m] = V.T
    Xb = np.zeros((nrhs, ldx), np.complex64)
    Xb[:, :m] = X.T
    Yb = np.zeros((nrhs, ldy), np.complex64)
    Yb[:, :rows] = Y.T
    sentinel = np.complex64(7.0 - 3.0j)
    Vd, Xd, Yd = _cuda(Vb), _cuda(Xb), _cuda(Yb)
    Yo = _cuda(np.full((nrhs, ldy), sentinel))
    Xo = _cuda(np.full((nrhs, ldx), sentinel))
    st = torch.cuda.current_stream().cuda_stream
    for op in (0, 1):
        n = lib.tv_aca_workspace_bytes(P.handle, op, nrhs)
        assert n >= 8 * rc * nrhs
        ws = torch.empty(n, dtype=torch.uint8, device="cuda")
        if op == 0:
            lib.tv_aca_matvec(P.handle, Vd.data_ptr(), m, ldv, Xd.data_ptr(),
                              ldx, nrhs, Yo.data_ptr(), ldy, ws.data_ptr(), n,
                              st)
        else:
            lib.tv_aca_rmatvec(P.handle, Vd.data_ptr(), m, ldv, Yd.data_ptr(),
                               ldy, nrhs, Xo.data_ptr(), ldx, ws.data_ptr(), n,
                               st)
    torch.cuda.synchronize()
    gy = Yo.cpu().numpy()
    gx = Xo.cpu().numpy()
    ref_y = oaca.aca_matvec(S, V, X)
    ref_x = oaca.aca_rmatvec(S, V, Y)
    for c in range(nrhs):
        assert_close(gy[c, :rows], ref_y[:, c], TOL_FP32)
        assert_close(gx[c, :m], ref_x[:, c], TOL_FP32)
        assert np.all(gy[c, rows:] == sentinel)      # padding untouched
        assert np.all(gx[c, m:] == sentinel)


def test_bf16x3_plan(gpu_lib):
    from paper_2103_06393_amd.ops import AcaTuckerOperator
    S = random_struct((48, 20, 16), 3, 12, 10, 9)
    V = _up(workloads.complex_normal((500, 12), 91))
    op = AcaTuckerOperator(_plan(S, precision=1), _cuda(V))
    x = _up(workloads.complex_normal(500, 92))
    y = _up(workloads.complex_normal(S.q * S.nv, 93))
    assert_close(op.matvec(_cuda(x)).cpu().numpy(), oaca.aca_matvec(S, V, x)[:, 0], TOL_BF16X3)
    assert_close(op.rmatvec(_cuda(y)).cpu().numpy(), oaca.aca_rmatvec(S, V, y)[:, 0], TOL_BF16X3)


def test_argument_errors(gpu_lib):
    import torch
    lib = gpu_lib
    S = random_struct((16, 8, 8), 3, 4, 4, 11)
    P = _plan(S)
    m, rows = 50, S.q * S.nv
    V = _cuda(np.ones((4, m)))
    x = _cuda(np.ones(m))
    y = _cuda(np.ones(rows))
    n = lib.tv_aca_workspace_bytes(P.handle, 0, 1)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    cases = [
        (dict(ws_bytes=n - 1), -8),                      # workspace too small
        (dict(ldv=m - 1), -2),                           # ldv < m
        (dict(ldy=rows - 1), -2),                        # ldy < rows
        (dict(nrhs=0), -1),
        (dict(y_ptr=x.data_ptr()), -1),                  # output overlaps input
        (dict(y_ptr=V.data_ptr()), -1),                  # output overlaps V
    ]
    for kw, code in cases:
        a = dict(v_ptr=V.data_ptr(), m=m, ldv=m, x_ptr=x.data_ptr(), ldx=m,
                 nrhs=1, y_ptr=y.data_ptr(), ldy=rows, ws_ptr=ws.data_ptr(),
                 ws_bytes=n, stream=st)
        a.update(kw)
        with pytest.raises(lib.TuckVsieError) as e:
            lib.tv_aca_matvec(P.handle, **a)
        assert e.value.status == code, kw


def test_body_coil_5mm_full(gpu_lib):
    """The 5 mm body-coil shape of Sec. IV.B.2: 81 x 44 x 108 voxels, PWC,
    r_c = 250 columns of U with ranks up to 18, 9450 coil elements; full
    forward and adjoint against the oracle."""
    from paper_2103_06393_amd.ops import AcaTuckerOperator
    S = random_struct((81, 44, 108), 3, 250, 18, 21)
    m = 9450
    V = _up(workloads.complex_normal((m, 250), 22))
    P = _plan(S)
    P.autotune()
    op = AcaTuckerOperator(P, _cuda(V))
    x = _up(workloads.complex_normal(m, 23))
    y = _up(workloads.complex_normal(S.q * S.nv, 24))
    assert_close(op.matvec(_cuda(x)).cpu().numpy(), oaca.aca_matvec(S, V, x)[:, 0], TOL_FP32)
    assert_close(op.rmatvec(_cuda(y)).cpu().numpy(), oaca.aca_rmatvec(S, V, y)[:, 0], TOL_FP32)


def test_body_coil_1mm_sampled(gpu_lib):
    """The 1 mm body-coil shape (409 x 219 x 541, PWC, r_c = 287, ranks
    15-18 as reported in Sec. IV.B.2, 9450 elements), autotuned as the
    benchmark runs it: sampled rows of U (V^* x) against single-element
    decompression, and the adjoint identity between the two GPU products."""
    import torch
    from paper_2103_06393_amd.ops import AcaTuckerOperator
    rng = np.random.default_rng(31)
    dims, rc, m = (409, 219, 541), 287, 9450
    cores, facs = [], []
    for _ in range(rc):
        cj, fj = [], []
        for _ in range(3):
            r = [int(v) for v in rng.integers(15, 19, size=3)]
            cj.append(rng.standard_normal(r) + 1j * rng.standard_normal(r))
            fj.append(tuple(np.linalg.qr(rng.standard_normal((n, k)) +
                                         1j * rng.standard_normal((n, k)))[0]
                            for n, k in zip(dims, r)))
        cores.append(cj)
        facs.append(fj)
    S = om.from_factors(dims, 3, cores, facs)
    V = _up(workloads.complex_normal((m, rc), 32))
    P = _plan(S)
    P.autotune()
    op = AcaTuckerOperator(P, _cuda(V))
    x = _up(workloads.complex_normal(m, 33))
    got_y = op.matvec(_cuda(x))
    yv = torch.from_numpy(_c64(workloads.complex_normal(S.q * S.nv, 34))).cuda()
    got_x = op.rmatvec(yv).cpu().numpy().astype(np.complex128)
    rows = np.random.default_rng(35).integers(0, S.q * S.nv, size=24)
    ref = oaca.aca_entries(S, V, x, rows)
    gy = got_y.cpu().numpy().astype(np.complex128)
    assert np.linalg.norm(gy[rows] - ref) <= TOL_FP32 * np.linalg.norm(ref)
    lhs = np.vdot(yv.cpu().numpy().astype(np.complex128), gy)
    rhs = np.vdot(got_x, x)
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    # U^* y itself on sampled columns against the oracle: with V the identity
    # (m = r_c) the adjoint returns U^* y, whose entry l is Algorithm 2's inner
    # product of U's column l with y
    opI = AcaTuckerOperator(P, torch.eye(rc, dtype=torch.complex64, device="cuda"))
    uy = opI.rmatvec(yv).cpu().numpy()
    y64 = yv.cpu().numpy().astype(np.complex128)
    cols = [0, rc // 2, rc - 1]
    ref = om.adjoint_entries(S, y64, cols)
    terms = np.abs(om.adjoint_entries(abs_struct(S), np.abs(y64), cols))
    assert_close(uy[cols], ref, TOL_FP32, terms=terms, what="1 mm U^* y columns")


def test_graph_replay(gpu_lib):
    """Both ACA + Tucker products allocate nothing and never synchronise, so
    they capture into a HIP graph; replays (eager work and syncs between
    them, fresh inputs each time) match eager calls exactly."""
    import torch
    lib = gpu_lib
    S = random_struct((40, 20, 12), 3, 9, 8, 51)
    P = _plan(S)
    m = 700
    V = _cuda(workloads.complex_normal((9, m), 52))          # column-major m x 9
    rows = S.q * S.nv
    x = _cuda(workloads.complex_normal(m, 53))
    y = _cuda(workloads.complex_normal(rows, 54))
    yo = torch.empty(rows, dtype=torch.complex64, device="cuda")
    xo = torch.empty(m, dtype=torch.complex64, device="cuda")
    n0 = lib.tv_aca_workspace_bytes(P.handle, 0, 1)
    n1 = lib.tv_aca_workspace_bytes(P.handle, 1, 1)
    ws0 = torch.empty(n0, dtype=torch.uint8, device="cuda")
    ws1 = torch.empty(n1, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())

    def run(stream):
        lib.tv_aca_matvec(P.handle, V.data_ptr(), m, m, x.data_ptr(), m, 1,
                          yo.data_ptr(), rows, ws0.data_ptr(), n0, stream)
        lib.tv_aca_rmatvec(P.handle, V.data_ptr(), m, m, y.data_ptr(), rows, 1,
                           xo.data_ptr(), m, ws1.data_ptr(), n1, stream)

    with torch.cuda.stream(s):
        run(s.cuda_stream)                                   # warm-up
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        run(s.cuda_stream)
    torch.cuda.synchronize()
    for rep in range(3):
        x.copy_(_cuda(workloads.complex_normal(m, 60 + rep)))
        y.copy_(_cuda(workloads.complex_normal(rows, 70 + rep)))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        gy, gx = yo.clone(), xo.clone()
        yo.zero_()
        xo.zero_()
        run(torch.cuda.current_stream().cuda_stream)         # eager reference
        torch.cuda.synchronize()
        assert torch.equal(gy, yo) and torch.equal(gx, xo), rep
