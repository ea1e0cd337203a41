"""GPU parity of tv_matvec / tv_rmatvec (FP32) against the FP64 oracle.

The library runs on the oracle's own factors (imported through the C ABI), so
the comparison isolates the kernels' arithmetic: the bar is a relative
2-norm error of at most 1e-5 (FP32 factors and accumulation), and every entry
within 1e-5 of the sum of the moduli of the terms that make it (the scale of
FP32 rounding in that entry's sums).
"""
import numpy as np
import pytest

import workloads
from oracle import matvec as om
from tests.plans import (adj_terms, assert_close, fwd_terms, random_struct, rel_err,
                         struct_to_abi)

pytestmark = pytest.mark.gpu
TOL_FP32 = 1e-5


def _plan(S, precision=0):
    from paper_2103_06393_amd.ops import TuckerPlan
    ranks, G, U1, U2, U3 = struct_to_abi(S)
    return TuckerPlan.from_factors(S.dims, S.q, S.m, ranks, G, U1, U2, U3,
                                   precision)


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.complex64)).cuda()


@pytest.mark.parametrize("dims,q,m,rmax,seed", [
    ((20, 13, 7), 2, 5, 5, 1),      # ragged everything, n1 not a multiple of 16
    ((32, 32, 32), 3, 9, 12, 2),    # full tiles
    ((17, 70, 9), 1, 4, 9, 3),      # odd n1, i2 ragged tiles
    ((48, 40, 33), 3, 6, 20, 4),    # 3 MFMA blocks, ragged i2 and i3
    ((96, 16, 8), 2, 3, 30, 5),     # n1 = 96 (6 blocks), large ranks
    ((160, 8, 6), 1, 2, 10, 6),     # n1 > 128: two waves along rows
])
def test_random_structs(gpu_lib, dims, q, m, rmax, seed):
    import torch
    S = random_struct(dims, q, m, rmax, seed)
    P = _plan(S)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    y = rng.standard_normal(S.q * S.nv) + 1j * rng.standard_normal(S.q * S.nv)
    ref_y = om.alg1(S, x)[:, 0]
    ref_x = om.alg2(S, y)[:, 0]
    got_y = P.matvec(_cuda(x)).cpu().numpy()
    got_x = P.rmatvec(_cuda(y)).cpu().numpy()
    torch.cuda.synchronize()
    assert_close(got_y, ref_y, TOL_FP32, terms=fwd_terms(S, x), what="Z x")
    assert_close(got_x, ref_x, TOL_FP32, terms=adj_terms(S, y), what="Z^* y")


@pytest.fixture(scope="module")
def c1_struct():
    wl = workloads.make("c1")
    return wl, om.compress_columns(wl)


def test_c1_forward_adjoint(gpu_lib, c1_struct):
    wl, S = c1_struct
    P = _plan(S)
    x = wl.x()[:, 0]
    y = wl.y()[:, 0]
    got_y = P.matvec(_cuda(x)).cpu().numpy()
    got_x = P.rmatvec(_cuda(y)).cpu().numpy()
    ref_y = om.alg1(S, x)[:, 0]
    ref_x = om.alg2(S, y)[:, 0]
    assert_close(got_y, ref_y, TOL_FP32, terms=fwd_terms(S, x), what="Z x")
    assert_close(got_x, ref_x, TOL_FP32, terms=adj_terms(S, y), what="Z^* y")
    # per component as well
    nv = wl.grid.nv
    for k in range(3):
        assert_close(got_y[k * nv:(k + 1) * nv], ref_y[k * nv:(k + 1) * nv], TOL_FP32)
    # adjoint identity on the GPU results
    lhs = np.vdot(got_y.astype(np.complex128), y)
    rhs = np.vdot(x, got_x.astype(np.complex128))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_c1_unit_vector_and_determinism(gpu_lib, c1_struct):
    wl, S = c1_struct
    P = _plan(S)
    e = np.zeros(wl.m, complex)
    e[17] = 1.0
    got = P.matvec(_cuda(e)).cpu().numpy()
    assert_close(got, om.column(S, 17), TOL_FP32)
    x = _cuda(wl.x()[:, 0])
    a = P.matvec(x).cpu().numpy()
    b = P.matvec(x).cpu().numpy()
    assert np.array_equal(a, b)
    y = _cuda(wl.y()[:, 0])
    assert np.array_equal(P.rmatvec(y).cpu().numpy(), P.rmatvec(y).cpu().numpy())


def test_multiple_rhs_and_leading_dims(gpu_lib):
    import torch
    from paper_2103_06393_amd import lib
    S = random_struct((24, 18, 10), 3, 7, 6, 9)
    P = _plan(S)
    rng = np.random.default_rng(0)
    p = 3
    X = rng.standard_normal((S.m, p)) + 1j * rng.standard_normal((S.m, p))
    ref = om.alg1(S, X)
    ldx, ldy = S.m + 5, S.q * S.nv + 3
    xb = np.zeros((p, ldx), np.complex64)
    xb[:, :S.m] = X.T
    xd = _cuda(xb)
    yd = torch.full((p, ldy), 7.0 + 7.0j, dtype=torch.complex64, device="cuda")
    ws = P.workspace(0, p)
    lib.tv_matvec(P.handle, xd.data_ptr(), ldx, p, yd.data_ptr(), ldy,
                  ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
    got = yd.cpu().numpy()
    assert_close(got[:, :S.q * S.nv].T, ref, TOL_FP32)
    assert np.all(got[:, S.q * S.nv:] == np.complex64(7 + 7j))    # padding untouched
    Yr = rng.standard_normal((S.q * S.nv, p)) + 1j * rng.standard_normal((S.q * S.nv, p))
    refx = om.alg2(S, Yr)
    got2 = P.rmatvec(_cuda(Yr)).cpu().numpy()
    assert_close(got2, refx, TOL_FP32)


def test_c2_subset_of_columns(gpu_lib):
    """The 64^3 grid of the headline workload, 24 of its 256 columns."""
    wl = workloads.make("c2")
    S = om.compress_columns(wl, cols=range(0, 256, 11))
    P = _plan(S)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(S.m) + 1j * rng.standard_normal(S.m)
    y = wl.y()[:, 0]
    assert_close(P.matvec(_cuda(x)).cpu().numpy(), om.alg1(S, x)[:, 0], TOL_FP32,
                 terms=fwd_terms(S, x), what="Z x")
    assert_close(P.rmatvec(_cuda(y)).cpu().numpy(), om.alg2(S, y)[:, 0], TOL_FP32,
                 terms=adj_terms(S, y), what="Z^* y")


def test_dipole_columns_match_oracle(gpu_lib):
    import torch
    from paper_2103_06393_amd import lib
    from oracle import fields
    import dataclasses
    for name, op in (("c1", "N"), ("tiny_pwl", "N"), ("c1", "K"), ("tiny_pwl", "K")):
        wl = dataclasses.replace(workloads.make(name), operator=op)
        cols = [0, 5 % wl.m, wl.m - 1]
        out = torch.empty(len(cols) * wl.q * wl.grid.nv * 2, dtype=torch.float64,
                          device="cuda")
        lib.tv_dipole_columns(*wl.grid.dims, wl.grid.h, wl.k0,
                              lib.field_code(wl.basis, wl.operator), wl.pos[cols],
                              wl.ori[cols], out.data_ptr(),
                              torch.cuda.current_stream().cuda_stream)
        got = out.cpu().numpy().view(np.complex128).reshape(len(cols), -1)
        for i, j in enumerate(cols):
            ref = fields.column_vector(wl, j)
            assert_close(got[i], ref, 1e-12)
