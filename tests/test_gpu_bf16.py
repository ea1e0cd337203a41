"""BF16X3 plans: every FP32 operand split into bf16 hi + lo, products formed
as hi*hi + hi*lo + lo*hi on BF16 MFMA with FP32 accumulation.

The bar against the FP64 oracle on the same factors is a relative error of
1e-3; the split keeps about 16 significant bits per operand, so the measured
error is far below that and is reported next to the FP32 plan's.
"""
import numpy as np
import pytest

import workloads
from oracle import matvec as om
from tests.plans import assert_close, abi_to_struct, random_struct, rel_err, struct_to_abi

pytestmark = pytest.mark.gpu
TOL_BF16 = 1e-3


def _plans(S):
    from paper_2103_06393_amd import lib
    from paper_2103_06393_amd.ops import TuckerPlan
    a = struct_to_abi(S)
    return (TuckerPlan.from_factors(S.dims, S.q, S.m, *a, lib.TV_PREC_FP32),
            TuckerPlan.from_factors(S.dims, S.q, S.m, *a, lib.TV_PREC_BF16X3))


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.complex64)).cuda()


@pytest.mark.parametrize("dims,q,m,rmax,seed", [
    ((20, 13, 7), 2, 5, 5, 11),
    ((32, 32, 32), 3, 9, 12, 12),
    ((48, 40, 33), 12, 3, 20, 13),
    ((96, 16, 8), 2, 3, 30, 14),
    ((160, 8, 6), 1, 2, 10, 15),
])
def test_random_structs_bf16(gpu_lib, dims, q, m, rmax, seed):
    S = random_struct(dims, q, m, rmax, seed)
    P32, P16 = _plans(S)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    y = rng.standard_normal(S.q * S.nv) + 1j * rng.standard_normal(S.q * S.nv)
    ry, rx = om.alg1(S, x)[:, 0], om.alg2(S, y)[:, 0]
    e16 = (rel_err(P16.matvec(_cuda(x)).cpu().numpy(), ry),
           rel_err(P16.rmatvec(_cuda(y)).cpu().numpy(), rx))
    e32 = (rel_err(P32.matvec(_cuda(x)).cpu().numpy(), ry),
           rel_err(P32.rmatvec(_cuda(y)).cpu().numpy(), rx))
    print(f"rel err bf16x3 {e16}, fp32 {e32}")
    assert max(e16) <= TOL_BF16
    assert max(e16) <= 1e-4          # the 3-term split keeps ~16 bits
    assert max(e32) <= 1e-5


@pytest.fixture(scope="module")
def c3s_struct():
    wl = workloads.make("c3s")          # 48^3 PWL (q = 12), 64 columns
    return wl, om.compress_columns(wl)


def test_pwl_workload_bf16_and_fp32(gpu_lib, c3s_struct):
    wl, S = c3s_struct
    P32, P16 = _plans(S)
    x, y = wl.x()[:, 0], wl.y()[:, 0]
    ry, rx = om.alg1(S, x)[:, 0], om.alg2(S, y)[:, 0]
    e16 = (rel_err(P16.matvec(_cuda(x)).cpu().numpy(), ry),
           rel_err(P16.rmatvec(_cuda(y)).cpu().numpy(), rx))
    e32 = (rel_err(P32.matvec(_cuda(x)).cpu().numpy(), ry),
           rel_err(P32.rmatvec(_cuda(y)).cpu().numpy(), rx))
    print(f"PWL 48^3: rel err bf16x3 {e16}, fp32 {e32}")
    assert max(e16) <= TOL_BF16 and max(e32) <= 1e-5


def test_device_compression_bf16_plan(gpu_lib):
    from paper_2103_06393_amd import lib
    from paper_2103_06393_amd.ops import TuckerPlan
    wl = workloads.make("c3s")
    P = TuckerPlan.compress_dipoles(wl.grid.dims, wl.grid.h, wl.k0, 1, wl.pos,
                                    wl.ori, wl.tol, 1, wl.rank_cap,
                                    precision=lib.TV_PREC_BF16X3)
    S = abi_to_struct(wl.grid.dims, wl.q, *P.export_factors())
    x, y = wl.x()[:, 0], wl.y()[:, 0]
    assert_close(P.matvec(_cuda(x)).cpu().numpy(), om.alg1(S, x)[:, 0], TOL_BF16)
    assert_close(P.rmatvec(_cuda(y)).cpu().numpy(), om.alg2(S, y)[:, 0], TOL_BF16)
