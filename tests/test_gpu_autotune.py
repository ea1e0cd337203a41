"""The project-written autotuner: any configuration it picks gives the same
products (to FP32 rounding), and its JSON cache is reused."""
import json

import numpy as np
import pytest

from oracle import matvec as om
from tests.plans import assert_close, random_struct, rel_err, struct_to_abi

pytestmark = pytest.mark.gpu


def test_autotune_keeps_results_and_caches(gpu_lib, tmp_path):
    import torch
    from paper_2103_06393_amd.ops import TuckerPlan
    S = random_struct((48, 40, 33), 3, 24, 10, 21)
    abi = struct_to_abi(S)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(S.m) + 1j * rng.standard_normal(S.m)
    y = rng.standard_normal(S.q * S.nv) + 1j * rng.standard_normal(S.q * S.nv)
    cx = lambda a: torch.from_numpy(a.astype(np.complex64)).cuda()  # noqa: E731
    cache = tmp_path / "tune.json"
    P = TuckerPlan.from_factors(S.dims, S.q, S.m, *abi)
    P.autotune(2, str(cache))
    assert_close(P.matvec(cx(x)).cpu().numpy(), om.alg1(S, x)[:, 0], 1e-5)
    assert_close(P.rmatvec(cx(y)).cpu().numpy(), om.alg2(S, y)[:, 0], 1e-5)
    entries = json.loads(cache.read_text())
    assert len(entries) == 2
    Q = TuckerPlan.from_factors(S.dims, S.q, S.m, *abi)
    Q.autotune(2, str(cache))                       # applied from the cache
    from paper_2103_06393_amd import lib
    for op in (0, 1):
        assert lib.tv_workspace_bytes(P.handle, op, 1) == lib.tv_workspace_bytes(Q.handle, op, 1)
    assert np.array_equal(P.matvec(cx(x)).cpu().numpy(), Q.matvec(cx(x)).cpu().numpy())
    # cached choices are [path, t2, split, row-block cap, slab, GEMM tile,
    # GEMM order]; the fused adjoint has a row-block cap of 2 or 3, the fused
    # forward 8
    for key, val in entries.items():
        assert len(val) == 7
        assert val[0] in (0, 1)
        if val[0] == 0:
            assert val[3] in ((2, 3) if key.endswith("op1") else (8,))


@pytest.mark.parametrize("cap,t2", [(2, 32), (3, 32), (3, 2), (2, 2)])
def test_adjoint_row_block_caps(gpu_lib, tmp_path, cap, t2):
    """Every adjoint tiling the autotuner may choose, forced through its
    cache: 81 voxel rows pad to 128 with 2 row blocks per wave and to 96
    with 3; t2 = 32 runs the warp-specialised kernel, t2 = 2 the phased one."""
    import torch
    from paper_2103_06393_amd.ops import TuckerPlan
    S = random_struct((81, 12, 10), 3, 9, 12, 41)
    abi = struct_to_abi(S)
    cache = tmp_path / "tune.json"
    P = TuckerPlan.from_factors(S.dims, S.q, S.m, *abi)
    P.autotune(1, str(cache))
    entries = json.loads(cache.read_text())
    (key,) = [k for k in entries if k.endswith("op1")]
    cache.write_text(json.dumps({key: [0, t2, 2, cap, 0, 0, 0]}))
    Q = TuckerPlan.from_factors(S.dims, S.q, S.m, *abi)
    Q.autotune(1, str(cache))
    info = Q.info
    assert info.tile_t2[1] == t2 and info.splits[1] == 2
    y = workloads_cn(S.q * S.nv, 42)
    got = Q.rmatvec(torch.from_numpy(y.astype(np.complex64)).cuda()).cpu().numpy()
    assert_close(got, om.alg2(S, y.astype(np.complex64).astype(np.complex128))[:, 0], 1e-5)


def workloads_cn(n, seed):
    import workloads
    return workloads.complex_normal(n, seed)
