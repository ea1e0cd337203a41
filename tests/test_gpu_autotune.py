"""The project-written autotuner: any configuration it picks gives the same
products (to FP32 rounding), and its JSON cache is reused."""
import json

import numpy as np
import pytest

from oracle import matvec as om
from tests.plans import random_struct, rel_err, struct_to_abi

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
    assert rel_err(P.matvec(cx(x)).cpu().numpy(), om.alg1(S, x)[:, 0]) <= 1e-5
    assert rel_err(P.rmatvec(cx(y)).cpu().numpy(), om.alg2(S, y)[:, 0]) <= 1e-5
    entries = json.loads(cache.read_text())
    assert len(entries) == 2
    Q = TuckerPlan.from_factors(S.dims, S.q, S.m, *abi)
    Q.autotune(2, str(cache))                       # applied from the cache
    from paper_2103_06393_amd import lib
    for op in (0, 1):
        assert lib.tv_workspace_bytes(P.handle, op, 1) == lib.tv_workspace_bytes(Q.handle, op, 1)
    assert np.array_equal(P.matvec(cx(x)).cpu().numpy(), Q.matvec(cx(x)).cpu().numpy())
