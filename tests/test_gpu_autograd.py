"""The adjoint kernel as the backward of a torch.autograd.Function.

For L(x) = ||Z x - b||^2 the gradient in PyTorch's convention is
dL/dRe x + i dL/dIm x = 2 Z^* (Z x - b) (the GMT cost gradient needs products
with Z^*, Sec. II.A.2).  It is checked against the oracle's gradient on the
same factors and against central differences, which are exact for a quadratic
loss up to rounding.
"""
import numpy as np
import pytest

import workloads
from oracle import matvec as om
from tests.plans import assert_close, rel_err, struct_to_abi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1_plan():
    from paper_2103_06393_amd.ops import TuckerPlan
    wl = workloads.make("c1")
    S = om.compress_columns(wl)
    P = TuckerPlan.from_factors(S.dims, S.q, S.m, *struct_to_abi(S))
    return wl, S, P


def _loss_torch(P, x, b):
    import torch
    from paper_2103_06393_amd.ops import TuckerMatvec
    y = TuckerMatvec.apply(x, P)
    r = y - b
    return torch.sum((r.conj() * r).real)


def test_gradient_matches_oracle(gpu_lib, c1_plan):
    import torch
    wl, S, P = c1_plan
    x_np = wl.x()[:, 0]
    b_np = workloads.complex_normal(wl.rows, 52) * 1e-3
    x = torch.from_numpy(x_np.astype(np.complex64)).cuda().requires_grad_(True)
    b = torch.from_numpy(b_np.astype(np.complex64)).cuda()
    L = _loss_torch(P, x, b)
    L.backward()
    g = x.grad.cpu().numpy()
    ref = om.loss_grad(S, x_np, b_np)
    assert_close(g, ref, 1e-5)
    assert abs(L.item() - om.loss(S, x_np, b_np)) <= 1e-5 * om.loss(S, x_np, b_np)


def test_gradient_central_differences(gpu_lib, c1_plan):
    import torch
    wl, S, P = c1_plan
    x_np = wl.x()[:, 0]
    b_np = workloads.complex_normal(wl.rows, 52) * 1e-3
    x = torch.from_numpy(x_np.astype(np.complex64)).cuda().requires_grad_(True)
    b = torch.from_numpy(b_np.astype(np.complex64)).cuda()
    _loss_torch(P, x, b).backward()
    g = x.grad.cpu().numpy().astype(np.complex128)
    L0 = om.loss(S, x_np, b_np)
    for d_np in workloads.complex_normal((8, wl.m), 53):
        t = np.linalg.norm(x_np) / np.linalg.norm(d_np)
        with torch.no_grad():
            d = torch.from_numpy((t * d_np).astype(np.complex64)).cuda()
            lp = _loss_torch(P, x + d, b).item()
            lm = _loss_torch(P, x - d, b).item()
        fd = (lp - lm) / (2 * t)
        assert abs(fd - np.vdot(g, d_np).real) <= 1e-4 * L0 / t


def test_backward_is_the_adjoint_kernel(gpu_lib, c1_plan):
    import torch
    from paper_2103_06393_amd.ops import TuckerMatvec
    wl, S, P = c1_plan
    x = torch.from_numpy(wl.x()[:, 0].astype(np.complex64)).cuda().requires_grad_(True)
    gy = torch.from_numpy(wl.y()[:, 0].astype(np.complex64)).cuda()
    y = TuckerMatvec.apply(x, P)
    (gx,) = torch.autograd.grad(y, x, grad_outputs=gy)
    assert torch.equal(gx, P.rmatvec(gy))
