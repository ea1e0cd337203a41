"""Differentiation at scale: 256^3 grid, 3 components, 2048 point currents on
16 rings, columns compressed on the GPU at tolerance 1e-4 (ranks capped at
32), complex64.

L(x) = ||Z x - b||^2 with b complex normal; its gradient is taken by the
adjoint kernel as the backward of TuckerMatvec.  Checked against central
differences on 8 random directions (exact for a quadratic up to rounding)
and against the oracle's 2 Z^* (Z x - b) on the plan's own factors at the
columns on both sides of every split of the adjoint's column ranges; the
forward product is checked on whole mode-1 fibres on the edges of the first
and last column tiles, every component, entry by entry (the full oracle
product would take hours on a CPU).
"""
import numpy as np
import pytest

import workloads
from oracle import matvec as om
from tests.plans import (abi_to_struct, abs_struct, assert_close, boundary_fibres,
                         fibre_check, split_boundary_columns)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c5():
    from paper_2103_06393_amd.ops import TuckerPlan
    wl = workloads.make("c5")
    P = TuckerPlan.compress_dipoles(wl.grid.dims, wl.grid.h, wl.k0, 0, wl.pos,
                                    wl.ori, wl.tol, 1, wl.rank_cap)
    return wl, P


def _loss(P, x, b):
    import torch
    from paper_2103_06393_amd.ops import TuckerMatvec
    r = TuckerMatvec.apply(x, P) - b
    return torch.sum((r.conj() * r).real.double())


def test_c5_gradient(gpu_lib, c5):
    import torch
    wl, P = c5
    x_np = wl.x()[:, 0]
    b_np = workloads.complex_normal(wl.rows, 52) * 1e-3
    x = torch.from_numpy(x_np.astype(np.complex64)).cuda().requires_grad_(True)
    b = torch.from_numpy(b_np.astype(np.complex64)).cuda()
    L = _loss(P, x, b)
    L.backward()
    g = x.grad.cpu().numpy().astype(np.complex128)
    L0 = L.item()
    # central differences on 8 random directions
    for d_np in workloads.complex_normal((8, wl.m), 53):
        t = np.linalg.norm(x_np) / np.linalg.norm(d_np)
        with torch.no_grad():
            d = torch.from_numpy((t * d_np).astype(np.complex64)).cuda()
            fd = (_loss(P, x + d, b).item() - _loss(P, x - d, b).item()) / (2 * t)
        assert abs(fd - np.vdot(g, d_np).real) <= 1e-4 * L0 / t
    # oracle gradient on sampled columns, with the GPU residual
    with torch.no_grad():
        from paper_2103_06393_amd.ops import TuckerMatvec
        r = (TuckerMatvec.apply(x, P) - b).cpu().numpy().astype(np.complex128)
    ranks, G, U1, U2, U3 = P.export_factors()
    S = abi_to_struct(wl.grid.dims, wl.q, ranks, G, U1, U2, U3)
    info = P.info
    cols = sorted(set(split_boundary_columns(ranks, wl.q, wl.m, info.splits[1]))
                  | {777})
    ref = 2.0 * om.adjoint_entries(S, r, cols)
    terms = 2.0 * np.abs(om.adjoint_entries(abs_struct(S), np.abs(r), cols))
    assert_close(g[cols], ref, 1e-5, terms=terms, what="gradient columns")
    # whole mode-1 fibres on the edges of the first and last column tiles of
    # the forward's tiling, every component
    y = P.matvec(x.detach()).cpu().numpy()
    for i2, i3 in boundary_fibres(wl.grid.dims, info.tile_t2[0], info.tile_t3[0]):
        for k in range(wl.q):
            fibre_check(S, y, x_np, k, i2, i3, 1e-5, what="c5 Z x")
