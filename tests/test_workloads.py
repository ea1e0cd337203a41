"""Checks of the seeded synthetic workloads and of the oracle on them."""
import math

import numpy as np

import workloads
from oracle import matvec


def test_ring_geometry():
    wl = workloads.make("c2")
    assert wl.m == 256 and wl.q == 3 and wl.grid.dims == (64, 64, 64)
    rad = np.hypot(wl.pos[:, 0], wl.pos[:, 1])
    assert np.allclose(rad, 1.2 * math.hypot(0.128, 0.128))
    assert set(np.round(wl.pos[:, 2], 12)) == {-0.064, 0.064}
    # tangential: orthogonal to the cylinder's radial direction
    radial = wl.pos[:, :2] / rad[:, None]
    assert np.allclose(np.sum(wl.ori[:, :2] * radial, axis=1), 0, atol=1e-12)
    assert np.allclose(np.linalg.norm(wl.ori, axis=1), 1)
    assert wl.min_distance() >= 2 * wl.grid.h


def test_named_sizes():
    assert workloads.make("c1").grid.nv == 32**3
    c3 = workloads.make("c3")
    assert c3.q == 12 and c3.m == 512 and c3.rows == 12 * 128**3
    c5 = workloads.make("c5")
    assert c5.m == 2048 and c5.grid.nv == 256**3
    for name in workloads.NAMES:
        assert workloads.make(name).min_distance() >= 2 * workloads.make(name).grid.h


def test_batch_geometry():
    plans = workloads.make_batch("c4")
    assert len(plans) == 16
    sizes = [p.m for p in plans]
    assert min(sizes) >= 64 and max(sizes) <= 1024
    for p in plans[:3]:
        g = p.grid
        ax, ay = g.half_extent(0), g.half_extent(1)
        gap = np.maximum(np.abs(p.pos[:, 0]) - ax, np.abs(p.pos[:, 1]) - ay)
        assert np.all(gap >= 0.5 * g.h * (1 - 1e-12))
        assert np.all(gap <= 128 * g.h * (1 + 1e-12))
        assert np.allclose(np.linalg.norm(p.ori, axis=1), 1)


def test_complex_normal_moments():
    z = workloads.complex_normal(200000, 9)
    assert abs(np.mean(np.abs(z) ** 2) - 1) < 0.02
    assert abs(np.mean(z.real ** 2) - 0.5) < 0.01
    assert abs(np.mean(z)) < 0.01


def test_c1_compression_error_and_ranks():
    wl = workloads.make("c1")
    S = matvec.compress_columns(wl, cols=range(0, 64, 16))
    R = S.ranks()
    assert R.min() >= 1 and R.max() <= 32
    for j, col in enumerate(S.t):
        for t in col:
            # relative error of every tensor within the tolerance
            assert np.sum(t.discarded) <= wl.tol ** 2 * t.norm2 * (1 + 1e-9)
