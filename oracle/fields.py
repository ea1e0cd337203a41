"""Coupling-matrix columns from unit point currents (oracle, FP64).

A coupling-matrix column j holds the field that coil element j produces in
every voxel (Sec. II.A.1).  The paper assembles it from 5-D MoM integrals over
RWG triangles; here the coil element is a unit point current p_j delta(r-r_j),
so the E-field operator N of eq. (2), with the free-space Green's function g of
eq. (3), reduces to a closed form.  Away from the source,

    N(p g) = curl curl (g p) = (grad grad + k0^2) g . p,

and with d/dR g = g (-i k0 - 1/R):

    (grad grad + k0^2) g = k0^2 g [ (1 - i/(k0 R) - 1/(k0 R)^2) I
                                  + (-1 + 3i/(k0 R) + 3/(k0 R)^2) Rhat Rhat ].

Piecewise-constant voxels (q = 3) sample it at the voxel centre, one point per
voxel as in Sec. IV.B.1.  Piecewise-linear voxels (q = 12) project it on
{1, (x-xc)/h, (y-yc)/h, (z-zc)/h} with a 2x2x2 Gauss-Legendre rule (eight
points per voxel, Sec. IV.B.1), normalised by the voxel volume; tensor index
k = 4 c + l for field component c and basis function l.

The physical E-field carries an extra constant 1/(i omega eps0); it scales
every column alike and is left out.

The magnetic coupling matrix Z_bc uses the K operator of eq. (5) instead,
K(s) = curl of the g-weighted integral of s; for a point current that is
curl(g p) = grad g x p = g (-i k0 - 1/R) Rhat x p (``point_hfield``).
A workload selects it with ``operator = "K"``; the voxel bases are the same.
"""
from __future__ import annotations

import math

import numpy as np


def scalar_green(R, k0: float):
    """Free-space Green's function g(R) = exp(-i k0 R) / (4 pi R), eq. (3)."""
    R = np.asarray(R, dtype=np.float64)
    return np.exp(-1j * k0 * R) / (4.0 * math.pi * R)


def point_field(points, src, p, k0: float):
    """N(p delta(r - src)) at ``points`` (..., 3) -> (..., 3) complex128.

    The dyadic form above, eq. (2) applied to a point current.
    """
    d = np.asarray(points, dtype=np.float64) - np.asarray(src, np.float64)
    R = np.sqrt(np.sum(d * d, axis=-1))
    rhat = d / R[..., None]
    kr = k0 * R
    g = np.asarray(scalar_green(R, k0))
    a = np.asarray(1.0 - 1j / kr - 1.0 / kr**2)     # coefficient of I
    b = np.asarray(-1.0 + 3j / kr + 3.0 / kr**2)    # coefficient of Rhat Rhat
    rp = np.sum(rhat * np.asarray(p, np.float64), axis=-1)
    return (k0 * k0 * g)[..., None] * (a[..., None] * np.asarray(p)
                                       + (b * rp)[..., None] * rhat)


def point_hfield(points, src, p, k0: float):
    """K(p delta(r - src)) = grad g x p at ``points`` (..., 3), eq. (5)."""
    d = np.asarray(points, dtype=np.float64) - np.asarray(src, np.float64)
    R = np.sqrt(np.sum(d * d, axis=-1))
    rhat = d / R[..., None]
    g = np.asarray(scalar_green(R, k0))
    dg = g * (-1j * k0 - 1.0 / R)                      # d g / d R
    return dg[..., None] * np.cross(rhat, np.asarray(p, np.float64))


def _field(wl):
    return point_hfield if getattr(wl, "operator", "N") == "K" else point_field


def voxel_centres(grid):
    """(n1, n2, n3, 3) array of voxel centres (domain centred at 0)."""
    x, y, z = (grid.axis(d) for d in range(3))
    X, Y, Z = np.meshgrid(x, y, z, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


_GL2 = 1.0 / (2.0 * math.sqrt(3.0))     # 2-point Gauss-Legendre node, in h


def column_tensors(wl, j: int) -> np.ndarray:
    """The q tensors Z^{kj} of column j, shape (q, n1, n2, n3) complex128.

    Sec. III.A: a column is q stacked vectors, each reshaped to an
    n1 x n2 x n3 tensor over the voxel grid.
    """
    centres = voxel_centres(wl.grid)
    src, p, k0 = wl.pos[j], wl.ori[j], wl.k0
    field = _field(wl)
    if wl.basis == "pwc":
        E = field(centres, src, p, k0)                  # (n1,n2,n3,3)
        return np.moveaxis(E, -1, 0).copy()
    h = wl.grid.h
    out = np.zeros((12,) + wl.grid.dims, dtype=np.complex128)
    for sx in (-1.0, 1.0):
        for sy in (-1.0, 1.0):
            for sz in (-1.0, 1.0):
                s = np.array([sx, sy, sz]) * _GL2
                E = field(centres + s * h, src, p, k0)
                phi = (1.0, s[0], s[1], s[2])           # basis values
                for c in range(3):
                    for l in range(4):
                        out[4 * c + l] += E[..., c] * (phi[l] / 8.0)
    return out


def column_vector(wl, j: int) -> np.ndarray:
    """Column j of the coupling matrix, length q * nv.

    Row order is [Y^1; ...; Y^q] (Algorithm 1's last step) with each block
    the column-major vectorisation (:) of its tensor.
    """
    T = column_tensors(wl, j)
    return np.concatenate([T[k].reshape(-1, order="F") for k in range(wl.q)])


def row_vector(wl, i: int) -> np.ndarray:
    """Row i of the coupling matrix (length m): the field of every coil
    element at one voxel and component.

    Row i is component k of voxel v = i1 + n1 (i2 + n2 i3), k nv + v = i
    (Algorithm 1's row order).  Evaluated dipole by dipole, independently of
    the voxel-vectorised ``column_tensors``.
    """
    nv = wl.grid.nv
    k, v = divmod(int(i), nv)
    n1, n2 = wl.grid.n1, wl.grid.n2
    idx = (v % n1, (v // n1) % n2, v // (n1 * n2))
    centre = np.array([wl.grid.axis(d)[idx[d]] for d in range(3)])
    field = _field(wl)
    if wl.basis == "pwc":
        return field(centre, wl.pos, wl.ori, wl.k0)[:, k]
    c, l = divmod(k, 4)
    h = wl.grid.h
    out = np.zeros(wl.m, dtype=np.complex128)
    for sx in (-1.0, 1.0):
        for sy in (-1.0, 1.0):
            for sz in (-1.0, 1.0):
                s = np.array([sx, sy, sz]) * _GL2
                E = field(centre + s * h, wl.pos, wl.ori, wl.k0)
                phi = (1.0, s[0], s[1], s[2])[l]
                out += E[:, c] * (phi / 8.0)
    return out
