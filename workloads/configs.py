"""Workload definitions for the Tucker-compressed coupling-matrix matvec.

The paper's experiments use a realistic head/body model and RWG coil meshes
(Sec. IV.B) that are not available here.  These seeded stand-ins keep the
paper's regime instead: a head-size voxel box (Sec. IV.B.1 uses 5/2/1 mm
voxels), 298 MHz (7 T, Sec. IV.B.1), coils made of unit point currents placed
outside the voxel domain.  Each coil element j gives one column of the
coupling matrix; its field is evaluated elsewhere (the oracle, the library).

Conventions shared by every consumer:

* voxel (i1, i2, i3) has centre ((i1 - (n1-1)/2) h, (i2 - (n2-1)/2) h,
  (i3 - (n3-1)/2) h): the domain is centred at the origin, as in Sec. IV.A;
* ``pos[j]`` is the position (metres) and ``ori[j]`` the unit orientation of
  the point current of column j;
* ``q`` is 3 for piecewise-constant and 12 for piecewise-linear voxel bases
  (Sec. II.A.1);
* random complex vectors are circular complex normal CN(0, 1): real and
  imaginary parts independent N(0, 1/2).

Named workloads (small -> large): ``c1`` 32^3 / 64 dipoles, ``c2`` 64^3 /
256 dipoles, ``c3`` 128^3 PWL / 512 dipoles, ``c4`` sixteen coil
configurations on a 96x128x112 grid, ``c5`` 256^3 / 2048 dipoles.
Reduced variants (``tiny``, ``c2s``...) exist for fast tests.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

C0 = 299_792_458.0          # speed of light in vacuum, m/s
FREQ_7T = 298.0e6           # Sec. IV.B.1 operating frequency, Hz


@dataclasses.dataclass(frozen=True)
class Grid:
    """Uniform voxel grid centred at the origin (h = voxel edge, metres)."""
    n1: int
    n2: int
    n3: int
    h: float

    @property
    def dims(self):
        return (self.n1, self.n2, self.n3)

    @property
    def nv(self) -> int:
        return self.n1 * self.n2 * self.n3

    def axis(self, d: int) -> np.ndarray:
        """Voxel-centre coordinates along axis d (0, 1, 2)."""
        n = self.dims[d]
        return (np.arange(n, dtype=np.float64) - (n - 1) / 2.0) * self.h

    def half_extent(self, d: int) -> float:
        """Distance from the origin to the domain face along axis d."""
        return self.dims[d] * self.h / 2.0


@dataclasses.dataclass
class Workload:
    name: str
    grid: Grid
    basis: str                  # 'pwc' (q = 3) or 'pwl' (q = 12)
    freq: float
    pos: np.ndarray             # (m, 3) float64
    ori: np.ndarray             # (m, 3) float64, unit rows
    tol: float                  # HOSVD tolerance per tensor
    rank_min: int = 1
    rank_cap: Optional[int] = None
    nrhs: int = 1
    seed_x: int = 0
    seed_y: int = 0
    operator: str = "N"         # 'N' (E-field, eq. 2) or 'K' (H-field, eq. 5)

    @property
    def q(self) -> int:
        return 3 if self.basis == "pwc" else 12

    @property
    def m(self) -> int:
        return int(self.pos.shape[0])

    @property
    def k0(self) -> float:
        return 2.0 * math.pi * self.freq / C0

    @property
    def rows(self) -> int:
        return self.q * self.grid.nv

    def x(self, nrhs: Optional[int] = None) -> np.ndarray:
        """Coil currents X (m x nrhs), CN(0,1), seed ``seed_x``."""
        p = self.nrhs if nrhs is None else nrhs
        return complex_normal((self.m, p), self.seed_x)

    def y(self, nrhs: Optional[int] = None) -> np.ndarray:
        """Voxel field Y (q*nv x nrhs), CN(0,1), seed ``seed_y``."""
        p = self.nrhs if nrhs is None else nrhs
        return complex_normal((self.rows, p), self.seed_y)

    def min_distance(self) -> float:
        """Smallest distance from any dipole to the box of voxel centres."""
        lo = np.array([self.grid.axis(d)[0] for d in range(3)])
        hi = np.array([self.grid.axis(d)[-1] for d in range(3)])
        nearest = np.clip(self.pos, lo, hi)
        return float(np.min(np.linalg.norm(self.pos - nearest, axis=1)))


def complex_normal(shape, seed: int) -> np.ndarray:
    """CN(0, 1) samples: real and imaginary parts i.i.d. N(0, 1/2)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * math.sqrt(0.5)


def _rings(n_rings: int, per_ring: int, radius: float, z_values, seed: int):
    """Dipoles on horizontal circles, tangent to the cylinder they lie on.

    Orientation p = cos(a) phi_hat + sin(a) z_hat with a ~ U[0, 2 pi).
    """
    rng = np.random.default_rng(seed)
    pos, ori = [], []
    for r in range(n_rings):
        z = z_values[r]
        for i in range(per_ring):
            phi = 2.0 * math.pi * i / per_ring
            pos.append((radius * math.cos(phi), radius * math.sin(phi), z))
            a = rng.uniform(0.0, 2.0 * math.pi)
            phat = np.array([-math.sin(phi), math.cos(phi), 0.0])
            zhat = np.array([0.0, 0.0, 1.0])
            ori.append(math.cos(a) * phat + math.sin(a) * zhat)
    pos = np.asarray(pos, dtype=np.float64)
    ori = np.asarray(ori, dtype=np.float64)
    ori /= np.linalg.norm(ori, axis=1, keepdims=True)
    return pos, ori


def _ring_radius(grid: Grid) -> float:
    """1.2 x the circumscribed half-width of the grid's (x, y) cross-section."""
    return 1.2 * math.hypot(grid.half_extent(0), grid.half_extent(1))


def _ring_workload(name, n, h, n_rings, per_ring, z_mode, basis, tol, cap,
                   seed_geo, seed_x, seed_y, rank_min=1) -> Workload:
    grid = Grid(n, n, n, h)
    a = grid.half_extent(2)
    if z_mode == "zero":
        zs = [0.0]
    elif z_mode == "pm_half":
        zs = [-a / 2.0, a / 2.0]
    else:                                   # equispaced in [-a, a]
        zs = list(np.linspace(-a, a, n_rings))
    pos, ori = _rings(n_rings, per_ring, _ring_radius(grid), zs, seed_geo)
    return Workload(name, grid, basis, FREQ_7T, pos, ori, tol, rank_min, cap,
                    1, seed_x, seed_y)


def _face_workload(name, grid: Grid, m: int, seed_geo: int, seed_x: int,
                   seed_y: int, tol=1e-6, rank_min=4, cap=32,
                   nrhs=32) -> Workload:
    """Dipoles on the four side faces (+-x, +-y) of the voxel domain.

    Each dipole sits at distance h * 2**U(-1, 7) outside a uniformly chosen
    face, at a uniform position over the face, oriented tangentially to it.
    """
    rng = np.random.default_rng(seed_geo)
    ax, ay, az = (grid.half_extent(d) for d in range(3))
    pos = np.zeros((m, 3))
    ori = np.zeros((m, 3))
    for j in range(m):
        face = int(rng.integers(0, 4))
        dist = grid.h * 2.0 ** rng.uniform(-1.0, 7.0)
        u = rng.uniform(-1.0, 1.0)
        w = rng.uniform(-az, az)
        beta = rng.uniform(0.0, 2.0 * math.pi)
        if face < 2:                        # +x / -x face, spans (y, z)
            s = 1.0 if face == 0 else -1.0
            pos[j] = (s * (ax + dist), u * ay, w)
            ori[j] = (0.0, math.cos(beta), math.sin(beta))
        else:                               # +y / -y face, spans (x, z)
            s = 1.0 if face == 2 else -1.0
            pos[j] = (u * ax, s * (ay + dist), w)
            ori[j] = (math.cos(beta), 0.0, math.sin(beta))
    return Workload(name, grid, "pwc", FREQ_7T, pos, ori, tol, rank_min, cap,
                    nrhs, seed_x, seed_y)


FREQ_3T = 123.0e6           # Sec. IV.B.2 operating frequency, Hz


def _bodycoil(name, dims, h, m, basis, tol, seed_geo, seed_x, seed_y,
              rank_min=1, cap=None) -> Workload:
    """Body-coil stand-in for Sec. IV.B.2 with point currents in place of
    the RWG functions, magnetic coupling matrix Z_bc (K operator, eq. 5): 32 legs (radius 35.5 cm, length 45 cm, z-directed),
    two end rings (phi-directed) and a conductive shield (radius 37.2 cm,
    length 1.5 m, tangential currents at seeded random positions and
    angles), all centred at the origin around the voxel box.  A quarter of
    the m elements lie on the coil (legs 3/4, rings 1/4), the rest on the
    shield.
    """
    rng = np.random.default_rng(seed_geo)
    rc, lc, rs, ls = 0.355, 0.45, 0.372, 1.5
    n_coil = m // 4
    per_leg = max(1, (3 * n_coil) // (4 * 32))
    n_ring = max(1, (n_coil - 32 * per_leg) // 2)
    pos, ori = [], []
    for leg in range(32):
        phi = 2.0 * math.pi * leg / 32
        for t in range(per_leg):
            z = -lc / 2 + lc * (t + 0.5) / per_leg
            pos.append((rc * math.cos(phi), rc * math.sin(phi), z))
            ori.append((0.0, 0.0, 1.0))
    for z in (-lc / 2, lc / 2):
        for t in range(n_ring):
            phi = 2.0 * math.pi * (t + 0.5) / n_ring
            pos.append((rc * math.cos(phi), rc * math.sin(phi), z))
            ori.append((-math.sin(phi), math.cos(phi), 0.0))
    for _ in range(m - len(pos)):
        phi = rng.uniform(0.0, 2.0 * math.pi)
        z = rng.uniform(-ls / 2, ls / 2)
        a = rng.uniform(0.0, 2.0 * math.pi)
        pos.append((rs * math.cos(phi), rs * math.sin(phi), z))
        ori.append((-math.cos(a) * math.sin(phi), math.cos(a) * math.cos(phi),
                    math.sin(a)))
    grid = Grid(dims[0], dims[1], dims[2], h)
    return Workload(name, grid, basis, FREQ_3T, np.asarray(pos, np.float64),
                    np.asarray(ori, np.float64), tol, rank_min, cap, 1,
                    seed_x, seed_y, operator="K")


# Body-coil workloads: the box of Sec. IV.B.2 (81 x 44 x 108 voxels at 5 mm,
# 205 x 109 x 270 at 2 mm, 409 x 219 x 541 at 1 mm), 9450 coil elements and
# the ACA ranks reported there (250 at 5 mm, 287 at 2 and 1 mm); ``aca_s``
# keeps the geometry at 2.5 cm voxels and 400 elements for the oracle.  The
# tolerance is the ACA tolerance of Sec. IV.B.2 (1e-3).
BODYCOIL = {
    "aca_s": ((16, 9, 22), 0.025, 400, None),
    "aca5": ((81, 44, 108), 0.005, 9450, 250),
    "aca2": ((205, 109, 270), 0.002, 9450, 287),
    "aca1": ((409, 219, 541), 0.001, 9450, 287),
}


def make_bodycoil(name: str, basis: str = "pwc") -> Workload:
    dims, h, m, _ = BODYCOIL[name]
    return _bodycoil(name, dims, h, m, basis, 1e-3, 6, 61, 62)


def aca_rank(name: str) -> int:
    """ACA rank of the body-coil coupling matrix reported in Sec. IV.B.2."""
    return BODYCOIL[name][3]


def make(name: str) -> Workload:
    """Build a named single-plan workload."""
    if name == "tiny":          # oracle-only unit tests: 8^3, 6 dipoles
        return _ring_workload("tiny", 8, 0.02, 1, 6, "zero", "pwc", 1e-6,
                              None, 1, 11, 12)
    if name == "tiny_pwl":
        return _ring_workload("tiny_pwl", 8, 0.02, 1, 4, "zero", "pwl", 1e-6,
                              None, 3, 31, 32)
    if name == "c1":            # 32^3, 5 mm, one ring of 64 at z = 0
        return _ring_workload("c1", 32, 0.005, 1, 64, "zero", "pwc", 1e-6,
                              None, 1, 11, 12)
    if name == "c2":            # 64^3, 4 mm, two rings of 128 at z = +-a/2
        return _ring_workload("c2", 64, 0.004, 2, 128, "pm_half", "pwc",
                              1e-4, 24, 2, 21, 22)
    if name == "c3":            # 128^3, 2 mm, PWL, 8 rings of 64
        return _ring_workload("c3", 128, 0.002, 8, 64, "spread", "pwl",
                              1e-4, 32, 3, 31, 32)
    if name == "c3s":           # reduced PWL case for parity tests: 48^3
        return _ring_workload("c3s", 48, 0.005, 4, 16, "spread", "pwl",
                              1e-4, 32, 3, 31, 32)
    if name == "c5":            # 256^3, 1 mm, 16 rings of 128
        return _ring_workload("c5", 256, 0.001, 16, 128, "spread", "pwc",
                              1e-4, 32, 5, 51, 52)
    raise KeyError(name)


def make_batch(name: str = "c4") -> List[Workload]:
    """The multi-configuration workload: 16 coils on a 96x128x112, 2 mm grid.

    Coil c has N_c ~ U{64..1024} dipoles (geometry seed 100 + c), currents
    X_c with seed 200 + c and fields with seed 300 + c, 32 right-hand sides.
    Tolerance 1e-6 with ranks clamped to [4, 32]: the paper's 1e-8 lies below
    what complex64 products and FP64 Gram matrices resolve.
    ``c4s`` is a reduced variant (4 coils, 24x32x28 grid, N_c in 8..40).
    """
    if name == "c4":
        grid = Grid(96, 128, 112, 0.002)
        rng = np.random.default_rng(100)
        sizes = rng.integers(64, 1025, size=16)
        return [_face_workload(f"c4.{c}", grid, int(sizes[c]), 100 + c,
                               200 + c, 300 + c) for c in range(16)]
    if name == "c4s":
        grid = Grid(24, 32, 28, 0.008)
        rng = np.random.default_rng(100)
        sizes = rng.integers(8, 41, size=4)
        return [_face_workload(f"c4s.{c}", grid, int(sizes[c]), 100 + c,
                               200 + c, 300 + c, nrhs=8) for c in range(4)]
    raise KeyError(name)


NAMES = ("tiny", "tiny_pwl", "c1", "c2", "c3", "c3s", "c5")
