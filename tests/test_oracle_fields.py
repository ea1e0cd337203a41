"""Pins for the oracle's closed-form columns (eq. 2 with eq. 3).

Each check is independent of the formula it tests: finite differences of the
scalar Green's function, the Helmholtz and divergence equations the field
must satisfy away from the source, its static and far-field limits, and a
brute-force quadrature of the PWL projection.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import fields

K0 = 2 * math.pi * workloads.FREQ_7T / workloads.C0
RNG = np.random.default_rng(7)
SRC = np.array([0.21, -0.05, 0.03])
P = np.array([0.3, -0.5, 0.81]) / np.linalg.norm([0.3, -0.5, 0.81])
PTS = RNG.uniform(-0.1, 0.1, size=(6, 3))


def _fd_hessian_g(x, src, k0, d):
    """Central-difference Hessian of g(|x - src|) (scalar eq. 3)."""
    H = np.zeros((3, 3), np.complex128)
    e = np.eye(3) * d
    g = lambda y: fields.scalar_green(np.linalg.norm(y - src), k0)  # noqa
    for a in range(3):
        for b in range(3):
            H[a, b] = (g(x + e[a] + e[b]) - g(x + e[a] - e[b])
                       - g(x - e[a] + e[b]) + g(x - e[a] - e[b])) / (4 * d * d)
    return H


def test_closed_form_matches_finite_difference_curl_curl():
    # curl curl (g p) = grad(div(g p)) - lap(g p) = H p + k0^2 g p
    for x in PTS:
        H = _fd_hessian_g(x, SRC, K0, 2e-4)
        g = fields.scalar_green(np.linalg.norm(x - SRC), K0)
        ref = H @ P + K0 * K0 * g * P
        got = fields.point_field(x, SRC, P, K0)
        assert np.linalg.norm(got - ref) <= 2e-5 * np.linalg.norm(ref)


def test_finite_difference_converges_second_order():
    x = PTS[0]
    errs = []
    ref = fields.point_field(x, SRC, P, K0)
    for d in (4e-3, 2e-3):
        H = _fd_hessian_g(x, SRC, K0, d)
        g = fields.scalar_green(np.linalg.norm(x - SRC), K0)
        errs.append(np.linalg.norm(H @ P + K0 * K0 * g * P - ref))
    assert 3.0 < errs[0] / errs[1] < 5.0       # O(d^2): ratio ~ 4


def _fd_field_derivs(x, d):
    E = lambda y: fields.point_field(y, SRC, P, K0)  # noqa
    e = np.eye(3) * d
    lap = sum((E(x + e[a]) - 2 * E(x) + E(x - e[a])) / (d * d)
              for a in range(3))
    div = sum((E(x + e[a])[a] - E(x - e[a])[a]) / (2 * d) for a in range(3))
    return lap, div


def test_helmholtz_and_divergence_free():
    # (lap + k0^2) E = 0 and div E = 0 away from the source; the residual
    # of the finite-difference check must vanish as O(d^2).
    for x in PTS:
        E = fields.point_field(x, SRC, P, K0)
        res = []
        for d in (5e-4, 2.5e-4):
            lap, div = _fd_field_derivs(x, d)
            R = np.linalg.norm(x - SRC)
            scale = np.linalg.norm(E) / R**2     # size of one 2nd derivative
            r = np.linalg.norm(lap + K0 * K0 * E)
            assert r <= 1e-3 * scale
            assert abs(div) <= 1e-3 * np.linalg.norm(E) / np.linalg.norm(x - SRC)
            res.append(r)
        assert 3.0 < res[0] / res[1] < 5.0


def test_static_limit_is_dipole_field():
    k0 = 1e-7
    for x in PTS:
        d = x - SRC
        R = np.linalg.norm(d)
        rh = d / R
        static = (3 * rh * (rh @ P) - P) / (4 * math.pi * R**3)
        got = fields.point_field(x, SRC, P, k0)
        assert np.linalg.norm(got - static) <= 1e-9 * np.linalg.norm(static)


def test_far_field_is_transverse_with_outgoing_phase():
    d = np.array([0.6, 0.8, 0.0])
    R1, R2 = 1e3, 1e3 + 0.25
    E1 = fields.point_field(SRC + d * R1, SRC, P, K0)
    E2 = fields.point_field(SRC + d * R2, SRC, P, K0)
    assert abs(d @ E1) <= 5e-3 * np.linalg.norm(E1)
    # far field: grad grad g -> -k0^2 d d g, so E -> k0^2 g (P - (d.P) d),
    # with the amplitude and phase of eq. (3)
    Pt = P - (d @ P) * d
    far = K0 * K0 * fields.scalar_green(R1, K0) * Pt
    assert np.linalg.norm(E1 - far) <= 5e-3 * np.linalg.norm(far)
    ratio = (E2 @ Pt) / (E1 @ Pt)
    assert abs(np.angle(ratio) - np.angle(np.exp(-1j * K0 * 0.25))) < 1e-3


def test_reciprocity():
    r1, r2 = np.array([0.02, 0.01, -0.03]), SRC
    p1 = np.array([1.0, 0.0, 0.0])
    a = p1 @ fields.point_field(r1, r2, P, K0)
    b = P @ fields.point_field(r2, r1, p1, K0)
    assert abs(a - b) <= 1e-13 * abs(a)


def test_green_function_value():
    R = 0.37
    g = fields.scalar_green(R, K0)
    assert abs(g - (math.cos(K0 * R) - 1j * math.sin(K0 * R))
               / (4 * math.pi * R)) < 1e-15


def test_pwc_tensor_layout_and_vectorisation():
    wl = workloads.make("tiny")
    T = fields.column_tensors(wl, 2)
    assert T.shape == (3, 8, 8, 8)
    # voxel (i1, i2, i3) holds the field at its centre, component k
    i1, i2, i3 = 1, 6, 3
    c = np.array([wl.grid.axis(0)[i1], wl.grid.axis(1)[i2],
                  wl.grid.axis(2)[i3]])
    E = fields.point_field(c, wl.pos[2], wl.ori[2], wl.k0)
    assert np.allclose(T[:, i1, i2, i3], E, rtol=1e-14, atol=0)
    col = fields.column_vector(wl, 2)
    nv = wl.grid.nv
    row = 1 * nv + i1 + 8 * (i2 + 8 * i3)
    assert col[row] == T[1, i1, i2, i3]


def test_pwl_projection_matches_brute_force_quadrature():
    wl = workloads.make("tiny_pwl")
    T = fields.column_tensors(wl, 1)
    h = wl.grid.h
    for (i1, i2, i3) in [(0, 0, 0), (7, 3, 5), (4, 4, 2)]:
        c = np.array([wl.grid.axis(0)[i1], wl.grid.axis(1)[i2],
                      wl.grid.axis(2)[i3]])
        # midpoint rule with 16^3 sub-cells
        s = (np.arange(16) + 0.5) / 16 - 0.5
        U = np.stack(np.meshgrid(s, s, s, indexing="ij"), -1).reshape(-1, 3)
        E = fields.point_field(c + U * h, wl.pos[1], wl.ori[1], wl.k0)
        phi = np.concatenate([np.ones((len(U), 1)), U], axis=1)
        ref = np.einsum("pc,pl->cl", E, phi) / len(U)      # (3, 4)
        got = T[:, i1, i2, i3].reshape(3, 4)
        assert np.allclose(got[:, 0], ref[:, 0], rtol=2e-3, atol=0)
        lin = np.abs(ref[:, 1:]).max()
        assert np.abs(got[:, 1:] - ref[:, 1:]).max() <= 2e-2 * lin


def test_pwl_linear_moments_follow_field_gradient():
    # (1/h^3) int E (x_l - c_l)/h = (h/12) dE/dx_l for a smooth field
    wl = workloads.make("tiny_pwl")
    T = fields.column_tensors(wl, 0)
    h = wl.grid.h
    i1, i2, i3 = 3, 4, 5
    c = np.array([wl.grid.axis(0)[i1], wl.grid.axis(1)[i2],
                  wl.grid.axis(2)[i3]])
    d = 1e-4
    for l in range(3):
        e = np.zeros(3)
        e[l] = d
        grad = (fields.point_field(c + e, wl.pos[0], wl.ori[0], wl.k0)
                - fields.point_field(c - e, wl.pos[0], wl.ori[0], wl.k0)) / (2 * d)
        got = np.array([T[4 * cc + 1 + l, i1, i2, i3] for cc in range(3)])
        assert np.linalg.norm(got - h / 12 * grad) <= 0.05 * np.linalg.norm(h / 12 * grad)


# ---- the K operator of eq. (5): H-field of a point current, curl(g p) ----

def _fd_grad_g(x, src, k0, d):
    e = np.eye(3) * d
    g = lambda y: fields.scalar_green(np.linalg.norm(y - src), k0)  # noqa
    return np.array([(g(x + e[a]) - g(x - e[a])) / (2 * d) for a in range(3)])


def test_hfield_matches_finite_difference_curl():
    """curl(g p) = grad g x p, with grad g by central differences of eq. (3)."""
    for x in PTS:
        ref = np.cross(_fd_grad_g(x, SRC, K0, 1e-4), P)
        got = fields.point_hfield(x, SRC, P, K0)
        assert np.linalg.norm(got - ref) <= 1e-6 * np.linalg.norm(ref)


def test_hfield_finite_difference_converges_second_order():
    x = PTS[1]
    ref = fields.point_hfield(x, SRC, P, K0)
    errs = [np.linalg.norm(np.cross(_fd_grad_g(x, SRC, K0, d), P) - ref)
            for d in (4e-3, 2e-3)]
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_hfield_orthogonal_and_divergence_free():
    for x in PTS:
        Hx = fields.point_hfield(x, SRC, P, K0)
        rhat = (x - SRC) / np.linalg.norm(x - SRC)
        assert abs(np.dot(Hx, rhat)) <= 1e-14 * np.linalg.norm(Hx)
        assert abs(np.dot(Hx, P)) <= 1e-14 * np.linalg.norm(Hx)
        d = 1e-4
        e = np.eye(3) * d
        div = sum((fields.point_hfield(x + e[a], SRC, P, K0)[a]
                   - fields.point_hfield(x - e[a], SRC, P, K0)[a]) / (2 * d)
                  for a in range(3))
        R = np.linalg.norm(x - SRC)
        assert abs(div) <= 1e-6 * np.linalg.norm(Hx) / R


def test_curl_of_hfield_is_efield():
    """N(p) = curl curl (g p) = curl K(p): eq. (2) is the curl of eq. (5)'s
    field, by central differences."""
    d = 1e-4
    e = np.eye(3) * d
    for x in PTS[:3]:
        J = np.zeros((3, 3), np.complex128)    # J[a, b] = d H_a / d x_b
        for b in range(3):
            J[:, b] = (fields.point_hfield(x + e[b], SRC, P, K0)
                       - fields.point_hfield(x - e[b], SRC, P, K0)) / (2 * d)
        curl = np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]])
        ref = fields.point_field(x, SRC, P, K0)
        assert np.linalg.norm(curl - ref) <= 1e-5 * np.linalg.norm(ref)


def test_hfield_static_limit_is_biot_savart():
    k0 = 1e-9
    for x in PTS:
        r = x - SRC
        R = np.linalg.norm(r)
        ref = -np.cross(r / R, P) / (4 * math.pi * R * R)
        got = fields.point_hfield(x, SRC, P, k0)
        assert np.linalg.norm(got - ref) <= 1e-8 * np.linalg.norm(ref)


@pytest.mark.parametrize("basis", ["pwc", "pwl"])
def test_hfield_rows_and_columns_agree(basis):
    import dataclasses
    wl = workloads.make("tiny" if basis == "pwc" else "tiny_pwl")
    wl = dataclasses.replace(wl, operator="K")
    for i in (0, 5, wl.rows // 2 + 3, wl.rows - 1):
        r = fields.row_vector(wl, i)
        c = np.array([fields.column_vector(wl, j)[i] for j in range(wl.m)])
        assert np.array_equal(r, c)
    # and the K columns differ from the N columns
    wn = dataclasses.replace(wl, operator="N")
    assert not np.allclose(fields.column_vector(wl, 0), fields.column_vector(wn, 0))
