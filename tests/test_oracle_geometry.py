"""Pins of the oracle's contact primitives, tangent basis and orientation update.

Each primitive is checked against something other than its own formula:
a dense brute-force sample of the box surface, point-in-shape signs, the
Rodrigues rotation matrix, and orthonormality identities.
"""
import math

import numpy as np
import pytest

import oracle


def quat_to_R(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def rodrigues(axis_angle):
    th = np.linalg.norm(axis_angle)
    if th == 0:
        return np.eye(3)
    k = axis_angle / th
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K


def box_surface_samples(c, half, R, n=60):
    """Dense grid on the six faces of a box (world coordinates)."""
    pts = []
    u = np.linspace(-1, 1, n)
    U, V = np.meshgrid(u, u)
    for ax in range(3):
        a1, a2 = [i for i in range(3) if i != ax]
        for sgn in (-1, 1):
            P = np.zeros((n * n, 3))
            P[:, ax] = sgn * half[ax]
            P[:, a1] = U.ravel() * half[a1]
            P[:, a2] = V.ravel() * half[a2]
            pts.append(P)
    P = np.concatenate(pts)
    return P @ R.T + c


def test_sphere_plane_closed_form():
    rng = np.random.default_rng(1)
    for _ in range(50):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        d = rng.uniform(-1, 1)
        c = rng.normal(size=3)
        r = rng.uniform(0, 0.3)
        phi, nn, p = oracle.pair(0, c, r, np.r_[n, d])
        # distance from a point to the plane n.x = d, minus the radius
        assert phi == pytest.approx(np.dot(n, c) - d - r, abs=1e-14)
        assert np.allclose(nn, n)
        # contact point lies on the sphere surface towards the plane
        assert np.linalg.norm(p - c) == pytest.approx(r, abs=1e-14)


def test_sphere_box_bruteforce():
    rng = np.random.default_rng(2)
    for trial in range(40):
        half = rng.uniform(0.05, 0.5, 3)
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        R = quat_to_R(q)
        bc = rng.normal(size=3)
        r = rng.uniform(0.0, 0.1)
        # centre outside (most trials) or inside the box
        loc = rng.uniform(-1.6, 1.6, 3) * half
        c = bc + R @ loc
        phi, n, p = oracle.pair(1, c, r, np.r_[bc, half, q])
        S = box_surface_samples(bc, half, R, n=80)
        dist = np.min(np.linalg.norm(S - c, axis=1))
        inside = np.all(np.abs(loc) <= half)
        signed = -dist if inside else dist
        spacing = 2 * half.max() / 79
        assert phi + r == pytest.approx(signed, abs=spacing), (trial, phi, signed)
        assert np.linalg.norm(n) == pytest.approx(1.0, abs=1e-12)
        # moving the sphere centre along n by eps raises phi by eps (away from the box)
        eps = 1e-6
        phi2, _, _ = oracle.pair(1, c + eps * n, r, np.r_[bc, half, q])
        assert phi2 - phi == pytest.approx(eps, rel=1e-3)
        assert np.allclose(p, c - r * n)


def test_sphere_box_inside_face_choice():
    # centre inside, nearest face +y (e - |c| smallest on axis 1)
    phi, n, p = oracle.pair(1, np.array([0.0, 0.9, 0.1]), 0.05,
                            np.r_[0, 0, 0, 1.0, 1.0, 1.0, 1, 0, 0, 0])
    assert phi == pytest.approx(-(1.0 - 0.9) - 0.05)
    assert np.allclose(n, [0, 1, 0])
    # tie between x and z faces -> lowest axis, + side for c_i >= 0
    phi, n, p = oracle.pair(1, np.array([0.5, 0.0, 0.5]), 0.0,
                            np.r_[0, 0, 0, 1.0, 2.0, 1.0, 1, 0, 0, 0])
    assert np.allclose(n, [1, 0, 0])
    assert phi == pytest.approx(-0.5)


def test_sphere_sphere_closed_form():
    rng = np.random.default_rng(3)
    for _ in range(50):
        ca, cb = rng.normal(size=3), rng.normal(size=3)
        ra, rb = rng.uniform(0, 0.5, 2)
        phi, n, p = oracle.pair(2, ca, ra, np.r_[cb, rb])
        assert phi == pytest.approx(np.linalg.norm(ca - cb) - ra - rb, abs=1e-13)
        assert np.allclose(n, (ca - cb) / np.linalg.norm(ca - cb))
    phi, n, p = oracle.pair(2, np.zeros(3), 0.1, np.r_[0, 0, 0, 0.2])
    assert np.allclose(n, [0, 0, 1]) and phi == pytest.approx(-0.3)


def test_onb_orthonormal_right_handed():
    rng = np.random.default_rng(4)
    normals = [np.array([0, 0, 1.0]), np.array([0, 0, -1.0]), np.array([1.0, 0, 0]), np.array([0, -1.0, 0])]
    normals += [v / np.linalg.norm(v) for v in rng.normal(size=(200, 3))]
    for n in normals:
        t1, t2 = oracle.onb(n)
        B = np.stack([t1, t2, n])
        assert np.allclose(B @ B.T, np.eye(3), atol=1e-12)
        assert np.allclose(np.cross(t1, t2), n, atol=1e-12)


def test_quat_update_matches_rodrigues():
    rng = np.random.default_rng(5)
    for _ in range(50):
        Q = rng.normal(size=4)
        Q /= np.linalg.norm(Q)
        w = rng.normal(size=3) * rng.choice([1e-9, 1e-3, 1.0, 20.0])
        h = 0.005
        Q2 = oracle.quat_update(Q, w, h)
        assert np.linalg.norm(Q2) == pytest.approx(1.0, abs=1e-14)
        assert np.allclose(quat_to_R(Q2), rodrigues(w * h) @ quat_to_R(Q), atol=1e-12)
