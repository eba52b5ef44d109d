"""Pins of the oracle's articulated-body kinematics and dynamics.

- planar two-link arm: forward kinematics, M(q) and C(q, qd) against the
  textbook closed forms (e.g. Spong, Hutchinson & Vidyasagar, Robot Modeling
  and Control, Sec. 7.4);
- Fetch-like and 7-R models: M symmetric positive definite, kinetic energy
  from link velocities equals 1/2 qd^T M qd, the RNEA bias equals the
  Lagrangian terms built from finite differences of the CRBA mass matrix and
  of the potential energy, and an FP64 articulated-body algorithm equals the
  CRBA + Cholesky solve (Featherstone 2008, chs. 6-7).
"""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg

G = 9.81


def two_link(m1=1.3, m2=0.7, l1=0.5, l2=0.35, lc1=0.2, lc2=0.15, I1=(0.01, 0.02, 0.015),
             I2=(0.004, 0.006, 0.003)):
    mb = sg.model_builder()
    b0 = mb.body(-1, sg.JT_REVOLUTE, (0, 1, 0), (0, 0, 0), m1, (lc1, 0, 0), I1)
    b1 = mb.body(b0, sg.JT_REVOLUTE, (0, 1, 0), (l1, 0, 0), m2, (lc2, 0, 0), I2)
    mb.segment(b1, (l2, 0, 0), (l2, 0, 0), 0.01, 1)
    batch = sg.custom_batch([mb.arrays()], [dict()])
    # the generator stores float32: read the rounded values back
    p = dict(m1=float(batch.model_mass[0, 0]), m2=float(batch.model_mass[0, 1]),
             l1=float(batch.model_xt_pos[0, 1, 0]), l2=float(batch.model_sph[0, 0, 0]),
             lc1=float(batch.model_com[0, 0, 0]), lc2=float(batch.model_com[0, 1, 0]),
             I1=float(batch.model_inertia[0, 0, 1]), I2=float(batch.model_inertia[0, 1, 1]))
    return batch, p


def test_two_link_fk_closed_form():
    b, p = two_link()
    o = oracle.Oracle(b)
    rng = np.random.default_rng(0)
    for _ in range(20):
        q = np.zeros(16)
        q[:2] = rng.uniform(-3, 3, 2)
        sph, org, rot = o.fk(0, q)
        l1, l2 = p["l1"], p["l2"]
        # rotation about +y by q maps the x axis to (cos q, 0, -sin q)
        elbow = np.array([l1 * math.cos(q[0]), 0, -l1 * math.sin(q[0])])
        tip = elbow + np.array([l2 * math.cos(q[0] + q[1]), 0, -l2 * math.sin(q[0] + q[1])])
        assert np.allclose(org[1], elbow, atol=1e-14)
        assert np.allclose(sph[0], tip, atol=1e-14)


def test_two_link_mass_matrix_and_bias_closed_form():
    b, p = two_link()
    o = oracle.Oracle(b)
    m1, m2, l1, lc1, lc2, I1, I2 = p["m1"], p["m2"], p["l1"], p["lc1"], p["lc2"], p["I1"], p["I2"]
    rng = np.random.default_rng(1)
    for _ in range(20):
        q = np.zeros(16)
        qd = np.zeros(16)
        q[:2] = rng.uniform(-3, 3, 2)
        qd[:2] = rng.normal(size=2) * 2
        M, Cb = o.dynamics(0, q, qd)
        c2 = math.cos(q[1])
        M_ref = np.array([[I1 + I2 + m1 * lc1 ** 2 + m2 * (l1 ** 2 + lc2 ** 2 + 2 * l1 * lc2 * c2),
                           I2 + m2 * (lc2 ** 2 + l1 * lc2 * c2)],
                          [I2 + m2 * (lc2 ** 2 + l1 * lc2 * c2), I2 + m2 * lc2 ** 2]])
        assert np.allclose(M, M_ref, atol=1e-12)
        h = -m2 * l1 * lc2 * math.sin(q[1])
        vel = np.array([h * qd[1] ** 2 + 2 * h * qd[0] * qd[1], -h * qd[0] ** 2])
        s1, s12 = math.cos(q[0]), math.cos(q[0] + q[1])
        grav = np.array([-G * (m1 * lc1 + m2 * l1) * s1 - m2 * G * lc2 * s12, -m2 * G * lc2 * s12])
        assert np.allclose(Cb, vel + grav, atol=1e-10)


@pytest.fixture(scope="module")
def robots():
    return [sg.make(1, 2), sg.make(2, 1)]


def _rand_state(b, rng):
    nb = int(b.model_nb[0])
    q = np.zeros(16)
    qd = np.zeros(16)
    q[:nb] = rng.uniform(-1.5, 1.5, nb)
    qd[:nb] = rng.normal(size=nb)
    return nb, q, qd


def test_mass_matrix_spd_and_energy(robots):
    rng = np.random.default_rng(2)
    for b in robots:
        o = oracle.Oracle(b)
        for _ in range(10):
            nb, q, qd = _rand_state(b, rng)
            M, _ = o.dynamics(0, q, qd)
            assert np.allclose(M, M.T, atol=1e-13)
            assert np.linalg.eigvalsh(M).min() > 0
            E = o.kinetic_energy(0, q, qd)
            assert E == pytest.approx(0.5 * qd[:nb] @ M @ qd[:nb], rel=1e-12)


def test_rnea_bias_equals_lagrangian_terms(robots):
    """C_i = sum_j dM_ij/dt qd_j - 1/2 qd^T dM/dq_i qd + dV/dq_i (central FD of CRBA M and V)."""
    rng = np.random.default_rng(3)
    for b in robots:
        o = oracle.Oracle(b)
        nb = int(b.model_nb[0])
        mass = b.model_mass[0].astype(np.float64)
        com = b.model_com[0].astype(np.float64)

        def V(q):
            _, org, rot = o.fk(0, q)
            return sum(mass[i] * G * (rot[i] @ com[i] + org[i])[2] for i in range(nb))

        for _ in range(4):
            _, q, qd = _rand_state(b, rng)
            _, Cb = o.dynamics(0, q, qd)
            eps = 1e-6
            dM = []
            dV = []
            for k in range(nb):
                e = np.zeros(16)
                e[k] = eps
                dM.append((o.dynamics(0, q + e, qd)[0] - o.dynamics(0, q - e, qd)[0]) / (2 * eps))
                dV.append((V(q + e) - V(q - e)) / (2 * eps))
            v = qd[:nb]
            Mdot = sum(dM[k] * v[k] for k in range(nb))
            ref = Mdot @ v - 0.5 * np.array([v @ dM[i] @ v for i in range(nb)]) + np.array(dV)
            assert np.allclose(Cb, ref, atol=1e-6 * max(1.0, np.abs(ref).max()))


def test_aba_equals_crba_cholesky(robots):
    rng = np.random.default_rng(4)
    for b in robots:
        o = oracle.Oracle(b)
        for _ in range(20):
            nb, q, qd = _rand_state(b, rng)
            tau = np.zeros(16)
            tau[:nb] = rng.normal(size=nb) * 5
            arm = np.zeros(16)
            arm[:nb] = rng.uniform(0, 0.5, nb)
            M, Cb = o.dynamics(0, q, qd)
            ref = np.linalg.solve(M + np.diag(arm[:nb]), tau[:nb] - Cb)
            got = o.aba(0, q, qd, tau, arm)
            assert np.allclose(got, ref, rtol=1e-10, atol=1e-10)


def test_sphere_intra_link_distances_invariant(robots):
    rng = np.random.default_rng(5)
    b = robots[1]
    o = oracle.Oracle(b)
    body = b.model_sph_body[0, : b.model_nsph[0]]
    s0, _, _ = o.fk(0, np.zeros(16))
    for _ in range(5):
        _, q, _ = _rand_state(b, rng)
        s, _, _ = o.fk(0, q)
        for link in np.unique(body):
            idx = np.nonzero(body == link)[0]
            d0 = np.linalg.norm(s0[idx][:, None] - s0[idx][None], axis=-1)
            d1 = np.linalg.norm(s[idx][:, None] - s[idx][None], axis=-1)
            assert np.allclose(d0, d1, atol=1e-12)
