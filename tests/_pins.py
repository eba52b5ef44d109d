"""Closed-form and conservation pins of the oracle's robot contact rows,
joint-limit rows and door / drawer joints, implicit PD drive, explicit
gyroscopic term, sliding sensitivity and robot contact cap.

Each pin takes ``mk(batch, **overrides) -> oracle`` so that the same check runs
against the oracle and against copies of it with one planted mistake
(``test_oracle_mutants.py``); a pin raises AssertionError when the physics it
states does not hold.  Every pin is a fact of mechanics that does not restate
the oracle's formula:

- angular momentum about a fixed frictionless hinge axis is conserved through
  contact impulses (no gravity, no other constraint), for the robot and for a
  door;
- a resting link's support force balances the gravity moment about its hinge;
- a single frictionless speculative contact after one sweep puts the contact
  point on the surface to second order in h (measured by independent forward
  kinematics);
- a joint-limit row lands the joint on its limit, and a free joint moves at
  constant velocity;
- a hinged door with a horizontal axis swings with the physical pendulum's
  exact period;
- implicit PD reaches its target with zero steady-state error, is stable at any
  stiffness, is monotone when overdamped and converges to the analytic damped
  oscillator at first order in h;
- a torque-free rigid body keeps its world angular momentum (first-order drift)
  and spins steadily about a principal axis;
- a box sliding on the floor has dx(T)/dv0 = T before it stops.
"""
from __future__ import annotations

import math

import numpy as np

import scenegen as sg

G = 9.81
FLOOR = [(0.0, 0.0, 1.0, 0.0)]


def _split(b, x):
    return sg.split_state(x, b.n_scenes, b.n_free, b.n_aux)


def _f(v):
    """A value as the scene arrays hold it (float32)."""
    return float(np.float32(v))


def _quat_R(q):
    w, a, b, c = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (b * b + c * c), 2 * (a * b - w * c), 2 * (a * c + w * b)],
                     [2 * (a * b + w * c), 1 - 2 * (a * a + c * c), 2 * (b * c - w * a)],
                     [2 * (a * c - w * b), 2 * (b * c + w * a), 1 - 2 * (a * a + b * b)]])


def _free_L(b, x, about=np.zeros(3), axis=None):
    """Sum of free-body angular momenta about a point: (x - o) x m v + R D R^T w."""
    fr = _split(b, x)["free"]
    L = np.zeros(3)
    for f in range(b.n_free):
        m = float(b.free_mass[f])
        R = _quat_R(fr[f, 4:8])
        Iw = R @ np.diag(b.free_inertia[f].astype(np.float64)) @ R.T
        L += np.cross(fr[f, 0:3] - about, m * fr[f, 8:11]) + Iw @ fr[f, 12:15]
    return L if axis is None else float(L @ axis)


# --------------------------------------------------------------------------
# robot contact rows
# --------------------------------------------------------------------------

def pin_robot_hinge_momentum(mk, mu=0.5):
    """A one-link robot turning about the world z axis through the origin
    (frictionless hinge, no gravity) strikes a free sphere and a free cube
    off-centre, with friction: the total angular momentum about z,
    M q_dot (the hinge's generalized momentum) plus each free body's
    (x m v + I_w w)_z, is conserved through every contact impulse."""
    mb = sg.model_builder()
    b0 = mb.body(-1, sg.JT_REVOLUTE, (0, 0, 1), (0, 0, 0), 2.0, (0.3, 0.02, 0.01), (0.01, 0.06, 0.05))
    mb.segment(b0, (0.15, 0, 0), (0.6, 0, 0.05), 0.05, 4)
    qd = np.zeros(16)
    qd[0] = 3.0
    ball = sg.sphere_object(0.06, 0.4, (0.45, 0.14, 0.06), angvel=(0.0, 2.0, -1.0))
    cube = sg.box_object((0.05, 0.05, 0.05), 0.3, (-0.2, 0.58, 0.0), quat=(0.9, 0.1, -0.2, 0.3),
                         vel=(0.1, -0.4, 0.0))
    b = sg.custom_batch([mb.arrays()], [dict(qd=qd, free=[ball, cube])], h=0.002, n_sub=5, pgs_iters=8, mu=mu,
                        gravity=(0.0, 0.0, 0.0))
    o = mk(b)
    x = b.state0.astype(np.float64)

    def Lz(x):
        st = _split(b, x)
        M, _ = o.dynamics(0, st["q"][0], st["qd"][0], g=(0.0, 0.0, 0.0))
        return float(M[0, 0] * st["qd"][0, 0]) + _free_L(b, x)[2]

    L0 = Lz(x)
    n_con = 0
    moved = 0.0
    for _ in range(12):
        x, d = o.step(x, np.zeros((1, 16)), debug=True)
        n_con += int(d["n_contacts"].sum())
        L = Lz(x)
        assert abs(L - L0) <= 1e-10 * abs(L0), (L, L0)
        moved = max(moved, abs(_free_L(b, x)[2] - _free_L(b, b.state0.astype(np.float64))[2]))
    assert n_con >= 10, n_con            # both bodies were struck, repeatedly
    assert moved >= 0.05 * abs(L0), moved  # and took a large share of the momentum
    return L0


def _rest_arm(theta, L=0.5, d=0.3, r=0.04, m=1.5):
    """One link hinged about the world y axis at height L sin(theta) + r, tilted
    down by theta, its tip sphere (radius r) on the floor."""
    mb = sg.model_builder()
    H = L * math.sin(theta) + r
    b0 = mb.body(-1, sg.JT_REVOLUTE, (0, 1, 0), (0, 0, H), m, (d, 0, 0), (0.002, 0.03, 0.03), damping=0.5)
    mb.segment(b0, (L, 0, 0), (L, 0, 0), r, 1)
    q = np.zeros(16)
    q[0] = theta
    return sg.custom_batch([mb.arrays()], [dict(q=q, planes=FLOOR)], h=0.002, n_sub=5, pgs_iters=10, mu=0.0)


def pin_robot_resting_moment(mk, theta=0.5):
    """A one-link arm resting on its tip sphere (frictionless floor) comes to
    rest with the support force N balancing the gravity moment about the
    hinge: N * (horizontal lever L cos th) = m g d cos th, i.e. N = m g d / L;
    its tip never sinks below the floor by more than the margin."""
    b = _rest_arm(theta)
    o = mk(b)
    x = b.state0.astype(np.float64)
    for _ in range(60):
        x, d = o.step(x, np.zeros((1, 16)), dump_cap=4)
        sph, _, _ = o.fk(0, _split(b, x)["q"][0])
        assert sph[0, 2] - float(b.model_sph[0, 0, 3]) >= -b.margin, sph[0, 2]
    m = float(b.model_mass[0, 0])
    dcom = float(b.model_com[0, 0, 0])
    Lt = float(b.model_sph[0, 0, 0])
    N = d["dump_lambda"][0, 0, 0] / b.h
    assert abs(_split(b, x)["qd"][0, 0]) < 1e-6
    N_ref = m * G * dcom / Lt
    assert abs(N - N_ref) <= 1e-6 * N_ref, (N, N_ref)
    return N


def pin_robot_speculative_landing(mk):
    """A three-joint chain (prismatic x slider, then two revolute joints about
    y) drives its tip sphere toward the floor faster than the gap closes in
    one substep.  One frictionless contact is exact after one sweep, so the
    tip lands on the floor: its signed distance after the substep, measured
    by forward kinematics of the new joint positions, is zero to second order
    in h."""
    mb = sg.model_builder()
    b0 = mb.body(-1, sg.JT_PRISMATIC, (1, 0, 0), (0, 0, 0.5), 3.0, (0, 0, 0), (0.01, 0.01, 0.01))
    b1 = mb.body(b0, sg.JT_REVOLUTE, (0, 1, 0), (0.05, 0, 0), 1.2, (0.15, 0, 0), (0.002, 0.01, 0.01))
    b2 = mb.body(b1, sg.JT_REVOLUTE, (0, 1, 0), (0.3, 0, 0), 0.7, (0.1, 0, 0.01), (0.001, 0.005, 0.005))
    mb.segment(b2, (0.25, 0, 0.02), (0.25, 0, 0.02), 0.03, 1)
    sc = mb.arrays()
    res = []
    for q1, q2 in [((0.7, 0.9), (0.4, 6.0, 4.0)), ((1.1, 0.2), (-0.6, 5.0, 8.0))]:
        q = np.zeros(16)
        qd = np.zeros(16)
        q[1], q[2] = q1
        qd[0], qd[1], qd[2] = q2
        b = sg.custom_batch([sc], [dict(q=q, qd=qd, planes=FLOOR)], h=1e-4, n_sub=1, pgs_iters=1, mu=0.0,
                            gravity=(0.0, 0.0, 0.0))
        o = mk(b)
        x = b.state0.astype(np.float64)
        st = _split(b, x)
        # the floor 0.05 mm below the tip sphere, which approaches at 1.5-1.8 m/s
        sph, _, _ = o.fk(0, st["q"][0])
        r = float(b.model_sph[0, 0, 3])
        b.plane[0, 3] = np.float32(sph[0, 2] - r - 5e-5)
        o = mk(b)
        x1, d = o.step(x, np.zeros((1, 16)), dump_cap=2)
        assert d["dump_lambda"][0, 0, 0] > 0.0
        sph1, _, _ = o.fk(0, _split(b, x1)["q"][0])
        gap = sph1[0, 2] - r - float(b.plane[0, 3])
        # tip travel per substep ~0.16 mm; second-order residual ~ h^2 w^2 l ~ 3e-7
        assert abs(gap) <= 1e-6, gap
        res.append(gap)
    return res


def pin_robot_contact_cap(mk):
    """Robot contact cap: with more robot contacts than the cap, the first
    `cap` robot-owned contacts in canonical order are kept, the rest of the
    robot's are dropped (status bit 8), free-body contacts are all kept."""
    mb = sg.model_builder()
    b0 = mb.body(-1, sg.JT_PRISMATIC, (0, 0, 1), (0, 0, 0.0), 2.0, (0, 0, 0), (0.01, 0.01, 0.01))
    mb.segment(b0, (-0.3, 0, 0.02), (0.3, 0, 0.02), 0.03, 7)
    box = sg.box_object((0.05, 0.05, 0.05), 0.3, (0.0, 0.5, 0.05))

    def run(rcap):
        b = sg.custom_batch([mb.arrays()], [dict(free=[box], planes=FLOOR)], h=0.002, n_sub=1, contact_cap=32)
        b.robot_contact_cap = rcap
        o = mk(b)
        _, d = o.step(b.state0.astype(np.float64), np.zeros((1, 16)), debug=True, dump_cap=32)
        k = d["dump_keys"][0]
        return k[k != np.uint64(~np.uint64(0))], int(d["status"][0] if "status" in d else 0), d

    full, _, dfull = run(32)
    robot = [k for k in full if (int(k) >> 56) == 0]   # robot-owned: owner class 0 in the key's top byte
    other = [k for k in full if (int(k) >> 56) != 0]
    assert len(robot) == 7 and len(other) == 4, (len(robot), len(other))
    capped, _, dcap = run(3)
    assert list(capped) == robot[:3] + other, capped
    return len(capped)


# --------------------------------------------------------------------------
# door / drawer joints and their limit rows
# --------------------------------------------------------------------------

def _door(q0, limit=(0.0, math.pi / 2), axis=(0, 0, 1), rot=(1.0, 0.0, 0.0, 0.0), pos=(0.0, 0.0, 0.01),
          box=(0.3, 0.0, 0.9, 0.3, 0.02, 0.9), m=10.0):
    full = 2 * np.array(box[3:])
    return dict(type=sg.JT_REVOLUTE, rot=rot, pos=pos, axis=axis, box=box, mass=m,
                inertia=sg._box_inertia(m, full), limit=limit, q0=q0)


def _drawer(q0, limit=(0.0, 0.4), rot=(1.0, 0.0, 0.0, 0.0), pos=(0.0, 0.0, 0.5)):
    full = np.array([0.5, 0.4, 0.2])
    return dict(type=sg.JT_PRISMATIC, rot=rot, pos=pos, axis=(1, 0, 0), box=(0.0, 0.0, 0.0, 0.25, 0.2, 0.1),
                mass=3.0, inertia=sg._box_inertia(3.0, full), limit=limit, q0=q0)


def _aux_batch(aux, free=(), h=0.004, n_sub=5, gravity=(0.0, 0.0, -G), pgs_iters=10, mu=0.5, planes=()):
    b = sg.custom_batch([sg.empty_model()], [dict(aux=list(aux), free=list(free), planes=list(planes))], h=h,
                        n_sub=n_sub, pgs_iters=pgs_iters, mu=mu, gravity=gravity)
    return b


def pin_limit_lands_on_limit(mk):
    """A drawer moving toward its upper limit (0.4 m) and a door turning toward
    its lower limit (0): the limit row, exact after one sweep, puts each joint
    on its limit at the end of the substep; afterwards they stay there."""
    yaw = (math.cos(0.35), 0.0, 0.0, math.sin(0.35))
    b = _aux_batch([_drawer(0.3995, rot=yaw), _door(0.0015, rot=yaw)], h=0.002, n_sub=1)
    ax = _split(b, b.state0)["aux"]
    ax[0, 1] = 0.5      # m/s toward 0.4
    ax[1, 1] = -1.2     # rad/s toward 0
    o = mk(b)
    x = b.state0.astype(np.float64)
    x1 = o.step(x, np.zeros((1, 16)))
    a1 = _split(b, x1)["aux"]
    assert abs(a1[0, 0] - _f(0.4)) <= 1e-12 and abs(a1[1, 0] - 0.0) <= 1e-12, a1[:, 0]
    for _ in range(50):
        x1 = o.step(x1, np.zeros((1, 16)))
    a1 = _split(b, x1)["aux"]
    assert abs(a1[0, 0] - _f(0.4)) <= 1e-9 and abs(a1[1, 0]) <= 1e-9, a1[:, 0]
    assert abs(a1[0, 1]) <= 1e-9 and abs(a1[1, 1]) <= 1e-9
    return a1[:, 0]


def pin_free_joints_constant_velocity(mk):
    """With no contact, no limit in reach and gravity along the door's hinge
    (no torque) and across the drawer's slide: q_n = q_0 + n h v_0 exactly,
    up to the drawer stopping at its 0.4 m limit."""
    yaw = (math.cos(-0.6), 0.0, 0.0, math.sin(-0.6))
    b = _aux_batch([_drawer(0.1, rot=yaw), _door(0.2, rot=yaw, pos=(2.0, 0.0, 0.01))], h=0.004, n_sub=5)
    ax = _split(b, b.state0)["aux"]
    ax[0, 1] = 0.25
    ax[1, 1] = 0.7
    o = mk(b)
    x = b.state0.astype(np.float64)
    v0, w0 = _f(0.25), _f(0.7)
    q0, a0 = _f(0.1), _f(0.2)
    hit = False
    for n in range(1, 80):
        x = o.step(x, np.zeros((1, 16)))
        a = _split(b, x)["aux"]
        t = n * b.n_sub * b.h
        assert abs(a[1, 0] - (a0 + t * w0)) <= 1e-10 and abs(a[1, 1] - w0) <= 1e-12, (n, a[1])
        if q0 + t * v0 < 0.4 - 0.002:
            assert abs(a[0, 0] - (q0 + t * v0)) <= 1e-10 and abs(a[0, 1] - v0) <= 1e-12, (n, a[0])
        elif q0 + t * v0 > 0.4 + 0.002:
            hit = True
            assert abs(a[0, 0] - _f(0.4)) <= 1e-6 and abs(a[0, 1]) <= 1e-6, (n, a[0])
    assert hit
    return float(a[1, 0])


def _door_pendulum_period(mk, h, th0=1.0):
    # hinge along world x at 2 m height, panel hanging below it (centre 0.5 m down)
    door = _door(th0, limit=(1.0, -1.0), axis=(1, 0, 0), pos=(0.0, 0.0, 2.0), box=(0.0, 0.0, -0.5, 0.3, 0.02, 0.5),
                 m=4.0)
    b = _aux_batch([door], h=h, n_sub=1)
    o = mk(b)
    x = b.state0.astype(np.float64)
    qs = [x[-4]]
    n = int(2.6 / h)
    for _ in range(n):
        x = o.step(x, np.zeros((1, 16)))
        qs.append(x[-4])
    qs = np.array(qs)
    t = np.arange(len(qs)) * h
    idx = np.nonzero((qs[:-1] > 0) & (qs[1:] <= 0))[0]
    assert len(idx) >= 2, "the door did not swing"
    tc = t[idx] + h * qs[idx] / (qs[idx] - qs[idx + 1])
    m = float(b.aux_mass[0])
    dd = -float(b.aux_box[0, 2])
    Ip = float(b.aux_inertia[0, 0]) + m * dd * dd
    th0 = float(b.state0[-4])
    a, c = 1.0, math.cos(th0 / 2)
    for _ in range(60):
        a, c = (a + c) / 2, math.sqrt(a * c)
    T = 2 * math.pi * math.sqrt(Ip / (m * G * dd)) / a
    return tc[1] - tc[0], T


def pin_door_pendulum_period(mk):
    """A door hinged about a horizontal axis is a physical pendulum: its period
    matches 2 pi sqrt(I_p / (m g d)) / AGM(1, cos(th0 / 2)) with an error
    that shrinks with h."""
    errs = []
    for h in (2e-3, 1e-3):
        Tm, T = _door_pendulum_period(mk, h)
        errs.append(abs(Tm - T))
    assert errs[1] < 2e-3 * T, errs
    assert errs[1] < 0.75 * errs[0], errs
    return errs


def pin_door_hinge_momentum(mk, mu=0.5):
    """Zero gravity: a free sphere strikes a turning door (vertical hinge, no
    limit in reach) off-centre, with friction; the door's hinge momentum
    M q_dot plus the sphere's angular momentum about the hinge axis is
    conserved.  A sphere striking a sliding drawer conserves the momentum
    along the slide."""
    # joint frame rotated by (0.5, 0.5, 0.5, 0.5) (exact in float32): its y axis is
    # the world z axis, its z axis the world x axis
    door = _door(0.3, limit=(1.0, -1.0), rot=(0.5, 0.5, 0.5, 0.5), axis=(0, 1, 0),
                 box=(0.0, 0.9, 0.3, 0.02, 0.9, 0.3))
    drawer = _drawer(0.1, limit=(1.0, -1.0), pos=(3.0, 0.0, 0.5))
    ball = sg.sphere_object(0.07, 0.8, (0.3, 0.25, 1.2), vel=(0.3, -1.5, 0.2), angvel=(1.0, 0.0, 3.0))
    ball2 = sg.sphere_object(0.05, 0.5, (3.45, 0.05, 0.52), vel=(-1.2, 0.1, 0.0))
    b = _aux_batch([door, drawer], free=[ball, ball2], h=0.002, n_sub=5, gravity=(0.0, 0.0, 0.0), mu=mu)
    _split(b, b.state0)["aux"][0, 1] = 0.8   # the door turns toward the ball
    o = mk(b)
    x = b.state0.astype(np.float64)
    hinge = b.aux_pos[0].astype(np.float64)
    z = np.array([0.0, 0.0, 1.0])
    Rd = _quat_R(b.aux_rot[1])
    slide = Rd @ np.array([1.0, 0.0, 0.0])
    # about the hinge (joint-frame y): I_yy + m (x^2 + z^2) of the panel centre
    Idoor = float(b.aux_inertia[0, 1]) + float(b.aux_mass[0]) * float(b.aux_box[0, 0]) ** 2 + \
        float(b.aux_mass[0]) * float(b.aux_box[0, 2]) ** 2

    def moments(x):
        a = _split(b, x)["aux"]
        fr = _split(b, x)["free"]
        Ld = Idoor * a[0, 1]
        m0 = float(b.free_mass[0])
        Ls = float(np.cross(fr[0, 0:3] - hinge, m0 * fr[0, 8:11]) @ z) + float(b.free_inertia[0, 0]) * fr[0, 14]
        P = float(b.aux_mass[1]) * a[1, 1] + float(b.free_mass[1]) * float(fr[1, 8:11] @ slide)
        return Ld + Ls, P

    L0, P0 = moments(x)
    n_con = 0
    for _ in range(12):
        x, d = o.step(x, np.zeros((1, 16)), debug=True)
        n_con += int(d["n_contacts"].sum())
        L, P = moments(x)
        assert abs(L - L0) <= 1e-10 * max(abs(L0), 1e-3), (L, L0)
        assert abs(P - P0) <= 1e-10 * abs(P0), (P, P0)
    a = _split(b, x)["aux"]
    assert n_con >= 12, n_con
    assert abs(a[1, 1]) > 0.1, a[1]   # the drawer was pushed
    assert abs(a[0, 1] - 0.8) > 0.1, a[0]   # the door was struck
    return L0, P0


# --------------------------------------------------------------------------
# implicit PD drive and joint damping
# --------------------------------------------------------------------------

def _slider(m, kp, kd, damping=0.0, veldof=0, h=0.002, n_sub=5, q0=0.0, mode=sg.CTRL_PD):
    mb = sg.model_builder()
    mb.body(-1, sg.JT_PRISMATIC, (1, 0, 0), (0, 0, 1.0), m, (0, 0, 0), (0.01, 0.01, 0.01), kp=kp, kd=kd,
            veldof=veldof, damping=damping)
    q = np.zeros(16)
    q[0] = q0
    return sg.custom_batch([mb.arrays()], [dict(q=q)], h=h, n_sub=n_sub, control_mode=mode)


def _run_slider(mk, b, target, n):
    o = mk(b)
    x = b.state0.astype(np.float64)
    u = np.zeros((1, 16))
    u[0, 0] = target
    qs, vs = [x[0]], [x[16]]
    for _ in range(n):
        x = o.step(x, u)
        qs.append(x[0])
        vs.append(x[16])
    return np.array(qs), np.array(vs)


def pin_pd_steady_state_and_stability(mk):
    """Implicit PD on a 1-DoF slider (no gravity along it): it settles on its
    target with zero steady-state error; at h^2 kp = 100 m and no damping gain
    (explicit PD would diverge) it stays bounded and settles; overdamped, it
    approaches the target monotonically without overshoot."""
    qs, vs = _run_slider(mk, _slider(0.5, 400.0, 40.0), 0.3, 300)
    assert abs(qs[-1] - 0.3) <= 1e-9 and abs(vs[-1]) <= 1e-9, (qs[-1], vs[-1])
    b = _slider(0.1, 1e5, 0.0, h=0.01, n_sub=1)
    qs, _ = _run_slider(mk, b, 0.2, 400)
    err = np.abs(qs - 0.2)[1:]
    assert np.all(err <= 0.05 * 0.2), err.max()   # after the first substep, never near the start error
    assert abs(qs[-1] - 0.2) <= 1e-9, qs[-1]
    # overdamped: kd^2 > 4 m kp
    qs, _ = _run_slider(mk, _slider(1.0, 100.0, 60.0), 0.25, 200)
    assert np.all(np.diff(qs) >= -1e-15) and np.all(qs <= 0.25 + 1e-12), (qs.max(), np.diff(qs).min())
    # a pure damping gain at h kd = 100 m (explicit damping would diverge):
    # the velocity decays monotonically, without changing sign
    b = _slider(0.1, 0.0, 1000.0, h=0.01, n_sub=1)
    _split(b, b.state0)["qd"][0, 0] = 1.0
    _, vs = _run_slider(mk, b, 0.0, 20)
    assert np.all(vs[1:] >= 0.0) and np.all(np.diff(vs) <= 0.0), vs
    return qs[-1]


def pin_pd_first_order_convergence(mk):
    """Implicit PD (with viscous joint damping) against the analytic damped
    oscillator m x'' = kp (x* - x) - (kd + c) x': the error at t = 0.4 s
    halves when h halves."""
    m, kp, kd, c, tgt = 0.8, 300.0, 4.0, 1.0, 0.2
    errs = []
    for h in (2e-3, 1e-3, 5e-4):
        n_sub = int(round(0.02 / h))
        b = _slider(m, kp, kd, damping=c, h=h, n_sub=n_sub)
        mf, kpf, kdf, cf = (float(b.model_mass[0, 0]), float(b.model_kp[0, 0]), float(b.model_kd[0, 0]),
                            float(b.model_damping[0, 0]))
        qs, _ = _run_slider(mk, b, tgt, 20)
        t = 0.4
        zeta = (kdf + cf) / (2 * math.sqrt(kpf * mf))
        w0 = math.sqrt(kpf / mf)
        wd = w0 * math.sqrt(1 - zeta * zeta)
        tg = _f(tgt)
        ex = tg - tg * math.exp(-zeta * w0 * t) * (math.cos(wd * t) + zeta * w0 / wd * math.sin(wd * t))
        errs.append(abs(qs[-1] - ex))
    assert errs[0] < 0.02, errs
    for a, b_ in zip(errs[:-1], errs[1:]):
        assert 0.4 * a < b_ < 0.6 * a, errs
    return errs


def pin_base_velocity_drive(mk):
    """A velocity-driven DoF (its position gain ignored) reaches the target
    velocity exactly; joint damping alone decays a free joint's velocity
    monotonically, approaching exp(-c t / m) at first order in h."""
    b = _slider(2.0, 500.0, 50.0, veldof=1)
    qs, vs = _run_slider(mk, b, 0.35, 200)
    assert abs(vs[-1] - 0.35) <= 1e-12, vs[-1]
    assert abs((qs[-1] - qs[-2]) - 0.35 * b.h * b.n_sub) <= 1e-12
    errs = []
    for h in (2e-3, 1e-3):
        b = _slider(2.0, 0.0, 0.0, damping=3.0, h=h, n_sub=int(round(0.02 / h)), mode=sg.CTRL_TORQUE)
        _split(b, b.state0)["qd"][0, 0] = 1.0
        qs, vs = _run_slider(mk, b, 0.0, 25)
        assert np.all(np.diff(vs) < 0) and vs[-1] > 0
        errs.append(abs(vs[-1] - math.exp(-float(b.model_damping[0, 0]) * 0.5 / float(b.model_mass[0, 0]))))
    assert 0.4 * errs[0] < errs[1] < 0.6 * errs[0], errs
    # stiff damping, h c = 10 m (explicit damping would diverge): monotone decay
    b = _slider(1.0, 0.0, 0.0, damping=1000.0, h=0.01, n_sub=1, mode=sg.CTRL_TORQUE)
    _split(b, b.state0)["qd"][0, 0] = 1.0
    _, vs = _run_slider(mk, b, 0.0, 20)
    assert np.all(vs[1:] >= 0.0) and np.all(np.diff(vs) <= 0.0), vs
    return errs


# --------------------------------------------------------------------------
# free-body gyroscopic term
# --------------------------------------------------------------------------

def _spinner(h, n_sub, w, quat):
    box = sg.box_object((0.2, 0.1, 0.05), 1.3, (0.0, 0.0, 1.0), quat=quat, angvel=w)
    return sg.custom_batch([sg.empty_model()], [dict(free=[box])], h=h, n_sub=n_sub, gravity=(0.0, 0.0, 0.0))


def pin_gyroscopic_torque_free(mk):
    """A torque-free box with three distinct principal moments, started in a
    general orientation with a general angular velocity: its world angular
    momentum R D R^T w keeps direction and magnitude with a drift that halves
    when h halves; spinning about a principal axis is a steady state."""
    quat = np.array([0.8, 0.3, -0.4, 0.33])
    quat = quat / np.linalg.norm(quat)
    w = (2.0, -1.0, 3.0)
    drifts = []
    for h in (1e-3, 5e-4):
        b = _spinner(h, int(round(0.02 / h)), w, quat)
        o = mk(b)
        x = b.state0.astype(np.float64)
        L0 = _free_L(b, x)
        for _ in range(25):
            x = o.step(x, np.zeros((1, 16)))
        L = _free_L(b, x)
        drifts.append(np.linalg.norm(L - L0) / np.linalg.norm(L0))
    assert drifts[0] < 0.05, drifts
    assert 0.4 * drifts[0] < drifts[1] < 0.6 * drifts[0], drifts
    # principal-axis spin: w along the world image of the body's second axis
    R = _quat_R(quat)
    wp = 2.5 * R[:, 1]
    b = _spinner(1e-3, 20, wp, quat)
    o = mk(b)
    x = b.state0.astype(np.float64)
    w0 = _split(b, x)["free"][0, 12:15].copy()
    for _ in range(10):
        x = o.step(x, np.zeros((1, 16)))
    w1 = _split(b, x)["free"][0, 12:15]
    assert np.linalg.norm(w1 - w0) <= 1e-5 * np.linalg.norm(w0), (w1, w0)
    return drifts


# --------------------------------------------------------------------------
# sliding sensitivity of the adjoint
# --------------------------------------------------------------------------

def pin_sliding_sensitivity(mk):
    """A box sliding on the floor under Coulomb friction, before it stops:
    x(T) = x0 + v0 T - mu g T^2 / 2 + ..., so dx(T)/dv0 = T and
    dv(T)/dv0 = 1 along the slide; the oracle's chained vector-Jacobian
    product over the control steps reproduces both."""
    half = (0.1, 0.08, 0.05)
    box = sg.box_object(half, 0.9, (0.0, 0.0, half[2]), vel=(2.0, 0.0, 0.0))
    b = sg.custom_batch([sg.empty_model()], [dict(free=[box], planes=FLOOR)], h=0.002, n_sub=10, pgs_iters=10,
                        mu=0.4)
    o = mk(b)
    xs = [b.state0.astype(np.float64)]
    n = 10
    u = np.zeros((1, 16))
    for _ in range(n):
        xs.append(o.step(xs[-1], u))
    T = n * b.n_sub * b.h
    vT = _split(b, xs[-1])["free"][0, 8]
    assert 0.5 < vT < 2.0   # still sliding
    out = []
    for comp in (0, 8):     # x position, x velocity
        g = np.zeros_like(xs[0])
        _split(b, g)["free"][0, comp] = 1.0
        for t in range(n - 1, -1, -1):
            g, _ = o.vjp(xs[t], u, g)
        out.append(_split(b, g)["free"][0, 8])
    assert abs(out[0] - T) <= 1e-9 * T, (out[0], T)
    assert abs(out[1] - 1.0) <= 1e-9, out[1]
    return out


ALL = [pin_robot_hinge_momentum, pin_robot_resting_moment, pin_robot_speculative_landing, pin_robot_contact_cap,
       pin_limit_lands_on_limit, pin_free_joints_constant_velocity, pin_door_pendulum_period,
       pin_door_hinge_momentum, pin_pd_steady_state_and_stability, pin_pd_first_order_convergence,
       pin_base_velocity_drive, pin_gyroscopic_torque_free, pin_sliding_sensitivity]
