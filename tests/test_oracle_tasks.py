"""Pins of the task oracle (subtask predicates, event labels, trajectory
categories of the appendix) against the definitions themselves: one
hand-built event list per success / failure mode, event transitions from
hand-set indicators, and kinematic invariants of the end-effector point."""
import math

import numpy as np
import pytest

import scenegen as sg
from oracle import tasks as ot

P, PL, O, CL = ot.PICK, ot.PLACE, ot.OPEN, ot.CLOSE

# (kind, event list, d0, expected mode): each list is built to satisfy the
# appendix's definition of that mode (and no mode tested before it)
CASES = [
    # Pick: success modes i-iv, failure modes v-ix
    (P, ["contact", "grasped", "success"], 0.0, 1),
    (P, ["contact", "grasped", "dropped", "contact", "grasped", "success"], 0.0, 2),
    (P, ["contact", "grasped", "success", "dropped"], 0.0, 3),
    (P, ["contact", "grasped", "success", "excessive_collisions"], 0.0, 4),
    (P, ["contact", "excessive_collisions"], 0.0, 5),
    (P, [], 0.0, 6),
    (P, ["contact"], 0.0, 7),
    (P, ["contact", "grasped", "dropped"], 0.0, 8),
    (P, ["contact", "grasped", "dropped", "grasped"], 0.0, 9),
    # Place: success i-v, failure vi-xii
    (PL, ["obj_at_goal", "released_at_goal", "success"], 0.5, 1),
    (PL, ["released_outside_goal", "obj_at_goal", "success"], 0.5, 2),
    (PL, ["obj_at_goal", "released_at_goal", "success", "obj_left_goal"], 0.5, 3),
    (PL, ["obj_at_goal", "obj_left_goal", "grasped", "obj_at_goal", "released_at_goal", "success"], 0.5, 4),
    (PL, ["obj_at_goal", "released_at_goal", "success", "excessive_collisions"], 0.5, 5),
    (PL, ["excessive_collisions"], 0.5, 6),
    (PL, [], 0.5, 7),
    (PL, ["released_outside_goal"], 0.5, 8),
    (PL, ["obj_at_goal", "released_at_goal", "obj_left_goal"], 0.5, 9),
    (PL, ["released_outside_goal", "obj_at_goal", "obj_left_goal"], 0.5, 10),
    (PL, ["obj_at_goal", "released_at_goal", "grasped"], 0.5, 11),
    (PL, ["obj_at_goal", "released_at_goal"], 0.5, 12),
    (PL, ["success"], 0.1, 1),           # already at the goal at the start, released there
    # Open: success i-iii, failure iv-ix
    (O, ["contact", "slightly_opened", "opened", "success"], 0.0, 1),
    (O, ["contact", "opened", "success", "closed"], 0.0, 2),
    (O, ["contact", "opened", "success", "excessive_collisions"], 0.0, 3),
    (O, ["contact", "excessive_collisions"], 0.0, 4),
    (O, [], 0.0, 5),
    (O, ["contact", "slightly_opened", "opened", "closed"], 0.0, 6),
    (O, ["contact", "slightly_opened"], 0.0, 7),
    (O, ["contact", "slightly_opened", "opened"], 0.0, 8),
    (O, ["contact"], 0.0, 9),
    # Close: success i-iii, failure iv-ix
    (CL, ["contact", "slightly_closed", "closed", "success"], 0.0, 1),
    (CL, ["contact", "closed", "success", "open"], 0.0, 2),
    (CL, ["contact", "closed", "success", "excessive_collisions"], 0.0, 3),
    (CL, ["excessive_collisions"], 0.0, 4),
    (CL, [], 0.0, 5),
    (CL, ["contact", "slightly_closed", "closed", "open"], 0.0, 6),
    (CL, ["contact", "slightly_closed"], 0.0, 7),
    (CL, ["contact", "slightly_closed", "closed"], 0.0, 8),
    (CL, ["contact"], 0.0, 9),
]


@pytest.mark.parametrize("kind,E,d0,mode", CASES)
def test_categories_from_definitions(kind, E, d0, mode):
    assert ot.categorize(kind, list(E), d0) == mode


def test_every_mode_has_a_case():
    n_modes = {P: 9, PL: 12, O: 9, CL: 9}
    for k, n in n_modes.items():
        assert sorted({m for kk, _, _, m in CASES if kk == k}) == list(range(1, n + 1))


def _ind(**kw):
    base = dict(grasped=False, contact=False, excessive=False, success=False, at_goal=False, state=False,
                slight=False)
    base.update(kw)
    return base


def test_event_transitions():
    # pick: touching and closing the gripper in one step gives contact then grasped
    assert ot.step_events(P, _ind(), _ind(contact=True, grasped=True)) == ["contact", "grasped"]
    assert ot.step_events(P, _ind(contact=True, grasped=True), _ind(contact=True)) == ["dropped"]
    assert ot.step_events(P, _ind(grasped=True), _ind(grasped=True, success=True, excessive=True)) == [
        "success", "excessive_collisions"]
    # staying in a state raises nothing
    assert ot.step_events(P, _ind(grasped=True), _ind(grasped=True)) == []
    # place: releasing inside / outside the goal region
    assert ot.step_events(PL, _ind(grasped=True, at_goal=True), _ind(at_goal=True)) == ["released_at_goal"]
    assert ot.step_events(PL, _ind(grasped=True), _ind()) == ["released_outside_goal"]
    assert ot.step_events(PL, _ind(grasped=True, at_goal=True), _ind()) == ["released_outside_goal",
                                                                            "obj_left_goal"]
    # open / close: reaching and leaving the goal state
    assert ot.step_events(O, _ind(), _ind(contact=True, slight=True, state=True)) == [
        "contact", "opened", "slightly_opened"]
    assert ot.step_events(CL, _ind(state=True), _ind()) == ["open"]


def _fetch_batch():
    return sg.make(2, 4)


def _robot(b):
    r = dict(sg.FETCH_TASK_ROBOT)
    r["ee_rest"] = (0.0, 0.0, 0.0)
    r["ee_rest"] = tuple(ot.ee_in_base(b, 0, np.asarray(sg.FETCH_REST), r))
    return r


def test_ee_point_is_invariant_to_the_base_pose():
    """Moving or turning the base leaves the end effector fixed in the base frame."""
    b = _fetch_batch()
    r = _robot(b)
    q = np.array(sg.FETCH_REST, np.float64)
    q[6:13] += np.array([0.3, -0.2, 0.5, 0.4, -0.6, 0.1, 0.7])
    e0 = ot.ee_in_base(b, 0, q, r)
    q2 = q.copy()
    q2[0] += 1.7
    q2[1] -= 0.4
    q2[2] += 2.1
    assert np.allclose(ot.ee_in_base(b, 0, q2, r), e0, atol=1e-12)
    # the world position turns with the yaw about the base origin (closed form)
    R0, p0 = ot.body_pose(b, 0, q, r["ee_body"])
    R1, p1 = ot.body_pose(b, 0, q2, r["ee_body"])
    c, s = math.cos(2.1), math.sin(2.1)
    Rz = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    base0 = np.array([q[0], q[1], 0.0])
    base1 = np.array([q2[0], q2[1], 0.0])
    assert np.allclose(p1 - base1, Rz @ (p0 - base0), atol=1e-12)
    assert np.allclose(R1, Rz @ R0, atol=1e-12)


def test_torso_lift_moves_the_ee_straight_up():
    b = _fetch_batch()
    r = _robot(b)
    q = np.array(sg.FETCH_REST, np.float64)
    e0 = ot.ee_in_base(b, 0, q, r)
    q[3] += 0.07
    assert np.allclose(ot.ee_in_base(b, 0, q, r) - e0, [0.0, 0.0, 0.07], atol=1e-12)


def test_rest_pose_predicates_and_success_limits():
    """At the rest pose with no motion: distances and joint errors vanish,
    the robot is static; pick succeeds iff grasped and C_t <= 5000 N."""
    b = _fetch_batch()
    r = _robot(b)
    S = b.n_scenes
    x = np.array(b.state0, np.float64)
    st = sg.split_state(x, S, b.n_free, b.n_aux)
    st["q"][:] = np.asarray(sg.FETCH_REST)
    st["qd"][:] = 0.0
    tk = [dict(kind=P, target=0, goal=(0, 0, 0), open_frac=0.9)] * S
    grip = np.zeros((b.n_free + b.n_aux, 2))
    grip[b.free_off[:-1], 1] = 0.6       # both fingers press with 0.6 N on object 0
    v = ot.predicates(b, x, tk, r, grip, 5, np.array([0.0, 5000.0, 5000.5, 1e4]))
    for s in range(S):
        assert v[s]["d_ee"] < 1e-12 and v[s]["j_arm"] == 0.0 and v[s]["static"] and v[s]["grasped"]
    ok = [ot.success(v[s], tk[s], 0.0)["success"] for s in range(S)]
    assert ok == [True, True, False, False]
    # a finger force below grasp_force is no grasp
    grip[b.free_off[:-1], 1] = 0.4
    v = ot.predicates(b, x, tk, r, grip, 5, np.zeros(S))
    assert not any(v[s]["grasped"] for s in range(S))


def test_open_close_thresholds():
    """open(a) / close(a) / slightly_* at the joint-range fractions of the
    definitions, on the config-5 drawer (stroke [0, 0.4] m)."""
    b = sg.make(5, 2)
    r = _robot(b)
    x = np.array(b.state0, np.float64)
    st = sg.split_state(x, b.n_scenes, b.n_free, b.n_aux)
    drawer = 1
    lo, hi = (float(v) for v in b.aux_limit[b.aux_off[0] + drawer])
    tk_open = [dict(kind=O, target=drawer, goal=(0, 0, 0), open_frac=0.9)] * 2
    tk_close = [dict(kind=CL, target=drawer, goal=(0, 0, 0), open_frac=0.9)] * 2
    for frac, exp_open, exp_slight in [(0.95, True, True), (0.85, False, True), (0.05, False, False)]:
        st["aux"][b.aux_off[0] + drawer, 0] = lo + frac * (hi - lo)
        v = ot.predicates(b, x, tk_open, r, None, 5, np.zeros(2))
        ind = ot.success(v[0], tk_open[0], 0.0)
        assert (ind["state"], ind["slight"]) == (exp_open, exp_slight)
    st["aux"][b.aux_off[0] + drawer, 0] = lo + 0.005 * (hi - lo)
    v = ot.predicates(b, x, tk_close, r, None, 5, np.zeros(2))
    ind = ot.success(v[0], tk_close[0], aq0=lo + 0.5 * (hi - lo))
    assert ind["state"] and ind["slight"]
    ind = ot.success(v[0], tk_close[0], aq0=lo + 0.04 * (hi - lo))
    assert ind["state"] and not ind["slight"]


def test_episode_bookkeeping_accumulates_collisions():
    """C_t adds the mean force per control step; crossing 5000 N raises
    excessive_collisions once."""
    b = _fetch_batch()
    r = _robot(b)
    tk = [dict(kind=P, target=0, goal=(0, 0, 0), open_frac=0.9)] * b.n_scenes
    ep = ot.Episodes(b, tk, r, n_sub=5)
    x = np.array(b.state0, np.float64)
    ep.begin(x)
    for _ in range(3):
        ep.update(x, np.full(b.n_scenes, 5 * 2000.0))
    assert np.allclose(ep.cumcol, 6000.0)
    assert all(E.count("excessive_collisions") == 1 for E in ep.events)
    assert all(ot.categorize(P, E) == 5 for E in ep.events)
