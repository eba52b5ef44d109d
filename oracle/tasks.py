"""Subtask success predicates, event labels and trajectory categories -- TEST
INFRASTRUCTURE ONLY (the oracle of the task kernels; only ``tests/`` may use it).

Written from the appendix's subtask definitions (success conditions of Pick,
Place, Open, Close), its event definitions (evaluated per step in the order
listed) and its success / failure modes.  Plain float64 Python; it shares no
code with the GPU path.

Readings of points the appendix leaves open or states inconsistently:
  - d is the Euclidean distance in m (the appendix writes a squared norm but
    gives the unit m);
  - is_static takes absolute values of the arm joint velocities and of the
    base x, y, yaw velocities;
  - C_t adds, per control step, the mean over its substeps of the robot's
    total normal contact force;
  - grasped(x): both finger bodies press on x with at least grasp_force in
    the control step's last substep (the smaller finger force >= grasp_force);
  - contact event: F_ee,x goes from 0 to > 0 (the text's ">= 0" is always true);
  - i_e is the list position of e's latest occurrence, -1 when absent;
  - the "success then excessive collisions" modes of Open and Close require
    e_excessive in the list (the text's "not in" would overlap the other modes);
  - Pick: the success modes are tried in the order iv, iii, i, ii (iii must
    precede ii, which it would otherwise never follow); Place: v first, then
    i .. iv; Open / Close: iii, i, ii; failure modes in the order listed;
  - an open / close target must be a joint with limits (a_qmin, a_qmax).

Parity status: pinned by hand-built event lists for every mode
(tests/test_oracle_tasks.py) and by kinematic invariants of the
end-effector position.
"""
from __future__ import annotations

import math

import numpy as np

PICK, PLACE, OPEN, CLOSE = 0, 1, 2, 3

# event names in the appendix's per-step evaluation order
EVENTS = {
    PICK: ["contact", "grasped", "dropped", "success", "excessive_collisions"],
    PLACE: ["grasped", "obj_at_goal", "released_at_goal", "released_outside_goal", "obj_left_goal", "success",
            "excessive_collisions"],
    OPEN: ["contact", "opened", "slightly_opened", "closed", "success", "excessive_collisions"],
    CLOSE: ["contact", "closed", "slightly_closed", "open", "success", "excessive_collisions"],
}
# collision limits of the success / failure conditions, N
COLLISION_LIMIT = {PICK: 5000.0, PLACE: 7500.0, OPEN: 10000.0, CLOSE: 10000.0}


# ------------------------------------------------------------ kinematics
def _rodrigues(axis, angle):
    """Rotation by `angle` about the unit `axis`: exp of the skew matrix."""
    k = np.asarray(axis, np.float64)
    K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
    return np.eye(3) + math.sin(angle) * K + (1.0 - math.cos(angle)) * (K @ K)


def _quat_matrix(wxyz):
    """Rotation matrix of the unit quaternion (w, x, y, z)."""
    w, x, y, z = (float(v) for v in wxyz)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def body_pose(batch, m, q, body):
    """World pose (R, p) of robot body `body` of model m at joint positions q:
    X_body = X_parent X_T X_J, walked from the root."""
    chain = []
    b = body
    while b >= 0:
        chain.append(b)
        b = int(batch.model_parent[m, b])
    R = np.eye(3)
    p = np.zeros(3)
    for j in reversed(chain):
        XR = _quat_matrix(batch.model_xt_rot[m, j])
        Xp = np.asarray(batch.model_xt_pos[m, j], np.float64)
        ax = np.asarray(batch.model_axis[m, j], np.float64)
        p = p + R @ Xp
        R = R @ XR
        if int(batch.model_jtype[m, j]) == 0:
            R = R @ _rodrigues(ax, float(q[j]))
        else:
            p = p + (R @ ax) * float(q[j])
    return R, p


def ee_in_base(batch, m, q, robot):
    """The end-effector point in the base frame."""
    Re, pe = body_pose(batch, m, q, robot["ee_body"])
    Rb, pb = body_pose(batch, m, q, robot["base_body"])
    ee = pe + Re @ np.asarray(robot["ee_offset"], np.float64)
    return Rb.T @ (ee - pb)


# ------------------------------------------------------------ predicates
def predicates(batch, x, tasks, robot, grip, n_sub, cumcol):
    """Per scene: the predicate values and indicators at state x.

    x: flat state (float64 view), tasks: list of dicts (kind, target, goal,
    open_frac), grip: [NF + NA][2] gripper outputs or None, cumcol: C_t per
    scene.  Returns a list of dicts (None for an invalid task)."""
    S = batch.n_scenes
    NF = batch.n_free
    x = np.asarray(x, np.float64)
    out = []
    for s in range(S):
        T = tasks[s]
        kind, tgt = int(T["kind"]), int(T["target"])
        f0, nf = int(batch.free_off[s]), int(batch.free_off[s + 1] - batch.free_off[s])
        a0, na = int(batch.aux_off[s]), int(batch.aux_off[s + 1] - batch.aux_off[s])
        obj = kind in (PICK, PLACE)
        if kind not in (PICK, PLACE, OPEN, CLOSE) or tgt < 0 or (obj and tgt >= nf) or (not obj and tgt >= na):
            out.append(None)
            continue
        if not obj:
            lo, hi = (float(v) for v in batch.aux_limit[a0 + tgt])
            if lo > hi:
                out.append(None)
                continue
        m = int(batch.scene_model[s])
        q = x[16 * s:16 * s + 16]
        qd = x[16 * S + 16 * s:16 * S + 16 * s + 16]
        d_ee = float(np.linalg.norm(ee_in_base(batch, m, q, robot) - np.asarray(robot["ee_rest"], np.float64)))
        arm = range(robot["arm0"], robot["arm0"] + robot["narm"])
        j_arm = max([abs(q[i] - robot["q_rest"][i]) for i in arm], default=0.0)
        qd_arm = max([abs(qd[i]) for i in arm], default=0.0)
        t = robot["torso"]
        j_tor = abs(q[t] - robot["q_rest"][t]) if t >= 0 else 0.0
        static = (qd_arm <= 0.2 and abs(qd[robot["base_x"]]) <= 0.05 and abs(qd[robot["base_y"]]) <= 0.05
                  and abs(qd[robot["base_yaw"]]) <= 0.05)
        row = f0 + tgt if obj else NF + a0 + tgt
        f_ee = float(grip[row][0]) / n_sub if grip is not None else 0.0
        f_fing = float(grip[row][1]) if grip is not None else 0.0
        v = dict(d_ee=d_ee, j_arm=float(j_arm), j_torso=float(j_tor), qd_arm=float(qd_arm), f_ee=f_ee,
                 f_finger=f_fing, static=static, cumcol=float(cumcol[s]), kind=kind)
        v["contact"] = f_ee > 0.0
        v["excessive"] = cumcol[s] > COLLISION_LIMIT[kind]
        if obj:
            xo = x[32 * S + 16 * row:32 * S + 16 * row + 3]
            v["d_goal"] = float(np.linalg.norm(xo - np.asarray(T["goal"], np.float64)))
            v["grasped"] = f_fing >= robot["grasp_force"]
            v["aq"] = 0.0
        else:
            v["d_goal"] = 0.0
            v["grasped"] = False
            v["aq"] = float(x[32 * S + 16 * NF + 4 * (a0 + tgt)])
            v["lo"], v["hi"] = lo, hi
        out.append(v)
    return out


def success(v, task, aq0):
    """The subtask's success condition (App. A.2) and its indicator set."""
    kind = v["kind"]
    col_ok = v["cumcol"] <= COLLISION_LIMIT[kind]
    ind = dict(grasped=v["grasped"], contact=v["contact"], excessive=v["excessive"])
    if kind == PICK:
        ok = v["grasped"] and v["d_ee"] <= 0.05 and v["j_arm"] <= 0.6 and v["static"] and col_ok
    elif kind == PLACE:
        ind["at_goal"] = v["d_goal"] <= 0.15
        ok = (not v["grasped"] and v["d_goal"] <= 0.15 and v["d_ee"] <= 0.05 and v["j_arm"] <= 0.2
              and v["j_torso"] <= 0.01 and v["static"] and col_ok)
    else:
        span = v["hi"] - v["lo"]
        if kind == OPEN:
            state = v["aq"] >= task["open_frac"] * span + v["lo"]       # open(a)
            slight = v["aq"] >= 0.1 * span + v["lo"]                    # slightly_opened(a)
        else:
            state = v["aq"] <= 0.01 * span + v["lo"]                    # close(a)
            slight = v["aq"] < aq0 - 0.05 * span                        # slightly_closed(a)
        ind["state"], ind["slight"] = state, slight
        ok = (state and v["d_ee"] <= 0.05 and v["j_arm"] <= 0.2 and v["j_torso"] <= 0.01 and v["static"]
              and col_ok)
    ind["success"] = ok
    return ind


def step_events(kind, a, b):
    """Events between indicator sets a (step t-1) and b (step t), in order."""
    rise = lambda k: (not a[k]) and b[k]
    fall = lambda k: a[k] and not b[k]
    if kind == PICK:
        hits = [rise("contact"), rise("grasped"), fall("grasped"), rise("success"), rise("excessive")]
    elif kind == PLACE:
        hits = [rise("grasped"), rise("at_goal"), b["at_goal"] and fall("grasped"),
                (not b["at_goal"]) and fall("grasped"), fall("at_goal"), rise("success"), rise("excessive")]
    else:
        hits = [rise("contact"), rise("state"), rise("slight"), fall("state"), rise("success"), rise("excessive")]
    return [EVENTS[kind][i] for i, h in enumerate(hits) if h]


class Episodes:
    """Episode bookkeeping of a batch: C_t, start values, indicators, events."""

    def __init__(self, batch, tasks, robot, n_sub):
        self.batch, self.tasks, self.robot, self.n_sub = batch, tasks, robot, n_sub
        S = batch.n_scenes
        self.cumcol = np.zeros(S)
        self.aq0 = np.zeros(S)
        self.d0 = np.zeros(S)
        self.ind = [None] * S
        self.events = [[] for _ in range(S)]
        self.t = np.zeros(S, np.int64)
        self.values = None

    def begin(self, x, grip=None, mask=None):
        v = predicates(self.batch, x, self.tasks, self.robot, grip, self.n_sub, np.zeros(self.batch.n_scenes))
        self.values = v
        for s in range(self.batch.n_scenes):
            if mask is not None and not mask[s]:
                continue
            self.cumcol[s] = 0.0
            self.t[s] = 0
            self.events[s] = []
            if v[s] is None:
                self.ind[s] = None
                continue
            self.aq0[s] = v[s]["aq"]
            self.d0[s] = v[s]["d_goal"]
            self.ind[s] = success(v[s], self.tasks[s], self.aq0[s])

    def update(self, x, robot_force, grip=None):
        cum = self.cumcol + np.asarray(robot_force, np.float64) / self.n_sub
        v = predicates(self.batch, x, self.tasks, self.robot, grip, self.n_sub, cum)
        self.values = v
        for s in range(self.batch.n_scenes):
            if v[s] is None or self.ind[s] is None:
                self.ind[s] = None
                continue
            b = success(v[s], self.tasks[s], self.aq0[s])
            self.events[s] += step_events(int(self.tasks[s]["kind"]), self.ind[s], b)
            self.ind[s] = b
            self.cumcol[s] = cum[s]
            self.t[s] += 1


# ------------------------------------------------------------ categories
def _idx(E, e):
    """i_e: position of e's latest occurrence in E, -1 when absent."""
    return max((i for i, x in enumerate(E) if x == e), default=-1)


def categorize(kind, E, d0=0.0):
    """Success / failure mode (roman numeral as 1, 2, ...; 0 none) of an
    event list E (App. A.3)."""
    i = lambda e: _idx(E, e)
    has = lambda e: e in E
    exc = has("excessive_collisions")
    if kind == PICK:
        if has("success"):
            modes = {
                1: E == ["contact", "grasped", "success"],
                2: E[:2] == ["contact", "grasped"] and len(E) > 3 and not exc,
                3: has("dropped") and i("dropped") > i("grasped") and not exc,
                4: exc,
            }
            order = [4, 3, 1, 2]
        else:
            modes = {
                5: exc,
                6: E == [],
                7: E == ["contact"],
                8: has("dropped") and i("dropped") > i("grasped") and not exc,
                9: has("grasped") and i("grasped") > i("dropped") and not exc,
            }
            order = [5, 6, 7, 8, 9]
    elif kind == PLACE:
        near0 = d0 <= 0.15
        if has("success"):
            modes = {
                1: len(E) <= 4 and (has("released_at_goal") or near0) and i("obj_left_goal") <= i("obj_at_goal")
                and not exc,
                2: len(E) <= 4 and (has("released_outside_goal") or not near0)
                and i("obj_left_goal") <= i("obj_at_goal") and not exc,
                3: i("obj_at_goal") < i("obj_left_goal") and not exc,
                4: len(E) > 4 and i("obj_at_goal") > i("obj_left_goal") and not exc,
                5: exc,
            }
            order = [5, 1, 2, 3, 4]
        else:
            placed_latest = (len(E) <= 2 and near0) or (
                i("released_at_goal") > i("released_outside_goal") and i("released_at_goal") > i("grasped"))
            dropped_latest = (len(E) <= 2 and not near0) or (
                i("released_outside_goal") > i("released_at_goal") and i("released_outside_goal") > i("grasped"))
            at, left = has("obj_at_goal"), i("obj_left_goal") > i("obj_at_goal")
            modes = {
                6: exc,
                7: E == [] and not exc,
                8: len(E) > 0 and not has("obj_at_goal") and not exc,
                9: at and placed_latest and left and not exc,
                10: at and dropped_latest and left and not exc,
                11: at and i("grasped") > i("released_at_goal") and i("grasped") > i("released_outside_goal")
                and not exc,
            }
            order = [6, 7, 8, 9, 10, 11]
            for k in order:
                if modes[k]:
                    return k
            return 12  # too slow: no other failure mode applies
    else:
        reach, slight, leave = ("opened", "slightly_opened", "closed") if kind == OPEN else \
            ("closed", "slightly_closed", "open")
        if has("success"):
            modes = {1: not exc and i(reach) > i(leave), 2: not exc and i(reach) < i(leave), 3: exc}
            order = [3, 1, 2]
        else:
            if kind == OPEN:
                undone = has("closed") and i("closed") > i("opened") and i("closed") > i("slightly_opened")
            else:
                undone = has("closed") and i("open") > i("closed") and i("open") > i("slightly_closed")
            modes = {
                4: exc,
                5: not has("contact") and not exc,
                6: undone and not exc,
                7: i(slight) > i(reach) and i(slight) > i(leave) and not exc,
                8: has(reach),
            }
            order = [4, 5, 6, 7, 8]
            for k in order:
                if modes[k]:
                    return k
            return 9  # can't open / close: no other failure mode applies
    for k in order:
        if modes[k]:
            return k
    return 0
