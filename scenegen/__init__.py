"""Seeded synthetic scene batches for the batched rigid-body step.

This module only draws inputs: robot descriptions, furniture boxes, free
objects, initial states and control sequences.  It contains none of the
physics step's arithmetic (no kinematics, dynamics, contact or solver code);
both the CPU oracle and the GPU library read the arrays it produces, each with
its own reader.

Workload shapes follow the paper's Interact benchmark (Sec. 4.2: a Fetch
mobile manipulator colliding with several dynamic objects in an apartment,
100 Hz simulation / 20 Hz control, up to 4096 parallel environments) and the
robot initialisation noise of Appendix A.1 (arm joints perturbed by
clip(N(0, 0.1), -0.2, 0.2), base position by clip(N(0, 0.1), -0.2, 0.2), base
yaw by clip(N(0, 0.25), -0.5, 0.5), zero velocities, z axis up).  The
apartment scenes, object meshes and robot description of the paper are not
available; boxes, spheres and a generic 15-DoF mobile manipulator stand in.

Every float is rounded to float32 before it is stored so that the FP64
oracle and the FP32 GPU path start from bit-identical inputs.

Scene ``s`` of configuration ``c`` draws from ``SeedSequence([seed, c, s])``;
its controls at control step ``t`` from ``SeedSequence([seed, c, s, t])``
(or the block ``t // 10`` for resampled PD targets), so any subset of scenes
is identical to the same scenes inside the full batch.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

NDOF = 16          # padded joint-space width of the robot articulation
SMAX = 128         # max robot collision spheres per model
BASE_SEED = 20241217

CTRL_TORQUE = 0    # controls are joint torques / forces
CTRL_PD = 1        # controls are PD targets (position, or velocity for base DoFs)
CTRL_TORQUE_HOLD = 2  # controls are torques added to an implicit PD hold
CTRL_ACTIONS = 3   # controls are normalized actions in [-1, 1] mapped to PD targets

# normalized-action channel of a DoF (target computed once per control step
# from the action a, clipped to [-1, 1], and the state q at the step start)
ACT_DELTA = 0         # position target q + a * scale (joint delta position)
ACT_BASE_FWD_X = 1    # velocity target a_fwd * scale * cos(yaw) (base linear velocity, world x)
ACT_BASE_FWD_Y = 2    # velocity target a_fwd * scale * sin(yaw) (a_fwd: the ACT_BASE_FWD_X action)
ACT_BASE_YAW = 3      # velocity target a * scale (base angular velocity)
ACT_ABSOLUTE = 4      # position target (a + 1) / 2 * scale (gripper opening)

JT_REVOLUTE = 0
JT_PRISMATIC = 1

FREE_BOX = 0
FREE_SPHERE = 1

SPH_SKIP_FLOOR = 1  # sphere flag: no contact with the scene's first plane


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


@dataclasses.dataclass
class SceneBatch:
    """Flat arrays describing ``n_scenes`` independent scenes (CSR-packed)."""
    name: str
    n_scenes: int
    # physics parameters
    h: float
    n_sub: int
    pgs_iters: int
    mu: float
    baumgarte: float
    margin: float
    gravity: tuple
    control_mode: int
    contact_cap: int
    n_steps: int
    robot_contact_cap: int
    # robot models
    model_nb: np.ndarray        # int32[M]
    model_parent: np.ndarray    # int32[M,16]
    model_jtype: np.ndarray     # int32[M,16]
    model_axis: np.ndarray      # f32[M,16,3]   joint axis in the joint frame
    model_xt_rot: np.ndarray    # f32[M,16,4]   joint frame rotation in parent (wxyz)
    model_xt_pos: np.ndarray    # f32[M,16,3]   joint frame origin in parent
    model_mass: np.ndarray      # f32[M,16]
    model_com: np.ndarray       # f32[M,16,3]   body frame
    model_inertia: np.ndarray   # f32[M,16,6]   about COM, body frame: xx yy zz xy xz yz
    model_kp: np.ndarray        # f32[M,16]
    model_kd: np.ndarray        # f32[M,16]
    model_veldof: np.ndarray    # int32[M,16]   1: PD target is a velocity
    model_armature: np.ndarray  # f32[M,16]     rotor inertia added to the mass-matrix diagonal
    model_damping: np.ndarray   # f32[M,16]     viscous joint damping (integrated implicitly)
    model_act_kind: np.ndarray  # int32[M,16]   normalized-action channel kind (ACT_*)
    model_act_scale: np.ndarray  # f32[M,16]    its scale (rad, m, m/s or rad/s per unit action)
    model_nsph: np.ndarray      # int32[M]
    model_sph_body: np.ndarray  # int32[M,SMAX]
    model_sph: np.ndarray       # f32[M,SMAX,4] local centre + radius
    model_sph_flags: np.ndarray  # int32[M,SMAX]
    # scenes
    scene_model: np.ndarray     # int32[S]
    free_off: np.ndarray        # int32[S+1]
    static_off: np.ndarray      # int32[S+1]
    plane_off: np.ndarray       # int32[S+1]
    aux_off: np.ndarray         # int32[S+1]
    scene_hold: np.ndarray      # f32[S,16] hold targets (torque-hold mode)
    free_type: np.ndarray       # int32[NF]
    free_size: np.ndarray       # f32[NF,3] half extents, or (radius, 0, 0)
    free_mass: np.ndarray       # f32[NF]
    free_inertia: np.ndarray    # f32[NF,3] principal moments, body frame
    static_box: np.ndarray      # f32[NS,6] centre, half extents
    plane: np.ndarray           # f32[NP,4] n, d with n.x = d
    aux_type: np.ndarray        # int32[NA]
    aux_rot: np.ndarray         # f32[NA,4] joint frame in world (wxyz)
    aux_pos: np.ndarray         # f32[NA,3]
    aux_axis: np.ndarray        # f32[NA,3] joint frame
    aux_box: np.ndarray         # f32[NA,6] OBB centre offset (body frame), half extents
    aux_mass: np.ndarray        # f32[NA]
    aux_inertia: np.ndarray     # f32[NA,3] principal moments about the box centre
    aux_limit: np.ndarray       # f32[NA,2] lo, hi (lo > hi: no limit)
    state0: np.ndarray          # f32[state_floats]
    cfg_id: int = 0
    seed: int = BASE_SEED
    # control recipe
    ctrl_kind: str = "torque_normal"
    ctrl_sigma: float = 2.0
    ctrl_rest: np.ndarray | None = None   # f32[M,16]
    ctrl_block: int = 10
    ctrl_clip: float = 0.3
    notes: str = ""

    @property
    def n_free(self):
        return int(self.free_off[-1])

    @property
    def n_aux(self):
        return int(self.aux_off[-1])

    @property
    def state_floats(self):
        return state_floats(self.n_scenes, self.n_free, self.n_aux)

    def controls(self, step: int, scenes=None) -> np.ndarray:
        """Controls u[len(scenes),16] for control step ``step`` (float32);
        ``scenes`` are rows of this batch (default: all).  The random stream
        of a scene is keyed by its id in the batch it was generated in, so a
        subset draws the same controls as the full batch."""
        rows = range(self.n_scenes) if scenes is None else scenes
        ids = self.scene_ids()
        out = np.zeros((len(rows), NDOF), np.float32)
        for r, row in enumerate(rows):
            s = int(ids[row])
            m = int(self.scene_model[row])
            nb = int(self.model_nb[m])
            if self.ctrl_kind == "torque_normal":
                g = _rng(self.seed, self.cfg_id, s, step)
                out[r, :nb] = f32(g.normal(0.0, self.ctrl_sigma, nb))
            elif self.ctrl_kind == "random_actions":
                # normalized actions drawn uniformly from [-1, 1] and clipped
                # to [-c, c], fresh every control step
                g = _rng(self.seed, self.cfg_id, s, 2_000_000 + step)
                c = self.ctrl_clip
                out[r, :nb] = f32(np.clip(g.uniform(-1.0, 1.0, nb), -c, c))
            elif self.ctrl_kind == "pd_targets":
                g = _rng(self.seed, self.cfg_id, s, 1_000_000 + step // self.ctrl_block)
                rest = self.ctrl_rest[m]
                u = np.zeros(NDOF)
                for j in range(nb):
                    if self.model_veldof[m, j]:
                        u[j] = g.uniform(-0.3, 0.3)
                    else:
                        u[j] = rest[j] + np.clip(g.normal(0.0, 0.3), -0.6, 0.6)
                # fingers (last two prismatic DoFs) stay in their stroke
                if nb == 15:
                    u[13] = g.uniform(0.0, 0.05)
                    u[14] = g.uniform(0.0, 0.05)
                out[r] = f32(u)
            else:
                raise ValueError(self.ctrl_kind)
        return out

    def push_goals(self, scenes=None) -> np.ndarray:
        """Differentiation workload: per scene a seeded goal for its first free
        body (the pushed box), its start position moved by U[-0.1, 0.1] m in
        x and y ([len(scenes), 3], float64)."""
        rows = range(self.n_scenes) if scenes is None else scenes
        ids = self.scene_ids()
        fr = split_state(self.state0, self.n_scenes, self.n_free, self.n_aux)["free"]
        out = np.zeros((len(rows), 3))
        for r, row in enumerate(rows):
            g = _rng(self.seed, self.cfg_id, int(ids[row]), 3_000_000)
            out[r] = fr[int(self.free_off[row]), 0:3]
            out[r, 0:2] += g.uniform(-0.1, 0.1, 2)
        return out

    def control_sequence(self, n_steps=None, scenes=None) -> np.ndarray:
        n = self.n_steps if n_steps is None else n_steps
        return np.stack([self.controls(t, scenes) for t in range(n)])

    def subset(self, scenes) -> "SceneBatch":
        """The same scenes as a smaller batch (models are kept whole)."""
        scenes = list(scenes)
        S = len(scenes)
        def gather_csr(off, arrays):
            new_off = np.zeros(S + 1, np.int32)
            parts = [[] for _ in arrays]
            for r, s in enumerate(scenes):
                a, b = int(off[s]), int(off[s + 1])
                new_off[r + 1] = new_off[r] + (b - a)
                for k, arr in enumerate(arrays):
                    parts[k].append(arr[a:b])
            out = [np.concatenate(p) if p else arr[:0] for p, arr in zip(parts, arrays)]
            return new_off, out
        fo, (ft, fs, fm, fi) = gather_csr(self.free_off, [self.free_type, self.free_size, self.free_mass, self.free_inertia])
        so, (sb,) = gather_csr(self.static_off, [self.static_box])
        po, (pl,) = gather_csr(self.plane_off, [self.plane])
        ao, aux = gather_csr(self.aux_off, [self.aux_type, self.aux_rot, self.aux_pos, self.aux_axis,
                                            self.aux_box, self.aux_mass, self.aux_inertia, self.aux_limit])
        st = split_state(self.state0, self.n_scenes, self.n_free, self.n_aux)
        fidx = np.concatenate([np.arange(self.free_off[s], self.free_off[s + 1]) for s in scenes]).astype(np.int64)
        aidx = np.concatenate([np.arange(self.aux_off[s], self.aux_off[s + 1]) for s in scenes]).astype(np.int64)
        state0 = join_state(st["q"][scenes], st["qd"][scenes], st["free"][fidx], st["aux"][aidx])
        sub = dataclasses.replace(
            self, n_scenes=S, scene_model=self.scene_model[scenes].copy(),
            free_off=fo, static_off=so, plane_off=po, aux_off=ao,
            scene_hold=self.scene_hold[scenes].copy(),
            free_type=ft, free_size=fs, free_mass=fm, free_inertia=fi,
            static_box=sb, plane=pl,
            aux_type=aux[0], aux_rot=aux[1], aux_pos=aux[2], aux_axis=aux[3],
            aux_box=aux[4], aux_mass=aux[5], aux_inertia=aux[6], aux_limit=aux[7],
            state0=state0)
        base = self.scene_ids()
        sub._scene_ids = [base[s] for s in scenes]
        return sub

    def scene_ids(self):
        return getattr(self, "_scene_ids", list(range(self.n_scenes)))

    def controls_for(self, step):
        """Controls at ``step`` for every scene of this batch."""
        return self.controls(step)


def state_floats(S, NF, NA):
    return 32 * S + 16 * NF + 4 * NA


def split_state(x, S, NF, NA):
    """Views of a flat state: q[S,16], qd[S,16], free[NF,16], aux[NA,4]."""
    x = np.asarray(x)
    q = x[: 16 * S].reshape(S, 16)
    qd = x[16 * S: 32 * S].reshape(S, 16)
    fr = x[32 * S: 32 * S + 16 * NF].reshape(NF, 16)
    ax = x[32 * S + 16 * NF: 32 * S + 16 * NF + 4 * NA].reshape(NA, 4)
    return {"q": q, "qd": qd, "free": fr, "aux": ax}


def join_state(q, qd, free, aux):
    return np.concatenate([np.asarray(q, np.float32).ravel(), np.asarray(qd, np.float32).ravel(),
                           np.asarray(free, np.float32).ravel(), np.asarray(aux, np.float32).ravel()])


def _rng(*key):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(k) for k in key])))


def _quat_z(yaw):
    return np.array([math.cos(yaw / 2), 0.0, 0.0, math.sin(yaw / 2)])


def _box_inertia(m, full):
    a, b, c = full
    return np.array([m * (b * b + c * c) / 12, m * (a * a + c * c) / 12, m * (a * a + b * b) / 12])


# ----------------------------------------------------------------------------
# robot models
# ----------------------------------------------------------------------------

class _ModelBuilder:
    def __init__(self):
        self.bodies = []
        self.spheres = []

    def body(self, parent, jtype, axis, pos, mass, com, inertia_diag, kp=0.0, kd=0.0, veldof=0,
             rot=(1.0, 0.0, 0.0, 0.0), armature=0.0, damping=0.0, act=(ACT_DELTA, 0.1)):
        """``act``: (kind, scale) of the DoF's normalized-action channel (ACT_*)."""
        self.bodies.append(dict(parent=parent, jtype=jtype, axis=np.array(axis, float), pos=np.array(pos, float),
                                rot=np.array(rot, float), mass=mass, com=np.array(com, float),
                                inertia=np.array(list(inertia_diag) + [0.0, 0.0, 0.0]), kp=kp, kd=kd, veldof=veldof,
                                armature=armature, damping=damping, act=act))
        return len(self.bodies) - 1

    def segment(self, body, a, b, r, n, flags=0):
        a = np.array(a, float)
        b = np.array(b, float)
        for k in range(n):
            t = 0.5 if n == 1 else k / (n - 1)
            self.spheres.append((body, a + t * (b - a), r, flags))

    def arrays(self):
        nb = len(self.bodies)
        assert nb <= NDOF and len(self.spheres) <= SMAX
        d = {k: np.zeros(s, t) for k, s, t in [
            ("parent", NDOF, np.int32), ("jtype", NDOF, np.int32), ("axis", (NDOF, 3), np.float64),
            ("xt_rot", (NDOF, 4), np.float64), ("xt_pos", (NDOF, 3), np.float64), ("mass", NDOF, np.float64),
            ("com", (NDOF, 3), np.float64), ("inertia", (NDOF, 6), np.float64), ("kp", NDOF, np.float64),
            ("kd", NDOF, np.float64), ("veldof", NDOF, np.int32), ("armature", NDOF, np.float64),
            ("damping", NDOF, np.float64), ("act_kind", NDOF, np.int32), ("act_scale", NDOF, np.float64),
            ("sph_body", SMAX, np.int32),
            ("sph", (SMAX, 4), np.float64), ("sph_flags", SMAX, np.int32)]}
        d["parent"][:] = -1
        d["xt_rot"][:, 0] = 1.0
        d["axis"][:, 2] = 1.0
        for i, b in enumerate(self.bodies):
            d["parent"][i] = b["parent"]
            d["jtype"][i] = b["jtype"]
            d["axis"][i] = b["axis"] / np.linalg.norm(b["axis"])
            d["xt_rot"][i] = b["rot"]
            d["xt_pos"][i] = b["pos"]
            d["mass"][i] = b["mass"]
            d["com"][i] = b["com"]
            d["inertia"][i] = b["inertia"]
            d["kp"][i] = b["kp"]
            d["kd"][i] = b["kd"]
            d["veldof"][i] = b["veldof"]
            d["armature"][i] = b["armature"]
            d["damping"][i] = b["damping"]
            d["act_kind"][i] = b["act"][0]
            d["act_scale"][i] = b["act"][1]
        for k, (body, c, r, fl) in enumerate(self.spheres):
            d["sph_body"][k] = body
            d["sph"][k, :3] = c
            d["sph"][k, 3] = r
            d["sph_flags"][k] = fl
        d["nb"] = nb
        d["nsph"] = len(self.spheres)
        return d


def arm7_model(g):
    """Fixed-base 7-revolute arm: capsule links approximated by 3 spheres each.

    Joint axes z, y, z, y, z, y, z; link i extends along its local +z by L_i;
    the base joint sits 0.1 m above the origin.  Capsule radius 0.04 m.
    Inertia: solid cylinder of length L and radius r about its centre.
    Every joint carries a rotor inertia of 0.01 kg m^2 and a viscous damping
    of 0.1 N m s/rad: without them the roll joints (axis along the link, inertia
    m r^2 / 2 ~ 1e-3 kg m^2) spin up without bound under N(0, 2) N m torques.
    """
    mb = _ModelBuilder()
    r = 0.04
    axes = [(0, 0, 1), (0, 1, 0), (0, 0, 1), (0, 1, 0), (0, 0, 1), (0, 1, 0), (0, 0, 1)]
    L = g.uniform(0.1, 0.4, 7)
    m = g.uniform(0.5, 3.0, 7)
    prev = -1
    for i in range(7):
        pos = (0.0, 0.0, 0.1) if i == 0 else (0.0, 0.0, float(L[i - 1]))
        Ia = m[i] * r * r / 2
        Ip = m[i] * (3 * r * r + L[i] ** 2) / 12
        prev = mb.body(prev, JT_REVOLUTE, axes[i], pos, float(m[i]), (0.0, 0.0, L[i] / 2), (Ip, Ip, Ia),
                       armature=0.01, damping=0.1)
        mb.segment(prev, (0, 0, 0), (0, 0, float(L[i])), r, 3)
    return mb.arrays()


FETCH_REST = np.zeros(NDOF)
# base x, y, yaw are velocity DoFs; torso, head pan/tilt, 7 arm joints, 2 fingers
FETCH_REST[3] = 0.15
FETCH_REST[5] = 0.3
FETCH_REST[6:13] = [0.0, 0.9, 0.0, -0.5, 0.0, 0.6, 0.0]
FETCH_REST[13] = 0.03
FETCH_REST[14] = 0.03


def fetch_like_model(g):
    """Generic 15-DoF mobile manipulator (dimensions chosen here, not a real robot).

    DoFs: 0 base x (prismatic, massless), 1 base y (prismatic, massless),
    2 base yaw (revolute z), 3 torso lift (prismatic z), 4-5 head pan/tilt,
    6-12 arm (axes z, y, x, y, x, y, x), 13-14 fingers (prismatic +-y).
    18 geometric links (13 moving + 5 fixed links merged into their parents),
    each approximated by U{2..6} spheres.
    """
    mb = _ModelBuilder()
    n = lambda: int(g.integers(2, 7))
    px = mb.body(-1, JT_PRISMATIC, (1, 0, 0), (0, 0, 0), 0.0, (0, 0, 0), (0, 0, 0), kd=2000.0, veldof=1,
                 act=(ACT_BASE_FWD_X, 1.0))
    py = mb.body(px, JT_PRISMATIC, (0, 1, 0), (0, 0, 0), 0.0, (0, 0, 0), (0, 0, 0), kd=2000.0, veldof=1,
                 act=(ACT_BASE_FWD_Y, 1.0))
    base = mb.body(py, JT_REVOLUTE, (0, 0, 1), (0, 0, 0), 60.0, (0, 0, 0.2),
                   _box_inertia(60.0, (0.56, 0.56, 0.36)), kd=500.0, veldof=1, act=(ACT_BASE_YAW, 1.0))
    torso = mb.body(base, JT_PRISMATIC, (0, 0, 1), (-0.08, 0, 0.37), 10.0, (0, 0, 0.3),
                    _box_inertia(10.0, (0.2, 0.24, 0.6)), kp=5000.0, kd=500.0, armature=0.1)
    hpan = mb.body(torso, JT_REVOLUTE, (0, 0, 1), (0.05, 0, 0.62), 2.0, (0.05, 0, 0.05),
                   _box_inertia(2.0, (0.2, 0.24, 0.1)), kp=200.0, kd=20.0, armature=0.01)
    htilt = mb.body(hpan, JT_REVOLUTE, (0, 1, 0), (0.1, 0, 0.1), 1.5, (0.05, 0, 0),
                    _box_inertia(1.5, (0.15, 0.25, 0.1)), kp=200.0, kd=20.0, armature=0.01)
    arm_axes = [(0, 0, 1), (0, 1, 0), (1, 0, 0), (0, 1, 0), (1, 0, 0), (0, 1, 0), (1, 0, 0)]
    arm_pos = [(0.12, 0, 0.35), (0.12, 0, 0.06), (0.2, 0, 0), (0.15, 0, 0), (0.14, 0, 0), (0.14, 0, 0), (0.14, 0, 0)]
    arm_len = [0.12, 0.2, 0.15, 0.14, 0.14, 0.14, 0.16]
    arm_m = [2.5, 2.2, 2.0, 1.8, 1.5, 1.2, 0.9]
    arm_r = [0.07, 0.065, 0.06, 0.055, 0.05, 0.05, 0.045]
    prev = torso
    arm = []
    for k in range(7):
        L = arm_len[k]
        prev = mb.body(prev, JT_REVOLUTE, arm_axes[k], arm_pos[k], arm_m[k], (L / 2, 0, 0),
                       _box_inertia(arm_m[k], (L, 2 * arm_r[k], 2 * arm_r[k])), kp=1000.0, kd=100.0,
                       armature=0.02)
        arm.append(prev)
    fl = mb.body(arm[-1], JT_PRISMATIC, (0, 1, 0), (0.16, 0, 0), 0.1, (0.03, 0, 0),
                 _box_inertia(0.1, (0.06, 0.015, 0.03)), kp=500.0, kd=50.0, armature=0.001, act=(ACT_ABSOLUTE, 0.05))
    fr = mb.body(arm[-1], JT_PRISMATIC, (0, -1, 0), (0.16, 0, 0), 0.1, (0.03, 0, 0),
                 _box_inertia(0.1, (0.06, 0.015, 0.03)), kp=500.0, kd=50.0, armature=0.001, act=(ACT_ABSOLUTE, 0.05))
    # geometric links: (body, segment a, segment b, radius, flags)
    links = [
        (base, (-0.18, 0, 0.2), (0.18, 0, 0.2), 0.2, SPH_SKIP_FLOOR),          # base
        (base, (0.3, -0.16, 0.09), (0.3, 0.16, 0.09), 0.08, SPH_SKIP_FLOOR),   # bumper (fixed)
        (base, (0.2, 0, 0.32), (0.24, 0, 0.32), 0.05, SPH_SKIP_FLOOR),         # laser (fixed)
        (base, (-0.2, -0.12, 0.38), (-0.2, -0.08, 0.38), 0.04, SPH_SKIP_FLOOR),  # estop (fixed)
        (base, (-0.08, 0, 0.38), (-0.08, 0, 0.7), 0.1, SPH_SKIP_FLOOR),        # torso column (fixed)
        (torso, (0, 0, 0.05), (0, 0, 0.6), 0.11, 0),                           # torso lift
        (hpan, (0, 0, 0.04), (0.1, 0, 0.08), 0.09, 0),                         # head pan
        (htilt, (0.0, 0, 0), (0.12, 0, 0), 0.08, 0),                           # head tilt
        (arm[0], (0, 0, 0), (0.12, 0, 0.06), arm_r[0], 0),                     # shoulder pan
    ]
    for k in range(1, 7):
        links.append((arm[k], (0, 0, 0), (arm_len[k], 0, 0), arm_r[k], 0))
    links.append((arm[-1], (0.1, 0, 0), (0.16, 0, 0), 0.05, 0))              # gripper palm (fixed)
    links.append((fl, (0.0, 0.01, 0), (0.06, 0.01, 0), 0.015, 0))           # finger L
    links.append((fr, (0.0, -0.01, 0), (0.06, -0.01, 0), 0.015, 0))         # finger R
    assert len(links) == 18
    for body, a, b, r, flags in links:
        mb.segment(body, a, b, r, n(), flags)
    return mb.arrays()


# Bodies and DoFs of the Fetch-like model as the subtask predicates use them:
# end effector = the last arm link with the point between the fingers, base
# frame = the yaw body, fingers = the two prismatic finger bodies.  The
# end-effector rest position is the caller's (e.g. the point at FETCH_REST).
FETCH_TASK_ROBOT = dict(ee_body=12, base_body=2, base_x=0, base_y=1, base_yaw=2, arm0=6, narm=7, torso=3,
                        finger_l=13, finger_r=14, ee_bodies=(1 << 12) | (1 << 13) | (1 << 14),
                        ee_offset=(0.19, 0.0, 0.0), q_rest=tuple(float(v) for v in FETCH_REST), grasp_force=0.5)

TASK_PICK, TASK_PLACE, TASK_OPEN, TASK_CLOSE = 0, 1, 2, 3


def tasks(batch, kinds=(TASK_PICK, TASK_PLACE, TASK_OPEN, TASK_CLOSE), seed=BASE_SEED):
    """Per-scene subtasks (list of dicts kind, target, goal, open_frac).

    Scene s takes kinds[s % len(kinds)] (a kind whose target does not exist
    in the scene falls back to pick / place); draws come from
    SeedSequence([seed, 1000 + cfg, s]): a random free body (pick, place), a
    place goal within 0.3 m of that body's start position in x and y, a
    random door / drawer joint (open, close) and open_frac 0.75 for every
    fourth scene (the fridge case) else 0.9."""
    ids = batch.scene_ids()
    st = split_state(batch.state0, batch.n_scenes, batch.n_free, batch.n_aux)
    out = []
    for s in range(batch.n_scenes):
        g = _rng(seed, 1000 + batch.cfg_id, int(ids[s]))
        kind = int(kinds[s % len(kinds)])
        nf = int(batch.free_off[s + 1] - batch.free_off[s])
        na = int(batch.aux_off[s + 1] - batch.aux_off[s])
        if kind in (TASK_OPEN, TASK_CLOSE) and na == 0:
            kind = TASK_PICK if kind == TASK_OPEN else TASK_PLACE
        t = dict(kind=kind, target=0, goal=(0.0, 0.0, 0.0), open_frac=0.75 if int(ids[s]) % 4 == 3 else 0.9)
        if kind in (TASK_PICK, TASK_PLACE):
            t["target"] = int(g.integers(0, max(nf, 1)))
            if nf:
                p = st["free"][batch.free_off[s] + t["target"], :3].astype(np.float64)
                t["goal"] = (float(p[0] + g.uniform(-0.3, 0.3)), float(p[1] + g.uniform(-0.3, 0.3)), float(p[2]))
        else:
            t["target"] = int(g.integers(0, na))
        out.append(t)
    return out


def _stack_models(models):
    keys = ["parent", "jtype", "axis", "xt_rot", "xt_pos", "mass", "com", "inertia", "kp", "kd", "veldof",
            "armature", "damping", "act_kind", "act_scale", "sph_body", "sph", "sph_flags"]
    out = {k: np.stack([m[k] for m in models]) for k in keys}
    out["nb"] = np.array([m["nb"] for m in models], np.int32)
    out["nsph"] = np.array([m["nsph"] for m in models], np.int32)
    return out


# ----------------------------------------------------------------------------
# scene content
# ----------------------------------------------------------------------------

ROOM = 3.0  # walls at x, y = +-ROOM


def _room_planes(walls=True):
    p = [(0.0, 0.0, 1.0, 0.0)]
    if walls:
        p += [(1.0, 0.0, 0.0, -ROOM), (-1.0, 0.0, 0.0, -ROOM), (0.0, 1.0, 0.0, -ROOM), (0.0, -1.0, 0.0, -ROOM)]
    return p


def _furniture(g, n, spawn, clear=1.5):
    """n axis-aligned boxes, extents U[0.2, 2] m, on the floor, inside the room,
    outside a clear disc around the robot spawn; overlaps between boxes allowed.
    Positions are drawn in blocks of 64 candidates; a box whose extents leave no
    admissible position after 4 blocks is shrunk by 20 % and tried again."""
    out = []
    for _ in range(n):
        ext = g.uniform(0.2, 2.0, 3)
        while True:
            half = ext / 2
            found = False
            for _blk in range(4):
                cx = g.uniform(-ROOM + half[0], ROOM - half[0], 64)
                cy = g.uniform(-ROOM + half[1], ROOM - half[1], 64)
                dx = np.maximum(np.abs(spawn[0] - cx) - half[0], 0.0)
                dy = np.maximum(np.abs(spawn[1] - cy) - half[1], 0.0)
                ok = np.nonzero(dx * dx + dy * dy >= clear * clear)[0]
                if len(ok):
                    cx, cy = float(cx[ok[0]]), float(cy[ok[0]])
                    found = True
                    break
            if found:
                break
            ext = ext * 0.8
        out.append((cx, cy, half[2], half[0], half[1], half[2]))
    return out


def _inside_any(p, boxes, pad):
    if len(boxes) == 0:
        return False
    b = boxes if isinstance(boxes, np.ndarray) else np.asarray(boxes, np.float64)
    d = np.abs(b[:, :3] - np.asarray(p)) < b[:, 3:] + pad
    return bool(np.any(d.all(axis=1)))


def _free_objects(g, n, spawn, yaw, statics, near=3, size=(0.04, 0.2), mass=(0.1, 1.0), first_box=False):
    """n resting boxes/spheres: the first `near` on the floor within 1 m in front
    of the robot, the rest on the floor or on furniture tops; no overlaps."""
    objs = []
    placed = []  # (x, y, z_bottom, z_top, radius_xy)
    sarr = np.asarray(statics, np.float64).reshape(len(statics), 6)
    for k in range(n):
        is_box = (g.uniform() < 0.5) or (first_box and k == 0)
        if first_box and k == 0:
            is_box = True
        if is_box:
            full = g.uniform(size[0], size[1], 3)
            half = full / 2
            rxy = float(np.hypot(half[0], half[1]))
            hz = half[2]
        else:
            rad = g.uniform(size[0], size[1]) / 2
            half = np.array([rad, 0.0, 0.0])
            rxy = rad
            hz = rad
        m = g.uniform(mass[0], mass[1])
        oyaw = g.uniform(-math.pi, math.pi) if is_box else 0.0
        pos = None
        for attempt in range(500):
            if k < near:
                d = g.uniform(0.55, 0.95)
                a = yaw + g.uniform(-0.7, 0.7)
                x, y, zb = spawn[0] + d * math.cos(a), spawn[1] + d * math.sin(a), 0.0
            elif statics and g.uniform() < 0.5:
                b = statics[int(g.integers(len(statics)))]
                if b[3] < rxy + 0.01 or b[4] < rxy + 0.01:
                    continue
                x = g.uniform(b[0] - b[3] + rxy, b[0] + b[3] - rxy)
                y = g.uniform(b[1] - b[4] + rxy, b[1] + b[4] - rxy)
                zb = b[2] + b[5]
            else:
                x = g.uniform(-ROOM + rxy + 0.02, ROOM - rxy - 0.02)
                y = g.uniform(-ROOM + rxy + 0.02, ROOM - rxy - 0.02)
                zb = 0.0
                if math.hypot(x - spawn[0], y - spawn[1]) < 0.5 + rxy:
                    continue
            if abs(x) > ROOM - rxy - 0.01 or abs(y) > ROOM - rxy - 0.01:
                continue
            cz = zb + hz
            # free of furniture (object centre region) and of other objects
            if _inside_any((x, y, cz), sarr, max(rxy, hz) + 0.02):
                continue
            ok = True
            for (px, py, pb, pt, pr) in placed:
                if math.hypot(px - x, py - y) < pr + rxy + 0.02 and not (zb >= pt + 0.02 or pb >= cz + hz + 0.02):
                    ok = False
                    break
            if ok and math.hypot(x - spawn[0], y - spawn[1]) < 0.45 + rxy:
                ok = False
            if ok:
                pos = (x, y, cz)
                break
        if pos is None:  # fall back to a far corner stack-free spot
            pos = (ROOM - 0.3, -ROOM + 0.3 + 0.2 * (k % 25), hz)
        placed.append((pos[0], pos[1], pos[2] - hz, pos[2] + hz, rxy))
        if is_box:
            inert = _box_inertia(m, 2 * half)
            objs.append(dict(type=FREE_BOX, size=half, mass=m, inertia=inert, pos=pos, quat=_quat_z(oyaw)))
        else:
            I = 0.4 * m * half[0] ** 2
            objs.append(dict(type=FREE_SPHERE, size=np.array([half[0], 0, 0]), mass=m, inertia=np.array([I, I, I]),
                             pos=pos, quat=np.array([1.0, 0, 0, 0])))
    return objs


def _init_noise(g):
    """Appendix A.1 robot initialisation noise (arm, base position, base yaw)."""
    arm = np.clip(g.normal(0.0, 0.1, 7), -0.2, 0.2)
    bpos = np.clip(g.normal(0.0, 0.1, 2), -0.2, 0.2)
    byaw = float(np.clip(g.normal(0.0, 0.25), -0.5, 0.5))
    return arm, bpos, byaw


def _assemble(name, cfg_id, S, params, models, per_scene, seed, **extra):
    """Pack per-scene dicts into CSR arrays."""
    mk = _stack_models(models)
    scene_model = np.array([p["model"] for p in per_scene], np.int32)
    def off(key):
        o = np.zeros(S + 1, np.int32)
        o[1:] = np.cumsum([len(p[key]) for p in per_scene])
        return o
    free = [o for p in per_scene for o in p["free"]]
    statics = [b for p in per_scene for b in p["static"]]
    planes = [pl for p in per_scene for pl in p["planes"]]
    aux = [a for p in per_scene for a in p["aux"]]
    NF, NA = len(free), len(aux)
    q = np.stack([p["q"] for p in per_scene])
    qd = np.zeros((S, NDOF))
    fr = np.zeros((NF, 16))
    for i, o in enumerate(free):
        fr[i, 0:3] = o["pos"]
        fr[i, 4:8] = o["quat"]
    ax = np.zeros((NA, 4))
    for i, a in enumerate(aux):
        ax[i, 0] = a["q0"]
    hold = np.stack([p.get("hold", np.zeros(NDOF)) for p in per_scene])
    sb = SceneBatch(
        name=name, n_scenes=S, cfg_id=cfg_id, seed=seed, **params,
        model_nb=mk["nb"], model_parent=mk["parent"].astype(np.int32), model_jtype=mk["jtype"].astype(np.int32),
        model_axis=f32(mk["axis"]), model_xt_rot=f32(mk["xt_rot"]), model_xt_pos=f32(mk["xt_pos"]),
        model_mass=f32(mk["mass"]), model_com=f32(mk["com"]), model_inertia=f32(mk["inertia"]),
        model_kp=f32(mk["kp"]), model_kd=f32(mk["kd"]), model_veldof=mk["veldof"].astype(np.int32),
        model_armature=f32(mk["armature"]), model_damping=f32(mk["damping"]),
        model_act_kind=mk["act_kind"].astype(np.int32), model_act_scale=f32(mk["act_scale"]),
        model_nsph=mk["nsph"], model_sph_body=mk["sph_body"].astype(np.int32), model_sph=f32(mk["sph"]),
        model_sph_flags=mk["sph_flags"].astype(np.int32),
        scene_model=scene_model, free_off=off("free"), static_off=off("static"), plane_off=off("planes"),
        aux_off=off("aux"), scene_hold=f32(hold),
        free_type=np.array([o["type"] for o in free], np.int32).reshape(NF),
        free_size=f32(np.array([o["size"] for o in free]).reshape(NF, 3)),
        free_mass=f32(np.array([o["mass"] for o in free]).reshape(NF)),
        free_inertia=f32(np.array([o["inertia"] for o in free]).reshape(NF, 3)),
        static_box=f32(np.array(statics, dtype=np.float64).reshape(len(statics), 6)),
        plane=f32(np.array(planes, dtype=np.float64).reshape(len(planes), 4)),
        aux_type=np.array([a["type"] for a in aux], np.int32).reshape(NA),
        aux_rot=f32(np.array([a["rot"] for a in aux]).reshape(NA, 4)),
        aux_pos=f32(np.array([a["pos"] for a in aux]).reshape(NA, 3)),
        aux_axis=f32(np.array([a["axis"] for a in aux]).reshape(NA, 3)),
        aux_box=f32(np.array([a["box"] for a in aux]).reshape(NA, 6)),
        aux_mass=f32(np.array([a["mass"] for a in aux]).reshape(NA)),
        aux_inertia=f32(np.array([a["inertia"] for a in aux]).reshape(NA, 3)),
        aux_limit=f32(np.array([a["limit"] for a in aux]).reshape(NA, 2)),
        state0=join_state(f32(q), f32(qd), f32(fr), f32(ax)),
        **extra)
    return sb


_PARAM_DEFAULTS = dict(mu=0.5, baumgarte=0.2, margin=0.01, gravity=(0.0, 0.0, -9.81))


def config1(seed=BASE_SEED, n_scenes=16):
    """16 fixed-base 7-R arms (capsules of 3 spheres), one resting cube each,
    ground plane; dt = 0.02 s control step, 4 substeps, 8 PGS sweeps, mu = 0.5,
    joint torques ~ N(0, 2) held over the control step, 100 control steps."""
    per, models = [], []
    for s in range(n_scenes):
        g = _rng(seed, 1, s)
        models.append(arm7_model(g))
        arm_noise, _, _ = _init_noise(g)
        q = np.zeros(NDOF)
        q[:7] = arm_noise
        e = g.uniform(0.05, 0.15)
        m = g.uniform(0.1, 1.0)
        r = g.uniform(0.3, 0.6)
        a = g.uniform(-math.pi, math.pi)
        half = np.array([e, e, e]) / 2
        box = dict(type=FREE_BOX, size=half, mass=m, inertia=_box_inertia(m, 2 * half),
                   pos=(r * math.cos(a), r * math.sin(a), e / 2), quat=_quat_z(g.uniform(-math.pi, math.pi)))
        per.append(dict(model=s, q=q, free=[box], static=[], planes=_room_planes(False), aux=[]))
    params = dict(h=0.02 / 4, n_sub=4, pgs_iters=8, control_mode=CTRL_TORQUE, contact_cap=48, n_steps=100,
                  robot_contact_cap=32, **_PARAM_DEFAULTS)
    return _assemble("cfg1_arm7", 1, n_scenes, params, models, per, seed, ctrl_kind="torque_normal",
                     ctrl_sigma=2.0)


def _fetch_scene(g, model_idx, n_free, n_static, first_box=False, near=3):
    arm_noise, bpos, byaw = _init_noise(g)
    spawn = g.uniform(-1.0, 1.0, 2) + bpos
    heading = g.uniform(-math.pi, math.pi)
    yaw = heading + byaw
    q = FETCH_REST.copy()
    q[0], q[1], q[2] = spawn[0], spawn[1], yaw
    q[6:13] += arm_noise
    statics = _furniture(g, n_static, spawn)
    objs = _free_objects(g, n_free, spawn, yaw, statics, near=min(near, n_free), first_box=first_box)
    return dict(model=model_idx, q=q, free=objs, static=statics, planes=_room_planes(True), aux=[],
                spawn=spawn, yaw=yaw)


def _fetch_batch(name, cfg_id, seed, n_scenes, n_free_fn, n_static_fn, params, aux_fn=None, post=None):
    gm = _rng(seed, cfg_id, 10_000_000)
    model = fetch_like_model(gm)
    per = []
    for s in range(n_scenes):
        g = _rng(seed, cfg_id, s)
        nf = n_free_fn(g)
        ns = n_static_fn(g)
        sc = _fetch_scene(g, 0, nf, ns)
        if aux_fn is not None:
            sc["aux"] = aux_fn(g, sc)
        if post is not None:
            post(g, sc)
        per.append(sc)
    rest = np.zeros((1, NDOF), np.float32)
    rest[0] = f32(FETCH_REST)
    return _assemble(name, cfg_id, n_scenes, params, [model], per, seed, ctrl_rest=rest, **(
        dict(ctrl_kind="pd_targets") if params["control_mode"] == CTRL_PD else dict(ctrl_kind="torque_normal",
                                                                                    ctrl_sigma=0.5)))


def config2(seed=BASE_SEED, n_scenes=1024, h=None, n_sub=5):
    """Fetch-like robot, 8 free boxes/spheres (U[0.04, 0.2] m), 64 furniture
    boxes (U[0.2, 2] m) in a 6 x 6 m room; dt = 0.01 s, 5 substeps, 10 PGS sweeps."""
    params = dict(h=(0.01 / n_sub if h is None else h), n_sub=n_sub, pgs_iters=10, control_mode=CTRL_PD,
                  contact_cap=64, n_steps=50, robot_contact_cap=24, **_PARAM_DEFAULTS)
    return _fetch_batch("cfg2_fetch", 2, seed, n_scenes, lambda g: 8, lambda g: 64, params)


def config3(seed=BASE_SEED, n_scenes=4096):
    """Uneven batch: free objects U{2..32}, furniture boxes U{32..256} per scene."""
    params = dict(h=0.01 / 5, n_sub=5, pgs_iters=10, control_mode=CTRL_PD, contact_cap=160, n_steps=50,
                  robot_contact_cap=24, **_PARAM_DEFAULTS)
    return _fetch_batch("cfg3_uneven", 3, seed, n_scenes, lambda g: int(g.integers(2, 33)),
                        lambda g: int(g.integers(32, 257)), params)


def config4(seed=BASE_SEED, n_scenes=256):
    """Differentiation workload: config-2 geometry, torque controls added to a PD
    hold, one box resting against the base bumper that the base pushes forward;
    50 control steps of dt = 0.02 s with 4 substeps."""
    params = dict(h=0.02 / 4, n_sub=4, pgs_iters=10, control_mode=CTRL_TORQUE_HOLD, contact_cap=64,
                  n_steps=50, robot_contact_cap=24, **_PARAM_DEFAULTS)

    def post(g, sc):
        yaw = sc["yaw"]
        c, s_ = math.cos(yaw), math.sin(yaw)
        full = np.array([g.uniform(0.1, 0.2), g.uniform(0.1, 0.2), g.uniform(0.1, 0.2)])
        half = full / 2
        m = g.uniform(0.1, 1.0)
        # near face 5 mm in front of the bumper spheres' surface (bumper x = 0.3, r = 0.08)
        d = 0.3 + 0.08 + 0.005 + half[0]
        pos = (sc["spawn"][0] + d * c, sc["spawn"][1] + d * s_, half[2])
        box = dict(type=FREE_BOX, size=half, mass=m, inertia=_box_inertia(m, full), pos=pos, quat=_quat_z(yaw))
        # drop other objects that would overlap the pushed box's path
        keep = []
        for o in sc["free"]:
            dx, dy = o["pos"][0] - sc["spawn"][0], o["pos"][1] - sc["spawn"][1]
            along = dx * c + dy * s_
            across = -dx * s_ + dy * c
            if -0.2 < along < 1.6 and abs(across) < 0.5 and o["pos"][2] < 0.3:
                continue
            keep.append(o)
        sc["free"] = [box] + keep[:7]
        hold = sc["q"].copy()
        hold[0] = 0.1 * c    # base forward velocity target (world x, y), m/s
        hold[1] = 0.1 * s_
        hold[2] = 0.0
        sc["hold"] = hold
    return _fetch_batch("cfg4_grad", 4, seed, n_scenes, lambda g: 8, lambda g: 64, params, post=post)


def config5(seed=BASE_SEED, n_scenes=16384):
    """Fetch-like robot + revolute door (0.6 x 1.8 m panel, 10 kg) + prismatic
    drawer (0.5 x 0.4 x 0.2 m, 3 kg, stroke [0, 0.4] m) + 4 free objects +
    64 furniture boxes; h = 0.002 s, 5 substeps, 20 control steps."""
    params = dict(h=0.002, n_sub=5, pgs_iters=10, control_mode=CTRL_PD, contact_cap=64, n_steps=20,
                  robot_contact_cap=32, **_PARAM_DEFAULTS)

    def aux_fn(g, sc):
        spawn, yaw = sc["spawn"], sc["yaw"]
        out = []
        # door: hinge line vertical, 1.3 m from the robot, panel along the joint frame's +x
        a = yaw + g.uniform(-1.0, 1.0)
        hx, hy = spawn[0] + 1.3 * math.cos(a), spawn[1] + 1.3 * math.sin(a)
        full = np.array([0.6, 0.04, 1.8])
        m = 10.0
        Ic = _box_inertia(m, full)
        q0 = 0.0 if g.uniform() < 0.5 else g.uniform(0.0, math.pi / 2)
        out.append(dict(type=JT_REVOLUTE, rot=_quat_z(a + math.pi / 2), pos=(hx, hy, 0.01), axis=(0, 0, 1),
                        box=(0.3, 0.0, 0.9, 0.3, 0.02, 0.9), mass=m, inertia=Ic, limit=(0.0, math.pi / 2), q0=q0))
        # drawer: slides along its joint frame's +x, box centred on the joint origin
        b = yaw + g.uniform(-1.0, 1.0) + math.pi
        dx, dy = spawn[0] + 1.2 * math.cos(b), spawn[1] + 1.2 * math.sin(b)
        full = np.array([0.5, 0.4, 0.2])
        m = 3.0
        q0 = 0.0 if g.uniform() < 0.5 else g.uniform(0.0, 0.4)
        out.append(dict(type=JT_PRISMATIC, rot=_quat_z(b + math.pi), pos=(dx, dy, 0.5), axis=(1, 0, 0),
                        box=(0.0, 0.0, 0.0, 0.25, 0.2, 0.1), mass=m, inertia=_box_inertia(m, full),
                        limit=(0.0, 0.4), q0=q0))
        return out
    return _fetch_batch("cfg5_articulated", 5, seed, n_scenes, lambda g: 4, lambda g: 64, params, aux_fn=aux_fn)


def config6(seed=BASE_SEED, n_scenes=1024):
    """Second physics regime: the config-2 scene at 120 Hz simulation under
    30 Hz control (4 substeps of h = 1/120 s), 300 control steps of random
    normalized actions clipped to [-0.3, 0.3] through the action front-end."""
    params = dict(h=1.0 / 120.0, n_sub=4, pgs_iters=10, control_mode=CTRL_ACTIONS, contact_cap=64, n_steps=300,
                  robot_contact_cap=24, **_PARAM_DEFAULTS)
    b = _fetch_batch("cfg6_random_actions", 6, seed, n_scenes, lambda g: 8, lambda g: 64, params)
    b.ctrl_kind = "random_actions"
    b.ctrl_clip = 0.3
    return b


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5, 6: config6}


def make(cfg: int, n_scenes=None, seed=BASE_SEED, **kw):
    fn = CONFIGS[cfg]
    if n_scenes is None:
        return fn(seed=seed, **kw)
    return fn(seed=seed, n_scenes=n_scenes, **kw)


# ----------------------------------------------------------------------------
# hand-built scenes (tests)
# ----------------------------------------------------------------------------

def model_builder():
    """A fresh robot-model builder (bodies with one DoF each, plus spheres)."""
    return _ModelBuilder()


def empty_model():
    """A robot model with no bodies (scenes holding only free bodies)."""
    return _ModelBuilder().arrays()


def box_object(half, mass, pos, quat=(1.0, 0.0, 0.0, 0.0), vel=(0, 0, 0), angvel=(0, 0, 0)):
    half = np.asarray(half, float)
    return dict(type=FREE_BOX, size=half, mass=mass, inertia=_box_inertia(mass, 2 * half), pos=tuple(pos),
                quat=np.asarray(quat, float), vel=vel, angvel=angvel)


def sphere_object(radius, mass, pos, vel=(0, 0, 0), angvel=(0, 0, 0)):
    I = 0.4 * mass * radius ** 2
    return dict(type=FREE_SPHERE, size=np.array([radius, 0, 0]), mass=mass, inertia=np.array([I, I, I]),
                pos=tuple(pos), quat=np.array([1.0, 0, 0, 0]), vel=vel, angvel=angvel)


def custom_batch(models, scenes, h=0.005, n_sub=1, pgs_iters=8, mu=0.5, baumgarte=0.2, margin=0.01,
                 gravity=(0.0, 0.0, -9.81), control_mode=CTRL_TORQUE, contact_cap=64, name="custom"):
    """Batch from explicit content.  Each scene dict may hold: model (index),
    q, qd (16-vectors), free (list of box_object / sphere_object dicts),
    static (list of (cx, cy, cz, hx, hy, hz)), planes (list of (nx, ny, nz, d)),
    aux (list of dicts as in config 5), hold (16-vector)."""
    per = []
    for sc in scenes:
        d = dict(model=sc.get("model", 0), q=np.asarray(sc.get("q", np.zeros(NDOF)), float),
                 free=sc.get("free", []), static=sc.get("static", []), planes=sc.get("planes", []),
                 aux=sc.get("aux", []))
        if "hold" in sc:
            d["hold"] = np.asarray(sc["hold"], float)
        per.append(d)
    params = dict(h=h, n_sub=n_sub, pgs_iters=pgs_iters, control_mode=control_mode, contact_cap=contact_cap,
                  n_steps=1, mu=mu, baumgarte=baumgarte, margin=margin, gravity=tuple(gravity),
                  robot_contact_cap=min(contact_cap, 32))
    b = _assemble(name, 0, len(per), params, models, per, BASE_SEED)
    st = split_state(b.state0, b.n_scenes, b.n_free, b.n_aux)
    k = 0
    for s, sc in enumerate(scenes):
        if "qd" in sc:
            st["qd"][s] = f32(sc["qd"])
        for o in sc.get("free", []):
            st["free"][k, 8:11] = f32(o.get("vel", (0, 0, 0)))
            st["free"][k, 12:15] = f32(o.get("angvel", (0, 0, 0)))
            k += 1
    return b
