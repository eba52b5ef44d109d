"""Batched rigid-body physics step on MI355X (gfx950) -- Python binding.

Argument marshalling over the C ABI of ``include/ms_phys.h`` (libms_phys.so,
built in-tree by ``_build.py``).  Every step of the physics runs in the HIP
kernels; PyTorch only provides device memory and streams.  There is no CPU
fallback: if the library cannot be loaded the import of :func:`lib` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libms_phys.so")

MS_OK = 0
MS_CTRL_TORQUE, MS_CTRL_PD, MS_CTRL_TORQUE_HOLD = 0, 1, 2
MS_SCHED_PERSISTENT = 1
MS_SCHED_GRAPH = 2
MS_SCHED_PER_SUBSTEP = 4
MS_SCHED_STAGE_STATIC = 8
MS_SCHED_CULL = 16
MS_SCHED_BWD_REFERENCE = 32
MS_SCHED_BWD_ONE_LAUNCH = 64
MS_SCHED_STATIC_ORDER = 128
MS_SCHED_FWD_ONE_LAUNCH = 256
MS_ST_NONFINITE, MS_ST_OVERFLOW, MS_ST_DEGENERATE, MS_ST_ROBOT_OVERFLOW = 1, 2, 4, 8

EXPORTS = ["ms_query_sizes", "ms_state_floats", "ms_create_batch", "ms_destroy_batch", "ms_set_schedule",
           "ms_get_schedule", "ms_set_backward_split", "ms_get_backward_split",
           "ms_set_forward_split", "ms_get_forward_split", "ms_autotune", "ms_autotune_backward",
           "ms_set_autotune_cache", "ms_autotune_key", "ms_step", "ms_step_backward",
           "ms_step_record", "ms_step_backward_recorded", "ms_get_state", "ms_set_state",
           "ms_scene_status", "ms_set_force_outputs", "ms_reset_robots", "ms_spawn_check", "ms_enable_debug",
           "ms_debug_contacts", "ms_enable_phase_profile", "ms_phase_cycles", "ms_set_task_robot",
           "ms_set_grip_outputs", "ms_task_begin", "ms_task_update", "ms_task_categorize", "ms_probe_copy",
           "ms_probe_fma", "ms_step_noalloc", "ms_last_error"]
PHASES = ["drive+kinematics", "contacts", "dynamics", "rows", "levels", "pgs", "integrate", "load/store"]


class MsError(RuntimeError):
    pass


class BatchDesc(C.Structure):
    _fields_ = [("n_scenes", C.c_int32), ("n_substeps", C.c_int32), ("pgs_iters", C.c_int32),
                ("control_mode", C.c_int32), ("contact_cap", C.c_int32), ("robot_contact_cap", C.c_int32),
                ("h", C.c_float), ("mu", C.c_float), ("baumgarte", C.c_float), ("margin", C.c_float),
                ("gravity", C.c_float * 3)]


SCENE_FIELDS = ["model_nb", "model_parent", "model_jtype", "model_axis", "model_xt_rot", "model_xt_pos",
                "model_mass", "model_com", "model_inertia", "model_kp", "model_kd", "model_veldof",
                "model_armature", "model_damping", "model_act_kind", "model_act_scale", "model_nsph", "model_sph_body", "model_sph", "model_sph_flags",
                "scene_model", "free_off", "static_off", "plane_off", "aux_off", "scene_hold", "free_type",
                "free_size", "free_mass", "free_inertia", "static_box", "plane", "aux_type", "aux_rot", "aux_pos",
                "aux_axis", "aux_box", "aux_mass", "aux_inertia", "aux_limit"]


class SceneDesc(C.Structure):
    _fields_ = [("n_models", C.c_int32)] + [(n, C.c_void_p) for n in SCENE_FIELDS]


class Sizes(C.Structure):
    _fields_ = [("params", C.c_size_t), ("state", C.c_size_t), ("scratch", C.c_size_t), ("tape", C.c_size_t),
                ("lds", C.c_size_t), ("record", C.c_size_t)]


class StateView(C.Structure):
    _fields_ = [("q", C.c_void_p), ("qd", C.c_void_p), ("free_body", C.c_void_p), ("aux", C.c_void_p),
                ("free_off_host", C.c_void_p), ("aux_off_host", C.c_void_p), ("n_scenes", C.c_int32),
                ("n_free", C.c_int32), ("n_aux", C.c_int32)]


class Schedule(C.Structure):
    _fields_ = [("flags", C.c_int32), ("grid", C.c_int32)]


# subtask predicates / events (ms_task_* calls)
MS_TASK_PICK, MS_TASK_PLACE, MS_TASK_OPEN, MS_TASK_CLOSE = 0, 1, 2, 3
MS_IND_GRASPED, MS_IND_SUCCESS, MS_IND_OPEN, MS_IND_SLIGHT = 1, 2, 4, 8
MS_IND_AT_GOAL, MS_IND_CONTACT, MS_IND_EXCESSIVE = 16, 32, 64
MS_EP_LIST = 16
PRED_FIELDS = ["d_ee", "j_arm", "j_torso", "qd_arm", "d_goal", "aq", "f_ee", "f_finger"]


class TaskRobot(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("ee_body", "base_body", "base_x", "base_y", "base_yaw", "arm0", "narm",
                                          "torso", "finger_l", "finger_r")] + [
        ("ee_bodies", C.c_uint32), ("ee_offset", C.c_float * 3), ("ee_rest", C.c_float * 3),
        ("q_rest", C.c_float * 16), ("grasp_force", C.c_float)]


# device layouts of ms_task [S] and ms_episode [S]
TASK_DTYPE = np.dtype([("kind", "<i4"), ("target", "<i4"), ("goal", "<f4", 3), ("open_frac", "<f4")])
EPISODE_DTYPE = np.dtype([("cumcol", "<f4"), ("aq0", "<f4"), ("d0", "<f4"), ("ind", "<u4"), ("t", "<i4"),
                          ("n", "<i4"), ("last", "<i4", 8), ("list", "u1", MS_EP_LIST)])


_lib = None


def lib():
    """Load libms_phys.so (building it first only if it does not exist)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import _build
            _build.build(force=False)
        L = C.CDLL(LIB_PATH)
        vp, i32 = C.c_void_p, C.c_int32
        sig = {
            "ms_query_sizes": [vp, vp, vp],
            "ms_state_floats": [vp, i32, vp],
            "ms_create_batch": [vp, vp, vp, vp, vp, vp, vp],
            "ms_destroy_batch": [vp],
            "ms_set_schedule": [vp, vp],
            "ms_get_schedule": [vp, vp],
            "ms_set_backward_split": [vp, i32, i32],
            "ms_get_backward_split": [vp, vp, vp],
            "ms_set_forward_split": [vp, i32],
            "ms_get_forward_split": [vp, vp, vp, vp],
            "ms_autotune": [vp, vp, vp, vp, i32, vp, vp, vp],
            "ms_autotune_backward": [vp, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp],
            "ms_set_autotune_cache": [vp, C.c_char_p],
            "ms_autotune_key": [vp, i32, C.c_char_p, C.c_size_t, vp],
            "ms_step": [vp, vp, vp, vp, vp],
            "ms_step_backward": [vp, vp, vp, vp, vp, vp, vp],
            "ms_step_record": [vp, vp, vp, vp, vp, vp],
            "ms_step_backward_recorded": [vp, vp, vp, vp, vp, vp, vp, vp],
            "ms_get_state": [vp, vp, vp],
            "ms_set_state": [vp, vp, vp, vp, vp],
            "ms_scene_status": [vp, vp],
            "ms_set_force_outputs": [vp, vp, vp],
            "ms_reset_robots": [vp, vp, vp, vp, vp, vp, vp],
            "ms_spawn_check": [vp, vp, vp, vp],
            "ms_enable_debug": [vp, i32],
            "ms_debug_contacts": [vp, vp],
            "ms_enable_phase_profile": [vp, i32],
            "ms_phase_cycles": [vp, vp],
            "ms_set_task_robot": [vp, vp],
            "ms_set_grip_outputs": [vp, vp],
            "ms_task_begin": [vp, vp, vp, vp, vp, vp, vp, vp],
            "ms_task_update": [vp, vp, vp, vp, vp, vp, vp, vp],
            "ms_task_categorize": [vp, vp, vp, vp, vp],
            "ms_probe_copy": [vp, vp, C.c_size_t, vp],
            "ms_probe_fma": [vp, i32, i32, vp, vp],
            "ms_step_noalloc": [vp, vp, vp, vp, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int32
        L.ms_last_error.argtypes = []
        L.ms_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc, what):
    if rc != MS_OK:
        msg = lib().ms_last_error().decode(errors="replace")
        raise MsError(f"{what} failed ({rc}): {msg}")


def _ptr_np(a):
    return C.c_void_p(a.ctypes.data) if a is not None and a.size else C.c_void_p(0)


def _ptr_t(t):
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def make_desc(batch, **over):
    g = lambda k, d=None: over.get(k, getattr(batch, k, d))
    d = BatchDesc()
    d.n_scenes = int(batch.n_scenes)
    d.n_substeps = int(g("n_sub"))
    d.pgs_iters = int(g("pgs_iters"))
    d.control_mode = int(g("control_mode"))
    d.contact_cap = int(g("contact_cap"))
    d.robot_contact_cap = int(over.get("robot_contact_cap",
                                       getattr(batch, "robot_contact_cap", min(int(g("contact_cap")), 32))))
    d.h = float(g("h"))
    d.mu = float(g("mu"))
    d.baumgarte = float(g("baumgarte"))
    d.margin = float(g("margin"))
    grav = g("gravity")
    for i in range(3):
        d.gravity[i] = float(grav[i])
    return d


def make_scene_desc(batch):
    keep = {}
    sd = SceneDesc()
    sd.n_models = int(len(batch.model_nb))
    for n in SCENE_FIELDS:
        a = np.ascontiguousarray(getattr(batch, n))
        a = a.astype(np.int32 if a.dtype.kind in "iu" else np.float32, copy=False)
        keep[n] = a
        setattr(sd, n, _ptr_np(a))
    return sd, keep


class MsBatch:
    """One batch of scenes bound to the current HIP device.

    ``batch`` is any object with the scene-description arrays (the scene
    generator's SceneBatch); keyword overrides replace its physics parameters.
    ``backward=True`` allocates the adjoint workspace that ``step_backward``
    needs (its size is ``sizes.tape`` bytes).
    """

    def __init__(self, batch, device=None, robot_contact_cap=None, backward=False, **over):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        if robot_contact_cap is not None:
            over["robot_contact_cap"] = robot_contact_cap
        self.desc = make_desc(batch, **over)
        self.sdesc, self._keep = make_scene_desc(batch)
        self.S = int(batch.n_scenes)
        self.n_sub = int(self.desc.n_substeps)
        sz = Sizes()
        _check(lib().ms_query_sizes(C.byref(self.desc), C.byref(self.sdesc), C.byref(sz)), "ms_query_sizes")
        self.sizes = sz
        self.state_floats = sz.state // 4
        with torch.cuda.device(self.device):
            self.params = torch.empty(max(sz.params, 256), dtype=torch.uint8, device=self.device)
            self.scratch = torch.empty(max(sz.scratch, 256), dtype=torch.uint8, device=self.device)
            self.tape = torch.empty(max(sz.tape, 256), dtype=torch.uint8, device=self.device) if backward else None
            h = C.c_void_p()
            _check(lib().ms_create_batch(C.byref(self.desc), C.byref(self.sdesc), _ptr_t(self.params),
                                         _ptr_t(self.scratch), _ptr_t(self.tape) if backward else None, _stream(),
                                         C.byref(h)),
                   "ms_create_batch")
        self.h = h
        self.n_free = int(batch.free_off[-1])
        self.n_aux = int(batch.aux_off[-1])

    def close(self):
        if getattr(self, "h", None):
            lib().ms_destroy_batch(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def new_state(self, x=None):
        t = self.torch.zeros(self.state_floats, dtype=self.torch.float32, device=self.device)
        if x is not None:
            t.copy_(self.torch.as_tensor(np.asarray(x, np.float32)))
        return t

    def _check_state(self, x, name):
        t = self.torch
        if not (isinstance(x, t.Tensor) and x.is_cuda and x.dtype == t.float32 and x.is_contiguous()
                and x.numel() == self.state_floats):
            raise MsError(f"{name}: expected a contiguous float32 device tensor of {self.state_floats} floats")

    def _check_controls(self, u):
        t = self.torch
        if not (isinstance(u, t.Tensor) and u.is_cuda and u.dtype == t.float32 and u.is_contiguous()
                and u.numel() == self.S * 16):
            raise MsError(f"controls: expected a contiguous float32 device tensor [{self.S}, 16]")

    def step(self, x, u, out=None, stream=None):
        """One control step: returns ``out`` (new tensor unless given; may be ``x``)."""
        self._check_state(x, "state_in")
        self._check_controls(u)
        if out is None:
            out = self.torch.empty_like(x)
        self._check_state(out, "state_out")
        _check(lib().ms_step(self.h, _ptr_t(x), _ptr_t(u), _ptr_t(out), _stream(stream)), "ms_step")
        return out

    def step_backward(self, x, u, gx_out, gx_in=None, gu=None, stream=None):
        """Vector-Jacobian product of one control step from ``x`` under ``u``:
        returns (dL/dx, dL/du) given dL/d(next state) ``gx_out``."""
        self._check_state(x, "state_in")
        self._check_controls(u)
        self._check_state(gx_out, "grad_state_out")
        if gx_in is None:
            gx_in = self.torch.empty_like(x)
        if gu is None:
            gu = self.torch.empty_like(u)
        _check(lib().ms_step_backward(self.h, _ptr_t(x), _ptr_t(u), _ptr_t(gx_out), _ptr_t(gx_in), _ptr_t(gu),
                                      _stream(stream)), "ms_step_backward")
        return gx_in, gu

    def new_record(self):
        """Device buffer for one control step's record (``step_record``)."""
        return self.torch.empty(max(self.sizes.record, 4) // 4, dtype=self.torch.float32, device=self.device)

    def step_record(self, x, u, rec, out=None, stream=None):
        """``step`` that also writes the step's record into ``rec`` (from
        ``new_record``) for ``step_backward_recorded``."""
        self._check_state(x, "state_in")
        self._check_controls(u)
        self._check_record(rec)
        if out is None:
            out = self.torch.empty_like(x)
        self._check_state(out, "state_out")
        _check(lib().ms_step_record(self.h, _ptr_t(x), _ptr_t(u), _ptr_t(out), _ptr_t(rec), _stream(stream)),
               "ms_step_record")
        return out

    def step_backward_recorded(self, x, u, rec, gx_out, gx_in=None, gu=None, stream=None):
        """``step_backward`` from the record ``step_record`` wrote for the
        same (x, u): the step is not run again."""
        self._check_state(x, "state_in")
        self._check_controls(u)
        self._check_record(rec)
        self._check_state(gx_out, "grad_state_out")
        if gx_in is None:
            gx_in = self.torch.empty_like(x)
        if gu is None:
            gu = self.torch.empty_like(u)
        _check(lib().ms_step_backward_recorded(self.h, _ptr_t(x), _ptr_t(u), _ptr_t(rec), _ptr_t(gx_out),
                                               _ptr_t(gx_in), _ptr_t(gu), _stream(stream)),
               "ms_step_backward_recorded")
        return gx_in, gu

    def _check_record(self, rec):
        if not (rec.is_cuda and rec.dtype == self.torch.float32 and rec.is_contiguous()
                and rec.numel() * 4 >= self.sizes.record):
            raise MsError(f"record must be a contiguous float32 device tensor of at least {self.sizes.record} bytes")

    def enable_forces(self, on=True):
        """Contact-force outputs written by every following ``step``: returns
        (robot_force [S], body_force [NF, 4]) device tensors (sums over the
        substeps of a control step), or None after ``enable_forces(False)``."""
        t = self.torch
        if on:
            self.robot_force = t.zeros(self.S, dtype=t.float32, device=self.device)
            self.body_force = t.zeros((max(self.n_free, 1), 4), dtype=t.float32, device=self.device)
            _check(lib().ms_set_force_outputs(self.h, _ptr_t(self.robot_force), _ptr_t(self.body_force)),
                   "ms_set_force_outputs")
            return self.robot_force, self.body_force
        _check(lib().ms_set_force_outputs(self.h, None, None), "ms_set_force_outputs")
        self.robot_force = self.body_force = None
        return None

    # ------------------------------------------------------------------ tasks
    def set_task_robot(self, robot):
        """The robot as the task predicates see it: a dict with the fields of
        ms_task_robot (ee_body, base_body, base_x, base_y, base_yaw, arm0, narm,
        torso, finger_l, finger_r, ee_bodies, ee_offset, ee_rest, q_rest,
        grasp_force)."""
        r = TaskRobot()
        for k, _ in TaskRobot._fields_:
            v = robot[k]
            if k in ("ee_offset", "ee_rest", "q_rest"):
                arr = getattr(r, k)
                for i, e in enumerate(np.asarray(v, np.float64).reshape(-1)):
                    arr[i] = float(e)
            else:
                setattr(r, k, float(v) if k == "grasp_force" else int(v))
        _check(lib().ms_set_task_robot(self.h, C.byref(r)), "ms_set_task_robot")

    def enable_grip(self, on=True):
        """Gripper contact outputs of every following ``step``: float32
        [NF + NA, 2] (end-effector normal force summed over the substeps; the
        smaller finger force in the last substep), or None when off."""
        t = self.torch
        if on:
            self.grip = t.zeros((max(self.n_free + self.n_aux, 1), 2), dtype=t.float32, device=self.device)
            _check(lib().ms_set_grip_outputs(self.h, _ptr_t(self.grip)), "ms_set_grip_outputs")
            return self.grip
        _check(lib().ms_set_grip_outputs(self.h, None), "ms_set_grip_outputs")
        self.grip = None
        return None

    def task_tensor(self, tasks):
        """Device copy of per-scene tasks (a TASK_DTYPE array or a list of dicts)."""
        if not (isinstance(tasks, np.ndarray) and tasks.dtype == TASK_DTYPE):
            arr = np.zeros(self.S, TASK_DTYPE)
            for s, tk in enumerate(tasks):
                arr[s]["kind"], arr[s]["target"] = int(tk["kind"]), int(tk["target"])
                arr[s]["goal"] = np.asarray(tk.get("goal", (0.0, 0.0, 0.0)), np.float32)
                arr[s]["open_frac"] = float(tk.get("open_frac", 0.9))
            tasks = arr
        if tasks.shape != (self.S,):
            raise MsError(f"tasks: expected {self.S} entries")
        return self.torch.from_numpy(np.ascontiguousarray(tasks).view(np.uint8).copy()).to(self.device)

    def new_episodes(self):
        return self.torch.zeros(self.S * EPISODE_DTYPE.itemsize, dtype=self.torch.uint8, device=self.device)

    @staticmethod
    def episodes(ep):
        """Host copy of an episode tensor as an EPISODE_DTYPE array."""
        return ep.cpu().numpy().view(EPISODE_DTYPE)

    def _pred(self, pred):
        if pred is True:
            return self.torch.zeros((self.S, 8), dtype=self.torch.float32, device=self.device)
        return pred if pred is not None and pred is not False else None

    def task_begin(self, x, tasks_t, ep=None, grip=None, mask=None, pred=None, stream=None):
        """Starts the episodes of the masked scenes (all when mask is None);
        returns (episodes, predicate values or None)."""
        self._check_state(x, "state")
        ep = self.new_episodes() if ep is None else ep
        pred = self._pred(pred)
        _check(lib().ms_task_begin(self.h, _ptr_t(x), _ptr_t(tasks_t), _ptr_t(grip) if grip is not None else None,
                                   _ptr_t(ep), _ptr_t(mask) if mask is not None else None,
                                   _ptr_t(pred) if pred is not None else None, _stream(stream)), "ms_task_begin")
        return ep, pred

    def task_update(self, x, tasks_t, ep, robot_force, grip=None, pred=None, stream=None):
        """Predicates and events after one control step; returns the
        predicate values (or None)."""
        self._check_state(x, "state")
        pred = self._pred(pred)
        _check(lib().ms_task_update(self.h, _ptr_t(x), _ptr_t(tasks_t), _ptr_t(robot_force),
                                    _ptr_t(grip) if grip is not None else None, _ptr_t(ep),
                                    _ptr_t(pred) if pred is not None else None, _stream(stream)), "ms_task_update")
        return pred

    def task_categorize(self, tasks_t, ep, stream=None):
        """int32 [S]: success / failure mode of every episode (0: none)."""
        out = self.torch.zeros(self.S, dtype=self.torch.int32, device=self.device)
        _check(lib().ms_task_categorize(self.h, _ptr_t(tasks_t), _ptr_t(ep), _ptr_t(out), _stream(stream)),
               "ms_task_categorize")
        return out

    def reset_robots(self, x, base, noise, clip, mask=None, stream=None):
        """Robot resets of the masked scenes in place: q = base + clip(noise), qd = 0."""
        self._check_state(x, "state")
        t = self.torch
        for v, n in ((base, "base"), (noise, "noise")):
            if not (isinstance(v, t.Tensor) and v.is_cuda and v.dtype == t.float32 and v.is_contiguous()
                    and v.numel() == self.S * 16):
                raise MsError(f"{n}: expected a contiguous float32 device tensor [{self.S}, 16]")
        if mask is not None and not (isinstance(mask, t.Tensor) and mask.is_cuda and mask.dtype == t.uint8
                                     and mask.numel() == self.S):
            raise MsError(f"mask: expected a uint8 device tensor of {self.S} entries")
        c = np.ascontiguousarray(np.asarray(clip, np.float32).reshape(16))
        _check(lib().ms_reset_robots(self.h, _ptr_t(x), _ptr_t(mask) if mask is not None else None, _ptr_t(base),
                                     _ptr_t(noise), _ptr_np(c), _stream(stream)), "ms_reset_robots")
        return x

    def spawn_check(self, x, out=None, stream=None):
        """uint8 [S]: 1 where a robot sphere penetrates another body."""
        self._check_state(x, "state")
        t = self.torch
        if out is None:
            out = t.empty(self.S, dtype=t.uint8, device=self.device)
        _check(lib().ms_spawn_check(self.h, _ptr_t(x), _ptr_t(out), _stream(stream)), "ms_spawn_check")
        return out

    def set_schedule(self, flags, grid=0):
        s = Schedule(flags, grid)
        _check(lib().ms_set_schedule(self.h, C.byref(s)), "ms_set_schedule")

    def get_schedule(self):
        s = Schedule()
        _check(lib().ms_get_schedule(self.h, C.byref(s)), "ms_get_schedule")
        return s.flags, s.grid

    def set_backward_split(self, contact_cap, robot_contact_cap=1):
        """Caps of the smaller adjoint layout (0: one launch; < 0: the
        library's choice)."""
        _check(lib().ms_set_backward_split(self.h, int(contact_cap), int(robot_contact_cap)),
               "ms_set_backward_split")

    def get_backward_split(self):
        cc, rc = C.c_int32(), C.c_int32()
        _check(lib().ms_get_backward_split(self.h, C.byref(cc), C.byref(rc)), "ms_get_backward_split")
        return cc.value, rc.value

    def set_forward_split(self, contact_cap):
        """Contact cap of the persistent step's smaller layout (0: one
        launch; < 0: the library's choice)."""
        _check(lib().ms_set_forward_split(self.h, int(contact_cap)), "ms_set_forward_split")

    def get_forward_split(self, counts=False):
        """The cap in use; with counts=True also (scenes routed to the full
        layout, scenes stepped again) of the last split step (synchronises)."""
        cc, nf, nr = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().ms_get_forward_split(self.h, C.byref(cc), C.byref(nf) if counts else None,
                                          C.byref(nr) if counts else None), "ms_get_forward_split")
        return (cc.value, nf.value, nr.value) if counts else cc.value

    def autotune(self, x, u, reps=5, stream=None):
        tmp = self.torch.empty_like(x)
        s = Schedule()
        ms = C.c_float()
        _check(lib().ms_autotune(self.h, _ptr_t(x), _ptr_t(u), _ptr_t(tmp), reps, _stream(stream), C.byref(s),
                                 C.byref(ms)), "ms_autotune")
        return (s.flags, s.grid), ms.value

    def autotune_backward(self, x, u, gx_out, reps=3, stream=None):
        """ms_autotune_backward: returns ((split_c, split_r), ms per step)."""
        gx_in = self.torch.empty_like(x)
        gu = self.torch.empty_like(u)
        c, r, ms = C.c_int32(), C.c_int32(), C.c_float()
        _check(lib().ms_autotune_backward(self.h, _ptr_t(x), _ptr_t(u), _ptr_t(gx_out), _ptr_t(gx_in), _ptr_t(gu),
                                          reps, _stream(stream), C.byref(c), C.byref(r), C.byref(ms)),
               "ms_autotune_backward")
        return (c.value, r.value), ms.value

    def set_autotune_cache(self, path):
        _check(lib().ms_set_autotune_cache(self.h, None if path is None else str(path).encode()),
               "ms_set_autotune_cache")

    def autotune_key(self, backward=False):
        """(cache key, whether the last tuning came from the cache)."""
        buf = C.create_string_buffer(256)
        fc = C.c_int32()
        _check(lib().ms_autotune_key(self.h, 1 if backward else 0, buf, C.c_size_t(256), C.byref(fc)),
               "ms_autotune_key")
        return buf.value.decode(), bool(fc.value)

    def status(self):
        out = np.zeros(self.S, np.uint32)
        rc = lib().ms_scene_status(self.h, _ptr_np(out))
        if rc not in (MS_OK, -5):
            _check(rc, "ms_scene_status")
        return out

    def enable_debug(self, on=True):
        _check(lib().ms_enable_debug(self.h, 1 if on else 0), "ms_enable_debug")

    def debug_contacts(self):
        out = np.zeros((self.S, self.n_sub, 4), np.uint32)
        _check(lib().ms_debug_contacts(self.h, _ptr_np(out)), "ms_debug_contacts")
        return out

    def enable_phase_profile(self, on=True):
        _check(lib().ms_enable_phase_profile(self.h, 1 if on else 0), "ms_enable_phase_profile")

    def phase_cycles(self):
        out = np.zeros((self.S, 8), np.uint64)
        _check(lib().ms_phase_cycles(self.h, _ptr_np(out)), "ms_phase_cycles")
        return out

    def set_state(self, x, src, mask=None, stream=None):
        m = C.c_void_p(0) if mask is None else _ptr_t(mask)
        _check(lib().ms_set_state(self.h, _ptr_t(x), _ptr_t(src), m, _stream(stream)), "ms_set_state")

    def get_state(self, x):
        """Typed device views of a state tensor through ms_get_state: q, qd
        [S,16], free [NF,16], aux [NA,4] (torch views sharing x's memory) and
        the CSR offsets free_off, aux_off (numpy copies)."""
        self._check_state(x, "state")
        v = StateView()
        _check(lib().ms_get_state(self.h, _ptr_t(x), C.byref(v)), "ms_get_state")
        base = x.data_ptr()
        elem = lambda p: (p - base) // 4
        S, NF, NA = v.n_scenes, v.n_free, v.n_aux
        out = {"q": x[elem(v.q): elem(v.q) + 16 * S].view(S, 16),
               "qd": x[elem(v.qd): elem(v.qd) + 16 * S].view(S, 16),
               "free": x[elem(v.free_body): elem(v.free_body) + 16 * NF].view(NF, 16),
               "aux": x[elem(v.aux): elem(v.aux) + 4 * NA].view(NA, 4)}
        out["free_off"] = np.ctypeslib.as_array(C.cast(v.free_off_host, C.POINTER(C.c_int32)), (S + 1,)).copy()
        out["aux_off"] = np.ctypeslib.as_array(C.cast(v.aux_off_host, C.POINTER(C.c_int32)), (S + 1,)).copy()
        return out

    def views(self, x):
        """Typed views of a state tensor: q, qd [S,16], free [NF,16], aux [NA,4]."""
        S, NF, NA = self.S, self.n_free, self.n_aux
        return {"q": x[: 16 * S].view(S, 16), "qd": x[16 * S: 32 * S].view(S, 16),
                "free": x[32 * S: 32 * S + 16 * NF].view(NF, 16),
                "aux": x[32 * S + 16 * NF: 32 * S + 16 * NF + 4 * NA].view(NA, 4)}


def probe_copy(src, dst, stream=None):
    """Enqueue the streaming-copy probe (ms_probe_copy) from ``src`` to ``dst``
    (contiguous device tensors of equal byte size, a multiple of 16)."""
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n:
        raise MsError("probe_copy: src and dst sizes differ")
    _check(lib().ms_probe_copy(_ptr_t(src), _ptr_t(dst), C.c_size_t(n), _stream(stream)), "ms_probe_copy")


def probe_fma(out, blocks, iters, stream=None):
    """Enqueue the FP32 FMA-chain probe (ms_probe_fma); ``out`` is a device
    tensor of at least 1024 floats.  Returns the FLOPs the launch executes."""
    if out.numel() < 1024:
        raise MsError("probe_fma: out needs 1024 floats")
    fl = C.c_double()
    _check(lib().ms_probe_fma(_ptr_t(out), int(blocks), int(iters), _stream(stream), C.byref(fl)), "ms_probe_fma")
    return fl.value
