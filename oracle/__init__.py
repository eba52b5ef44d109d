"""FP64 CPU oracle of the batched rigid-body step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The GPU library never links or calls it, and it
shares no code with the GPU path: it reads the same generated scene arrays
through its own reader (``ms_oracle.hpp``).

Parity status per function (details in the design notes):
  or_step      pinned by closed forms and invariants (tests/test_oracle_*.py),
               including the robot and door / drawer contact rows, joint-limit
               rows, implicit PD drive, joint damping, gyroscopic term and the
               robot contact cap (tests/_pins.py); each of those pins is shown
               to fail on a copy with a planted mistake (tests/_mutants.py)
  or_vjp/jvp   pinned by central finite differences, the dot-product test and
               the ballistic and sliding closed-form sensitivities
  multi-contact friction at finite PGS sweeps: parity unpinned beyond the
  single-contact closed forms and physical-plausibility checks.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = [os.path.join(HERE, "ms_oracle.cpp")]
HDR = [os.path.join(HERE, "ms_oracle.hpp"), os.path.join(HERE, "ms_ad.hpp")]


def build(force=False):
    """Compile the oracle with g++ (FP64, no fast-math, no FMA contraction)."""
    newest = max(os.path.getmtime(p) for p in SRC + HDR)
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= newest:
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", tmp] + SRC + ["-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def source_texts():
    """The oracle's source files by name (ms_oracle.cpp and its headers)."""
    out = {}
    for p in SRC + HDR:
        with open(p) as f:
            out[os.path.basename(p)] = f.read()
    return out


def build_variant(texts, out_dir, opt="-O1"):
    """Compile another text of the oracle's sources (the tests plant single
    mistakes in a copy to show that a pin catches them) in ``out_dir``;
    ``texts`` maps file names to contents, as source_texts() returns them.
    Returns the library's path."""
    os.makedirs(out_dir, exist_ok=True)
    for name, text in texts.items():
        with open(os.path.join(out_dir, name), "w") as f:
            f.write(text)
    src = os.path.join(out_dir, "ms_oracle.cpp")
    out_path = os.path.join(out_dir, "liboracle_variant.so")
    subprocess.check_call(["g++", opt, "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                           "-w", "-o", out_path, src, "-lpthread"])
    return out_path


class OrScene(C.Structure):
    _fields_ = [("n_scenes", C.c_int32), ("n_models", C.c_int32)] + [
        (n, C.c_void_p) for n in [
            "model_nb", "model_parent", "model_jtype", "model_axis", "model_xt_rot", "model_xt_pos",
            "model_mass", "model_com", "model_inertia", "model_kp", "model_kd", "model_veldof", "model_armature",
            "model_damping", "model_act_kind", "model_act_scale", "model_nsph",
            "model_sph_body", "model_sph", "model_sph_flags", "scene_model", "free_off", "static_off",
            "plane_off", "aux_off", "scene_hold", "free_type", "free_size", "free_mass", "free_inertia",
            "static_box", "plane", "aux_type", "aux_rot", "aux_pos", "aux_axis", "aux_box", "aux_mass",
            "aux_inertia", "aux_limit"]]


class OrParams(C.Structure):
    _fields_ = [("h", C.c_double), ("mu", C.c_double), ("baumgarte", C.c_double), ("margin", C.c_double),
                ("gravity", C.c_double * 3), ("n_sub", C.c_int32), ("pgs_iters", C.c_int32),
                ("control_mode", C.c_int32), ("contact_cap", C.c_int32), ("robot_contact_cap", C.c_int32)]


class OrDebug(C.Structure):
    _fields_ = [("status", C.c_void_p), ("n_contacts", C.c_void_p), ("key_hash", C.c_void_p),
                ("act_hash", C.c_void_p), ("dump_cap", C.c_int32), ("dump_keys", C.c_void_p),
                ("dump_phi", C.c_void_p), ("dump_lambda", C.c_void_p), ("dump_y", C.c_void_p),
                ("robot_force", C.c_void_p),
                ("robot_body_force", C.c_void_p), ("grip_ee", C.c_uint32), ("grip_finger_l", C.c_int32),
                ("grip_finger_r", C.c_int32), ("grip", C.c_void_p)]


_libs = {}


def lib(path=None):
    """The oracle library (ctypes), built on first use; ``path`` loads another
    build of the same source (the tests' planted-mistake copies)."""
    path = LIB if path is None else path
    if path not in _libs:
        if path == LIB and not os.path.exists(LIB):
            build()
        L = C.CDLL(path)
        vp = C.c_void_p
        for name, args in [("or_step", [vp, vp, vp, vp, vp, C.c_int, vp]),
                           ("or_vjp", [vp, vp, vp, vp, vp, vp, vp, C.c_int]),
                           ("or_step_f32", [vp, vp, vp, vp, vp, C.c_int, vp]),
                           ("or_jvp", [vp, vp, vp, vp, vp, vp, vp, C.c_int]),
                           ("or_flops", [vp, vp, vp, vp, vp]),
                           ("or_fk", [vp, C.c_int, vp, vp, vp, vp]),
                           ("or_dynamics", [vp, C.c_int, vp, vp, vp, vp, vp]),
                           ("or_aba", [vp, C.c_int, vp, vp, vp, vp, vp, vp]),
                           ("or_pair", [C.c_int, vp, C.c_double, vp, vp]),
                           ("or_spawn_check", [vp, vp, vp, vp, C.c_int])]:
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.or_kinetic_energy.argtypes = [vp, C.c_int, vp, vp]
        L.or_kinetic_energy.restype = C.c_double
        L.or_onb.argtypes = [vp, vp, vp]
        L.or_onb.restype = None
        L.or_quat_update.argtypes = [vp, vp, C.c_double, vp]
        L.or_quat_update.restype = None
        _libs[path] = L
    return _libs[path]


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None and a.size else C.c_void_p(0)


class Oracle:
    """FP64 oracle bound to one generated scene batch."""

    _ARRS = ["model_nb", "model_parent", "model_jtype", "model_axis", "model_xt_rot", "model_xt_pos",
             "model_mass", "model_com", "model_inertia", "model_kp", "model_kd", "model_veldof", "model_armature",
            "model_damping", "model_act_kind", "model_act_scale", "model_nsph",
             "model_sph_body", "model_sph", "model_sph_flags", "scene_model", "free_off", "static_off",
             "plane_off", "aux_off", "scene_hold", "free_type", "free_size", "free_mass", "free_inertia",
             "static_box", "plane", "aux_type", "aux_rot", "aux_pos", "aux_axis", "aux_box", "aux_mass",
             "aux_inertia", "aux_limit"]

    def __init__(self, batch, threads=0, lib_path=None, **overrides):
        self.batch = batch
        self._L = lib(lib_path)
        self.threads = threads
        self._keep = {}
        sc = OrScene()
        sc.n_scenes = batch.n_scenes
        sc.n_models = len(batch.model_nb)
        for n in self._ARRS:
            a = np.ascontiguousarray(getattr(batch, n))
            a = a.astype(np.int32 if a.dtype.kind in "iu" else np.float32, copy=False)
            self._keep[n] = a
            setattr(sc, n, _ptr(a))
        self.sc = sc
        p = OrParams()
        get = lambda k: overrides.get(k, getattr(batch, k))
        p.h = get("h")
        p.mu = get("mu")
        p.baumgarte = get("baumgarte")
        p.margin = get("margin")
        g = get("gravity")
        for i in range(3):
            p.gravity[i] = g[i]
        p.n_sub = get("n_sub")
        p.pgs_iters = get("pgs_iters")
        p.control_mode = get("control_mode")
        p.contact_cap = get("contact_cap")
        p.robot_contact_cap = get("robot_contact_cap")
        self.params = p
        self.S = batch.n_scenes
        self.nsf = batch.state_floats
        # gripper outputs of step(debug=True): (end-effector body mask, finger L, finger R) or None
        self.grip_cfg = None

    # ------------------------------------------------------------------
    def step(self, x, u, debug=False, dump_cap=0):
        """One control step; returns the new state (float64) [and diagnostics]."""
        x = np.ascontiguousarray(x, np.float64)
        u = np.ascontiguousarray(u, np.float64).reshape(self.S, 16)
        out = np.empty(self.nsf, np.float64)
        dbg = None
        d = {}
        if debug or dump_cap:
            ns = self.params.n_sub
            d = dict(status=np.zeros(self.S, np.uint32), n_contacts=np.zeros((self.S, ns), np.int32),
                     key_hash=np.zeros((self.S, ns), np.uint64), act_hash=np.zeros((self.S, ns), np.uint64),
                     robot_force=np.zeros(self.S, np.float64),
                     robot_body_force=np.zeros((max(self.batch.n_free, 1), 3), np.float64))
            if self.grip_cfg is not None:
                d["grip"] = np.zeros((max(self.batch.n_free + self.batch.n_aux, 1), 2), np.float64)
            if dump_cap:
                d["dump_keys"] = np.zeros((self.S, dump_cap), np.uint64)
                d["dump_phi"] = np.zeros((self.S, dump_cap), np.float64)
                d["dump_lambda"] = np.zeros((self.S, dump_cap, 3), np.float64)
                d["dump_y"] = np.zeros((self.S, self.params.pgs_iters, dump_cap, 3), np.float64)
            dbg = OrDebug()
            for k, v in d.items():
                setattr(dbg, k, _ptr(v))
            dbg.dump_cap = dump_cap
            if self.grip_cfg is not None:
                dbg.grip_ee, dbg.grip_finger_l, dbg.grip_finger_r = self.grip_cfg
        rc = self._L.or_step(C.byref(self.sc), C.byref(self.params), _ptr(x), _ptr(u), _ptr(out), self.threads,
                           C.byref(dbg) if dbg is not None else None)
        if rc != 0:
            raise RuntimeError(f"or_step failed: {rc}")
        return (out, d) if dbg is not None else out

    def step_f32(self, x, u, dump_cap=0):
        """The same step in IEEE single precision (error floor of an FP32
        evaluation); with dump_cap also the last substep's impulses and
        pre-projection values, as step() gives them."""
        x = np.ascontiguousarray(x, np.float64)
        u = np.ascontiguousarray(u, np.float64).reshape(self.S, 16)
        out = np.empty(self.nsf, np.float64)
        d = {}
        dbg = None
        if dump_cap:
            d = dict(dump_keys=np.zeros((self.S, dump_cap), np.uint64),
                     dump_phi=np.zeros((self.S, dump_cap), np.float64),
                     dump_lambda=np.zeros((self.S, dump_cap, 3), np.float64),
                     dump_y=np.zeros((self.S, self.params.pgs_iters, dump_cap, 3), np.float64))
            dbg = OrDebug()
            for k, v in d.items():
                setattr(dbg, k, _ptr(v))
            dbg.dump_cap = dump_cap
        if self._L.or_step_f32(C.byref(self.sc), C.byref(self.params), _ptr(x), _ptr(u), _ptr(out), self.threads,
                               C.byref(dbg) if dbg is not None else None):
            raise RuntimeError("or_step_f32 failed")
        return (out, d) if dump_cap else out

    def rollout(self, x0, controls, debug=False):
        xs = [np.asarray(x0, np.float64)]
        dbgs = []
        for t in range(len(controls)):
            r = self.step(xs[-1], controls[t], debug=debug)
            if debug:
                xs.append(r[0])
                dbgs.append(r[1])
            else:
                xs.append(r)
        return (xs, dbgs) if debug else xs

    def spawn_check(self, x, with_phi=False):
        """Per scene 1 where a robot sphere penetrates another body (phi < 0);
        with_phi: also the smallest signed distance per scene."""
        x = np.ascontiguousarray(x, np.float64)
        out = np.zeros(self.S, np.int32)
        phi = np.zeros(self.S, np.float64)
        if self._L.or_spawn_check(C.byref(self.sc), _ptr(x), _ptr(out), _ptr(phi), self.threads):
            raise RuntimeError("or_spawn_check failed")
        return (out, phi) if with_phi else out

    def vjp(self, x, u, gx_out):
        x = np.ascontiguousarray(x, np.float64)
        u = np.ascontiguousarray(u, np.float64).reshape(self.S, 16)
        g = np.ascontiguousarray(gx_out, np.float64)
        gx = np.zeros(self.nsf, np.float64)
        gu = np.zeros((self.S, 16), np.float64)
        rc = self._L.or_vjp(C.byref(self.sc), C.byref(self.params), _ptr(x), _ptr(u), _ptr(g), _ptr(gx), _ptr(gu),
                          self.threads)
        if rc != 0:
            raise RuntimeError("or_vjp failed")
        return gx, gu

    def jvp(self, x, u, dx, du):
        x = np.ascontiguousarray(x, np.float64)
        u = np.ascontiguousarray(u, np.float64).reshape(self.S, 16)
        dx = np.ascontiguousarray(dx, np.float64)
        du = np.ascontiguousarray(du, np.float64).reshape(self.S, 16)
        out = np.zeros(self.nsf, np.float64)
        rc = self._L.or_jvp(C.byref(self.sc), C.byref(self.params), _ptr(x), _ptr(u), _ptr(dx), _ptr(du), _ptr(out),
                          self.threads)
        if rc != 0:
            raise RuntimeError("or_jvp failed")
        return out

    def flops(self, x, u):
        x = np.ascontiguousarray(x, np.float64)
        u = np.ascontiguousarray(u, np.float64).reshape(self.S, 16)
        out = np.zeros(self.S, np.float64)
        self._L.or_flops(C.byref(self.sc), C.byref(self.params), _ptr(x), _ptr(u), _ptr(out))
        return out

    # ---- probes -------------------------------------------------------
    def fk(self, model, q):
        q = np.ascontiguousarray(q, np.float64)
        ns = int(self.batch.model_nsph[model])
        sph = np.zeros((max(ns, 1), 3))
        org = np.zeros((16, 3))
        rot = np.zeros((16, 9))
        nb = self._L.or_fk(C.byref(self.sc), model, _ptr(q), _ptr(sph), _ptr(org), _ptr(rot))
        return sph[:ns], org[:nb], rot[:nb].reshape(nb, 3, 3)

    def dynamics(self, model, q, qd, g=(0.0, 0.0, -9.81)):
        q = np.ascontiguousarray(q, np.float64)
        qd = np.ascontiguousarray(qd, np.float64)
        g = np.ascontiguousarray(g, np.float64)
        M = np.zeros((16, 16))
        Cb = np.zeros(16)
        nb = self._L.or_dynamics(C.byref(self.sc), model, _ptr(q), _ptr(qd), _ptr(g), _ptr(M), _ptr(Cb))
        return M[:nb, :nb], Cb[:nb]

    def aba(self, model, q, qd, tau, arm=None, g=(0.0, 0.0, -9.81)):
        q = np.ascontiguousarray(q, np.float64)
        qd = np.ascontiguousarray(qd, np.float64)
        tau = np.ascontiguousarray(tau, np.float64)
        arm = np.zeros(16) if arm is None else np.ascontiguousarray(arm, np.float64)
        g = np.ascontiguousarray(g, np.float64)
        out = np.zeros(16)
        nb = self._L.or_aba(C.byref(self.sc), model, _ptr(q), _ptr(qd), _ptr(tau), _ptr(arm), _ptr(g), _ptr(out))
        return out[:nb]

    def kinetic_energy(self, model, q, qd):
        q = np.ascontiguousarray(q, np.float64)
        qd = np.ascontiguousarray(qd, np.float64)
        return self._L.or_kinetic_energy(C.byref(self.sc), model, _ptr(q), _ptr(qd))


def pair(kind, c, r, prim):
    c = np.ascontiguousarray(c, np.float64)
    prim = np.ascontiguousarray(prim, np.float64)
    out = np.zeros(7)
    lib().or_pair(kind, _ptr(c), float(r), _ptr(prim), _ptr(out))
    return out[0], out[1:4], out[4:7]


def onb(n):
    n = np.ascontiguousarray(n, np.float64)
    t1 = np.zeros(3)
    t2 = np.zeros(3)
    lib().or_onb(_ptr(n), _ptr(t1), _ptr(t2))
    return t1, t2


def quat_update(Q, w, h):
    Q = np.ascontiguousarray(Q, np.float64)
    w = np.ascontiguousarray(w, np.float64)
    out = np.zeros(4)
    lib().or_quat_update(_ptr(Q), _ptr(w), float(h), _ptr(out))
    return out
