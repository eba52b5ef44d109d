"""Shared helpers of the GPU parity tests: error metrics against the oracle.

Position error (m): max Euclidean error over robot body origins, robot
sphere centres, free-body centres of mass and free-box vertices, computed by
the oracle's forward kinematics on both states.  Velocity error: max
absolute error over joint velocities and free-body linear / angular
velocities.  Quaternions are compared through the vertices they place.
"""
import numpy as np

import oracle
import scenegen as sg


def world_points(o, batch, x):
    """Per scene: array of world points (robot origins + spheres + free COMs + box vertices)."""
    st = sg.split_state(np.asarray(x, np.float64), batch.n_scenes, batch.n_free, batch.n_aux)
    pts = []
    for s in range(batch.n_scenes):
        m = int(batch.scene_model[s])
        sph, org, _ = o.fk(m, st["q"][s])
        P = [sph, org]
        for f in range(batch.free_off[s], batch.free_off[s + 1]):
            fr = st["free"][f]
            x0 = fr[0:3]
            P.append(x0[None])
            if batch.free_type[f] == sg.FREE_BOX:
                q = fr[4:8] / np.linalg.norm(fr[4:8])
                w, a, b, c = q
                R = np.array([[1 - 2 * (b * b + c * c), 2 * (a * b - w * c), 2 * (a * c + w * b)],
                              [2 * (a * b + w * c), 1 - 2 * (a * a + c * c), 2 * (b * c - w * a)],
                              [2 * (a * c - w * b), 2 * (b * c + w * a), 1 - 2 * (a * a + b * b)]])
                h = batch.free_size[f].astype(np.float64)
                V = np.array([[(k & 1) * 2 - 1, ((k >> 1) & 1) * 2 - 1, ((k >> 2) & 1) * 2 - 1] for k in range(8)]) * h
                P.append(V @ R.T + x0)
        pts.append(np.concatenate(P))
    return pts


def velocities(batch, x):
    st = sg.split_state(np.asarray(x, np.float64), batch.n_scenes, batch.n_free, batch.n_aux)
    out = []
    for s in range(batch.n_scenes):
        v = [st["qd"][s]]
        for f in range(batch.free_off[s], batch.free_off[s + 1]):
            v.append(st["free"][f, 8:11])
            v.append(st["free"][f, 12:15])
        for a in range(batch.aux_off[s], batch.aux_off[s + 1]):
            v.append(st["aux"][a, 1:2])
        out.append(np.concatenate(v))
    return out


def aux_positions(batch, x):
    st = sg.split_state(np.asarray(x, np.float64), batch.n_scenes, batch.n_free, batch.n_aux)
    return [st["aux"][batch.aux_off[s]:batch.aux_off[s + 1], 0] for s in range(batch.n_scenes)]


def errors(o, batch, xa, xb):
    """Per-scene (position error, velocity error) between two states."""
    pa, pb = world_points(o, batch, xa), world_points(o, batch, xb)
    va, vb = velocities(batch, xa), velocities(batch, xb)
    aa, ab = aux_positions(batch, xa), aux_positions(batch, xb)
    pos = np.array([np.max(np.linalg.norm(a - b, axis=1)) if len(a) else 0.0 for a, b in zip(pa, pb)])
    aux = np.array([np.max(np.abs(a - b)) if len(a) else 0.0 for a, b in zip(aa, ab)])
    vel = np.array([np.max(np.abs(a - b)) for a, b in zip(va, vb)])
    return np.maximum(pos, aux), vel


def oracle_debug_hash(d):
    """Oracle per-substep (count, key-sum) comparable with the GPU debug words."""
    return d["n_contacts"].astype(np.int64), d["key_hash"].astype(np.uint64)


def gpu_debug_hash(dbg):
    cnt = dbg[:, :, 0].astype(np.int64)
    ks = dbg[:, :, 2].astype(np.uint64) | (dbg[:, :, 3].astype(np.uint64) << np.uint64(32))
    return cnt, ks


def same_contacts(d_oracle, dbg_gpu):
    """Per scene: True when every substep's contact key set agrees (count and key sum)."""
    oc, ok = oracle_debug_hash(d_oracle)
    gc, gk = gpu_debug_hash(dbg_gpu)
    return np.all(oc == gc, axis=1) & np.all(ok == gk, axis=1)


def _ulp_perturb(x, rng):
    """Round to float32 and move each component by -1, 0 or +1 ulp (seeded)."""
    xp = np.asarray(x, np.float64).astype(np.float32)
    sgn = rng.integers(0, 3, xp.shape) - 1
    up = np.nextafter(xp, np.float32(np.inf))
    dn = np.nextafter(xp, np.float32(-np.inf))
    return np.where(sgn > 0, up, np.where(sgn < 0, dn, xp)).astype(np.float64)


def fp32_sensitivity(o, batch, x, u, trials=8, seed=0):
    """Per scene: the oracle's own output change (position, velocity) when its
    float32 input state is moved by random 1-ulp steps, over the trials that
    keep the scene's contact sets.  This is the floor any float32 evaluation
    of the same step faces; the parity bar is scaled by it where it exceeds
    the fixed bar (ill-conditioned contact configurations)."""
    rng = np.random.default_rng(seed)
    x0, d0 = o.step(x, u, debug=True)
    ps = np.zeros(batch.n_scenes)
    vs = np.zeros(batch.n_scenes)
    for _ in range(trials):
        xp = _ulp_perturb(x, rng)
        x1, d1 = o.step(xp, u, debug=True)
        keep = np.all(d1["key_hash"] == d0["key_hash"], axis=1) & np.all(d1["n_contacts"] == d0["n_contacts"], axis=1)
        pe, ve = errors(o, batch, x0, x1)
        ps = np.where(keep, np.maximum(ps, pe), ps)
        vs = np.where(keep, np.maximum(vs, ve), vs)
    return ps, vs


def noisy_fp32_rollout(o, batch, x0, controls, seed=0):
    """Oracle rollout whose state is rounded to float32 and moved by random
    1-ulp steps after every control step (the chaos screen)."""
    rng = np.random.default_rng(seed)
    x = np.asarray(x0, np.float64)
    for u in controls:
        x = _ulp_perturb(o.step(x, u), rng)
    return x
