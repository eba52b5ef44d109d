"""The action front-end (normalized actions in [-1, 1] to PD targets, once per
control step; the action space of the paper's Sec. 4.1): the oracle's mode
equals PD-target mode on targets computed here from the definition; clipping;
its adjoint against central differences."""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg


def targets_by_definition(b, x, a):
    q = sg.split_state(x, b.n_scenes, b.n_free, b.n_aux)["q"]
    out = np.zeros((b.n_scenes, 16))
    for s in range(b.n_scenes):
        m = int(b.scene_model[s])
        kind, sc = b.model_act_kind[m], b.model_act_scale[m].astype(np.float64)
        nb = int(b.model_nb[m])
        ac = np.clip(a[s], -1.0, 1.0)
        jx = [j for j in range(nb) if kind[j] == sg.ACT_BASE_FWD_X][0]
        jy = [j for j in range(nb) if kind[j] == sg.ACT_BASE_YAW][0]
        yaw = q[s, jy]
        for j in range(nb):
            k = kind[j]
            if k == sg.ACT_DELTA:
                out[s, j] = q[s, j] + ac[j] * sc[j]
            elif k == sg.ACT_BASE_FWD_X:
                out[s, j] = ac[j] * sc[j] * math.cos(yaw)
            elif k == sg.ACT_BASE_FWD_Y:
                out[s, j] = ac[jx] * sc[j] * math.sin(yaw)
            elif k == sg.ACT_BASE_YAW:
                out[s, j] = ac[j] * sc[j]
            else:
                out[s, j] = (ac[j] + 1.0) / 2.0 * sc[j]
    return out


@pytest.fixture(scope="module")
def batch_state():
    b = sg.make(6, 6)
    o = oracle.Oracle(b)
    x = b.state0.astype(np.float64)
    for t in range(4):
        x = o.step(x, b.controls_for(t))
    return b, x


def test_actions_equal_pd_targets_by_definition(batch_state):
    b, x = batch_state
    a = np.random.default_rng(3).uniform(-1.2, 1.2, (b.n_scenes, 16))
    xa = oracle.Oracle(b).step(x, a)
    xp = oracle.Oracle(b, control_mode=sg.CTRL_PD).step(x, targets_by_definition(b, x, a))
    np.testing.assert_allclose(xa, xp, rtol=0, atol=1e-12)


def test_actions_are_clipped(batch_state):
    b, x = batch_state
    a = np.random.default_rng(4).uniform(-1, 1, (b.n_scenes, 16))
    a[:, ::3] = 1.0
    big = a.copy()
    big[:, ::3] = 7.5
    o = oracle.Oracle(b)
    np.testing.assert_array_equal(o.step(x, a), o.step(x, big))


def test_action_adjoint_central_differences(batch_state):
    b, x = batch_state
    o = oracle.Oracle(b)
    rng = np.random.default_rng(5)
    a = rng.uniform(-0.9, 0.9, (b.n_scenes, 16))
    g = rng.normal(size=x.size)
    _, ga = o.vjp(x, a, g)
    du = rng.normal(size=a.shape)
    eps = 1e-6
    fd = (g @ o.step(x, a + eps * du) - g @ o.step(x, a - eps * du)) / (2 * eps)
    assert abs(fd - np.sum(ga * du)) <= 1e-5 * max(1.0, abs(fd))


def test_spawn_check_detects_penetration_only():
    """Spawn check: a clear scene passes; a free box moved onto a robot sphere,
    or the robot base pushed into a furniture box, is flagged."""
    b = sg.make(2, 4)
    o = oracle.Oracle(b)
    x = b.state0.astype(np.float64)
    assert np.all(o.spawn_check(x) == 0)
    sph, org, _ = o.fk(int(b.scene_model[0]), sg.split_state(x, b.n_scenes, b.n_free, b.n_aux)["q"][0])
    x1 = x.copy()
    fr = sg.split_state(x1, b.n_scenes, b.n_free, b.n_aux)["free"]
    fr[b.free_off[0], 0:3] = sph[20]               # scene 0: a free body centred on robot sphere 20
    q = sg.split_state(x1, b.n_scenes, b.n_free, b.n_aux)["q"]
    box = b.static_box[b.static_off[1]]
    q[1, 0:2] = box[0:2]                          # scene 1: base moved into its first furniture box
    res = o.spawn_check(x1)
    assert res[0] == 1 and res[1] == 1 and res[2] == 0 and res[3] == 0
