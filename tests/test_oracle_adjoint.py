"""Pins of the oracle's vector-Jacobian product (reverse-mode tape).

- central finite differences (eps = 1e-4) of the FP64 step, on components
  whose contact set and PGS active set do not switch between u +- eps e_i;
- forward / reverse dot-product test <J s, w> = <s, J^T w>;
- closed form: for a ballistic body dx_N / dv_0 = N h.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg


def _batches():
    return [sg.make(1, 3), sg.make(2, 2), sg.make(4, 2), sg.make(5, 2)]


@pytest.fixture(scope="module")
def warm_states():
    """Each batch advanced a few control steps so that contacts are established."""
    out = []
    for b in _batches():
        o = oracle.Oracle(b)
        x = b.state0.astype(np.float64)
        for t in range(3):
            x = o.step(x, b.controls(t))
        out.append((b, o, x, b.controls(3).astype(np.float64)))
    return out


def test_dot_product_forward_reverse(warm_states):
    rng = np.random.default_rng(0)
    for b, o, x, u in warm_states:
        dx = rng.normal(size=x.shape)
        du = rng.normal(size=u.shape)
        w = rng.normal(size=x.shape)
        Js = o.jvp(x, u, dx, du)
        gx, gu = o.vjp(x, u, w)
        lhs = float(Js @ w)
        rhs = float(dx @ gx + (du * gu).sum())
        assert lhs == pytest.approx(rhs, rel=1e-9, abs=1e-9), b.name


def test_vjp_matches_central_fd_non_switching(warm_states):
    rng = np.random.default_rng(1)
    eps = 1e-4
    checked = 0
    for b, o, x, u in warm_states:
        w = rng.normal(size=x.shape)
        gx, gu = o.vjp(x, u, w)
        _, d0 = o.step(x, u, debug=True)
        S = b.n_scenes
        for trial in range(12):
            s = int(rng.integers(S))
            j = int(rng.integers(int(b.model_nb[b.scene_model[s]])))
            e = np.zeros_like(u)
            e[s, j] = eps
            xp, dp = o.step(x, u + e, debug=True)
            xm, dm = o.step(x, u - e, debug=True)
            same = all(np.array_equal(dp[k][s], d0[k][s]) and np.array_equal(dm[k][s], d0[k][s])
                       for k in ("key_hash", "act_hash"))
            if not same:
                continue
            fd = float(w @ (xp - xm)) / (2 * eps)
            assert gu[s, j] == pytest.approx(fd, rel=1e-5, abs=1e-7 * max(1.0, abs(fd))), (b.name, s, j)
            checked += 1
        # a few state components too
        for trial in range(6):
            i = int(rng.integers(x.size))
            e = np.zeros_like(x)
            e[i] = eps
            xp, dp = o.step(x + e, u, debug=True)
            xm, dm = o.step(x - e, u, debug=True)
            same = all(np.array_equal(dp[k], d0[k]) and np.array_equal(dm[k], d0[k]) for k in ("key_hash", "act_hash"))
            if not same:
                continue
            fd = float(w @ (xp - xm)) / (2 * eps)
            assert gx[i] == pytest.approx(fd, rel=1e-5, abs=1e-7 * max(1.0, abs(fd))), (b.name, i)
            checked += 1
    assert checked >= 30


def test_ballistic_sensitivity_closed_form():
    b = sg.custom_batch([sg.empty_model()], [dict(free=[sg.box_object((0.1, 0.1, 0.1), 1.0, (0, 0, 5.0),
                                                                      vel=(0.3, 0, 0))])], h=0.005, n_sub=20)
    o = oracle.Oracle(b)
    x = b.state0.astype(np.float64)
    w = np.zeros_like(x)
    w[32 + 0] = 1.0     # x position of the box after the step
    gx, gu = o.vjp(x, np.zeros((1, 16)), w)
    assert gx[32 + 8] == pytest.approx(20 * 0.005, rel=1e-12)   # dx_N / dv_0 = N h
    assert gx[32 + 0] == pytest.approx(1.0, rel=1e-12)
    assert np.abs(gu).max() == 0.0


def test_differentiation_workload_horizon_central_fd():
    """The differentiation workload's gradient over its whole horizon: two
    scenes of the 256-scene batch, 50 control steps, loss = squared distance
    of the pushed box to its seeded goal; the chained VJP against central
    differences (eps = 1e-4) of the FP64 rollout on sampled torque components
    whose perturbed rollouts keep every substep's contact and active sets."""
    b = sg.make(4)
    pick = [3, 117]
    sub = b.subset(pick)
    o = oracle.Oracle(sub)
    T = b.n_steps
    U = np.stack([b.controls(t, pick) for t in range(T)]).astype(np.float64)
    goals = b.push_goals(pick)
    box = np.array([sub.free_off[s] for s in range(sub.n_scenes)])

    def rollout(Uv):
        xs, hashes = [sub.state0.astype(np.float64)], []
        for t in range(T):
            x, d = o.step(xs[-1], Uv[t], debug=True)
            xs.append(x)
            hashes.append((d["key_hash"].copy(), d["act_hash"].copy()))
        return xs, hashes

    def losses(x):
        fr = sg.split_state(x, sub.n_scenes, sub.n_free, sub.n_aux)["free"]
        return ((fr[box, 0:3] - goals) ** 2).sum(axis=1)

    xs, h0 = rollout(U)
    fr = sg.split_state(xs[-1], sub.n_scenes, sub.n_free, sub.n_aux)["free"]
    g = np.zeros_like(xs[0])
    sg.split_state(g, sub.n_scenes, sub.n_free, sub.n_aux)["free"][box, 0:3] = 2 * (fr[box, 0:3] - goals)
    gU = np.zeros_like(U)
    for t in range(T - 1, -1, -1):
        g, gu = o.vjp(xs[t], U[t], g)
        gU[t] = gu
    rng = np.random.default_rng(5)
    eps = 1e-4
    checked = 0
    for trial in range(16):
        s, t, j = int(rng.integers(2)), int(rng.integers(T)), int(rng.integers(15))
        e = np.zeros_like(U)
        e[t, s, j] = eps
        xp, hp = rollout(U + e)
        xm, hm = rollout(U - e)
        same = all(np.array_equal(a[k][s], c[k][s]) and np.array_equal(a2[k][s], c[k][s])
                   for a, a2, c in zip(hp, hm, h0) for k in (0, 1))
        if not same:
            continue
        fd = (losses(xp[-1])[s] - losses(xm[-1])[s]) / (2 * eps)
        scale = np.abs(gU[:, s]).max()
        assert abs(gU[t, s, j] - fd) <= 1e-3 * scale, (s, t, j, gU[t, s, j], fd)
        checked += 1
    print(f"horizon FD: {checked} of 16 sampled components keep their contact and active sets")
    assert checked >= 6, checked
