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
