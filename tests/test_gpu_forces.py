"""GPU contact-force outputs (ms_set_force_outputs) against the FP64 oracle's
own impulses: the robot's summed normal force and the force its contacts
exert on every free body, over one control step from oracle states.

Bar: per value, |gpu - oracle| <= max(1e-3 |oracle|, 0.05 N, 10 x the spread of
the oracle's forces under 1-ulp float32 perturbations of the state).  0.05 N is
the force a 1e-4 m/s velocity error (the velocity bar of the step) implies for a
1 kg body over a 2 ms substep.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg
from _parity import _ulp_perturb

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def oracle_forces(o, x, u):
    _, d = o.step(x, u, debug=True)
    return d["robot_force"], d["robot_body_force"]


@pytest.mark.parametrize("cfg,n,steps", [(2, 32, 6), (5, 32, 6), (1, 16, 20)])
def test_contact_forces_match_oracle(cfg, n, steps):
    import paper_2412_13211_amd as ms
    b = sg.make(cfg, n)
    o = oracle.Oracle(b, threads=8)
    x = b.state0.astype(np.float64)
    for t in range(steps):
        x = o.step(x, b.controls_for(t))
    x = x.astype(np.float32).astype(np.float64)
    u = b.controls_for(steps)
    fr, fb = oracle_forces(o, x, u)
    rng = np.random.default_rng(0)
    spread_r = np.zeros_like(fr)
    spread_b = np.zeros_like(fb)
    for _ in range(3):
        pr, pb = oracle_forces(o, _ulp_perturb(x, rng), u)
        spread_r = np.maximum(spread_r, np.abs(pr - fr))
        spread_b = np.maximum(spread_b, np.abs(pb - fb))
    mb = ms.MsBatch(b)
    robot_force, body_force = mb.enable_forces()
    xt = torch.as_tensor(x.astype(np.float32)).cuda()
    ut = torch.as_tensor(np.asarray(u, np.float32)).cuda().contiguous()
    mb.step(xt, ut)
    torch.cuda.synchronize()
    gr32, gb32 = robot_force.cpu().numpy().copy(), body_force.cpu().numpy().copy()
    gr = gr32.astype(np.float64)
    gb = gb32[: b.n_free, :3].astype(np.float64)
    bar_r = np.maximum(np.maximum(1e-3 * np.abs(fr), 0.05), 10 * spread_r)
    bar_b = np.maximum(np.maximum(1e-3 * np.abs(fb[: b.n_free]), 0.05), 10 * spread_b[: b.n_free])
    say(f"cfg{cfg}: robot force max {fr.max():.2f} N, max err {np.abs(gr - fr).max():.2e}; "
        f"body force max {np.abs(fb).max():.2f} N, max err {np.abs(gb - fb[: b.n_free]).max():.2e}; "
        f"scenes with robot contact {int(np.count_nonzero(fr))}")
    assert np.all(np.abs(gr - fr) <= bar_r)
    assert np.all(np.abs(gb - fb[: b.n_free]) <= bar_b)
    # the plain per-substep form continues each launch's sums from the last
    # one's: the same outputs bit for bit
    mb.set_schedule(ms.MS_SCHED_PER_SUBSTEP | ms.MS_SCHED_CULL)
    mb.step(xt, ut)
    torch.cuda.synchronize()
    assert np.array_equal(robot_force.cpu().numpy(), gr32)
    assert np.array_equal(body_force.cpu().numpy(), gb32)
    mb.enable_forces(False)
