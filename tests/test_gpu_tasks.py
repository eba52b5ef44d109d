"""GPU subtask predicates, event labels and trajectory categories
(ms_task_begin / ms_task_update / ms_task_categorize) against the task
oracle, and the gripper contact outputs of the step (ms_set_grip_outputs)
against the FP64 step oracle.

Task kernels: both sides get the same inputs (states, robot forces, gripper
outputs).  The scripted inputs keep every predicate value far from its
threshold, so the decisions are compared exactly; predicate values to 1e-5
relative.  Gripper outputs: the bar of the contact-force outputs, per value
|gpu - oracle| <= max(1e-3 |oracle|, 0.05 N, 10 x the oracle's spread under
1-ulp float32 perturbations of the state).
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import scenegen as sg
from oracle import tasks as ot
from _parity import _ulp_perturb
from test_oracle_tasks import CASES

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def robot_for(b):
    r = dict(sg.FETCH_TASK_ROBOT)
    r["ee_rest"] = (0.0, 0.0, 0.0)
    r["ee_rest"] = tuple(float(v) for v in ot.ee_in_base(b, 0, np.asarray(sg.FETCH_REST), r))
    return r


def grasp_batch(n=4):
    """Fetch-like robot at rest, fingers open 0.03 m, a 3 x 6 x 4 cm box
    between the finger tips (each finger sphere overlaps it by 5 mm); PD
    targets close the fingers."""
    model = sg.fetch_like_model(np.random.default_rng(11))
    q = np.array(sg.FETCH_REST, np.float64)
    bare = sg.custom_batch([model], [dict(q=q)], h=0.002, n_sub=5, control_mode=sg.CTRL_PD)
    r = robot_for(bare)
    R, p = ot.body_pose(bare, 0, q, r["ee_body"])
    centre = p + R @ np.array([0.23, 0.0, 0.0])
    wxyz = np.roll(Rotation.from_matrix(R).as_quat(), 1)
    scenes = [dict(q=q, free=[sg.box_object((0.015, 0.03, 0.02), 0.2, centre, quat=wxyz)],
                   planes=[(0.0, 0.0, 1.0, 0.0)]) for _ in range(n)]
    b = sg.custom_batch([model], scenes, h=0.002, n_sub=5, control_mode=sg.CTRL_PD)
    u = np.tile(np.array(sg.FETCH_REST, np.float32), (n, 1))
    u[:, 13:15] = 0.0
    return b, u


def oracle_grip(o, x, u):
    _, d = o.step(x, u, debug=True)
    return d["grip"], d["robot_force"]


@pytest.mark.parametrize("which", ["grasp", "cfg5", "cfg2"])
def test_grip_outputs_match_oracle(which):
    import paper_2412_13211_amd as ms
    if which == "grasp":
        b, u = grasp_batch()
        x = b.state0.astype(np.float64)
    else:
        b = sg.make(5 if which == "cfg5" else 2, 32)
        x = b.state0.astype(np.float64)
        o0 = oracle.Oracle(b, threads=8)
        for t in range(6):
            x = o0.step(x, b.controls_for(t))
        u = b.controls_for(6)
    r = robot_for(b)
    o = oracle.Oracle(b, threads=8)
    o.grip_cfg = (r["ee_bodies"], r["finger_l"], r["finger_r"])
    x = x.astype(np.float32).astype(np.float64)
    g_o, _ = oracle_grip(o, x, u)
    rng = np.random.default_rng(1)
    spread = np.zeros_like(g_o)
    for _ in range(3):
        gp, _ = oracle_grip(o, _ulp_perturb(x, rng), u)
        spread = np.maximum(spread, np.abs(gp - g_o))
    mb = ms.MsBatch(b)
    mb.set_task_robot(r)
    grip = mb.enable_grip()
    mb.enable_forces()
    xt = torch.as_tensor(x.astype(np.float32)).cuda()
    ut = torch.as_tensor(np.asarray(u, np.float32)).cuda().contiguous()
    mb.step(xt, ut)
    torch.cuda.synchronize()
    g_g = grip.cpu().numpy().astype(np.float64)[: b.n_free + b.n_aux]
    g_o = g_o[: b.n_free + b.n_aux]
    bar = np.maximum(np.maximum(1e-3 * np.abs(g_o), 0.05), 10 * spread[: b.n_free + b.n_aux])
    say(f"{which}: ee force rows with contact {int(np.count_nonzero(g_o[:, 0]))}, max {g_o[:, 0].max():.2f} N; "
        f"finger rows {int(np.count_nonzero(g_o[:, 1]))}, max {g_o[:, 1].max():.3f} N; "
        f"max err {np.abs(g_g - g_o).max():.2e}")
    assert np.all(np.abs(g_g - g_o) <= bar)
    if which == "grasp":
        # every scene grasps its box: both fingers press on it
        assert np.all(g_o[:, 1] > 0.5) and np.all(g_g[:, 1] > 0.5)
    # the per-substep schedule writes the same outputs
    mb.set_schedule(ms.MS_SCHED_PER_SUBSTEP | ms.MS_SCHED_CULL)
    mb.step(xt, ut)
    torch.cuda.synchronize()
    assert np.allclose(grip.cpu().numpy()[: b.n_free + b.n_aux], g_g, rtol=1e-4, atol=1e-3)
    mb.enable_grip(False)


def scripted_inputs(b, tasks, r, steps, seed=3):
    """Per step: state, robot force [S] and gripper outputs chosen from
    far-from-threshold alternatives (rest / away, static / moving, object at /
    away from the goal, joint fractions 0, 0.3, 0.5, 0.95, fingers 0 / 2 N,
    end-effector force 0 / 3 N, robot force 0 / 1700 N)."""
    rng = np.random.default_rng(seed)
    S, NF, NA = b.n_scenes, b.n_free, b.n_aux
    out = []
    for t in range(steps + 1):
        x = np.array(b.state0, np.float32)
        st = sg.split_state(x, S, NF, NA)
        grip = np.zeros((NF + NA, 2), np.float32)
        for s in range(S):
            q = np.array(r["q_rest"], np.float32) + rng.normal(0, 1e-4, 16).astype(np.float32)
            if rng.uniform() < 0.3:
                q[6:13] += rng.choice([-1, 1], 7) * rng.uniform(0.3, 0.5, 7)
            q[0:3] = rng.uniform(-1, 1, 3)
            st["q"][s] = q
            st["qd"][s] = 0.0
            if rng.uniform() < 0.3:
                st["qd"][s, rng.integers(0, 13)] = rng.choice([-1.0, 1.0])
            tk = tasks[s]
            f0, a0 = int(b.free_off[s]), int(b.aux_off[s])
            if tk["kind"] in (ot.PICK, ot.PLACE):
                row = f0 + tk["target"]
                d = rng.normal(size=3)
                d /= np.linalg.norm(d)
                st["free"][row, :3] = np.asarray(tk["goal"], np.float32) + d * (0.05 if rng.uniform() < 0.5 else 0.5)
            else:
                row = NF + a0 + tk["target"]
                lo, hi = b.aux_limit[a0 + tk["target"]]
                st["aux"][a0 + tk["target"], 0] = lo + rng.choice([0.0, 0.3, 0.5, 0.95]) * (hi - lo)
            grip[row, 0] = 3.0 * b.n_sub if rng.uniform() < 0.5 else 0.0
            grip[row, 1] = 2.0 if rng.uniform() < 0.5 else 0.0
        rf = np.where(rng.uniform(size=S) < 0.4, 1700.0 * b.n_sub, 0.0).astype(np.float32)
        out.append((x, rf, grip))
    return out


def test_task_kernels_match_oracle_on_scripted_inputs():
    import paper_2412_13211_amd as ms
    b = sg.make(5, 48)
    tasks = sg.tasks(b)
    tasks[5]["target"] = 99                     # an invalid task: no episode
    r = robot_for(b)
    steps = 14
    seq = scripted_inputs(b, tasks, r, steps)
    mb = ms.MsBatch(b)
    mb.set_task_robot(r)
    tt = mb.task_tensor(tasks)
    dev = lambda a: torch.as_tensor(a).cuda().contiguous()
    eo = ot.Episodes(b, tasks, r, n_sub=b.n_sub)
    x0, _, g0 = seq[0]
    ep, pred = mb.task_begin(dev(x0), tt, grip=dev(g0), pred=True)
    eo.begin(x0.astype(np.float64), grip=g0.astype(np.float64))
    n_events = 0
    for t in range(1, steps + 1):
        x, rf, gr = seq[t]
        pred = mb.task_update(dev(x), tt, ep, dev(rf), grip=dev(gr), pred=True)
        eo.update(x.astype(np.float64), rf.astype(np.float64), grip=gr.astype(np.float64))
        E = mb.episodes(ep)
        pv = pred.cpu().numpy()
        for s in range(b.n_scenes):
            v = eo.values[s]
            if v is None:
                assert E[s]["ind"] == 0xFFFFFFFF
                continue
            ref = [v["d_ee"], v["j_arm"], v["j_torso"], v["qd_arm"], v["d_goal"], v["aq"], v["f_ee"], v["f_finger"]]
            assert np.allclose(pv[s], ref, rtol=1e-5, atol=2e-6), (t, s, pv[s], ref)
            ind = eo.ind[s]
            bits = (ms.MS_IND_GRASPED * ind["grasped"] | ms.MS_IND_SUCCESS * ind["success"]
                    | ms.MS_IND_CONTACT * ind["contact"] | ms.MS_IND_EXCESSIVE * ind["excessive"]
                    | ms.MS_IND_AT_GOAL * ind.get("at_goal", False) | ms.MS_IND_OPEN * ind.get("state", False)
                    | ms.MS_IND_SLIGHT * ind.get("slight", False))
            assert int(E[s]["ind"]) == bits, (t, s)
            assert abs(float(E[s]["cumcol"]) - eo.cumcol[s]) <= 1e-3
    E = mb.episodes(ep)
    for s in range(b.n_scenes):
        if eo.ind[s] is None:
            continue
        kind = tasks[s]["kind"]
        names = [ot.EVENTS[kind][c] for c in E[s]["list"][: min(int(E[s]["n"]), ms.MS_EP_LIST)]]
        assert int(E[s]["n"]) == len(eo.events[s])
        assert names == eo.events[s][: ms.MS_EP_LIST], (s, names, eo.events[s])
        for c, nm in enumerate(ot.EVENTS[kind]):
            assert int(E[s]["last"][c]) == ot._idx(eo.events[s], nm)
        n_events += len(eo.events[s])
    modes = mb.task_categorize(tt, ep).cpu().numpy()
    ref = [0 if eo.ind[s] is None else ot.categorize(tasks[s]["kind"], eo.events[s], eo.d0[s])
           for s in range(b.n_scenes)]
    say(f"scripted: {n_events} events over {b.n_scenes} scenes; modes {np.bincount(modes)}")
    assert list(modes) == ref
    assert n_events > 5 * b.n_scenes


def test_categories_on_crafted_episodes():
    """Every success / failure mode from the hand-built lists of the oracle pins."""
    import paper_2412_13211_amd as ms
    b = sg.make(5, len(CASES))
    mb = ms.MsBatch(b)
    tasks = [dict(kind=k, target=0, goal=(0, 0, 0), open_frac=0.9) for k, _, _, _ in CASES]
    ep = np.zeros(len(CASES), ms.EPISODE_DTYPE)
    for s, (kind, E, d0, _) in enumerate(CASES):
        codes = [ot.EVENTS[kind].index(e) for e in E]
        ep[s]["n"] = len(codes)
        ep[s]["list"][: len(codes)] = codes
        ep[s]["last"][:] = -1
        for i, c in enumerate(codes):
            ep[s]["last"][c] = i
        ep[s]["d0"] = d0
    ept = torch.from_numpy(ep.view(np.uint8).copy()).cuda()
    modes = mb.task_categorize(mb.task_tensor(tasks), ept).cpu().numpy()
    assert list(modes) == [m for _, _, _, m in CASES]


def test_rollout_tasks_match_oracle():
    """Predicates and events along a physics rollout (config 5, door and
    drawer tasks included), fed with the GPU's own states and force outputs;
    scenes with a predicate within 1e-4 of a threshold are left out."""
    import paper_2412_13211_amd as ms
    b = sg.make(5, 64)
    tasks = sg.tasks(b)
    r = robot_for(b)
    mb = ms.MsBatch(b)
    mb.set_task_robot(r)
    rfo, _ = mb.enable_forces()
    grip = mb.enable_grip()
    tt = mb.task_tensor(tasks)
    x = torch.as_tensor(b.state0).cuda()
    ep, _ = mb.task_begin(x, tt)
    eo = ot.Episodes(b, tasks, r, n_sub=b.n_sub)
    eo.begin(x.cpu().numpy().astype(np.float64))
    near = np.zeros(b.n_scenes, bool)
    for t in range(10):
        x = mb.step(x, torch.as_tensor(b.controls_for(t)).cuda().contiguous())
        mb.task_update(x, tt, ep, rfo, grip=grip)
        xh = x.cpu().numpy().astype(np.float64)
        eo.update(xh, rfo.cpu().numpy().astype(np.float64), grip=grip.cpu().numpy().astype(np.float64))
        for s, v in enumerate(eo.values):
            if v is None:
                continue
            span = v.get("hi", 1.0) - v.get("lo", 0.0)
            checks = [(v["d_ee"], 0.05), (v["j_arm"], 0.6 if v["kind"] == ot.PICK else 0.2), (v["j_torso"], 0.01),
                      (v["qd_arm"], 0.2), (v["d_goal"], 0.15), (v["f_finger"], r["grasp_force"])]
            if v["kind"] in (ot.OPEN, ot.CLOSE):
                for f in (0.01, 0.1, tasks[s]["open_frac"]):
                    checks.append((v["aq"], v["lo"] + f * span))
                checks.append((v["aq"], eo.aq0[s] - 0.05 * span))
            q = xh[32 * b.n_scenes:]  # noqa: F841 (state views are not needed here)
            near[s] |= any(abs(a - c) < 1e-4 for a, c in checks)
    E = mb.episodes(ep)
    modes = mb.task_categorize(tt, ep).cpu().numpy()
    cmp = 0
    for s in range(b.n_scenes):
        if near[s] or eo.ind[s] is None:
            continue
        kind = tasks[s]["kind"]
        names = [ot.EVENTS[kind][c] for c in E[s]["list"][: min(int(E[s]["n"]), ms.MS_EP_LIST)]]
        assert names == eo.events[s][: ms.MS_EP_LIST], (s, names, eo.events[s])
        assert modes[s] == ot.categorize(kind, eo.events[s], eo.d0[s])
        cmp += 1
    say(f"rollout: {cmp} of {b.n_scenes} scenes compared; events {sum(len(e) for e in eo.events)}")
    assert cmp >= b.n_scenes // 2


def test_task_argument_errors():
    import paper_2412_13211_amd as ms
    b = sg.make(5, 4)
    mb = ms.MsBatch(b)
    with pytest.raises(ms.MsError, match="ms_set_task_robot first"):
        mb.enable_grip()
    x = torch.as_tensor(b.state0).cuda()
    tt = mb.task_tensor(sg.tasks(b))
    with pytest.raises(ms.MsError, match="ms_set_task_robot first"):
        mb.task_begin(x, tt)
    bad = dict(robot_for(b))
    bad["finger_l"] = 16
    with pytest.raises(ms.MsError, match="out of range"):
        mb.set_task_robot(bad)
