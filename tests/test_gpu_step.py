"""GPU parity of ms_step against the FP64 oracle (through the C ABI).

Single control steps are teacher-forced: both sides start from the same
float32-representable states taken along oracle trajectories.  Bars: position
error <= 1e-5 m and velocity error <= 1e-4 m/s (rad/s) per step, or, where
larger, 4x the deviation of the oracle's own IEEE single-precision evaluation
from its FP64 result, or 10x the oracle's change under 1-ulp float32 input
perturbations (contact-rich states amplify rounding: the speculative bias
scales position rounding by 1/h, a float32 position near 3 m rounds by
2.4e-7 m, i.e. 1.2e-4 m/s at h = 2 ms); at most 35 % of the scene-steps may
need the scaled bar.  100-step trajectories <= 1e-3 m where the per-substep
contact sets agree all along and the oracle with float32 rounding noise
injected every step stays within 1e-3 m of itself (chaos screen); at least
half of the scenes must be kept.  Contact sets are compared per substep
through the count and an order-independent sum of mixed keys.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg
from _parity import errors, fp32_sensitivity, noisy_fp32_rollout, same_contacts

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

POS_TOL = 1e-5
VEL_TOL = 1e-4


def _ms():
    import paper_2412_13211_amd as ms
    return ms


def say(*a):
    print(*a, flush=True)


def gpu_step(mb, x, u):
    xt = torch.as_tensor(np.asarray(x, np.float32)).cuda()
    ut = torch.as_tensor(np.asarray(u, np.float32)).cuda().contiguous()
    out = mb.step(xt, ut)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def oracle_states(b, o, steps):
    """States along the oracle trajectory at the given control steps (float32-rounded)."""
    x = b.state0.astype(np.float64)
    out = {}
    for t in range(max(steps) + 1):
        if t in steps:
            out[t] = x.astype(np.float32).astype(np.float64)
        x = o.step(x, b.controls_for(t))
    return out


CASES = [
    ("cfg1", lambda: sg.make(1), [0, 10, 40, 80]),
    ("cfg2", lambda: sg.make(2, 48), [0, 5, 20]),
    ("cfg3", lambda: sg.make(3, 32), [0, 5, 20]),
    ("cfg4", lambda: sg.make(4, 16), [0, 10, 30]),
    ("cfg5", lambda: sg.make(5, 48), [0, 5, 15]),
    ("cfg6", lambda: sg.make(6, 32), [0, 10, 40]),
]


@pytest.mark.parametrize("name,mk,steps", CASES, ids=[c[0] for c in CASES])
def test_single_step_parity(name, mk, steps):
    ms = _ms()
    b = mk()
    o = oracle.Oracle(b)
    say(f"[single-step] {name}: S={b.n_scenes} NF={b.n_free} NA={b.n_aux} steps={steps}")
    mb = ms.MsBatch(b)
    mb.enable_debug(True)
    states = oracle_states(b, o, steps)
    n_match = n_tot = 0
    worst = (0.0, 0.0)
    n_relaxed = 0
    worst_ratio = 0.0
    for t, x in states.items():
        u = b.controls_for(t)
        xo, d = o.step(x, u, debug=True)
        xg = gpu_step(mb, x, u)
        st = mb.status()
        assert not np.any(st & (ms.MS_ST_NONFINITE | ms.MS_ST_OVERFLOW | ms.MS_ST_ROBOT_OVERFLOW)), st
        same = same_contacts(d, mb.debug_contacts())
        pe, ve = errors(o, b, xo, xg)
        ps, vs = fp32_sensitivity(o, b, x, u)
        pf, vf = errors(o, b, xo, o.step_f32(x, u))
        tol_p = np.maximum.reduce([np.full_like(ps, POS_TOL), 10 * ps, 4 * pf])
        tol_v = np.maximum.reduce([np.full_like(vs, VEL_TOL), 10 * vs, 4 * vf])
        n_match += int(same.sum())
        n_tot += len(same)
        strict = same & (pe <= POS_TOL) & (ve <= VEL_TOL)
        n_relaxed += int((same & ~strict).sum())
        if same.any():
            worst = (max(worst[0], pe[same].max()), max(worst[1], ve[same].max()))
            worst_ratio = max(worst_ratio, float(np.max(np.maximum(pe / tol_p, ve / tol_v)[same])))
        say(f"  t={t}: contact sets equal in {same.sum()}/{len(same)} scenes; "
            f"max pos err {pe[same].max() if same.any() else 0:.3e} m, vel err {ve[same].max() if same.any() else 0:.3e}; "
            f"within the fixed bars {strict.sum()}")
        for i in np.nonzero(same & ~strict)[0]:
            say(f"    scene {i}: pos {pe[i]:.2e} (1-ulp sens {ps[i]:.2e}, fp32 oracle {pf[i]:.2e}), "
                f"vel {ve[i]:.2e} (1-ulp sens {vs[i]:.2e}, fp32 oracle {vf[i]:.2e})")
        assert np.all(pe[same] <= tol_p[same]), (t, np.nonzero(pe > tol_p))
        assert np.all(ve[same] <= tol_v[same]), (t, np.nonzero(ve > tol_v))
    assert n_match >= 0.8 * n_tot, f"contact sets differ in {n_tot - n_match} of {n_tot} scene-steps"
    assert n_relaxed <= 0.35 * n_tot, f"{n_relaxed} of {n_tot} scene-steps needed the conditioning-scaled bar"
    say(f"  summary {name}: contact sets equal in {n_match}/{n_tot} scene-steps; worst pos {worst[0]:.3e} m, "
        f"vel {worst[1]:.3e}; scaled bar used in {n_relaxed}/{n_tot}; max err/bar {worst_ratio:.3f}")


def test_robot_heavy_scenes_parity():
    """The scenes with the most robot contacts (robot rows beyond those whose
    w = M~^-1 J^T the sweeps keep in LDS, so both paths of the robot row run):
    found by stepping a 512-scene cfg3 batch on the GPU, then one step from
    the GPU's state compared with the oracle's step from the same state."""
    ms = _ms()
    b = sg.make(3, 512)
    mb = ms.MsBatch(b)
    mb.enable_debug(True)
    x = torch.as_tensor(b.state0).cuda()
    best = []  # (robot contacts in one substep, step, scene, state before the step)
    for t in range(10):
        xs = x.cpu().numpy().copy()
        x = mb.step(x, torch.as_tensor(b.controls_for(t)).cuda())
        torch.cuda.synchronize()
        nr = mb.debug_contacts()[:, :, 1].max(axis=1).astype(int)
        for s in np.argsort(-nr)[:8]:
            best.append((int(nr[s]), t, int(s), xs))
    best.sort(key=lambda e: -e[0])
    picked, seen = [], set()
    for nr, t, s, xs in best:
        if s not in seen:
            seen.add(s)
            picked.append((nr, t, s, xs))
        if len(picked) == 6:
            break
    say(f"[robot-heavy] robot contacts per substep of the picked scenes: {[p[0] for p in picked]}")
    assert picked[0][0] >= 12
    scenes = [p[2] for p in picked]
    sub = b.subset(scenes)
    parts = []
    for nr, t, s, xs in picked:
        st = sg.split_state(xs, b.n_scenes, b.n_free, b.n_aux)
        parts.append((st["q"][s], st["qd"][s], st["free"][b.free_off[s]:b.free_off[s + 1]],
                      st["aux"][b.aux_off[s]:b.aux_off[s + 1]]))
    x0 = sg.join_state(np.stack([p[0] for p in parts]), np.stack([p[1] for p in parts]),
                       np.concatenate([p[2] for p in parts]), np.concatenate([p[3] for p in parts]))
    u = np.stack([b.controls_for(t)[s] for nr, t, s, xs in picked]).astype(np.float32)
    x0 = x0.astype(np.float64)
    o = oracle.Oracle(sub)
    smb = ms.MsBatch(sub)
    smb.enable_debug(True)
    xo, d = o.step(x0, u, debug=True)
    xg = gpu_step(smb, x0, u)
    st = smb.status()
    assert not np.any(st & (ms.MS_ST_NONFINITE | ms.MS_ST_OVERFLOW | ms.MS_ST_ROBOT_OVERFLOW)), st
    dbg = smb.debug_contacts()
    say(f"  robot contacts per substep on the GPU: {dbg[:, :, 1].max(axis=1).tolist()}")
    same = same_contacts(d, dbg)
    pe, ve = errors(o, sub, xo, xg)
    ps, vs = fp32_sensitivity(o, sub, x0, u)
    pf, vf = errors(o, sub, xo, o.step_f32(x0, u))
    tol_p = np.maximum.reduce([np.full_like(ps, POS_TOL), 10 * ps, 4 * pf])
    tol_v = np.maximum.reduce([np.full_like(vs, VEL_TOL), 10 * vs, 4 * vf])
    for i in range(len(scenes)):
        say(f"    scene {scenes[i]}: contacts equal {same[i]}; pos err {pe[i]:.2e} (bar {tol_p[i]:.2e}), "
            f"vel err {ve[i]:.2e} (bar {tol_v[i]:.2e})")
    assert same.sum() >= len(scenes) // 2
    assert np.all(pe[same] <= tol_p[same]) and np.all(ve[same] <= tol_v[same])


FREE_RUNS = [("cfg1", lambda: sg.make(1)), ("cfg2", lambda: sg.make(2, 32)), ("cfg5", lambda: sg.make(5, 32))]


@pytest.mark.parametrize("name,mk", FREE_RUNS, ids=[c[0] for c in FREE_RUNS])
def test_free_run_100_steps(name, mk):
    ms = _ms()
    b = mk()
    o = oracle.Oracle(b)
    say(f"[free-run] {name} S={b.n_scenes}: 100 control steps")
    mb = ms.MsBatch(b)
    mb.enable_debug(True)
    xo = b.state0.astype(np.float64)
    controls = [b.controls_for(t) for t in range(100)]
    xg = torch.as_tensor(b.state0.copy()).cuda()
    same_all = np.ones(b.n_scenes, bool)
    for t in range(100):
        u = controls[t]
        xo, d = o.step(xo, u, debug=True)
        xg = mb.step(xg, torch.as_tensor(u).cuda())
        torch.cuda.synchronize()
        same_all &= same_contacts(d, mb.debug_contacts())
    xn = noisy_fp32_rollout(o, b, b.state0, controls)
    pe, _ = errors(o, b, xo, xg.cpu().numpy())
    pc, _ = errors(o, b, xo, xn)
    chaotic = pc > 1e-3
    keep = same_all & ~chaotic
    say(f"  contact sets equal all along in {same_all.sum()}/{b.n_scenes}; chaotic {chaotic.sum()}; "
        f"pos err (kept) max {pe[keep].max() if keep.any() else 0:.3e} m; all scenes max {pe.max():.3e}")
    for i in range(b.n_scenes):
        say(f"    scene {i}: gpu err {pe[i]:.2e} m, noisy-oracle err {pc[i]:.2e} m, contacts equal {same_all[i]}")
    say(f"  summary {name}: kept {keep.sum()}/{b.n_scenes}; worst kept pos err "
        f"{pe[keep].max() if keep.any() else 0:.3e} m")
    assert keep.sum() >= b.n_scenes // 2
    assert np.all(pe[keep] <= 1e-3)


def _run_sched(ms, b, flags, x, u, steps=2):
    mb = ms.MsBatch(b)
    mb.set_schedule(flags)
    xt = torch.as_tensor(np.asarray(x, np.float32)).cuda()
    ut = torch.as_tensor(np.asarray(u, np.float32)).cuda()
    for _ in range(steps):
        xt = mb.step(xt, ut, out=xt)
    torch.cuda.synchronize()
    return xt.cpu().numpy()


def test_schedules_bitwise_equal():
    """Grid shape, persistent queue, graph replay, per-substep launches and LDS
    staging change only where and when the same arithmetic runs."""
    ms = _ms()
    b = sg.make(3, 40)
    x = b.state0
    u = b.controls(0)
    say("[schedules] cfg3 S=40")
    for cull in (0, ms.MS_SCHED_CULL):
        ref = _run_sched(ms, b, ms.MS_SCHED_STAGE_STATIC | cull, x, u)
        for flags in [0, ms.MS_SCHED_PERSISTENT, ms.MS_SCHED_GRAPH | ms.MS_SCHED_STAGE_STATIC,
                      ms.MS_SCHED_GRAPH | ms.MS_SCHED_PERSISTENT | ms.MS_SCHED_STAGE_STATIC,
                      ms.MS_SCHED_PER_SUBSTEP | ms.MS_SCHED_STAGE_STATIC]:
            say(f"  flags={flags | cull}")
            got = _run_sched(ms, b, flags | cull, x, u)
            assert np.array_equal(got, ref), flags | cull


def _split_outputs(mb, ms, x, u, record):
    """One step: (state out, record or None, status, robot force, body force)."""
    xt = torch.as_tensor(np.asarray(x, np.float32)).cuda()
    ut = torch.as_tensor(np.asarray(u, np.float32)).cuda()
    if record:
        rec = mb.new_record()
        rec.zero_()
        y = mb.step_record(xt, ut, rec)
    else:
        rec = None
        y = mb.step(xt, ut)
    torch.cuda.synchronize()
    rf, bf = getattr(mb, "robot_force", None), getattr(mb, "body_force", None)
    fr = rf.cpu().numpy().copy() if rf is not None else None
    fb = bf.cpu().numpy().copy() if bf is not None else None
    return (y.cpu().numpy(), None if rec is None else rec.cpu().numpy(), mb.status().copy(), fr, fb)


def _same(a, b):
    ok = True
    for name, p, q in zip(("state", "record", "status", "robot force", "body force"), a, b):
        if (p is None) != (q is None) or (p is not None and not np.array_equal(p, q)):
            bad = np.flatnonzero(p != q) if p is not None and q is not None and p.shape == q.shape else []
            say(f"   {name} differs at {len(bad)} entries, first {bad[:8]}")
            ok = False
    return ok


@pytest.mark.parametrize("extra", ["plain", "graph", "record", "forces"])
def test_forward_split_bitwise_equal(extra):
    """The persistent step split into a smaller and the full LDS layout
    (scenes routed by their previous contact counts, a scene that overflows
    the smaller layout stepped again in the full one) gives the single
    launch's state, record, forces and status bit for bit.  A fresh batch's
    first step routes every scene to the smaller layout, so the scenes with
    more contacts than its cap take the retry path; the second step routes
    them to the full layout."""
    ms = _ms()
    b = sg.make(3, 64)
    x, u = b.state0, b.controls(0)
    flags = ms.MS_SCHED_PERSISTENT | ms.MS_SCHED_CULL | (ms.MS_SCHED_GRAPH if extra == "graph" else 0)
    ref_mb = ms.MsBatch(b, backward=extra == "record")
    ref_mb.set_schedule(flags | ms.MS_SCHED_FWD_ONE_LAUNCH)
    if extra == "forces":
        ref_mb.enable_forces(True)
    auto = ref_mb.get_forward_split()
    ref = _split_outputs(ref_mb, ms, x, u, extra == "record")
    # the step's contact counts (the diagnostics of a plain step)
    cnt_mb = ms.MsBatch(b)
    cnt_mb.set_schedule(ms.MS_SCHED_CULL)
    cnt_mb.enable_debug(True)
    _split_outputs(cnt_mb, ms, x, u, False)
    dbg = cnt_mb.debug_contacts()
    nmax = dbg[:, :, 0].max(axis=1).astype(int)
    rmax = dbg[:, :, 1].max(axis=1).astype(int)
    cc = max(int(np.median(nmax)), 9)
    rc = b.robot_contact_cap           # robot contacts of the smaller layout
    over = (nmax > cc) | (rmax > rc)                # overflow the smaller layout
    routed = (nmax + 8 > cc) | (rmax + 2 > rc)      # sent to the full layout by last step's counts
    say(f"[forward split, {extra}] automatic cap {auto}, forced cap {cc}; scenes above it {over.sum()}")
    assert auto > 0 and over.any() and (~routed).any()
    mb = ms.MsBatch(b, backward=extra == "record")
    mb.set_schedule(flags)
    if extra == "forces":
        mb.enable_forces(True)
    mb.set_forward_split(cc)
    # a captured step (graph schedule) runs in one launch: a replayed graph
    # would run the two branches one after the other
    split = extra != "graph"
    got = _split_outputs(mb, ms, x, u, extra == "record")
    cap, n_full, n_retry = mb.get_forward_split(counts=True)
    say(f"   first step: {n_full} scenes in the full layout, {n_retry} stepped again")
    assert cap == cc and n_full == 0 and n_retry == (int(over.sum()) if split else 0)
    assert _same(got, ref)
    got = _split_outputs(mb, ms, x, u, extra == "record")
    cap, n_full, n_retry = mb.get_forward_split(counts=True)
    say(f"   second step: {n_full} scenes in the full layout, {n_retry} stepped again")
    assert n_full == (int(routed.sum()) if split else 0) and n_retry == 0
    assert _same(got, ref)
    # the library's own cap
    mb.set_forward_split(-1)
    assert mb.get_forward_split() == auto
    assert _same(_split_outputs(mb, ms, x, u, extra == "record"), ref)
    with pytest.raises(ms.MsError, match="split cap"):
        mb.set_forward_split(b.contact_cap)


def test_culled_contacts_equal_brute_force_full_size():
    """The bounding-volume pre-test keeps exactly the brute-force contact sets
    (4096 uneven scenes, 5 control steps, every substep)."""
    ms = _ms()
    b = sg.make(3)
    say("[culling] cfg3 S=4096: culled vs brute-force contact sets")
    out = {}
    for cull in (0, ms.MS_SCHED_CULL):
        mb = ms.MsBatch(b)
        mb.set_schedule(ms.MS_SCHED_STAGE_STATIC | cull)
        mb.enable_debug(True)
        x = torch.as_tensor(b.state0).cuda()
        dbgs = []
        for t in range(5):
            x = mb.step(x, torch.as_tensor(b.controls(t)).cuda())
            torch.cuda.synchronize()
            dbgs.append(mb.debug_contacts().copy())
        out[cull] = (x.cpu().numpy(), dbgs)
    for d0, d1 in zip(out[0][1], out[ms.MS_SCHED_CULL][1]):
        assert np.array_equal(d0, d1)
    x0, x1 = out[0][0], out[ms.MS_SCHED_CULL][0]
    assert np.allclose(x0, x1, rtol=1e-5, atol=1e-6)


def test_deterministic_reruns():
    ms = _ms()
    b = sg.make(2, 24)
    say("[determinism] cfg2 S=24")
    a1 = _run_sched(ms, b, ms.MS_SCHED_STAGE_STATIC, b.state0, b.controls(0), steps=3)
    a2 = _run_sched(ms, b, ms.MS_SCHED_STAGE_STATIC, b.state0, b.controls(0), steps=3)
    assert np.array_equal(a1, a2)


def test_full_size_cfg3_sampled_scenes():
    """4096 uneven scenes in the benchmark's launch configuration; 24 sampled
    scenes checked one by one against the oracle on the same scenes."""
    ms = _ms()
    b = sg.make(3)
    say("[full-size] cfg3 S=4096 graph+persistent")
    mb = ms.MsBatch(b)
    mb.set_schedule(ms.MS_SCHED_GRAPH | ms.MS_SCHED_PERSISTENT | ms.MS_SCHED_STAGE_STATIC)
    mb.enable_debug(True)
    u = b.controls(0)
    xg = gpu_step(mb, b.state0, u)
    dbg = mb.debug_contacts()
    st = mb.status()
    assert not np.any(st & (ms.MS_ST_NONFINITE | ms.MS_ST_OVERFLOW | ms.MS_ST_ROBOT_OVERFLOW))
    rng = np.random.default_rng(0)
    pick = sorted(rng.choice(b.n_scenes, 24, replace=False).tolist())
    sub = b.subset(pick)
    o = oracle.Oracle(sub)
    xo, d = o.step(sub.state0.astype(np.float64), u[pick], debug=True)
    # gather the sampled scenes from the full GPU state
    full = sg.split_state(xg, b.n_scenes, b.n_free, b.n_aux)
    fidx = np.concatenate([np.arange(b.free_off[s], b.free_off[s + 1]) for s in pick])
    aidx = np.concatenate([np.arange(b.aux_off[s], b.aux_off[s + 1]) for s in pick]).astype(int)
    xs = sg.join_state(full["q"][pick], full["qd"][pick], full["free"][fidx], full["aux"][aidx])
    same = same_contacts(d, dbg[pick])
    pe, ve = errors(o, sub, xo, xs)
    say(f"  sampled: contacts equal {same.sum()}/24; pos {pe[same].max():.3e} vel {ve[same].max():.3e}")
    assert same.sum() >= 20
    assert np.all(pe[same] <= POS_TOL) and np.all(ve[same] <= VEL_TOL)


def test_edge_cases_empty_robot_and_no_objects():
    ms = _ms()
    box = sg.box_object((0.1, 0.1, 0.1), 1.0, (0.0, 0.0, 0.1), vel=(0.5, 0.0, 0.0))
    sph = sg.sphere_object(0.05, 0.3, (0.3, 0.0, 0.2))
    scenes = [dict(free=[box, sph], planes=[(0, 0, 1, 0)]), dict(planes=[(0, 0, 1, 0)]),
              dict(free=[sph]), dict(free=[box], static=[(0.0, 0.0, -0.5, 1.0, 1.0, 0.5)])]
    b = sg.custom_batch([sg.empty_model()], scenes, h=0.002, n_sub=5, pgs_iters=10)
    say("[edge] empty robot / no objects / no planes")
    o = oracle.Oracle(b)
    mb = ms.MsBatch(b)
    mb.enable_debug(True)
    x = b.state0.astype(np.float64)
    for t in range(5):
        xo, d = o.step(x, np.zeros((b.n_scenes, 16)), debug=True)
        xg = gpu_step(mb, x, np.zeros((b.n_scenes, 16)))
        same = same_contacts(d, mb.debug_contacts())
        pe, ve = errors(o, b, xo, xg)
        assert same.all()
        assert np.all(pe <= POS_TOL) and np.all(ve <= VEL_TOL), (pe, ve)
        x = xo


def test_contact_cap_overflow_flagged():
    ms = _ms()
    boxes = [sg.box_object((0.05, 0.05, 0.05), 0.5, (0.3 * k, 0.0, 0.05)) for k in range(4)]
    b = sg.custom_batch([sg.empty_model()], [dict(free=boxes, planes=[(0, 0, 1, 0)])], contact_cap=6)
    say("[edge] contact cap overflow")
    mb = ms.MsBatch(b)
    gpu_step(mb, b.state0, np.zeros((1, 16)))
    st = mb.status()
    assert st[0] & ms.MS_ST_OVERFLOW
    # the oracle keeps the same first 6 contacts in canonical order
    o = oracle.Oracle(b)
    xo = o.step(b.state0.astype(np.float64), np.zeros((1, 16)))
    xg = gpu_step(mb, b.state0, np.zeros((1, 16)))
    pe, ve = errors(o, b, xo, xg)
    assert pe.max() <= POS_TOL and ve.max() <= VEL_TOL


def test_robot_contact_cap_matches_oracle():
    """Robot contact cap: an arm lying on the floor with more robot contacts
    than the cap keeps the first ones in canonical order on both sides (the
    rest dropped, status bit 8), with the same step."""
    ms = _ms()
    b = sg.make(1)
    o64 = oracle.Oracle(b)
    x = b.state0.astype(np.float64)
    for t in range(80):
        x = o64.step(x, b.controls_for(t))
    x = x.astype(np.float32).astype(np.float64)
    u = b.controls_for(80)
    rcap = 4
    o = oracle.Oracle(b, robot_contact_cap=rcap)
    xo, d = o.step(x, u, debug=True)
    mb = ms.MsBatch(b, robot_contact_cap=rcap)
    mb.enable_debug(True)
    xg = gpu_step(mb, x, u)
    st = mb.status()
    capped = (d["status"] & ms.MS_ST_ROBOT_OVERFLOW) != 0
    say(f"[robot cap] cfg1 t=80, cap {rcap}: scenes over the cap {capped.sum()}/{b.n_scenes}")
    assert capped.sum() >= 4
    assert np.array_equal(capped, (st & ms.MS_ST_ROBOT_OVERFLOW) != 0)
    same = same_contacts(d, mb.debug_contacts())
    pe, ve = errors(o, b, xo, xg)
    pf, vf = errors(o, b, xo, o.step_f32(x, u))
    ps, vs = fp32_sensitivity(o, b, x, u)
    tol_p = np.maximum.reduce([np.full_like(ps, POS_TOL), 10 * ps, 4 * pf])
    tol_v = np.maximum.reduce([np.full_like(vs, VEL_TOL), 10 * vs, 4 * vf])
    say(f"  contact sets equal {same.sum()}/{b.n_scenes}; max pos {pe[same].max():.2e} vel {ve[same].max():.2e}")
    assert same.all()
    assert np.all(pe <= tol_p) and np.all(ve <= tol_v)


def test_invalid_arguments_leave_state_untouched():
    ms = _ms()
    b = sg.make(1, 2)
    mb = ms.MsBatch(b)
    x = torch.as_tensor(b.state0.copy()).cuda()
    before = x.clone()
    with pytest.raises(ms.MsError):
        mb.step(x, torch.zeros(3, 16, device="cuda"))           # wrong control shape
    with pytest.raises(ms.MsError):
        mb.step(x[:-1], torch.zeros(2, 16, device="cuda"))      # wrong state size
    with pytest.raises(ms.MsError):
        mb.set_schedule(1 << 10)
    torch.cuda.synchronize()
    assert torch.equal(x, before)
