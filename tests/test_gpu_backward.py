"""GPU adjoint of the control step (ms_step_backward) against the FP64
oracle's exact adjoint, through the C ABI.

Bar: on every scene, the Euclidean norm of the error over the locally smooth
components of the oracle's adjoint is <= 1e-3 of the norm of that adjoint;
at least a stated share of the components must be smooth, so the check is
not vacuous.  Hand-built single-contact scenes (no redundant contacts) are
smooth everywhere and must meet the bar on every component.  Rollouts through
the torch.autograd.Function (checkpoint + recompute) are checked against the
oracle adjoint chained over the same horizon.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg
from _grad import GRAD_TOL, compare, oracle_vjp_smooth, scene_vectors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ms():
    import paper_2412_13211_amd as ms
    return ms


def say(*a):
    print(*a, flush=True)


def gpu_vjp(mb, x, u, g):
    xt = torch.as_tensor(np.asarray(x, np.float32)).cuda()
    ut = torch.as_tensor(np.asarray(u, np.float32)).cuda().contiguous()
    gt = torch.as_tensor(np.asarray(g, np.float32)).cuda()
    gx, gu = mb.step_backward(xt, ut, gt)
    torch.cuda.synchronize()
    return gx.cpu().numpy().astype(np.float64), gu.cpu().numpy().astype(np.float64)


def advanced_state(b, steps):
    o = oracle.Oracle(b, threads=8)
    x = b.state0.astype(np.float64)
    for t in range(steps):
        x = o.step(x, b.controls_for(t))
    return x.astype(np.float32).astype(np.float64)


def _tilted(angle, axis):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    return (math.cos(angle / 2), *(math.sin(angle / 2) * a))


def primitive_scenes():
    q = _tilted(0.2, (1, 0.3, 0))
    floor = [(0, 0, 1, 0)]
    return [
        dict(free=[sg.box_object((0.1, 0.1, 0.1), 1.0, (0, 0, 0.118), quat=q, vel=(0.1, 0, -0.1),
                                 angvel=(0.3, 0.2, 0.1))], planes=floor),
        dict(free=[sg.sphere_object(0.1, 1.0, (0, 0, 0.098), vel=(0.1, 0, -0.1))], planes=floor),
        dict(free=[sg.box_object((0.1, 0.1, 0.1), 1.0, (0, 0, 0.595), quat=q, vel=(0.1, 0, -0.1))],
             static=[(0, 0, 0.25, 1, 1, 0.25)], planes=floor),
        dict(free=[sg.sphere_object(0.1, 1.0, (0.03, 0, 0.598), vel=(0.1, 0, -0.1))],
             static=[(0, 0, 0.25, 1, 1, 0.25)], planes=floor),
        dict(free=[sg.sphere_object(0.1, 1.0, (0, 0, 0.1)),
                   sg.sphere_object(0.1, 1.0, (0.03, 0, 0.295), vel=(0.1, 0, -0.1))], planes=floor),
        dict(free=[sg.sphere_object(0.1, 1.0, (0, 0, 0.1)),
                   sg.box_object((0.1, 0.1, 0.1), 1.0, (0.02, 0.01, 0.296), quat=q, vel=(0.1, 0, -0.1))],
             planes=floor),
    ]


@pytest.mark.parametrize("mu,iters,n_sub", [(0.0, 1, 1), (0.5, 3, 1), (0.5, 10, 3)])
def test_backward_contact_primitives(mu, iters, n_sub):
    """Sphere / box against plane, static box, free sphere: every component."""
    ms = _ms()
    b = sg.custom_batch([sg.empty_model()], primitive_scenes(), n_sub=n_sub, pgs_iters=iters, mu=mu)
    x = b.state0.astype(np.float64)
    u = np.zeros((b.n_scenes, 16), np.float32)
    g = np.random.default_rng(3).normal(size=x.size)
    o = oracle.Oracle(b)
    ref = scene_vectors(b, *o.vjp(x, u, g))
    mb = ms.MsBatch(b, backward=True)
    mine = scene_vectors(b, *gpu_vjp(mb, x, u, g))
    for s in range(b.n_scenes):
        err = np.linalg.norm(mine[s] - ref[s]) / np.linalg.norm(ref[s])
        say(f"primitive scene {s} mu={mu} K={iters} n_sub={n_sub}: rel err {err:.2e}")
        assert err <= GRAD_TOL, (s, err)


GEN_CASES = [("cfg1", 1, 6, 10), ("cfg2", 2, 8, 5), ("cfg4", 4, 8, 3), ("cfg5", 5, 8, 3), ("cfg6", 6, 8, 6)]


@pytest.mark.parametrize("name,cfg,n,steps", GEN_CASES)
def test_backward_generated_scenes(name, cfg, n, steps):
    ms = _ms()
    b = sg.make(cfg, n)
    x = advanced_state(b, steps)
    u = b.controls_for(steps)
    g = np.random.default_rng(5).normal(size=x.size)
    o = oracle.Oracle(b, threads=8)
    ref, mask, scale = oracle_vjp_smooth(o, b, x, u, g)
    mb = ms.MsBatch(b, backward=True)
    mine = scene_vectors(b, *gpu_vjp(mb, x, u, g))
    err = compare(ref, mask, scale, mine)
    share = np.mean(np.concatenate(mask))
    say(f"{name}: smooth share {share:.3f}, per-scene rel err {np.array2string(err, precision=2)}")
    assert share >= 0.8
    assert np.all(err <= GRAD_TOL), err


def test_backward_full_size_sampled():
    """Full-size batch (16384 scenes with door and drawer), sampled scenes."""
    ms = _ms()
    b = sg.make(5)
    steps = 2
    pick = [0, 1, 777, 4096, 9001, 16383]
    sub = b.subset(pick)
    xs = advanced_state(sub, steps)
    # place the sampled scenes' states into the full batch state (others from the generator)
    x = b.state0.astype(np.float64).copy()
    full = sg.split_state(x, b.n_scenes, b.n_free, b.n_aux)
    part = sg.split_state(xs, sub.n_scenes, sub.n_free, sub.n_aux)
    for r, s in enumerate(pick):
        full["q"][s] = part["q"][r]
        full["qd"][s] = part["qd"][r]
        full["free"][b.free_off[s]:b.free_off[s + 1]] = part["free"][sub.free_off[r]:sub.free_off[r + 1]]
        full["aux"][b.aux_off[s]:b.aux_off[s + 1]] = part["aux"][sub.aux_off[r]:sub.aux_off[r + 1]]
    u = b.controls_for(steps)
    g = np.random.default_rng(7).normal(size=x.size).astype(np.float32)
    mb = ms.MsBatch(b, backward=True)
    say(f"full-size backward: {b.n_scenes} scenes, workspace {mb.sizes.tape / 2**20:.0f} MiB")
    gx, gu = gpu_vjp(mb, x, u, g)
    assert np.isfinite(gx).all() and np.isfinite(gu).all()
    mine_all = scene_vectors(b, gx, gu)
    gsub = np.zeros(sub.state_floats, np.float64)
    gs = sg.split_state(gsub, sub.n_scenes, sub.n_free, sub.n_aux)
    gf = sg.split_state(g.astype(np.float64), b.n_scenes, b.n_free, b.n_aux)
    for r, s in enumerate(pick):
        gs["q"][r] = gf["q"][s]
        gs["qd"][r] = gf["qd"][s]
        gs["free"][sub.free_off[r]:sub.free_off[r + 1]] = gf["free"][b.free_off[s]:b.free_off[s + 1]]
        gs["aux"][sub.aux_off[r]:sub.aux_off[r + 1]] = gf["aux"][b.aux_off[s]:b.aux_off[s + 1]]
    o = oracle.Oracle(sub, threads=8)
    ref, mask, scale = oracle_vjp_smooth(o, sub, xs, u[pick], gsub)
    err = compare(ref, mask, scale, [mine_all[s] for s in pick])
    say(f"full-size sampled per-scene rel err {np.array2string(err, precision=2)}")
    assert np.all(err <= GRAD_TOL), err


def test_reference_kernel_agrees():
    """The lane-per-scene kernel (recomputes everything itself) and the
    wavefront kernel (reads the forward kernel's record) both meet the bar."""
    ms = _ms()
    b = sg.make(5, 8)
    x = advanced_state(b, 3)
    u = b.controls_for(3)
    g = np.random.default_rng(21).normal(size=x.size)
    o = oracle.Oracle(b, threads=8)
    ref, mask, scale = oracle_vjp_smooth(o, b, x, u, g)
    mb = ms.MsBatch(b, backward=True)
    wave = scene_vectors(b, *gpu_vjp(mb, x, u, g))
    mb.set_schedule(mb.get_schedule()[0] | ms.MS_SCHED_BWD_REFERENCE)
    lane = scene_vectors(b, *gpu_vjp(mb, x, u, g))
    e_wave, e_lane = compare(ref, mask, scale, wave), compare(ref, mask, scale, lane)
    say(f"wavefront kernel rel err {np.array2string(e_wave, precision=2)}")
    say(f"lane kernel rel err {np.array2string(e_lane, precision=2)}")
    assert np.all(e_wave <= GRAD_TOL) and np.all(e_lane <= GRAD_TOL)


def test_backward_alias_and_determinism():
    ms = _ms()
    b = sg.make(2, 16)
    x = advanced_state(b, 3)
    u = b.controls_for(3)
    g = np.random.default_rng(9).normal(size=x.size)
    mb = ms.MsBatch(b, backward=True)
    a1 = gpu_vjp(mb, x, u, g)
    a2 = gpu_vjp(mb, x, u, g)
    assert np.array_equal(a1[0], a2[0]) and np.array_equal(a1[1], a2[1])
    xt = torch.as_tensor(x.astype(np.float32)).cuda()
    ut = torch.as_tensor(u.astype(np.float32)).cuda().contiguous()
    gt = torch.as_tensor(g.astype(np.float32)).cuda()
    gx, gu = mb.step_backward(xt, ut, gt, gx_in=gt)
    torch.cuda.synchronize()
    assert gx.data_ptr() == gt.data_ptr()
    assert np.array_equal(gx.cpu().numpy().astype(np.float64), a1[0])
    assert np.array_equal(gu.cpu().numpy().astype(np.float64), a1[1])


def test_split_launch_matches_one_launch():
    """Scenes reversed in the smaller LDS layout and the others in the full
    one, on two streams, give the single launch's result bit for bit; the
    split caps are forced so that both launches get scenes."""
    ms = _ms()
    b = sg.make(2, 32)
    x = advanced_state(b, 3)
    u = b.controls_for(3)
    g = np.random.default_rng(5).normal(size=x.size)
    mb = ms.MsBatch(b, backward=True)
    auto = mb.get_backward_split()
    say(f"automatic split caps {auto}")
    assert 0 < auto[0] <= b.contact_cap and 0 < auto[1] <= b.robot_contact_cap
    # contact counts of the same step from the forward kernel's diagnostics
    mb.enable_debug(True)
    mb.step(torch.as_tensor(x.astype(np.float32)).cuda(), torch.as_tensor(u.astype(np.float32)).cuda())
    dbg = mb.debug_contacts()
    mb.enable_debug(False)
    nmax, rmax = dbg[:, :, 0].max(axis=1).astype(int), dbg[:, :, 1].max(axis=1).astype(int)
    cc = max(int(np.median(nmax)), 1)
    rc = max(int(rmax.max()), 1)
    small = (nmax <= cc) & (rmax <= rc)
    say(f"forced caps ({cc}, {rc}): {small.sum()} scenes in the smaller layout, {(~small).sum()} in the full one")
    assert small.any() and not small.all()
    flags = mb.get_schedule()[0]
    mb.set_schedule(flags | ms.MS_SCHED_BWD_ONE_LAUNCH)
    one = gpu_vjp(mb, x, u, g)
    mb.set_schedule(flags)
    for caps in [(cc, rc), auto]:
        mb.set_backward_split(*caps)
        assert mb.get_backward_split() == caps
        sp = gpu_vjp(mb, x, u, g)
        assert np.array_equal(sp[0], one[0]) and np.array_equal(sp[1], one[1]), caps
    mb.set_backward_split(0)
    assert mb.get_backward_split() == (0, 0)
    assert np.array_equal(gpu_vjp(mb, x, u, g)[0], one[0])
    mb.set_backward_split(-1)
    assert mb.get_backward_split() == auto
    with pytest.raises(ms.MsError, match="split caps"):
        mb.set_backward_split(b.contact_cap + 1, 1)
    assert np.all(mb.status() == 0)


@pytest.mark.parametrize("cfg,n", [(2, 16), (5, 8)])
def test_recorded_step_and_backward_match(cfg, n):
    """ms_step_record gives ms_step's state bit for bit and a record from
    which ms_step_backward_recorded gives ms_step_backward's results bit for
    bit (also when the record is reused after other steps ran)."""
    ms = _ms()
    b = sg.make(cfg, n)
    x = advanced_state(b, 2)
    u = b.controls_for(2)
    g = np.random.default_rng(17).normal(size=x.size)
    mb = ms.MsBatch(b, backward=True)
    xt = torch.as_tensor(x.astype(np.float32)).cuda()
    ut = torch.as_tensor(np.asarray(u, np.float32)).cuda().contiguous()
    gt = torch.as_tensor(g.astype(np.float32)).cuda()
    rec = mb.new_record()
    assert rec.numel() * 4 >= mb.sizes.record > 0
    y_ref = mb.step(xt, ut)
    y_rec = mb.step_record(xt, ut, rec)
    torch.cuda.synchronize()
    assert torch.equal(y_ref, y_rec)
    gx_ref, gu_ref = mb.step_backward(xt, ut, gt)
    mb.step(y_ref, ut)                      # other work between the record and its use
    gx_rec, gu_rec = mb.step_backward_recorded(xt, ut, rec, gt)
    torch.cuda.synchronize()
    assert torch.equal(gx_ref, gx_rec) and torch.equal(gu_ref, gu_rec)
    # in place on the state: out aliases x
    x2 = xt.clone()
    mb.step_record(x2, ut, rec, out=x2)
    torch.cuda.synchronize()
    assert torch.equal(x2, y_ref)
    with pytest.raises(ms.MsError, match="record"):
        mb.step_record(xt, ut, rec[:8])
    assert not np.any(mb.status() & 16)     # record and recomputation agree


def test_backward_without_workspace_is_an_error():
    ms = _ms()
    b = sg.make(2, 4)
    mb = ms.MsBatch(b)
    x = torch.as_tensor(b.state0).cuda()
    u = torch.zeros((4, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(ms.MsError, match="tape"):
        mb.step_backward(x, u, x.clone())


def test_rollout_gradient_checkpointed():
    """Differentiation workload: squared distance of one box to a goal plus
    the robot's squared distance to a joint-space goal after T control steps,
    gradient with respect to the torque sequence, through the autograd
    function with a checkpoint every 5 steps."""
    ms = _ms()
    from paper_2412_13211_amd.autograd import rollout
    b = sg.make(4, 6)
    T, every = 10, 5
    x0 = advanced_state(b, 2)
    U = np.stack([b.controls_for(2 + t) for t in range(T)]).astype(np.float32)
    goal = np.random.default_rng(11).uniform(-0.05, 0.05, (b.n_scenes, 3))
    qgoal = np.random.default_rng(12).uniform(-0.1, 0.1, (b.n_scenes, 16))
    S = b.n_scenes
    box = np.array([b.free_off[s] for s in range(S)])  # first free body of each scene

    def loss_grad_oracle(x0v, Uv):
        o = oracle.Oracle(b, threads=8)
        xs = [x0v]
        for t in range(T):
            xs.append(o.step(xs[-1], Uv[t]))
        fr = sg.split_state(xs[-1], S, b.n_free, b.n_aux)["free"]
        start = sg.split_state(x0v, S, b.n_free, b.n_aux)["free"]
        d = fr[box, 0:3] - (start[box, 0:3] + goal)
        g = np.zeros_like(x0v)
        gf = sg.split_state(g, S, b.n_free, b.n_aux)["free"]
        gf[box, 0:3] = 2 * d
        q = sg.split_state(xs[-1], S, b.n_free, b.n_aux)["q"]
        q0 = sg.split_state(x0v, S, b.n_free, b.n_aux)["q"]
        sg.split_state(g, S, b.n_free, b.n_aux)["q"][:] = 2 * (q - (q0 + qgoal))
        gU = np.zeros_like(Uv, dtype=np.float64)
        for t in range(T - 1, -1, -1):
            g, gu = o.vjp(xs[t], Uv[t], g)
            gU[t] = gu
        return gU

    ref = loss_grad_oracle(x0, U.astype(np.float64))
    rng = np.random.default_rng(13)
    stable = np.ones(ref.shape, bool)
    for _ in range(2):
        xp = x0 + 1e-7 * (np.abs(x0) + 1) * rng.uniform(-1, 1, x0.size)
        up = U.astype(np.float64) + 1e-7 * rng.uniform(-1, 1, U.shape)
        stable &= np.abs(loss_grad_oracle(xp, up) - ref) <= 1e-4 * np.abs(ref).max()

    mb = ms.MsBatch(b, backward=True)
    x0t = torch.as_tensor(x0.astype(np.float32)).cuda()
    Ut = torch.as_tensor(U).cuda().requires_grad_(True)
    start = x0t[32 * S: 32 * S + 16 * b.n_free].view(b.n_free, 16)
    goal_t = torch.as_tensor(goal, dtype=torch.float32, device="cuda")
    bi = torch.as_tensor(box, device="cuda")
    qg = torch.as_tensor(qgoal, dtype=torch.float32, device="cuda")

    def loss_of(xT):
        fr = xT[32 * S: 32 * S + 16 * b.n_free].view(b.n_free, 16)
        return ((fr[bi, 0:3] - (start[bi, 0:3] + goal_t)) ** 2).sum() + \
            ((xT[:16 * S].view(S, 16) - (x0t[:16 * S].view(S, 16) + qg)) ** 2).sum()

    xT = rollout(mb, x0t, Ut, every=every)
    loss_of(xT).backward()
    mine = Ut.grad.cpu().numpy().astype(np.float64)
    share = stable.mean()
    err = np.linalg.norm((mine - ref)[stable]) / np.linalg.norm(ref)
    say(f"rollout T={T} every={every}: smooth share {share:.3f} rel err {err:.2e}")
    assert share >= 0.5
    assert err <= GRAD_TOL
    # keeping every step's record instead of checkpoints: the same, bit for bit
    Ut2 = torch.as_tensor(U).cuda().requires_grad_(True)
    xT2 = rollout(mb, x0t, Ut2, records=True)
    assert torch.equal(xT2.detach(), xT.detach())
    loss_of(xT2).backward()
    assert torch.equal(Ut2.grad, Ut.grad)


def test_cfg4_box_push_gradient_stated_shape():
    """The differentiation workload as stated: 256 scenes, 50 control steps of
    20 ms (4 substeps of 5 ms), loss = squared distance of the pushed box to
    its seeded goal, gradient with respect to the 50 x 15 torque sequence
    through the autograd function with a checkpoint every 10 steps.  The whole
    batch runs on the GPU; a seeded sample of 32 of its scenes is checked
    against the oracle's adjoint chained along the same trajectory: its
    one-substep VJP at every substep state the GPU recorded (teacher-forced
    like the single-step parity, at the granularity of the record), per
    scene ||g - g*|| / ||g*|| <= 1e-3 over the components of g* that are
    locally smooth (they move < 1e-4 of the scene's scale under 1e-7
    perturbations), both norms over those components.  Forcing per control
    step instead lets the oracle's own substeps drift from the GPU's by
    FP32 rounding, and a resting contact whose gap crosses zero within a
    step (bias switching from Baumgarte to speculative) then sits between
    the two sides' substep states: the step's VJP jumps by percents there
    though each substep's VJP agrees to 1e-5.

    The precondition of gradient parity is that both sides differentiate the
    same branch of the piecewise-smooth step (no contact or active-set
    switch).  So for every sampled scene, every substep of the 50 steps is
    run by the oracle from the GPU's recorded substep state, and the contact
    count and the branch of every Gauss-Seidel row update in every sweep
    (normal clamp, friction disk projection) are compared with the GPU's
    record.  A row's bias branch (speculative for a gap >= 0, Baumgarte for
    a penetration) flips at gap 0, where resting contacts sit: the bias is
    continuous there and the 1e-7 perturbations of the smoothness mask cross
    it, so it is left to the mask; the count of such rows is reported.  dL/dU[t] depends on the steps t .. T-1 only, so it is compared
    where both sides agree in all of them: the components after a scene's
    last difference (a row within FP32 rounding of its kink, mostly a
    redundant resting contact).  At least a quarter of all components and 16
    scenes must be compared.  The error against the oracle's gradient along
    its own FP64 trajectory is reported beside it."""
    ms = _ms()
    from paper_2412_13211_amd.autograd import rollout
    from _record import counts, decisions, gaps, layout, substep_state, tape
    b = sg.make(4)
    S, T, every = b.n_scenes, 50, 10
    assert S == 256
    U = np.stack([b.controls_for(t) for t in range(T)]).astype(np.float32)
    goals = b.push_goals()
    box = np.array([b.free_off[s] for s in range(S)])
    pick = sorted(np.random.default_rng(41).choice(S, 32, replace=False).tolist())

    # GPU: the whole batch, gradient through the checkpointed autograd rollout
    mb = ms.MsBatch(b, backward=True)
    x0t = torch.as_tensor(b.state0).cuda()
    Ut = torch.as_tensor(U).cuda().requires_grad_(True)
    bi = torch.as_tensor(box, device="cuda")
    gt = torch.as_tensor(goals, dtype=torch.float32, device="cuda")
    nf = b.n_free
    xT = rollout(mb, x0t, Ut, every=every)
    fr = xT[32 * S: 32 * S + 16 * nf].view(nf, 16)
    ((fr[bi, 0:3] - gt) ** 2).sum().backward()
    torch.cuda.synchronize()
    mine_all = Ut.grad.cpu().numpy().astype(np.float64)
    assert np.isfinite(mine_all).all()
    # the same forward again with records (bitwise the same steps): the GPU's
    # states at every substep and its Gauss-Seidel branch decisions
    L = layout(b)
    rec = mb.new_record()
    x = x0t.clone()
    recs = []
    rows = torch.as_tensor(np.concatenate([np.arange(s * L["total"], (s + 1) * L["total"]) for s in pick]),
                           device="cuda")
    for t in range(T):
        rec.zero_()
        x = mb.step_record(x, torch.as_tensor(U[t]).cuda(), rec)
        recs.append(rec[rows].view(len(pick), L["total"]).cpu().numpy())
    torch.cuda.synchronize()
    assert torch.equal(x, xT.detach())

    sub = b.subset(pick)
    o = oracle.Oracle(sub, threads=16)
    o1 = [oracle.Oracle(sub.subset([i]), n_sub=1) for i in range(len(pick))]
    Us = U[:, pick].astype(np.float64)
    sbox = np.array([sub.free_off[s] for s in range(len(pick))])

    # the branch screen: steps at which the GPU and the oracle (from the GPU's
    # recorded substep states) differ in a contact count or a Gauss-Seidel branch
    flips = []
    ngap = [0] * len(pick)
    for i in range(len(pick)):
        f = []
        for t in range(T):
            r = recs[t][i]
            for k in range(b.n_sub):
                xk = substep_state(sub, L, r, i, k)
                _, d = o1[i].step(xk, Us[t, i:i + 1], dump_cap=b.contact_cap)
                nc, nl, nr = counts(L, r, k)
                no = int(np.sum(d["dump_keys"][0] != np.uint64(~np.uint64(0))))
                if no != nc:
                    f.append(t)
                    break
                cg, pg = decisions(tape(b, L, r, k, nc), b.mu)
                co, po = decisions(d["dump_y"][0, :, :nc], b.mu)
                if not (np.array_equal(cg, co) and np.array_equal(pg, po)):
                    f.append(t)
                    break
                # bias branches (gap sign) are counted, not screened: the
                # bias is continuous in the gap, and a gap within rounding of
                # zero is inside the smoothness mask's perturbation radius
                ngap[i] += int(np.sum((gaps(L, r, k, nc) >= 0.0) != (d["dump_phi"][0, :nc] >= 0.0)))
        flips.append(f)

    # batch states along the GPU trajectory: the start of every substep of
    # every control step, and the end
    def batch_state(t, k):
        per = [substep_state(sub, L, recs[t][i], i, k) for i in range(len(pick))]
        parts = [sg.split_state(v, 1, int(sub.free_off[i + 1] - sub.free_off[i]),
                                int(sub.aux_off[i + 1] - sub.aux_off[i])) for i, v in enumerate(per)]
        return sg.join_state(np.concatenate([p["q"] for p in parts]), np.concatenate([p["qd"] for p in parts]),
                             np.concatenate([p["free"] for p in parts]),
                             np.concatenate([p["aux"] for p in parts])).astype(np.float64)

    def loss_adjoint(xT):
        frT = sg.split_state(xT, sub.n_scenes, sub.n_free, sub.n_aux)["free"]
        g = np.zeros_like(xT)
        sg.split_state(g, sub.n_scenes, sub.n_free, sub.n_aux)["free"][sbox, 0:3] = 2 * (frT[sbox, 0:3] - goals[pick])
        return g

    def chain_substeps(xs, Uv):
        # xs[t][k]: state at substep k of step t (xs[T][0]: the end); the
        # control is held over a step, so dL/dU[t] sums its substeps' terms
        g = loss_adjoint(xs[T][0])
        gU = np.zeros_like(Uv)
        for t in range(T - 1, -1, -1):
            for k in range(b.n_sub - 1, -1, -1):
                g, gu = os1.vjp(xs[t][k], Uv[t], g)
                gU[t] += gu
        return gU

    def chain_steps(xs, Uv):
        g = loss_adjoint(xs[T])
        gU = np.zeros_like(Uv)
        for t in range(T - 1, -1, -1):
            g, gU[t] = o.vjp(xs[t], Uv[t], g)
        return gU

    os1 = oracle.Oracle(sub, n_sub=1, threads=16)
    xs_gpu = [[batch_state(t, k) for k in range(b.n_sub)] for t in range(T)]
    xs_gpu.append([batch_state(T - 1, b.n_sub)])
    ref = chain_substeps(xs_gpu, Us)
    xs_own = [sub.state0.astype(np.float64)]
    for t in range(T):
        xs_own.append(o.step(xs_own[-1], Us[t]))
    ref_own = chain_steps(xs_own, Us)
    rng = np.random.default_rng(43)
    stable = np.ones(ref.shape, bool)
    for _ in range(4):
        xp = [[xx + 1e-7 * (np.abs(xx) + 1) * rng.uniform(-1, 1, xx.size) for xx in row] for row in xs_gpu]
        up = Us + 1e-7 * rng.uniform(-1, 1, Us.shape)
        pert = chain_substeps(xp, up)
        for i in range(len(pick)):
            stable[:, i] &= np.abs(pert[:, i] - ref[:, i]) <= 1e-4 * np.abs(ref[:, i]).max()
    # dL/dU[t] depends on the steps t .. T-1 only: it is comparable where both
    # sides take the same branches in all of them (and the oracle's adjoint is
    # locally smooth there)
    mine = mine_all[:, pick]
    errs, shares = [], []
    for i in range(len(pick)):
        last = max(flips[i]) if flips[i] else -1
        m = stable[:, i, :15].copy()
        m[:last + 1] = False
        r, g_m = ref[:, i, :15][m], mine[:, i, :15][m]
        den = max(np.linalg.norm(r), 1e-12)
        err = np.linalg.norm(g_m - r) / den if m.any() else 0.0
        ms_ = stable[:, i, :15]
        err_all = np.linalg.norm((mine[:, i, :15] - ref[:, i, :15])[ms_]) / max(np.linalg.norm(ref[:, i, :15][ms_]), 1e-12)
        err_own = np.linalg.norm((mine[:, i, :15] - ref_own[:, i, :15])[ms_]) / max(np.linalg.norm(ref_own[:, i, :15][ms_]), 1e-12)
        say(f"  scene {pick[i]}: branch differences at steps {flips[i]} (gap-sign rows {ngap[i]}); "
            f"compared {m.mean():.3f} of the "
            f"components, err {err:.2e}; over every smooth component {err_all:.2e} "
            f"(vs the oracle's own trajectory {err_own:.2e})")
        shares.append(m.mean())
        if m.any():
            errs.append(err)
    say(f"  summary cfg4 256 x 50 (checkpoint 10): compared share {np.mean(shares):.3f}, scenes with compared "
        f"components {len(errs)}/32, worst rel err {max(errs) if errs else 0:.2e}")
    assert np.mean(shares) >= 0.25 and len(errs) >= 16
    assert max(errs) <= GRAD_TOL
