#!/usr/bin/env python3
"""Benchmark: physics env-steps/s of the batched rigid-body step on one MI355X.

Workload (default): 4096 uneven Fetch-like scenes (free objects U{2..32},
furniture boxes U{32..256}), h = 2 ms, 5 substeps per control step, 10 PGS
sweeps; one "step" is one control step of every scene with the inputs
resident in HBM.  Prints ONE JSON line (see the keys below).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 3] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("ms_kernels.hip", "ms_internal.h"):
        with open(os.path.join(ROOT, "paper_2412_13211_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes_per_env_step(b):
    """HBM bytes one control step must move for the whole batch: state in +
    out, controls in, the per-scene description (free-body parameters, static
    boxes, planes, door/drawer, scene record); the shared robot model once."""
    S, NF, NA = b.n_scenes, b.n_free, b.n_aux
    state = (32 * S + 16 * NF + 4 * NA) * 4
    controls = 16 * S * 4
    desc = NF * 32 + int(b.static_off[-1]) * 24 + int(b.plane_off[-1]) * 16 + NA * 128 + S * 112
    model = len(b.model_nb) * 6 * 1024
    return 2 * state + controls + desc + model


def algorithmic_flops_per_env_step(b, sample=64, seed=0):
    """Floating-point operations of one control step (the oracle's definition,
    counted by its op-counting scalar) averaged over a scene sample."""
    import oracle
    rng = np.random.default_rng(seed)
    pick = sorted(rng.choice(b.n_scenes, min(sample, b.n_scenes), replace=False).tolist())
    sub = b.subset(pick)
    o = oracle.Oracle(sub)
    return float(np.mean(o.flops(sub.state0.astype(np.float64), b.controls(0, pick)))) / 1.0


def host_cpu():
    """(model name, logical cores of the host, cores this process may use)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    return model, os.cpu_count() or 1, allowed


def cpu_baseline(b, seconds=12.0, n=256, threads=None):
    """The FP64 oracle as it stands, on a seeded scene subset, on every host
    core allotted to this process (at most 16: the CPU share of one GPU on a
    shared box)."""
    import oracle
    oracle.build(force=False)
    model, host_cores, allowed = host_cpu()
    cores = threads or min(16, allowed)
    rng = np.random.default_rng(1)
    pick = sorted(rng.choice(b.n_scenes, min(n, b.n_scenes), replace=False).tolist())
    sub = b.subset(pick)
    o = oracle.Oracle(sub, threads=cores)
    x = sub.state0.astype(np.float64)
    steps = 0
    t0 = time.perf_counter()
    while True:
        x = o.step(x, b.controls(steps, pick))
        steps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": len(pick) * steps / dt, "unit": "env-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(pick)} seeded scenes of the same workload x {steps} control steps, FP64, {dt:.1f} s",
            "cpu_model": model, "host_cores": host_cores, "allotted_cores": allowed}


def measured_peaks(ms, torch, stream):
    """Achievable rates of this device as the library is built: a streaming
    copy of 2 x 1 GiB (HBM, far above the 256 MB Infinity Cache) and an FP32
    FMA-chain kernel (packed FP32 is off in this build, so about half the
    157.3 TFLOP/s published peak is the ceiling)."""
    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = torch.zeros(1024, dtype=torch.float32, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for _ in range(2):
        ms.probe_copy(src, dst, stream)
    ev[0].record(stream)
    reps = 5
    for _ in range(reps):
        ms.probe_copy(src, dst, stream)
    ev[1].record(stream)
    blocks, iters = 256 * 64, 256
    ms.probe_fma(out, blocks, iters, stream)
    ev[2].record(stream)
    fl = 0.0
    for _ in range(reps):
        fl += ms.probe_fma(out, blocks, iters, stream)
    ev[3].record(stream)
    torch.cuda.synchronize()
    copy_gbs = reps * 2 * 4 * n / (ev[0].elapsed_time(ev[1]) * 1e-3) / 1e9
    fma_tflops = fl / (ev[2].elapsed_time(ev[3]) * 1e-3) / 1e12
    del src, dst
    return {"hbm_copy_gbs": round(copy_gbs, 1), "fp32_fma_tflops": round(fma_tflops, 2),
            "copy_bytes_per_launch": 2 * 4 * n, "fma_launch": f"{blocks} x 256 lanes, 8 chains x {16 * iters} FMAs"}


def load_traffic(name, nscenes, src_hash, flags, graph_bit):
    """HBM traffic of the dominant kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source, the same batch
    size and the same schedule (graph replay or direct launch of the same
    kernel does not change its traffic)."""
    p = os.path.join(ROOT, "profiles", f"k_step_{name.split('_')[0]}_{nscenes}_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("kernel_source_hash") != src_hash or d.get("scenes") != nscenes:
        return None
    if (int(d.get("schedule_flags", -1)) & ~graph_bit) != (int(flags) & ~graph_bit):
        return None
    # per control step (all of the step's launches), like `achieved`
    return d.get("bytes_per_control_step", d.get("bytes_per_launch"))


def time_fwd_bwd(mb, x0, U, args, flags, stream, torch, keep_records=True, grid=0):
    """Forward + backward over a horizon of T control steps: T steps forward
    keeping every state, then T vector-Jacobian products in reverse.  With
    keep_records every forward step also writes its record (substep states,
    contact lists, Gauss-Seidel tape: T x sizes.record bytes resident in HBM)
    and the backward reads it; without, each backward step runs its forward
    step again to record it.  Inputs resident in HBM; HIP events on the
    launch stream."""
    T = max(1, args.bwd_steps)
    S = mb.S
    mb.set_schedule(flags, grid)
    xs = [x0.clone() for _ in range(T + 1)]
    g0 = torch.randn_like(x0) * 1e-3
    gx = g0.clone()
    gu = torch.empty((S, 16), dtype=torch.float32, device=x0.device)
    recs = [mb.new_record() for _ in range(T)] if keep_records else None

    def once():
        for t in range(T):
            if recs is not None:
                mb.step_record(xs[t], U[t % U.shape[0]], recs[t], out=xs[t + 1])
            else:
                mb.step(xs[t], U[t % U.shape[0]], out=xs[t + 1])
        ev_mid.record(stream)
        gx.copy_(g0)
        for t in range(T - 1, -1, -1):
            if recs is not None:
                mb.step_backward_recorded(xs[t], U[t % U.shape[0]], recs[t], gx, gx_in=gx, gu=gu)
            else:
                mb.step_backward(xs[t], U[t % U.shape[0]], gx, gx_in=gx, gu=gu)

    ev0, ev_mid, ev1 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    once()  # warm-up (graph capture for the forward)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    once()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd_ms = ev0.elapsed_time(ev_mid)
    bwd_ms = ev_mid.elapsed_time(ev1)
    ok = bool(torch.isfinite(gx).all().item() and torch.isfinite(gu).all().item())
    out = {"value": round(S * T / wall, 1), "unit": "env-steps/s", "horizon": T,
           "ms_per_step": round(1e3 * wall / T, 4), "fwd_ms_per_step": round(fwd_ms / T, 4),
           "bwd_ms_per_step": round(bwd_ms / T, 4), "finite": ok}
    if recs is not None:
        out["record_bytes_per_step"] = int(mb.sizes.record)
    del recs
    return out


def time_env_outputs(mb, b, x0, U, args, flags, stream, torch, ms, sg):
    """Cost of the environment outputs around the step: the forward step with
    the contact-force and gripper outputs on, and one subtask predicate /
    event update (ms_task_update) per control step.  Fetch-like robots only.
    The end-effector rest position is the paper's (0.5, 0, 1.25) m; it does
    not change the cost."""
    r = dict(sg.FETCH_TASK_ROBOT)
    r["ee_rest"] = (0.5, 0.0, 1.25)
    try:
        mb.set_task_robot(r)
    except ms.MsError:
        return None
    rf, _ = mb.enable_forces()
    grip = mb.enable_grip()
    tt = mb.task_tensor(sg.tasks(b))
    mb.set_schedule(flags)
    xa, xb = x0.clone(), torch.empty_like(x0)
    ep, _ = mb.task_begin(xa, tt)
    for t in range(min(args.warmup, U.shape[0])):
        mb.step(xa, U[t], out=xb)
        mb.task_update(xb, tt, ep, rf, grip=grip)
        xa, xb = xb, xa
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    n = args.steps
    ev[0].record(stream)
    for t in range(n):
        mb.step(xa, U[t % U.shape[0]], out=xb)
        xa, xb = xb, xa
    ev[1].record(stream)
    ev[2].record(stream)
    for t in range(n):
        mb.task_update(xa, tt, ep, rf, grip=grip)
    ev[3].record(stream)
    torch.cuda.synchronize()
    events = int(mb.episodes(ep)["n"].sum())
    mb.enable_grip(False)
    mb.enable_forces(False)
    return {"fwd_with_outputs_ms_per_step": round(ev[0].elapsed_time(ev[1]) / n, 4),
            "task_update_ms": round(ev[2].elapsed_time(ev[3]) / n, 4), "events_recorded": events}


def time_cfg4(ms, sg, torch, stream, every=10):
    """Differentiation workload as stated: 256 scenes, 50 control steps of
    20 ms, loss = squared distance of each scene's pushed box to its seeded
    goal; forward and backward through the checkpointed autograd function
    (a checkpoint every 10 steps).  Inputs resident in HBM; HIP events on the
    launch stream."""
    from paper_2412_13211_amd.autograd import rollout
    b = sg.make(4)
    S, T = b.n_scenes, b.n_steps
    mb = ms.MsBatch(b, backward=True)
    mb.set_schedule(ms.MS_SCHED_GRAPH | ms.MS_SCHED_PERSISTENT | ms.MS_SCHED_CULL)
    U0 = torch.as_tensor(np.stack([b.controls(t) for t in range(T)])).cuda()
    x0 = torch.as_tensor(b.state0).cuda()
    goals = torch.as_tensor(b.push_goals(), dtype=torch.float32, device="cuda")
    bi = torch.as_tensor(np.asarray(b.free_off[:-1], np.int64), device="cuda")
    nf = b.n_free

    def once():
        U = U0.clone().requires_grad_(True)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(stream)
        xT = rollout(mb, x0, U, every=every)
        fr = xT[32 * S: 32 * S + 16 * nf].view(nf, 16)
        loss = ((fr[bi, 0:3] - goals) ** 2).sum()
        ev[1].record(stream)
        loss.backward()
        ev[2].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), bool(torch.isfinite(U.grad).all().item())

    once()
    t0 = time.perf_counter()
    f_ms, b_ms, ok = once()
    wall = time.perf_counter() - t0
    return {"value": round(S * T / wall, 1), "unit": "env-steps/s", "scenes": S, "horizon": T,
            "checkpoint_every": every, "ms_per_step": round(1e3 * wall / T, 4),
            "fwd_ms_per_step": round(f_ms / T, 4), "bwd_ms_per_step": round(b_ms / T, 4), "finite": ok,
            "workload": f"{b.name}: {S} scenes, h={b.h:g} s x {b.n_sub} substeps, loss = squared box-goal distance"}


def time_cfg5(ms, sg, torch, stream, T=20):
    """Articulated furniture at scale: 16384 scenes, forward plus backward
    over a 20-step horizon; the forward steps replay a captured hipGraph of
    the persistent step, the backward chains ms_step_backward (each call
    records its step again); algorithmic HBM bytes: state in + out,
    controls, scene description per forward step, and per backward step the
    state and controls in, the state adjoint in and out, the control adjoint
    out and the scene description."""
    t_gen = time.perf_counter()
    b = sg.make(5)
    gen_s = time.perf_counter() - t_gen
    S = b.n_scenes
    mb = ms.MsBatch(b, backward=True)
    flags = ms.MS_SCHED_GRAPH | ms.MS_SCHED_PERSISTENT | ms.MS_SCHED_CULL | ms.MS_SCHED_STAGE_STATIC
    mb.set_schedule(flags)
    blocks = {}   # PD targets are resampled every ctrl_block steps
    for t in range(T):
        if t // b.ctrl_block not in blocks:
            blocks[t // b.ctrl_block] = b.controls(t)
    U = torch.as_tensor(np.stack([blocks[t // b.ctrl_block] for t in range(T)])).cuda()
    xs = [torch.as_tensor(b.state0).cuda()] + [torch.empty(b.state_floats, device="cuda") for _ in range(T)]
    g0 = torch.randn(b.state_floats, device="cuda") * 1e-3
    gx = g0.clone()
    gu = torch.empty((S, 16), dtype=torch.float32, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def once():
        ev[0].record(stream)
        for t in range(T):
            mb.step(xs[t], U[t], out=xs[t + 1])
        ev[1].record(stream)
        gx.copy_(g0)
        for t in range(T - 1, -1, -1):
            mb.step_backward(xs[t], U[t], gx, gx_in=gx, gu=gu)
        ev[2].record(stream)

    once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    once()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    f_ms, b_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    fwd_bytes = algorithmic_bytes_per_env_step(b)
    state = b.state_floats * 4
    bwd_bytes = fwd_bytes - state + 2 * state + 16 * S * 4     # + adjoint in and out + control adjoint
    gbs = T * (fwd_bytes + bwd_bytes) / ((f_ms + b_ms) * 1e-3) / 1e9
    return {"value": round(S * T / wall, 1), "unit": "env-steps/s", "scenes": S, "horizon": T,
            "ms_per_step": round(1e3 * wall / T, 4), "fwd_ms_per_step": round(f_ms / T, 4),
            "bwd_ms_per_step": round(b_ms / T, 4), "fwd_env_steps_per_s": round(S * T / (f_ms * 1e-3), 1),
            "hbm_gbs": round(gbs, 2), "hbm_frac": round(gbs / HBM_PEAK_GBS, 6),
            "bytes_per_env_step_batch": {"fwd": fwd_bytes, "bwd": bwd_bytes},
            "finite": bool(torch.isfinite(gx).all().item() and torch.isfinite(gu).all().item()),
            "schedule_flags": flags, "generated_s": round(gen_s, 1),
            "workload": f"{b.name}: {S} scenes, door + drawer + {b.n_free // S} free objects + 64 boxes, "
                        f"h={b.h:g} s x {b.n_sub} substeps"}


def time_cfg2_paper_rate(ms, sg, torch, stream, steps=20):
    """The config-2 scene at the paper's own rate: 100 Hz physics (h = 10 ms)
    under 20 Hz control (5 substeps), 1024 scenes, forward."""
    b = sg.make(2, h=0.01, n_sub=5)
    S = b.n_scenes
    mb = ms.MsBatch(b)
    mb.set_schedule(ms.MS_SCHED_GRAPH | ms.MS_SCHED_PERSISTENT | ms.MS_SCHED_CULL | ms.MS_SCHED_STAGE_STATIC)
    blocks = {}
    for t in range(steps):
        if t // b.ctrl_block not in blocks:
            blocks[t // b.ctrl_block] = b.controls(t)
    U = torch.as_tensor(np.stack([blocks[t // b.ctrl_block] for t in range(steps)])).cuda()
    xa = torch.as_tensor(b.state0).cuda()
    xb = torch.empty_like(xa)
    for t in range(3):
        mb.step(xa, U[t], out=xb)
        xa, xb = xb, xa
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for t in range(steps):
        mb.step(xa, U[t], out=xb)
        xa, xb = xb, xa
    ev[1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = mb.status()
    return {"value": round(S * steps / wall, 1), "unit": "env-steps/s", "scenes": S, "h": b.h, "substeps": b.n_sub,
            "ms_per_step": round(ev[0].elapsed_time(ev[1]) / steps, 4), "scene_status_nonzero": int(np.count_nonzero(st))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--scenes", type=int, default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-bwd", action="store_true", help="skip the forward+backward measurement")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-substep comparison run")
    ap.add_argument("--bwd-steps", type=int, default=10, help="control steps in the timed forward+backward horizon")
    ap.add_argument("--schedule", default="auto", help="auto | graph | graph-persistent | persistent | fused | plain")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2412_13211_amd", "autotune_cache.jsonl"),
                    help="autotune cache file (JSON lines; '' for none)")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-captured comparison runs")
    ap.add_argument("--no-peaks", action="store_true", help="skip the copy and FMA-chain probes")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (cfg4 and cfg5 forward+backward, cfg2 at the paper's rate)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: scenes are independent and the step has no cross-GPU "
              f"exchange, so G GPUs run G independent batches (asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        n = args.calibrate_copy // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n, "launches": 5}), flush=True)
        return
    import paper_2412_13211_amd as ms
    import scenegen as sg

    t_gen = time.perf_counter()
    b = sg.make(args.config, args.scenes)
    S = b.n_scenes
    print(f"[bench] workload {b.name}: {S} scenes, {b.n_free} free bodies, {int(b.static_off[-1])} boxes "
          f"(generated in {time.perf_counter() - t_gen:.1f} s)", file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    mb = ms.MsBatch(b, backward=not args.no_bwd)
    # controls for every timed step, resident in HBM before timing
    n_ctrl = args.warmup + args.steps
    blocks = {}
    U = torch.empty((n_ctrl, S, 16), dtype=torch.float32, device=dev)
    for t in range(n_ctrl):
        key = t // b.ctrl_block if b.ctrl_kind == "pd_targets" else t
        if key not in blocks:
            blocks[key] = torch.as_tensor(b.controls(t)).to(dev)
        U[t].copy_(blocks[key])
    x0 = torch.as_tensor(b.state0).to(dev)
    xa = x0.clone()
    xb = torch.empty_like(x0)
    stream = torch.cuda.current_stream()

    def run(n, flags, time_it, grid=0):
        nonlocal xa, xb
        mb.set_schedule(flags, grid)
        xa.copy_(x0)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        # warm-up (also captures the graphs for both ping-pong directions)
        for t in range(min(args.warmup, n_ctrl)):
            mb.step(xa, U[t], out=xb)
            xa, xb = xb, xa
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record(stream)
        for t in range(args.steps):
            mb.step(xa, U[(args.warmup + t) % n_ctrl], out=xb)
            xa, xb = xb, xa
        ev[1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gpu_ms = ev[0].elapsed_time(ev[1])
        return wall, gpu_ms

    flags_graph = ms.MS_SCHED_GRAPH | ms.MS_SCHED_STAGE_STATIC | ms.MS_SCHED_CULL
    tune = None
    grid = 0
    if args.schedule == "auto":
        mb.set_autotune_cache(args.tune_cache or None)
        # tune on the state the timed steps start from (after the warm-up)
        xw = x0.clone()
        for t in range(min(args.warmup, n_ctrl)):
            xw = mb.step(xw, U[t])
        uw = U[min(args.warmup, n_ctrl - 1)]
        (flags, grid), t_auto = mb.autotune(xw, uw, reps=5)
        key, hit = mb.autotune_key()
        tune = {"key": key, "from_cache": hit, "flags": int(flags), "grid": int(grid),
                "fwd_split_cap": int(mb.get_forward_split()), "tuned_ms_per_step": round(float(t_auto), 4)}
        if not args.no_bwd:
            g0 = torch.randn_like(x0) * 1e-3
            (bc, br), t_b = mb.autotune_backward(xw, uw, g0, reps=2)
            bkey, bhit = mb.autotune_key(backward=True)
            tune["backward"] = {"key": bkey, "from_cache": bhit, "split_cap": [int(bc), int(br)],
                                "tuned_ms_per_step": round(float(t_b), 4)}
        print(f"[bench] autotune: {tune}", file=sys.stderr, flush=True)
    elif args.schedule == "graph":
        flags = flags_graph
    elif args.schedule == "graph-persistent":
        flags = flags_graph | ms.MS_SCHED_PERSISTENT
    elif args.schedule == "persistent":
        flags = ms.MS_SCHED_PERSISTENT | ms.MS_SCHED_CULL
    elif args.schedule == "fused":
        flags = ms.MS_SCHED_STAGE_STATIC | ms.MS_SCHED_CULL
    else:
        flags = ms.MS_SCHED_STAGE_STATIC | ms.MS_SCHED_PER_SUBSTEP | ms.MS_SCHED_CULL
    print(f"[bench] schedule flags {flags}", file=sys.stderr, flush=True)
    wall, gpu_ms = run(args.steps, flags, True, grid)
    # the plain form: one launch per substep, no graph, same kernel
    if args.no_plain:
        wall_plain = float("nan")
    else:
        wall_plain, gpu_ms_plain = run(args.steps, ms.MS_SCHED_STAGE_STATIC | ms.MS_SCHED_PER_SUBSTEP |
                                       ms.MS_SCHED_CULL, True)
    # the batched graph-captured form: one persistent launch per control step
    # replayed from a hipGraph (with and without furniture staged in LDS)
    graph_forms = {}
    for gf in (() if args.no_graph else
               (ms.MS_SCHED_GRAPH | ms.MS_SCHED_PERSISTENT | ms.MS_SCHED_CULL,
                ms.MS_SCHED_GRAPH | ms.MS_SCHED_PERSISTENT | ms.MS_SCHED_CULL | ms.MS_SCHED_STAGE_STATIC)):
        graph_forms[gf] = run(args.steps, gf, True)
    gflags = min(graph_forms, key=lambda k: graph_forms[k][0]) if graph_forms else 0
    wall_graph, gpu_ms_graph = graph_forms[gflags] if graph_forms else (float("nan"), float("nan"))
    print(f"[bench] main form {1e3 * wall / args.steps:.3f} ms, graph-captured {1e3 * wall_graph / args.steps:.3f} ms, "
          f"plain {1e3 * wall_plain / args.steps:.3f} ms", file=sys.stderr, flush=True)
    fwd_bwd = None if args.no_bwd else time_fwd_bwd(mb, x0, U, args, flags, stream, torch, grid=grid)
    fwd_bwd_rc = None if args.no_bwd else time_fwd_bwd(mb, x0, U, args, flags, stream, torch, keep_records=False,
                                                      grid=grid)
    st = mb.status()
    env_out = time_env_outputs(mb, b, x0, U, args, flags, stream, torch, ms, sg)
    peaks = None if args.no_peaks else measured_peaks(ms, torch, stream)
    extra = {}
    if not args.no_extra:
        print("[bench] cfg4 forward+backward", file=sys.stderr, flush=True)
        extra["cfg4_fwd_bwd"] = time_cfg4(ms, sg, torch, stream)
        print("[bench] cfg2 at the paper's rate", file=sys.stderr, flush=True)
        extra["cfg2_paper_rate"] = time_cfg2_paper_rate(ms, sg, torch, stream)
        print("[bench] cfg5 forward+backward", file=sys.stderr, flush=True)
        extra["cfg5_fwd_bwd"] = time_cfg5(ms, sg, torch, stream)
    value = S * args.steps / wall
    ms_per_step = 1e3 * wall / args.steps
    # one control step = the step's launches on the launch stream (the
    # scene-order kernel, the persistent step; in the split form also the
    # second stream's launch, joined back before the event)
    launch_ms = gpu_ms / args.steps
    bytes_step = algorithmic_bytes_per_env_step(b)
    flops_env = algorithmic_flops_per_env_step(b)
    flops_launch = flops_env * S
    achieved_tflops = flops_launch / (launch_ms * 1e-3) / 1e12
    hbm_gbs = bytes_step / (launch_ms * 1e-3) / 1e9
    src_hash = kernel_source_hash()
    traffic = load_traffic(b.name, S, src_hash, flags, ms.MS_SCHED_GRAPH)
    out = {
        "metric": f"physics env-steps/sec at {S} scenes (fwd)",
        "value": round(value, 1),
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{b.name}: {S} scenes, {b.n_free} free objects, {int(b.static_off[-1])} furniture "
                               f"boxes, h={b.h:g} s x {b.n_sub} substeps, {b.pgs_iters} PGS sweeps",
                   "scenes": S, "substeps": b.n_sub, "schedule_flags": int(flags)},
        "autotune": tune,
        "roofline": {"bound": "alu", "achieved": round(achieved_tflops, 4), "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved_tflops / FP32_VECTOR_PEAK_TFLOPS, 6),
                     "traffic": traffic, "flops_per_env_step": round(flops_env),
                     "flops_model": "oracle op count of one control step (64-scene mean); each emit decision "
                                    "charged its signed-distance cost",
                     "kernel_ms_per_launch": round(launch_ms, 5),
                     "measured_peak": peaks and peaks["fp32_fma_tflops"],
                     "frac_of_measured_peak": peaks and round(achieved_tflops / peaks["fp32_fma_tflops"], 6)},
        "hbm_roofline": {"achieved": round(hbm_gbs, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(hbm_gbs / HBM_PEAK_GBS, 6), "bytes_per_env_step_batch": bytes_step,
                         "measured_peak": peaks and peaks["hbm_copy_gbs"],
                         "frac_of_measured_peak": peaks and round(hbm_gbs / peaks["hbm_copy_gbs"], 6)},
        "measured_peaks": peaks,
        "plain_per_substep": None if args.no_plain else {
            "value": round(S * args.steps / wall_plain, 1), "unit": "env-steps/s",
            "ms_per_step": round(1e3 * wall_plain / args.steps, 4)},
        "graph_captured": None if args.no_graph else {
            "value": round(S * args.steps / wall_graph, 1), "unit": "env-steps/s",
            "ms_per_step": round(1e3 * wall_graph / args.steps, 4),
            "kernel_ms_per_step": round(gpu_ms_graph / args.steps, 5), "schedule_flags": int(gflags),
            "vs_plain_per_substep": None if args.no_plain else round(wall_plain / wall_graph, 3)},
        "scene_status_nonzero": int(np.count_nonzero(st)),
    }
    if fwd_bwd is not None:
        out["fwd_bwd"] = fwd_bwd
        out["fwd_bwd_recompute"] = fwd_bwd_rc
    if env_out is not None:
        out["env_outputs"] = env_out
    out.update(extra)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(b)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
