"""The state and schedule helpers of the C ABI on the GPU: ms_get_state views,
masked ms_set_state, ms_autotune, ms_scene_status, argument errors."""
import numpy as np
import pytest

import scenegen as sg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_get_state_views_share_memory():
    import paper_2412_13211_amd as ms
    b = sg.make(5, 32)
    mb = ms.MsBatch(b)
    x = torch.as_tensor(b.state0).cuda()
    v = mb.get_state(x)
    ref = sg.split_state(b.state0, b.n_scenes, b.n_free, b.n_aux)
    for k in ("q", "qd", "free", "aux"):
        assert np.array_equal(v[k].cpu().numpy(), ref[k])
    assert np.array_equal(v["free_off"], b.free_off) and np.array_equal(v["aux_off"], b.aux_off)
    v["q"][3, 4] = 123.0
    assert float(x[16 * 3 + 4]) == 123.0


def test_set_state_masked_copy():
    import paper_2412_13211_amd as ms
    b = sg.make(3, 40)
    mb = ms.MsBatch(b)
    rng = np.random.default_rng(1)
    a = rng.normal(size=b.state0.size).astype(np.float32)
    src = rng.normal(size=b.state0.size).astype(np.float32)
    mask = (rng.uniform(size=b.n_scenes) < 0.5).astype(np.uint8)
    x = torch.as_tensor(a).cuda()
    mb.set_state(x, torch.as_tensor(src).cuda(), torch.as_tensor(mask).cuda())
    torch.cuda.synchronize()
    got = sg.split_state(x.cpu().numpy(), b.n_scenes, b.n_free, b.n_aux)
    A = sg.split_state(a, b.n_scenes, b.n_free, b.n_aux)
    B = sg.split_state(src, b.n_scenes, b.n_free, b.n_aux)
    for s in range(b.n_scenes):
        pick = B if mask[s] else A
        assert np.array_equal(got["q"][s], pick["q"][s]) and np.array_equal(got["qd"][s], pick["qd"][s])
        f0, f1 = b.free_off[s], b.free_off[s + 1]
        assert np.array_equal(got["free"][f0:f1], pick["free"][f0:f1])
    # no mask: every scene
    mb.set_state(x, torch.as_tensor(src).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), src)


def test_autotune_status_and_errors(tmp_path):
    import paper_2412_13211_amd as ms
    b = sg.make(2, 256)
    mb = ms.MsBatch(b)
    x = torch.as_tensor(b.state0).cuda()
    u = torch.as_tensor(b.controls(0)).cuda()
    cache = tmp_path / "tune.jsonl"
    mb.set_autotune_cache(cache)
    (flags, grid), t = mb.autotune(x, u, reps=2)
    key, hit = mb.autotune_key()
    known = ms.MS_SCHED_PERSISTENT | ms.MS_SCHED_GRAPH | ms.MS_SCHED_STAGE_STATIC | ms.MS_SCHED_CULL | \
        ms.MS_SCHED_FWD_ONE_LAUNCH
    assert flags & ~known == 0 and t > 0 and grid >= 0
    assert key.startswith("gfx950:fwd:") and not hit
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and f'"key": "{key}"' in lines[0] and f'"flags": {flags}' in lines[0]
    # a second batch of the same configuration takes the cached choice without timing
    mb2 = ms.MsBatch(b)
    mb2.set_autotune_cache(cache)
    (flags2, grid2), t2 = mb2.autotune(x, u, reps=2)
    assert (flags2, grid2) == (flags, grid) and mb2.autotune_key() == (key, True)
    assert mb2.get_forward_split() == mb.get_forward_split()
    assert len(cache.read_text().splitlines()) == 1
    # a different configuration has a different key
    mb3 = ms.MsBatch(sg.make(2, 128))
    assert mb3.autotune_key()[0] != key
    # backward tuning needs the adjoint workspace; with it, a choice and its key
    with pytest.raises(ms.MsError, match="tape"):
        mb.autotune_backward(x, u, x.clone())
    mbb = ms.MsBatch(b, backward=True)
    mbb.set_autotune_cache(cache)
    (sc, sr), tb = mbb.autotune_backward(x, u, torch.randn_like(x) * 1e-3, reps=1)
    assert tb > 0 and (sc, sr) == mbb.get_backward_split()
    assert mbb.autotune_key(backward=True)[0].startswith("gfx950:bwd:")
    y = mb.step(x, u)
    torch.cuda.synchronize()
    assert np.count_nonzero(mb.status()) == 0
    assert np.array_equal(x.cpu().numpy(), b.state0)  # the input is not modified
    with pytest.raises(ms.MsError):
        mb.step(x[:-1].contiguous(), u)
    with pytest.raises(ms.MsError):
        mb.set_schedule(1 << 12)
    with pytest.raises(ms.MsError):
        mb.step_backward(x, u, y)  # no adjoint workspace
