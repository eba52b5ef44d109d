"""The allocation-free entry point ms_step_noalloc, called through the C ABI,
gives ms_step's results bit for bit on two calls in a row, the second on a
smaller batch (its scratch is one device array every call shares; the work
counter must start from zero each time), in the persistent and one-workgroup-
per-scene forms and with normalized actions (PD targets staged in it)."""
import ctypes as C

import numpy as np
import pytest

import scenegen as sg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ms():
    import paper_2412_13211_amd as ms
    return ms


def say(*a):
    print(*a, flush=True)


def _noalloc(ms, mb, x, u, out):
    rc = ms.lib().ms_step_noalloc(mb.h, C.c_void_p(x.data_ptr()), C.c_void_p(u.data_ptr()),
                                  C.c_void_p(out.data_ptr()), C.c_void_p(0))
    if rc != 0:
        raise ms.MsError(ms.lib().ms_last_error().decode())


@pytest.mark.parametrize("flags_name", ["persistent", "per_scene"])
def test_noalloc_step_equals_step(flags_name):
    ms = _ms()
    ms.lib().ms_step_noalloc.argtypes = [C.c_void_p] * 5
    ms.lib().ms_step_noalloc.restype = C.c_int32
    flags = ms.MS_SCHED_CULL | ms.MS_SCHED_STATIC_ORDER | (ms.MS_SCHED_PERSISTENT if flags_name == "persistent" else 0)
    for cfg, S, steps in [(3, 96, 3), (6, 40, 2), (2, 24, 2)]:   # each call after a larger one
        b = sg.make(cfg, S)
        say(f"[noalloc] {flags_name}: cfg{cfg} S={S}")
        ref_mb = ms.MsBatch(b)
        ref_mb.set_schedule(flags)
        mb = ms.MsBatch(b)
        mb.set_schedule(flags)
        x_ref = torch.as_tensor(b.state0).cuda()
        x = x_ref.clone()
        for t in range(steps):
            u = torch.as_tensor(b.controls(t)).cuda()
            y_ref = ref_mb.step(x_ref, u)
            y = torch.empty_like(x)
            _noalloc(ms, mb, x, u, y)
            torch.cuda.synchronize()
            assert torch.equal(y, y_ref), (cfg, t, (y - y_ref).abs().max().item())
            assert np.array_equal(mb.status(), ref_mb.status())
            x_ref, x = y_ref, y


def test_noalloc_rejects_too_many_scenes_and_bad_arguments():
    ms = _ms()
    ms.lib().ms_step_noalloc.argtypes = [C.c_void_p] * 5
    ms.lib().ms_step_noalloc.restype = C.c_int32
    b = sg.make(1, 2)
    mb = ms.MsBatch(b)
    x = torch.as_tensor(b.state0).cuda()
    u = torch.zeros((2, 16), device="cuda")
    rc = ms.lib().ms_step_noalloc(mb.h, C.c_void_p(x.data_ptr()), None, C.c_void_p(x.data_ptr()), None)
    assert rc == -1   # MS_E_INVALID
    big = sg.custom_batch([sg.empty_model()], [dict()] * 16385)
    mbb = ms.MsBatch(big)
    xb = torch.as_tensor(big.state0).cuda()
    ub = torch.zeros((16385, 16), device="cuda")
    rc = ms.lib().ms_step_noalloc(mbb.h, C.c_void_p(xb.data_ptr()), C.c_void_p(ub.data_ptr()),
                                  C.c_void_p(xb.data_ptr()), None)
    assert rc == -1   # MS_E_INVALID
    assert b"16384" in ms.lib().ms_last_error()
    del u
