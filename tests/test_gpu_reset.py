"""GPU robot resets and spawn check (ms_reset_robots / ms_spawn_check):
resets follow their definition exactly; the spawn check equals the oracle's
brute-force penetration test scene by scene, except where the smallest signed
distance is within 1e-5 m of zero (the decision then depends on the
precision the distances are computed in)."""
import numpy as np
import pytest

import oracle
import scenegen as sg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# clip per DoF of the Fetch-like model: base x, y 0.2 m, yaw 0.5 rad, arm joints 0.2 rad
CLIP = np.zeros(16, np.float32)
CLIP[0:2] = 0.2
CLIP[2] = 0.5
CLIP[6:13] = 0.2


def test_reset_robots_definition():
    import paper_2412_13211_amd as ms
    b = sg.make(2, 64)
    mb = ms.MsBatch(b)
    rng = np.random.default_rng(0)
    x0 = b.state0.copy()
    st = sg.split_state(x0, b.n_scenes, b.n_free, b.n_aux)
    st["qd"][:] = rng.normal(size=st["qd"].shape).astype(np.float32)
    base = rng.normal(size=(b.n_scenes, 16)).astype(np.float32)
    noise = rng.normal(0, 0.3, (b.n_scenes, 16)).astype(np.float32)
    mask = (rng.uniform(size=b.n_scenes) < 0.5).astype(np.uint8)
    x = torch.as_tensor(x0).cuda()
    mb.reset_robots(x, torch.as_tensor(base).cuda(), torch.as_tensor(noise).cuda(), CLIP,
                    mask=torch.as_tensor(mask).cuda())
    got = x.cpu().numpy()
    want = x0.copy()
    ws = sg.split_state(want, b.n_scenes, b.n_free, b.n_aux)
    m = mask.astype(bool)
    ws["q"][m] = base[m] + np.clip(noise[m], -CLIP, CLIP)
    ws["qd"][m] = 0.0
    assert np.array_equal(got, want)


@pytest.mark.parametrize("cfg", [2, 5])
def test_spawn_check_matches_oracle(cfg):
    import paper_2412_13211_amd as ms
    b = sg.make(cfg, 96)
    o = oracle.Oracle(b, threads=8)
    rng = np.random.default_rng(cfg)
    x = b.state0.astype(np.float64).copy()
    st = sg.split_state(x, b.n_scenes, b.n_free, b.n_aux)
    # large base and arm perturbations make some spawns collide
    st["q"][:, 0:2] += rng.uniform(-1.5, 1.5, (b.n_scenes, 2))
    st["q"][:, 6:13] += rng.uniform(-1.0, 1.0, (b.n_scenes, 7))
    x = x.astype(np.float32).astype(np.float64)
    want, phi = o.spawn_check(x, with_phi=True)
    clear = np.abs(phi) >= 1e-5
    mb = ms.MsBatch(b)
    got = mb.spawn_check(torch.as_tensor(x.astype(np.float32)).cuda()).cpu().numpy()
    print(f"cfg{cfg}: {int(want.sum())} of {b.n_scenes} spawns collide, {int((~clear).sum())} within 1e-5 m of "
          f"contact", flush=True)
    assert 0 < want.sum() < b.n_scenes and clear.sum() >= 0.9 * b.n_scenes
    assert np.array_equal(got.astype(np.int32)[clear], want[clear])
