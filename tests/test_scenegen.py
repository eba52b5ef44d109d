"""The seeded scene generator: subsets reproduce the full batch's scenes."""
import numpy as np

import scenegen as sg


def test_subset_draws_the_same_controls_and_state():
    b = sg.make(3, 64)
    pick = [0, 5, 17, 63]
    sub = b.subset(pick)
    for t in (0, 7, 25):
        assert np.array_equal(sub.controls_for(t), b.controls(t, pick))
    sub2 = sub.subset([1, 3])
    assert np.array_equal(sub2.controls_for(3), b.controls(3, [5, 63]))
    full = sg.split_state(b.state0, b.n_scenes, b.n_free, b.n_aux)
    part = sg.split_state(sub.state0, sub.n_scenes, sub.n_free, sub.n_aux)
    assert np.array_equal(part["q"], full["q"][pick])
    for r, s in enumerate(pick):
        assert np.array_equal(part["free"][sub.free_off[r]:sub.free_off[r + 1]],
                              full["free"][b.free_off[s]:b.free_off[s + 1]])


def test_torque_controls_subset():
    b = sg.make(1)
    sub = b.subset([3, 9])
    assert np.array_equal(sub.controls_for(4), b.controls(4, [3, 9]))
