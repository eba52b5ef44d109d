"""The C-ABI library loads and exports every function include/ms_phys.h declares;
argument validation (which needs no GPU) rejects malformed inputs."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2412_13211_amd as ms
import scenegen as sg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ms_phys.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ms_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = ms.lib()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(ms.EXPORTS) <= set(names)


def test_library_is_gfx950_code_object():
    # the shared object carries an embedded gfx950 offload bundle
    data = open(ms.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def _sizes(batch, **over):
    d = ms.make_desc(batch, **over)
    sd, keep = ms.make_scene_desc(batch)
    sz = ms.Sizes()
    rc = ms.lib().ms_query_sizes(C.byref(d), C.byref(sd), C.byref(sz))
    return rc, sz, keep


def test_query_sizes_valid():
    b = sg.make(1)
    rc, sz, _ = _sizes(b)
    assert rc == 0
    assert sz.state == b.state_floats * 4
    assert sz.params > 0 and sz.scratch > 0 and sz.lds > 0
    n = C.c_size_t()
    sd, keep = ms.make_scene_desc(b)
    assert ms.lib().ms_state_floats(C.byref(sd), b.n_scenes, C.byref(n)) == 0
    assert n.value == b.state_floats


@pytest.mark.parametrize("mutate,msg", [
    (lambda b: setattr(b, "contact_cap", 0), "contact_cap"),
    (lambda b: setattr(b, "n_sub", 0), "n_substeps"),
    (lambda b: setattr(b, "h", 0.0), "h must"),
    (lambda b: setattr(b, "control_mode", 7), "control_mode"),
    (lambda b: b.free_off.__setitem__(1, b.free_off[2] + 1), "not monotone"),
    (lambda b: b.model_parent.__setitem__((0, 1), 3), "parent"),
    (lambda b: b.free_mass.__setitem__(0, 0.0), "mass"),
    (lambda b: b.scene_model.__setitem__(0, 5), "model"),
])
def test_query_sizes_rejects(mutate, msg):
    b = sg.make(1, 4)
    mutate(b)
    rc, _, _ = _sizes(b)
    assert rc == -1
    assert msg in ms.lib().ms_last_error().decode()


def test_null_arguments_rejected():
    L = ms.lib()
    assert L.ms_step(None, None, None, None, None) == -1
    assert L.ms_destroy_batch(None) == -1
    assert L.ms_query_sizes(None, None, None) == -1


def test_python_constants_match_header():
    """Every MS_* enumerator the binding defines has the header's value (the
    binding marshals flags and reads status bits by these numbers)."""
    hdr = open(os.path.join(ROOT, "include", "ms_phys.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    values = {}
    for body in re.findall(r"enum\s*\{(.*?)\}", hdr, flags=re.S):
        for name, val in re.findall(r"(MS_[A-Z0-9_]+)\s*=\s*(-?\w+)", body):
            values[name] = int(val.rstrip("uU"), 0)
    names = [n for n in dir(ms) if re.fullmatch(r"MS_[A-Z0-9_]+", n) and isinstance(getattr(ms, n), int)]
    checked = [n for n in names if n in values]
    assert len(checked) >= 20, checked
    for n in checked:
        assert getattr(ms, n) == values[n], (n, getattr(ms, n), values[n])
