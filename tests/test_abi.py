"""C ABI checks that need no GPU: the library loads, exports every function
include/vuda.h declares, and rejects malformed descriptors before touching
the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2605_01352_amd import scenegen as sg
from paper_2605_01352_amd import vuda

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "vuda.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vuda_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    L = vuda.lib()
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(vuda.EXPORTS)


def test_library_matches_its_sources(monkeypatch):
    """The in-tree library was built from the sources the tree holds, and the
    binding refuses one built from others (its manifest, written by build.py,
    against the sources' digests now)."""
    assert vuda.stale_sources() == []
    from paper_2605_01352_amd import build as vb
    real = vb.source_digests()
    edited = dict(real)
    key = sorted(k for k in real if k.endswith("raster.hip"))[0]
    edited[key] = "0" * 64
    monkeypatch.setattr(vb, "source_digests", lambda: edited)
    assert vuda.stale_sources() == [key]
    monkeypatch.setattr(vuda, "_lib", None)
    with pytest.raises(RuntimeError, match="built from other sources"):
        vuda.lib()


def test_strerror():
    L = vuda.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.vuda_strerror(code)
    assert L.vuda_strerror(-99) == b"unknown error"


def _desc(scene, keep, **kw):
    d = vuda.WorldDesc()
    d.phys = vuda.PhysParams(1 / 240, 4, 1e4, 10.0, (C.c_float * 3)(0, 0, -9.81))
    d.render = vuda.render_desc(keep)
    d.initial = vuda.env_batch(keep, scene)
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def _create(d):
    w = C.c_void_p()
    rc = vuda.lib().vuda_create_world(C.byref(d), None, C.byref(w))
    return rc, w


@pytest.mark.parametrize("mutate", ["substeps", "dt", "bodies", "type", "size", "camsize", "near"])
def test_malformed_descriptors_rejected(mutate):
    s = sg.config_scene(1, n_envs=2)
    keep = vuda._Keep()
    if mutate == "bodies":
        s = sg.make_scene(1, [129], 64, mixed=True)
    if mutate == "type":
        s.btype[3] = 7
    if mutate == "size":
        s.size[0] = -1.0
    if mutate == "camsize":
        s.cam_w[0] = 0
    d = _desc(s, keep)
    if mutate == "substeps":
        d.phys.substeps = 0
    if mutate == "dt":
        d.phys.dt = float("nan")
    if mutate == "near":
        d.render.near_w = 0.0
    rc, w = _create(d)
    assert rc == vuda.EINVAL
    assert not w.value
    assert vuda.lib().vuda_last_error_message()


def test_null_arguments():
    L = vuda.lib()
    assert L.vuda_create_world(None, None, None) == vuda.EINVAL
    assert L.vuda_step(None, 0, 1, 1) == vuda.EINVAL
    assert L.vuda_render(None, 0, 1) == vuda.EINVAL
    assert L.vuda_wait(None, 3) == vuda.EINVAL
    assert L.vuda_cosched(None, C.c_float(0.5)) == vuda.EINVAL
    assert L.vuda_destroy_world(None) == vuda.EINVAL


def test_binding_constants_match_header():
    """Every numeric #define of include/vuda.h has the same value in the
    Python binding (VUDA_X -> vuda.X)."""
    src = open(os.path.join(ROOT, "include", "vuda.h")).read()
    found = 0
    for name, val in re.findall(r"#define VUDA_([A-Z0-9_]+)\s+\(?(-?\d+)u?\)?(?=\s|$)", src):
        py = name[:-1] if name.endswith("_H") else name
        if not hasattr(vuda, py):
            continue
        assert getattr(vuda, py) == int(val), name
        found += 1
    assert found >= 30
