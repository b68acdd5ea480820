"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol the header declares, and rejects invalid input before any launch."""
import os
import re

import numpy as np
import pytest

import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def rb():
    import paper_1508_07803_amd as rb
    return rb


def test_header_symbols_exported(rb):
    hdr = open(os.path.join(ROOT, "include", "robast.h")).read()
    declared = set(re.findall(r"^(?:int|void|const char\*)\s+(robast_[a-z_]+)\s*\(", hdr, re.M))
    assert declared == set(rb.SYMBOLS)
    for name in declared:
        assert hasattr(rb.lib(), name), name
    assert rb.lib().robast_abi_version() == 1


def test_volume_desc_layout_matches_inputs(rb):
    import ctypes
    assert ctypes.sizeof(rb.VolumeDesc) == scenes.VOLUME_DTYPE.itemsize == 464
    for name, _ in rb.VolumeDesc._fields_:
        assert getattr(rb.VolumeDesc, name).offset == scenes.VOLUME_DTYPE.fields[name][1]


def _try(rb, sc, **over):
    kw = dict(volumes=sc.volumes, precision=sc.precision, max_events=sc.max_events,
              n_groups=sc.n_groups, seed=sc.seed, l_ref=sc.l_ref, params=sc.params)
    kw.update(over)
    st, h = rb.build_scene_raw(**kw)
    return st


@pytest.mark.parametrize("field,value", [
    ("role", 9), ("shape", 0), ("outline", 7), ("shape_param", 5), ("tilt_param", 0),
    ("reflectivity", 1.5), ("reflectivity", np.nan)])
def test_invalid_volume_rejected(rb, field, value):
    sc = scenes.single_mirror()
    v = sc.volumes.copy()
    v[0][field] = value
    assert _try(rb, sc, volumes=v) == rb.EINVAL


@pytest.mark.parametrize("over", [dict(precision=16), dict(max_events=0), dict(max_events=300),
                                  dict(n_groups=0), dict(l_ref=0.0), dict(l_ref=np.inf)])
def test_invalid_scene_rejected(rb, over):
    assert _try(rb, scenes.single_mirror(), **over) == rb.EINVAL


def test_invalid_geometry_rejected(rb):
    sc = scenes.single_mirror()
    v = sc.volumes.copy()
    v[0]["p"][0] = 1.0 / 1.5          # aperture r = 2 m beyond the equator of R = 1.5 m
    assert _try(rb, sc, volumes=v) == rb.EINVAL
    v = sc.volumes.copy()
    v[0]["Q"][:] = 0.0                # singular frame
    assert _try(rb, sc, volumes=v) == rb.EINVAL
    v = sc.volumes.copy()
    v[1]["o"][0] = -1.0               # degenerate outline
    assert _try(rb, sc, volumes=v) == rb.EINVAL
    assert _try(rb, sc, params=np.array([np.nan])) == rb.EINVAL


def test_null_arguments_rejected(rb):
    import ctypes
    lib = rb.lib()
    h = ctypes.c_void_p()
    assert lib.robast_build_scene(None, None, 0, ctypes.byref(h)) == rb.EINVAL
    assert lib.robast_trace(None, None, 10, None, 0, None) == rb.EINVAL
    assert lib.robast_trace_backward(None, None, 10, None, None, None, None) == rb.EINVAL
    assert lib.robast_figures(None, None, None, None) == rb.EINVAL
    assert b"NULL" in lib.robast_last_error()
    assert lib.robast_status_string(rb.EINVAL) == b"invalid argument"


def test_batch_arguments_rejected(rb):
    """Batch entry points validate before touching a device."""
    import ctypes
    lib = rb.lib()
    h = ctypes.c_void_p()
    offs = (ctypes.c_int64 * 3)(0, 10, 5)
    scenes_null = (ctypes.c_void_p * 2)(None, None)
    assert lib.robast_build_batch(None, 1, offs, 64, None) == rb.EINVAL
    assert lib.robast_build_batch(None, 1, offs, 64, ctypes.byref(h)) == rb.EINVAL
    assert lib.robast_build_batch(scenes_null, 0, offs, 64, ctypes.byref(h)) == rb.EINVAL
    assert lib.robast_build_batch(scenes_null, 2, offs, 0, ctypes.byref(h)) == rb.EINVAL
    assert lib.robast_build_batch(scenes_null, 2, offs, 64, ctypes.byref(h)) == rb.EINVAL
    assert h.value is None
    assert lib.robast_trace_batch(None, None, None, 0, None) == rb.EINVAL
    assert lib.robast_figures_batch(None, None, None, None) == rb.EINVAL
    assert lib.robast_trace_backward_batch(None, None, None, None, None, None) == rb.EINVAL
    assert lib.robast_batch_sizes(None, None, None, None) == rb.EINVAL
    lib.robast_destroy_batch(None)


def test_tuning_arguments_rejected(rb):
    import ctypes
    lib = rb.lib()
    t = rb.Tuning(1, 128, 1, 0)
    assert lib.robast_get_tuning(None, ctypes.byref(t)) == rb.EINVAL
    assert lib.robast_set_tuning(None, ctypes.byref(t)) == rb.EINVAL
    assert lib.robast_autotune(None, None, 10, None, None) == rb.EINVAL
