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
    assert rb.lib().robast_abi_version() == rb.ABI_VERSION == 2


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


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("name", sorted(scenes.ALL))
def test_every_scene_passes_validation(rb, name, precision):
    """Each stand-in scene, rounded to either precision, gets past the
    library's checks of volumes and parameters (without a device the build
    then stops at its first HIP call)."""
    f = scenes.ALL[name]
    sc = f() if name == "single_mirror" else f(precision=precision)
    assert _try(rb, sc) in (rb.OK, rb.EHIP)


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


def test_lens_face_rules(rb):
    """Lens faces: planes, spheres, aspheres and boxes pass the checks; a
    cylinder lens has no kernel; the absorption length p[15] must be finite
    and >= 0."""
    sc = scenes.aspheric_lens(precision=64)
    assert _try(rb, sc) in (rb.OK, rb.EHIP)                  # asphere + plane lens faces
    v = sc.volumes.copy()
    v[2]["role"] = scenes.ROLE_LENS                          # the absorbing rim cylinder as a lens
    v[2]["n_inside"] = 1.49
    assert _try(rb, sc, volumes=v) == rb.EUNSUPPORTED
    for bad in (-1.0, np.nan, np.inf):
        v = sc.volumes.copy()
        v[0]["p"][15] = bad
        assert _try(rb, sc, volumes=v) == rb.EINVAL, bad
    v = sc.volumes.copy()
    v[0]["p"][15] = 0.3
    assert _try(rb, sc, volumes=v) in (rb.OK, rb.EHIP)


def test_null_arguments_rejected(rb):
    import ctypes
    lib = rb.lib()
    h = ctypes.c_void_p()
    assert lib.robast_build_scene(None, None, 0, ctypes.byref(h)) == rb.EINVAL
    assert lib.robast_trace(None, None, 10, None, 0, None) == rb.EINVAL
    assert lib.robast_trace_backward(None, None, 10, None, None, None, None, 0, None) == rb.EINVAL
    assert lib.robast_figures(None, None, None, None) == rb.EINVAL
    assert lib.robast_update_params(None, None, None, None) == rb.EINVAL
    assert lib.robast_set_params(None, None, 0) == rb.EINVAL
    assert lib.robast_update_params_batch(None, None, None, None) == rb.EINVAL
    assert b"NULL" in lib.robast_last_error()
    assert lib.robast_status_string(rb.EINVAL) == b"invalid argument"


def test_backward_arguments_rejected(rb):
    """robast_trace_backward rejects an unknown flag, a group cotangent
    without the forward sums and the sequence check without the forward
    hashes, before it reads the scene (a stand-in handle is never touched)."""
    import ctypes
    lib = rb.lib()
    fake = ctypes.create_string_buffer(64)
    scene = ctypes.cast(fake, ctypes.c_void_p)
    rays = rb.Rays()
    grad = ctypes.cast(ctypes.create_string_buffer(64), ctypes.c_void_p)
    cot = ctypes.cast(ctypes.create_string_buffer(64), ctypes.c_void_p)
    no_sums = rb.Hits()
    assert lib.robast_trace_backward(scene, ctypes.byref(rays), 10, None, None, None, grad, 2, None) == rb.EINVAL
    assert b"flag" in lib.robast_last_error()
    assert lib.robast_trace_backward(scene, ctypes.byref(rays), 10, None, cot, None, grad, 0, None) == rb.EINVAL
    assert lib.robast_trace_backward(scene, ctypes.byref(rays), 10, ctypes.byref(no_sums), cot, None, grad, 0,
                                     None) == rb.EINVAL
    assert b"group_sums" in lib.robast_last_error()
    assert lib.robast_trace_backward(scene, ctypes.byref(rays), 10, ctypes.byref(no_sums), None, None, grad,
                                     rb.BACKWARD_CHECK_SEQ, None) == rb.EINVAL
    assert b"seq_hash" in lib.robast_last_error()


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
    assert lib.robast_autotune_batch(None, None, None, None, None) == rb.EINVAL
    assert lib.robast_gd_step(None, None, None, None, None, None) == rb.EINVAL
    assert lib.robast_gd_step_batch(None, None, None, None, None, None) == rb.EINVAL
    assert lib.robast_boundary_grad(None, None, 10, None, None, 0.01, None, None) == rb.EINVAL


def test_binding_checks_extents_before_launch(rb):
    """The C ABI takes plain pointers, so the binding checks every tensor a
    call reads or writes against the photon count and the scene sizes
    (CPU tensors: the checks run before anything reaches the library)."""
    import torch
    f32 = torch.float32
    n = 100
    rays = {k: torch.zeros(n, dtype=f32) for k in ("ox", "oy", "oz", "dx", "dy", "dz")}
    rays["group"] = torch.zeros(n, dtype=torch.int32)
    hits = {"fate": torch.zeros(n, dtype=torch.uint8), "x": torch.zeros(n, dtype=f32),
            "seq_hash": torch.zeros(n, dtype=torch.int64)}
    sums = torch.zeros(16, dtype=torch.float64)
    rb._check_extents(n, f32, rays, hits, [("sums", sums, 16)])          # consistent: no error
    bad_cases = [
        dict(n=n + 1),                                                   # more photons than the arrays hold
        dict(rays={**rays, "dz": torch.zeros(n - 1, dtype=f32)}),
        dict(rays={**rays, "ox": torch.zeros(n, dtype=torch.float64)}),   # wrong precision
        dict(rays={**rays, "group": torch.zeros(n, dtype=torch.int64)}),
        dict(hits={**hits, "x": torch.zeros(n - 1, dtype=f32)}),
        dict(hits={**hits, "fate": torch.zeros(n, dtype=torch.int32)}),
        dict(hits={**hits, "seq_hash": torch.zeros(n, dtype=torch.float64)}),
        dict(f64=[("sums", sums, 17)]),
        dict(f64=[("sums", sums.float(), 16)]),
    ]
    for case in bad_cases:
        args = dict(n=n, rays=rays, hits=hits, f64=[("sums", sums, 16)])
        args.update(case)
        with pytest.raises(ValueError):
            rb._check_extents(args["n"], f32, args["rays"], args["hits"], args["f64"])
