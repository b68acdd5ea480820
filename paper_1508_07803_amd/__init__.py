"""Python binding of librobast (MI355X non-sequential photon tracer).

Argument marshalling only: every step of the trace, the figures and the
adjoint runs in the HIP library behind the C ABI declared in
``include/robast.h``.  PyTorch supplies device memory and the stream.  There
is no CPU fallback: if the library is missing this module raises on import.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librobast.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")

_lib = ctypes.CDLL(LIB_PATH)
ABI_VERSION = 2   # the layouts below (robast_tuning with bin_dirs)
if _lib.robast_abi_version() != ABI_VERSION:
    raise ImportError(f"{LIB_PATH} has ABI version {_lib.robast_abi_version()}, this binding expects "
                      f"{ABI_VERSION}; rebuild it")

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED, EMISMATCH = 0, -1, -2, -3, -4, -5
GROUP_STRIDE = 8
FIGURE_STRIDE = 8
TRACE_KEEP_ORDER = 1
BACKWARD_CHECK_SEQ = 1

SYMBOLS = ["robast_build_scene", "robast_trace", "robast_figures", "robast_trace_backward",
           "robast_update_params", "robast_destroy_scene", "robast_status_string",
           "robast_last_error", "robast_abi_version", "robast_build_batch", "robast_trace_batch",
           "robast_figures_batch", "robast_trace_backward_batch", "robast_batch_sizes", "robast_destroy_batch",
           "robast_get_tuning", "robast_set_tuning", "robast_autotune", "robast_bin_photons",
           "robast_arrival_figures", "robast_trace_static", "robast_set_params", "robast_update_params_batch",
           "robast_gd_step", "robast_gd_step_batch", "robast_autotune_batch", "robast_boundary_grad"]


class VolumeDesc(ctypes.Structure):
    _fields_ = [("role", ctypes.c_int32), ("shape", ctypes.c_int32), ("outline", ctypes.c_int32),
                ("shape_param", ctypes.c_int32), ("tilt_param", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("Q", ctypes.c_double * 9), ("c", ctypes.c_double * 3), ("p", ctypes.c_double * 16),
                ("o", ctypes.c_double * 4), ("reflectivity", ctypes.c_double), ("n_inside", ctypes.c_double),
                ("Q0", ctypes.c_double * 9), ("c0", ctypes.c_double * 3), ("pivot", ctypes.c_double * 3),
                ("e1", ctypes.c_double * 3), ("e2", ctypes.c_double * 3)]


class SceneDesc(ctypes.Structure):
    _fields_ = [("volumes", ctypes.c_void_p), ("n_volumes", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_events", ctypes.c_int32), ("n_groups", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("l_ref", ctypes.c_double)]


class Rays(ctypes.Structure):
    _fields_ = [("ox", ctypes.c_void_p), ("oy", ctypes.c_void_p), ("oz", ctypes.c_void_p),
                ("dx", ctypes.c_void_p), ("dy", ctypes.c_void_p), ("dz", ctypes.c_void_p),
                ("group", ctypes.c_void_p), ("id_base", ctypes.c_uint64), ("lam", ctypes.c_void_p)]


class Hits(ctypes.Structure):
    _fields_ = [("fate", ctypes.c_void_p), ("n_events", ctypes.c_void_p), ("last_vol", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("ux", ctypes.c_void_p), ("uy", ctypes.c_void_p), ("uz", ctypes.c_void_p),
                ("opl", ctypes.c_void_p), ("seq_hash", ctypes.c_void_p), ("group_sums", ctypes.c_void_p),
                ("seq_log", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("bin_photons", ctypes.c_uint32), ("bin_target", ctypes.c_uint32),
                ("waves_mult", ctypes.c_uint32), ("block", ctypes.c_uint32), ("bin_dirs", ctypes.c_uint32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


assert ctypes.sizeof(VolumeDesc) == 464

_lib.robast_build_scene.argtypes = [ctypes.POINTER(SceneDesc), ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_void_p)]
_lib.robast_trace.argtypes = [ctypes.c_void_p, ctypes.POINTER(Rays), ctypes.c_int64, ctypes.POINTER(Hits),
                              ctypes.c_uint32, ctypes.c_void_p]
_lib.robast_trace_static.argtypes = [ctypes.c_void_p, ctypes.POINTER(Rays), ctypes.c_int64, ctypes.POINTER(Hits),
                                     ctypes.c_void_p]
_lib.robast_figures.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
_lib.robast_trace_backward.argtypes = [ctypes.c_void_p, ctypes.POINTER(Rays), ctypes.c_int64, ctypes.POINTER(Hits),
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                       ctypes.c_void_p]
_lib.robast_update_params.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
_lib.robast_set_params.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
_lib.robast_update_params_batch.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
_lib.robast_gd_step.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 5
_lib.robast_boundary_grad.argtypes = [ctypes.c_void_p, ctypes.POINTER(Rays), ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
_lib.robast_gd_step_batch.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 5
_lib.robast_autotune_batch.argtypes = [ctypes.c_void_p, ctypes.POINTER(Rays), ctypes.POINTER(ctypes.c_uint32),
                                       ctypes.POINTER(ctypes.c_uint32), ctypes.c_void_p]
_lib.robast_destroy_scene.argtypes = [ctypes.c_void_p]
_lib.robast_destroy_scene.restype = None
_lib.robast_status_string.argtypes = [ctypes.c_int]
_lib.robast_status_string.restype = ctypes.c_char_p
_lib.robast_last_error.restype = ctypes.c_char_p
_lib.robast_build_batch.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_uint32,
                                    ctypes.POINTER(ctypes.c_void_p)]
_lib.robast_trace_batch.argtypes = [ctypes.c_void_p, ctypes.POINTER(Rays), ctypes.POINTER(Hits), ctypes.c_uint32,
                                    ctypes.c_void_p]
_lib.robast_figures_batch.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
_lib.robast_trace_backward_batch.argtypes = [ctypes.c_void_p, ctypes.POINTER(Rays), ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
_lib.robast_batch_sizes.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int64)] * 3
_lib.robast_get_tuning.argtypes = [ctypes.c_void_p, ctypes.POINTER(Tuning)]
_lib.robast_set_tuning.argtypes = [ctypes.c_void_p, ctypes.POINTER(Tuning)]
_lib.robast_autotune.argtypes = [ctypes.c_void_p, ctypes.POINTER(Rays), ctypes.c_int64, ctypes.POINTER(Tuning),
                                 ctypes.c_void_p]
_lib.robast_bin_photons.argtypes = [ctypes.c_void_p, ctypes.POINTER(Rays), ctypes.c_int64, ctypes.c_void_p]
_lib.robast_arrival_figures.argtypes = [ctypes.c_void_p, ctypes.POINTER(Rays), ctypes.POINTER(Hits), ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_void_p]
_lib.robast_destroy_batch.argtypes = [ctypes.c_void_p]
_lib.robast_destroy_batch.restype = None
for _name in ("robast_build_scene", "robast_trace", "robast_figures", "robast_trace_backward",
              "robast_update_params", "robast_abi_version", "robast_build_batch", "robast_trace_batch",
              "robast_figures_batch", "robast_trace_backward_batch", "robast_batch_sizes", "robast_get_tuning",
              "robast_set_tuning", "robast_autotune", "robast_bin_photons", "robast_arrival_figures",
              "robast_trace_static", "robast_set_params", "robast_update_params_batch", "robast_gd_step",
              "robast_gd_step_batch", "robast_autotune_batch", "robast_boundary_grad"):
    getattr(_lib, _name).restype = ctypes.c_int


class RobastError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        msg = _lib.robast_last_error().decode()
        super().__init__(f"{what}: {_lib.robast_status_string(status).decode()} ({status}): {msg}")


def _check(status, what):
    if status != OK:
        raise RobastError(status, what)


def lib():
    return _lib


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr()) if hasattr(t, "data_ptr") else t


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def build_scene_raw(volumes, precision, max_events, n_groups, seed, l_ref, params):
    """Call robast_build_scene on a VOLUME_DTYPE array; returns (status, handle)."""
    vols = np.ascontiguousarray(volumes)
    assert vols.dtype.itemsize == 464 or len(vols) == 0
    P = np.ascontiguousarray(params, dtype=np.float64)
    desc = SceneDesc(vols.ctypes.data if len(vols) else None, len(vols), precision, max_events, n_groups,
                     seed, l_ref)
    h = ctypes.c_void_p()
    st = _lib.robast_build_scene(ctypes.byref(desc), P.ctypes.data if len(P) else None, len(P),
                                 ctypes.byref(h))
    return st, h


_HIT_KEYS = ("fate", "n_events", "last_vol", "x", "y", "z", "ux", "uy", "uz", "opl", "seq_hash")


def _rays_struct(rays, id_base=0, offset=0):
    def p(k):
        t = rays[k]
        return t.data_ptr() + offset * t.element_size()
    g = rays.get("group")
    lam = rays.get("lam")
    return Rays(p("ox"), p("oy"), p("oz"), p("dx"), p("dy"), p("dz"),
                (g.data_ptr() + offset * g.element_size()) if g is not None else None, id_base + offset,
                p("lam") if lam is not None else None)


_HIT_ITEM = {"fate": 1, "n_events": 1, "last_vol": 4, "seq_hash": 8}


def _check_extents(n, dtype, rays=None, hits=None, f64=()):
    """The C ABI takes plain pointers: extents and element types of the
    tensors a call reads or writes are checked here, before any launch."""
    import torch
    if rays is not None:
        for k in ("ox", "oy", "oz", "dx", "dy", "dz", "lam"):
            t = rays.get(k)
            if t is None and k == "lam":
                continue
            if t.dtype != dtype:
                raise ValueError(f"rays[{k!r}] is {t.dtype}, the scene computes in {dtype}")
            if t.numel() < n:
                raise ValueError(f"rays[{k!r}] holds {t.numel()} < {n} photons")
        g = rays.get("group")
        if g is not None and (g.element_size() != 4 or g.dtype.is_floating_point or g.numel() < n):
            raise ValueError(f"rays['group'] must hold >= {n} 32-bit integers")
    for k, t in (hits or {}).items():
        if t is None or k not in _HIT_KEYS:
            continue
        if k in _HIT_ITEM:
            if t.element_size() != _HIT_ITEM[k] or t.dtype.is_floating_point:
                raise ValueError(f"hits[{k!r}] must be {8 * _HIT_ITEM[k]}-bit integers")
        elif t.dtype != dtype:
            raise ValueError(f"hits[{k!r}] is {t.dtype}, the scene computes in {dtype}")
        if t.numel() < n:
            raise ValueError(f"hits[{k!r}] holds {t.numel()} < {n} photons")
    for name, t, need in f64:     # FP64 buffers: (name, tensor, values needed)
        if t is None:
            continue
        if t.dtype != torch.float64:
            raise ValueError(f"{name} must be float64")
        if t.numel() < need:
            raise ValueError(f"{name} holds {t.numel()} < {need} values")


def _hits_struct(hits, sums):
    hits = hits or {}
    log = hits.get("seq_log")
    return Hits(*[(hits[k].data_ptr() if hits.get(k) is not None else None) for k in _HIT_KEYS],
                sums.data_ptr() if sums is not None else None, log.data_ptr() if log is not None else None)


class Scene:
    """A compiled scene on the current HIP device."""

    def __init__(self, scene):
        self.src = scene
        self.precision = scene.precision
        self.n_groups = scene.n_groups
        self.n_params = len(scene.params)
        self.params = np.array(scene.params, dtype=np.float64)
        st, h = build_scene_raw(scene.volumes, scene.precision, scene.max_events, scene.n_groups,
                                scene.seed, scene.l_ref, scene.params)
        _check(st, "robast_build_scene")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.robast_destroy_scene(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- tensors
    @property
    def dtype(self):
        import torch
        return torch.float32 if self.precision == 32 else torch.float64

    def upload_rays(self, rays, device="cuda", wavelengths=False):
        """Host ray dict (numpy, from `scenes`) -> dict of device tensors;
        with wavelengths, each photon's rays["lam"] goes along as "lam"."""
        import torch
        keys = ("ox", "oy", "oz", "dx", "dy", "dz") + (("lam",) if wavelengths else ())
        out = {k: torch.from_numpy(np.ascontiguousarray(rays[k])).to(device=device, dtype=self.dtype)
               for k in keys}
        out["group"] = torch.from_numpy(np.ascontiguousarray(rays["group"]).astype(np.int32)).to(device)
        return out

    def alloc_hits(self, n, device="cuda", sums=False):
        import torch
        h = dict(fate=torch.zeros(n, dtype=torch.uint8, device=device),
                 n_events=torch.zeros(n, dtype=torch.uint8, device=device),
                 last_vol=torch.zeros(n, dtype=torch.int32, device=device),
                 opl=torch.zeros(n, dtype=self.dtype, device=device),
                 seq_hash=torch.zeros(n, dtype=torch.int64, device=device))
        for k in ("x", "y", "z", "ux", "uy", "uz"):
            h[k] = torch.zeros(n, dtype=self.dtype, device=device)
        if sums:
            h["group_sums"] = self.new_sums(device)
        return h

    def new_sums(self, device="cuda"):
        import torch
        return torch.zeros(self.n_groups * GROUP_STRIDE, dtype=torch.float64, device=device)

    @staticmethod
    def _rays_struct(rays, id_base=0, offset=0):
        return _rays_struct(rays, id_base, offset)

    # -------------------------------------------------------------- calls
    def trace(self, rays, n=None, hits=None, sums=None, id_base=0, stream=None, keep_order=False):
        """Trace n photons; writes the given hit tensors and/or accumulates sums.

        keep_order: keep the binned photon order, and each photon's path
        record, for the next backward call on the same photon tensors (which
        must not be modified in between): that call then replays the
        recorded surface sequences instead of searching for them again.
        """
        n = int(rays["ox"].numel()) if n is None else int(n)
        hits = hits or {}
        _check_extents(n, self.dtype, rays, hits, [("sums", sums, self.n_groups * GROUP_STRIDE)])
        H = _hits_struct(hits, sums)
        R = self._rays_struct(rays, id_base)
        flags = TRACE_KEEP_ORDER if keep_order else 0
        _check(_lib.robast_trace(self._h, ctypes.byref(R), n, ctypes.byref(H), flags, _stream(stream)),
               "robast_trace")
        return hits

    def trace_static(self, rays, n=None, hits=None, sums=None, id_base=0, stream=None):
        """robast_trace_static: the trace of `trace`, binning in the library's
        fixed per-GPU workspace (no device allocation)."""
        n = int(rays["ox"].numel()) if n is None else int(n)
        hits = hits or {}
        _check_extents(n, self.dtype, rays, hits, [("sums", sums, self.n_groups * GROUP_STRIDE)])
        H = _hits_struct(hits, sums)
        R = self._rays_struct(rays, id_base)
        _check(_lib.robast_trace_static(self._h, ctypes.byref(R), n, ctypes.byref(H), _stream(stream)),
               "robast_trace_static")
        return hits

    def bin_photons(self, rays, n=None, id_base=0, stream=None):
        """Bin the photons now and keep the order for the next trace / backward calls."""
        n = int(rays["ox"].numel()) if n is None else int(n)
        _check_extents(n, self.dtype, rays)
        R = self._rays_struct(rays, id_base)
        _check(_lib.robast_bin_photons(self._h, ctypes.byref(R), n, _stream(stream)), "robast_bin_photons")

    def figures(self, sums, fig=None, stream=None):
        import torch
        if fig is None:
            fig = torch.zeros(self.n_groups * FIGURE_STRIDE, dtype=torch.float64, device=sums.device)
        _check_extents(0, None, f64=[("sums", sums, self.n_groups * GROUP_STRIDE),
                                     ("fig", fig, self.n_groups * FIGURE_STRIDE)])
        _check(_lib.robast_figures(self._h, _ptr(sums), _ptr(fig), _stream(stream)), "robast_figures")
        return fig.view(self.n_groups, FIGURE_STRIDE)

    def arrival_figures(self, rays, hits, n=None, out=None, stream=None):
        """Per group (count, mean optical path, RMS optical path spread, 0) of
        the FOCUSED photons in the per-photon records `hits` (fate, opl) of a
        trace of these photons; returns an (n_groups, 4) FP64 tensor."""
        import torch
        n = int(rays["ox"].numel()) if n is None else int(n)
        if out is None:
            out = torch.zeros(self.n_groups * 4, dtype=torch.float64, device=hits["fate"].device)
        _check_extents(n, self.dtype, rays, {k: hits[k] for k in ("fate", "opl")}, [("out", out, self.n_groups * 4)])
        H = _hits_struct(hits, None)
        R = self._rays_struct(rays, 0)
        _check(_lib.robast_arrival_figures(self._h, ctypes.byref(R), ctypes.byref(H), n, _ptr(out), _stream(stream)),
               "robast_arrival_figures")
        return out.view(self.n_groups, 4)

    def backward(self, rays, sums, cot, grad, n=None, id_base=0, stream=None, photon_cot=None, fwd_hash=None,
                 check=False):
        """Accumulate dL/dparams into grad for L = sum_g cot[g,0] RMS_g + cot[g,1] effw_g
        (sums: the forward group sums; cot may be None) plus, per FOCUSED
        photon, photon_cot[p] . (x, y, z, ux, uy, uz) of its exit state
        (an (n, 6) float64 tensor, or None).  check: compare every photon's
        re-derived surface sequence with fwd_hash (the forward seq_hash);
        raises RobastError(EMISMATCH) if any differs."""
        n = int(rays["ox"].numel()) if n is None else int(n)
        f64 = [("grad", grad, self.n_params), ("photon_cot", photon_cot, 6 * n)]
        if cot is not None:
            f64 += [("sums", sums, self.n_groups * GROUP_STRIDE), ("cot", cot, self.n_groups * 2)]
        _check_extents(n, self.dtype, rays, {"seq_hash": fwd_hash} if fwd_hash is not None else None, f64)
        R = self._rays_struct(rays, id_base)
        H = _hits_struct({"seq_hash": fwd_hash} if fwd_hash is not None else None, sums)
        flags = BACKWARD_CHECK_SEQ if check else 0
        _check(_lib.robast_trace_backward(self._h, ctypes.byref(R), n, ctypes.byref(H), _ptr(cot), _ptr(photon_cot),
                                          _ptr(grad), flags, _stream(stream)), "robast_trace_backward")
        return grad

    def boundary_grad(self, rays, sums, cot, grad, band=0.02, n=None, id_base=0, stream=None):
        """Accumulate into grad the boundary (fate-flip) terms of
        d/dparams sum_g cot[g] eta_g, eta_g the collection efficiency of
        group g (robast_boundary_grad; sums: the forward group sums of the
        same photons; cot: n_groups float64)."""
        n = int(rays["ox"].numel()) if n is None else int(n)
        _check_extents(n, self.dtype, rays, None, [("grad", grad, self.n_params),
                                                   ("sums", sums, self.n_groups * GROUP_STRIDE),
                                                   ("cot", cot, self.n_groups)])
        R = self._rays_struct(rays, id_base)
        _check(_lib.robast_boundary_grad(self._h, ctypes.byref(R), n, _ptr(sums), _ptr(cot), float(band), _ptr(grad),
                                         _stream(stream)), "robast_boundary_grad")
        return grad

    @property
    def tuning(self):
        t = Tuning()
        _check(_lib.robast_get_tuning(self._h, ctypes.byref(t)), "robast_get_tuning")
        return t.as_dict()

    def set_tuning(self, **fields):
        """Change launch parameters (bin_photons, bin_target, waves_mult, block)."""
        cur = self.tuning
        unknown = set(fields) - set(cur)
        if unknown:
            raise KeyError(f"unknown tuning fields {sorted(unknown)}")
        cur.update(fields)
        t = Tuning(**cur)
        _check(_lib.robast_set_tuning(self._h, ctypes.byref(t)), "robast_set_tuning")
        return self.tuning

    def autotune(self, rays, n=None, stream=None):
        """Time candidate launch parameters on these photons; keeps and returns the fastest."""
        n = int(rays["ox"].numel()) if n is None else int(n)
        _check_extents(n, self.dtype, rays)
        R = self._rays_struct(rays, 0)
        t = Tuning()
        _check(_lib.robast_autotune(self._h, ctypes.byref(R), n, ctypes.byref(t), _stream(stream)),
               "robast_autotune")
        return t.as_dict()

    def update_params(self, params):
        """New parameters from the host: robast_set_params (checked first,
        tables rebuilt on the host, synchronous)."""
        P = np.ascontiguousarray(params, dtype=np.float64)
        _check(_lib.robast_set_params(self._h, P.ctypes.data if len(P) else None, len(P)),
               "robast_set_params")
        self.params = P.copy()

    def update_params_device(self, params, status=None, stream=None):
        """New parameters already on the device (float64 tensor of n_params):
        robast_update_params, in stream order (graph-capturable).  status: an
        int32 device tensor that receives 0 or the rejection code.  The
        host copy self.params no longer describes the scene afterwards."""
        import torch
        _check_extents(0, None, f64=[("params", params, self.n_params)])
        if status is not None and (status.dtype != torch.int32 or status.numel() < 1):
            raise ValueError("status must hold an int32")
        _check(_lib.robast_update_params(self._h, _ptr(params), _ptr(status), _stream(stream)),
               "robast_update_params")
        self.params = None

    def gd_step(self, params, grad, lr, status=None, stream=None):
        """robast_gd_step: params <- params - lr * grad on the device, applied
        to the scene in stream order (graph-capturable); params (float64
        device tensor) is overwritten where the update is applied."""
        import torch
        _check_extents(0, None, f64=[("params", params, self.n_params), ("grad", grad, self.n_params),
                                     ("lr", lr, self.n_params)])
        if status is not None and (status.dtype != torch.int32 or status.numel() < 1):
            raise ValueError("status must hold an int32")
        _check(_lib.robast_gd_step(self._h, _ptr(params), _ptr(grad), _ptr(lr), _ptr(status), _stream(stream)),
               "robast_gd_step")
        self.params = None


class Batch:
    """Scene variants traced together: one persistent launch per call.

    ``counts[v]`` photons of variant ``v`` occupy rays
    ``[offsets[v], offsets[v+1])`` of one concatenated bundle and are
    numbered from ``offsets[v]``; sums, cotangents, figures and gradients are
    concatenated per variant (``goff`` / ``poff`` give each variant's first
    group / parameter).  The member scenes are kept alive by the batch.
    """

    def __init__(self, scenes, counts, chunk=8192):
        self.scenes = list(scenes)
        precisions = {s.precision for s in self.scenes}
        self.precision = self.scenes[0].precision if len(precisions) == 1 else None
        counts = np.asarray(counts, dtype=np.int64)
        self.offsets = np.zeros(len(self.scenes) + 1, dtype=np.int64)
        self.offsets[1:] = np.cumsum(counts) if len(counts) else []
        self.goff = np.concatenate([[0], np.cumsum([s.n_groups for s in self.scenes])]).astype(np.int64)
        self.poff = np.concatenate([[0], np.cumsum([s.n_params for s in self.scenes])]).astype(np.int64)
        handles = (ctypes.c_void_p * max(1, len(self.scenes)))(*[s.handle.value for s in self.scenes])
        offs = np.ascontiguousarray(self.offsets)
        h = ctypes.c_void_p()
        _check(_lib.robast_build_batch(handles, len(self.scenes), offs.ctypes.data, int(chunk), ctypes.byref(h)),
               "robast_build_batch")
        self._h = h
        n = [ctypes.c_int64() for _ in range(3)]
        _check(_lib.robast_batch_sizes(h, *[ctypes.byref(x) for x in n]), "robast_batch_sizes")
        self.n_photons, self.n_groups, self.n_params = (int(x.value) for x in n)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.robast_destroy_batch(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_sums(self, device="cuda"):
        import torch
        return torch.zeros(self.n_groups * GROUP_STRIDE, dtype=torch.float64, device=device)

    def _check_sizes(self, rays, hits=None, sums=None, grad=None, cot=None):
        import torch
        _check_extents(self.n_photons, torch.float32, rays, hits,
                       [("sums", sums, self.n_groups * GROUP_STRIDE), ("cot", cot, self.n_groups * 2),
                        ("grad", grad, self.n_params)])

    def trace(self, rays, hits=None, sums=None, id_base=0, stream=None, keep_order=False):
        self._check_sizes(rays, hits, sums)
        H = _hits_struct(hits, sums)
        R = _rays_struct(rays, id_base)
        flags = TRACE_KEEP_ORDER if keep_order else 0
        _check(_lib.robast_trace_batch(self._h, ctypes.byref(R), ctypes.byref(H), flags, _stream(stream)),
               "robast_trace_batch")
        return hits

    def figures(self, sums, fig=None, stream=None):
        import torch
        if fig is None:
            fig = torch.zeros(self.n_groups * FIGURE_STRIDE, dtype=torch.float64, device=sums.device)
        _check_extents(0, None, f64=[("sums", sums, self.n_groups * GROUP_STRIDE),
                                     ("fig", fig, self.n_groups * FIGURE_STRIDE)])
        _check(_lib.robast_figures_batch(self._h, _ptr(sums), _ptr(fig), _stream(stream)), "robast_figures_batch")
        return fig.view(self.n_groups, FIGURE_STRIDE)

    def update_params(self, params, status=None, stream=None):
        """robast_update_params_batch: every variant's parameters from the
        concatenated float64 device tensor (status: int32 per variant)."""
        import torch
        _check_extents(0, None, f64=[("params", params, self.n_params)])
        if status is not None and (status.dtype != torch.int32 or status.numel() < len(self.scenes)):
            raise ValueError("status must hold one int32 per variant")
        _check(_lib.robast_update_params_batch(self._h, _ptr(params), _ptr(status), _stream(stream)),
               "robast_update_params_batch")
        for s in self.scenes:
            s.params = None

    def gd_step(self, params, grad, lr, status=None, stream=None):
        """robast_gd_step_batch: one gradient-descent step of every variant
        (concatenated float64 device tensors; status: int32 per variant)."""
        import torch
        _check_extents(0, None, f64=[("params", params, self.n_params), ("grad", grad, self.n_params),
                                     ("lr", lr, self.n_params)])
        if status is not None and (status.dtype != torch.int32 or status.numel() < len(self.scenes)):
            raise ValueError("status must hold one int32 per variant")
        _check(_lib.robast_gd_step_batch(self._h, _ptr(params), _ptr(grad), _ptr(lr), _ptr(status),
                                         _stream(stream)), "robast_gd_step_batch")
        for s in self.scenes:
            s.params = None

    def autotune(self, rays, id_base=0, stream=None):
        """robast_autotune_batch: the fastest work-item size and workgroup
        size of the forward launch, kept in the batch; returns both."""
        self._check_sizes(rays)
        R = _rays_struct(rays, id_base)
        c, b = ctypes.c_uint32(), ctypes.c_uint32()
        _check(_lib.robast_autotune_batch(self._h, ctypes.byref(R), ctypes.byref(c), ctypes.byref(b),
                                          _stream(stream)), "robast_autotune_batch")
        return {"chunk": int(c.value), "block": int(b.value)}

    def backward(self, rays, sums, cot, grad, id_base=0, stream=None):
        self._check_sizes(rays, None, sums, grad, cot)
        R = _rays_struct(rays, id_base)
        _check(_lib.robast_trace_backward_batch(self._h, ctypes.byref(R), _ptr(sums), _ptr(cot), _ptr(grad),
                                                _stream(stream)), "robast_trace_backward_batch")
        return grad


def _autograd():
    import torch

    class RobastTrace(torch.autograd.Function):
        """figures (n_groups x 8) = trace(params); backward via robast_trace_backward.

        Gradients flow from the RMS spot radius (column 4) and the weighted
        collection (column 6); the other figure columns are counts and means
        whose pathwise derivative is not propagated.
        """

        @staticmethod
        def forward(ctx, params, scene, rays):
            p = params.detach().to("cpu", torch.float64).numpy()
            if not np.array_equal(p, scene.params):
                scene.update_params(p)
            sums = scene.new_sums(rays["ox"].device)
            scene.trace(rays, sums=sums, keep_order=True)
            fig = scene.figures(sums)
            ctx.scene, ctx.rays = scene, rays
            ctx.params = p.copy()
            ctx.pdev, ctx.pdtype = params.device, params.dtype
            ctx.save_for_backward(sums)
            return fig

        @staticmethod
        def backward(ctx, gfig):
            (sums,) = ctx.saved_tensors
            scene = ctx.scene
            # the scene may have moved on (another forward call since): the
            # gradient is taken at this forward call's parameters
            if not np.array_equal(ctx.params, scene.params):
                scene.update_params(ctx.params)
            cot = torch.stack([gfig[:, 4], gfig[:, 6]], 1).contiguous().to(torch.float64)
            grad = torch.zeros(scene.n_params, dtype=torch.float64, device=sums.device)
            scene.backward(ctx.rays, sums, cot, grad)
            return grad.to(device=ctx.pdev, dtype=ctx.pdtype), None, None

    return RobastTrace


def __getattr__(name):
    if name == "RobastTrace":
        return _autograd()
    raise AttributeError(name)
