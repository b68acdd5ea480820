"""FP64 reference tracer (the oracle) -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP
library: the tracing arithmetic lives in ``oracle.cpp`` (plain C++17, FP64),
and this module marshals the scene descriptors and photon bundles built by
``scenes`` into it, then computes the focal-plane figures in numpy.

What is computed (paper §2.1, §2.2, §3):
  * ``trace``: each photon is carried through the scene by brute-force
    nearest-surface search over every face of every volume, with the role of
    the volume hit deciding reflection / refraction / detection / absorption.
  * ``figures``: per group (field angle or incidence angle) the centroid and
    RMS spot radius of the FOCUSED photons (the spot diagrams of §3, Fig. 1),
    the collection efficiency (Fig. 2b) and the cosine-weighted collection.
  * ``forced`` / ``forced_jac``: re-evaluation of each photon along its
    recorded surface sequence with changed parameters (central finite
    differences) and with dual numbers (forward-mode derivatives).

Parity pins are in ``tests/test_oracle_*.py``; functions without a pin are
listed there as "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

FATE_FOCUSED, FATE_ABSORBED, FATE_EXITED, FATE_SUSPENDED, FATE_FAILED = 1, 2, 3, 4, 5
ACT_REFLECT, ACT_REFRACT, ACT_STOP = 0, 1, 2


def build(force=True):
    """Compile oracle.cpp into liboracle.so (g++, -O2, FP64; no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _lib.oracle_draw.restype = ctypes.c_uint32
        _lib.oracle_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int]
        _lib.oracle_fresnel.restype = ctypes.c_double
        _lib.oracle_fresnel.argtypes = [ctypes.c_double] * 3
    return _lib


def default_threads():
    """Host threads the oracle uses by default: the cores this process may
    run on, at most 16 (a GPU machine's share of its host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def pack_volumes(volumes):
    """Oracle's own flat layout: 5 ints and 55 doubles per volume."""
    n = len(volumes)
    vi = np.zeros((n, 5), dtype=np.int32)
    vd = np.zeros((n, 55), dtype=np.float64)
    for k in range(n):
        v = volumes[k]
        vi[k] = [v["role"], v["shape"], v["outline"], v["shape_param"], v["tilt_param"]]
        vd[k] = np.concatenate([v["Q"], v["c"], v["p"], v["o"], [v["reflectivity"], v["n_inside"]],
                                v["Q0"], v["c0"], v["pivot"], v["e1"], v["e2"]])
    return np.ascontiguousarray(vi), np.ascontiguousarray(vd)


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32); k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def draw(seed, photon_id, event):
    return int(lib().oracle_draw(seed, photon_id, event))


def fresnel(cos_i, n1, n2):
    return float(lib().oracle_fresnel(cos_i, n1, n2))


def outline(volume, x, y):
    """(inside, boundary distance) of the outline of one volume descriptor
    at local points (x, y): the trace's bounds test and its diagnostic."""
    vi, vd = pack_volumes(np.array([volume]))
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    inside = np.zeros(len(x), np.uint8)
    bd = np.zeros(len(x))
    lib().oracle_outline(_p(vi), _p(vd), ctypes.c_int64(len(x)), _p(x), _p(y), _p(inside), _p(bd))
    return inside.astype(bool), bd


def _rays64(rays):
    return [np.ascontiguousarray(rays[k], dtype=np.float64) for k in ("ox", "oy", "oz", "dx", "dy", "dz")]


def _lam(rays, wavelengths):
    if not wavelengths:
        return None
    return np.ascontiguousarray(rays["lam"], dtype=np.float64)


def trace(scene, rays, id_base=0, log=False, nthreads=None, culled=True, volumes=None, wavelengths=False):
    """Trace every photon; returns a dict of per-photon exit records (and the event log).

    wavelengths: each photon carries its wavelength rays["lam"] (m), and a
    lens with a dispersion law refracts it with n(lam) (§2.1: lenses; the
    law is the Cauchy form A + B / lam^2 of the lens descriptor); otherwise
    every lens has its fixed index."""
    L = lib()
    vols = scene.volumes if volumes is None else volumes
    vi, vd = pack_volumes(vols)
    cols = _rays64(rays)
    lam = _lam(rays, wavelengths)
    n = len(cols[0])
    me = scene.max_events
    out = dict(fate=np.zeros(n, np.uint8), n_events=np.zeros(n, np.uint8),
               last_vol=np.zeros(n, np.int32), pos=np.zeros((n, 3)), dir=np.zeros((n, 3)),
               opl=np.zeros(n), seq_hash=np.zeros(n, np.uint64))
    lg = None
    if log:
        lg = dict(vol=np.full((n, me), -1, np.int32), face=np.full((n, me), -1, np.int32),
                  act=np.full((n, me), -1, np.int32), t=np.zeros((n, me)), s=np.zeros((n, me)),
                  diag=np.full((n, me, 5), np.inf))
    nth = nthreads or default_threads()
    rc = L.oracle_trace(ctypes.c_int(len(vols)), _p(vi), _p(vd), ctypes.c_int(me),
                        ctypes.c_uint64(scene.seed), ctypes.c_double(scene.l_ref),
                        ctypes.c_int64(n), *[_p(c) for c in cols], _p(lam), ctypes.c_uint64(id_base),
                        _p(out["fate"]), _p(out["n_events"]), _p(out["last_vol"]), _p(out["pos"]),
                        _p(out["dir"]), _p(out["opl"]), _p(out["seq_hash"]),
                        _p(lg["vol"]) if lg else None, _p(lg["face"]) if lg else None,
                        _p(lg["act"]) if lg else None, _p(lg["t"]) if lg else None,
                        _p(lg["s"]) if lg else None, _p(lg["diag"]) if lg else None,
                        ctypes.c_int(nth), ctypes.c_int(1 if culled else 0))
    if rc != 0:
        raise ValueError("oracle_trace rejected its input")
    out["group"] = np.asarray(rays["group"])
    out["lam"] = lam
    if log:
        out["log"] = lg
    return out


def grazing(rec, l_ref, tol_len=1e-5, tol_cos=1e-4, tol_draw=1e-5):
    """Photons whose oracle path is ill-conditioned: at some interaction two
    candidate surfaces lie within tol_len * l_ref, the hit or a rejected root
    nearer than it lies within tol_len * l_ref of a face boundary, the ray
    meets the surface with |d . n| < tol_cos, or the random draw lies within
    tol_draw of its threshold.  Needs a trace with log=True."""
    dg = rec["log"]["diag"]
    ne = rec["n_events"].astype(np.int64)
    live = np.arange(dg.shape[1])[None, :] <= np.minimum(ne, dg.shape[1] - 1)[:, None]
    L = tol_len * l_ref
    bad = ((dg[:, :, 0] < L) | (dg[:, :, 1] < L) | (dg[:, :, 2] < L) | (dg[:, :, 3] < tol_cos) |
           (dg[:, :, 4] < tol_draw)) & live
    return bad.any(axis=1)


def timed_trace(scene, rays, nthreads=None, **kw):
    t0 = time.perf_counter()
    out = trace(scene, rays, nthreads=nthreads, **kw)
    return out, time.perf_counter() - t0


def forced(scene, rays, rec, params, nthreads=None):
    """Final (pos, dir, status) of each photon along its recorded sequence with `params`."""
    L = lib()
    vi, vd = pack_volumes(scene.volumes)
    cols = _rays64(rays)
    n = len(cols[0])
    lg = rec["log"]
    P = np.ascontiguousarray(params, dtype=np.float64)
    pos, dirv = np.zeros((n, 3)), np.zeros((n, 3))
    st = np.zeros(n, np.int32)
    L.oracle_forced(ctypes.c_int(len(scene.volumes)), _p(vi), _p(vd), _p(P), ctypes.c_int64(n),
                    *[_p(c) for c in cols], _p(rec.get("lam")), ctypes.c_int(scene.max_events), _p(rec["n_events"]),
                    _p(lg["vol"]), _p(lg["face"]), _p(lg["act"]), _p(lg["t"]), _p(lg["s"]),
                    _p(pos), _p(dirv), _p(st), ctypes.c_int(nthreads or default_threads()))
    return pos, dirv, st


def forced_jac(scene, rays, rec, params, p0, cnt, nthreads=None):
    """Dual-number derivatives d(pos, dir)/d(params[p0:p0+cnt]), shapes (n, 3, cnt)."""
    L = lib()
    vi, vd = pack_volumes(scene.volumes)
    cols = _rays64(rays)
    n = len(cols[0])
    lg = rec["log"]
    P = np.ascontiguousarray(params, dtype=np.float64)
    dpos, ddir = np.zeros((n, 3, cnt)), np.zeros((n, 3, cnt))
    st = np.zeros(n, np.int32)
    rc = L.oracle_forced_jac(ctypes.c_int(len(scene.volumes)), _p(vi), _p(vd), _p(P),
                             ctypes.c_int(len(P)), ctypes.c_int(p0), ctypes.c_int(cnt),
                             ctypes.c_int64(n), *[_p(c) for c in cols], _p(rec.get("lam")),
                             ctypes.c_int(scene.max_events),
                             _p(rec["n_events"]), _p(lg["vol"]), _p(lg["face"]), _p(lg["act"]),
                             _p(lg["t"]), _p(lg["s"]), _p(dpos), _p(ddir), _p(st),
                             ctypes.c_int(nthreads or default_threads()))
    if rc != 0:
        raise ValueError("oracle_forced_jac rejected its input")
    return dpos, ddir, st


# ------------------------------------------------------------------ figures (§3)
def figures(rec, n_groups):
    """Per group: launched, focused, centroid, RMS spot radius, efficiency, weighted collection.

    RMS = sqrt(mean over FOCUSED photons of (x - xbar)^2 + (y - ybar)^2) in
    the focal surface's global (x, y).  Efficiency = N_FOCUSED / N_launched;
    the weighted collection sums the cosine of the exit direction to the
    detector normal, |d_z|, over FOCUSED photons, divided by N_launched.
    """
    g = rec["group"].astype(np.int64)
    foc = rec["fate"] == FATE_FOCUSED
    out = []
    for k in range(n_groups):
        m = g == k
        f = m & foc
        nl, nf = int(m.sum()), int(f.sum())
        x, y = rec["pos"][f, 0], rec["pos"][f, 1]
        cx = x.mean() if nf else 0.0
        cy = y.mean() if nf else 0.0
        rms = float(np.sqrt(np.mean((x - cx) ** 2 + (y - cy) ** 2))) if nf else 0.0
        w = float(np.abs(rec["dir"][f, 2]).sum())
        out.append(dict(launched=nl, focused=nf, cx=float(cx), cy=float(cy), rms=rms,
                        eff=nf / nl if nl else 0.0, eff_w=w / nl if nl else 0.0))
    return out


def arrival_figures(rec, n_groups):
    """Per group: FOCUSED photons, the mean and the RMS spread of their
    optical path length from the start point to the focal surface (arrival
    time x c): the spread is the isochronicity of the optics.  Two passes
    (mean, then mean squared deviation), in FP64."""
    g = rec["group"].astype(np.int64)
    foc = rec["fate"] == FATE_FOCUSED
    out = []
    for k in range(n_groups):
        p = np.asarray(rec["opl"], dtype=np.float64)[foc & (g == k)]
        nf = len(p)
        mean = float(p.mean()) if nf else 0.0
        rms = float(np.sqrt(np.mean((p - mean) ** 2))) if nf else 0.0
        out.append(dict(focused=nf, mean=mean, rms=rms))
    return out


def rms_cotangent(rec, n_groups, dL_drms):
    """dL/d(x, y) per photon for L = sum_g dL_drms[g] * RMS_g (zero for non-FOCUSED)."""
    fig = figures(rec, n_groups)
    g = rec["group"].astype(np.int64)
    foc = rec["fate"] == FATE_FOCUSED
    cot = np.zeros((len(g), 3))
    for k in range(n_groups):
        f = (g == k) & foc
        if fig[k]["focused"] == 0 or fig[k]["rms"] == 0.0:
            continue
        a = dL_drms[k] / (fig[k]["focused"] * fig[k]["rms"])
        cot[f, 0] = a * (rec["pos"][f, 0] - fig[k]["cx"])
        cot[f, 1] = a * (rec["pos"][f, 1] - fig[k]["cy"])
    return cot


def gradient_rms(scene, rays, rec, dL_drms, params=None, chunk=8):
    """Pathwise gradient of sum_g dL_drms[g] RMS_g by dual numbers, (n_params,)."""
    P = scene.params if params is None else params
    cot = rms_cotangent(rec, scene.n_groups, dL_drms)
    foc = rec["fate"] == FATE_FOCUSED
    grad = np.zeros(len(P))
    for p0 in range(0, len(P), chunk):
        cnt = min(chunk, len(P) - p0)
        dpos, _, st = forced_jac(scene, rays, rec, P, p0, cnt)
        m = foc & (st == 0)
        grad[p0:p0 + cnt] = np.einsum("nk,nkj->j", cot[m], dpos[m])
    return grad


def gradient_eff_w(scene, rays, rec, dL_deffw, params=None, chunk=8):
    """Pathwise gradient of sum_g dL_deffw[g] eff_w_g by dual numbers."""
    P = scene.params if params is None else params
    g = rec["group"].astype(np.int64)
    foc = rec["fate"] == FATE_FOCUSED
    nl = np.bincount(g, minlength=scene.n_groups).astype(np.float64)
    w = np.where(foc, np.asarray(dL_deffw)[g] / np.maximum(nl[g], 1.0), 0.0)
    # d|d_z|/dp = sign(d_z) d(d_z)/dp
    grad = np.zeros(len(P))
    for p0 in range(0, len(P), chunk):
        cnt = min(chunk, len(P) - p0)
        _, ddir, st = forced_jac(scene, rays, rec, P, p0, cnt)
        m = foc & (st == 0)
        sgn = np.sign(rec["dir"][m, 2])
        grad[p0:p0 + cnt] = np.einsum("n,nj->j", w[m] * sgn, ddir[m, 2, :])
    return grad
