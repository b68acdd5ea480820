"""Seeded synthetic scenes and photon bundles.

This module is the only code shared by the FP64 reference tracer under
``oracle/`` and the HIP library.  It builds *inputs*: volume descriptors (a
role from the paper's set of lens / mirror / focal surface / obscuration,
§2.1, and a shape from §2.2) and photon bundles (position plus direction,
§2.1).  It contains no tracing arithmetic: no intersection, no interaction
physics, no random draws made during tracing.

Every stand-in telescope follows the optics the paper applies ROBAST to (§3):
a single spherical mirror, a Davies-Cotton segmented dish, a two-mirror
Schwarzschild-Couder telescope with segmented aspheric mirrors, and an array
of hexagonal Bezier-profile light concentrators behind a PMMA window.  The
paper prints no design tables, so the layouts are synthetic and every
number below is stated where it is chosen.

Conventions
-----------
* A volume's local frame is ``x_l = Q (x - c)`` (rows of ``Q`` are the local
  axes in world coordinates).
* Each face has a *front* side.  Mirrors reflect on the front, focal
  surfaces detect on the front; both absorb on the back.  Closed solids
  (box, cylinder) have the front outside, hexagonal cone walls inside.
* For single-precision scenes every descriptor and ray value is rounded to
  float32 here, so the reference tracer and the GPU read identical numbers.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Dict, List, Optional

import numpy as np

# ---------------------------------------------------------------- codes
ROLE_MIRROR, ROLE_LENS, ROLE_FOCAL, ROLE_OBSCURATION = 1, 2, 3, 4
SHAPE_PLANE, SHAPE_SPHERE, SHAPE_ASPHERE, SHAPE_CYLINDER, SHAPE_BOX, SHAPE_HEXCONE = 1, 2, 3, 4, 5, 6
OUTLINE_NONE, OUTLINE_DISC, OUTLINE_ANNULUS, OUTLINE_RECT, OUTLINE_HEX, OUTLINE_SECTOR = 0, 1, 2, 3, 4, 5
FATE_NONE, FATE_FOCUSED, FATE_ABSORBED, FATE_EXITED, FATE_SUSPENDED, FATE_FAILED = 0, 1, 2, 3, 4, 5

VOLUME_DTYPE = np.dtype([
    ("role", "<i4"), ("shape", "<i4"), ("outline", "<i4"),
    ("shape_param", "<i4"), ("tilt_param", "<i4"), ("flags", "<i4"),
    ("Q", "<f8", (9,)), ("c", "<f8", (3,)),
    ("p", "<f8", (16,)), ("o", "<f8", (4,)),
    ("reflectivity", "<f8"), ("n_inside", "<f8"),
    # untilted frame, pivot and the two tilt axes (world); used only by
    # volumes with tilt parameters: the effective frame is the untilted one
    # rotated about `pivot` by R = Rot(e2, beta) Rot(e1, alpha).
    ("Q0", "<f8", (9,)), ("c0", "<f8", (3,)),
    ("pivot", "<f8", (3,)), ("e1", "<f8", (3,)), ("e2", "<f8", (3,)),
])

SEED_BASE = 150807803


def _q(x, precision):
    """Round to the kernel precision (float32 values kept in float64)."""
    a = np.asarray(x, dtype=np.float64)
    if precision == 32:
        return a.astype(np.float32).astype(np.float64)
    return a


def rot(axis, angle):
    """Rotation matrix about a unit axis (Rodrigues)."""
    e = np.asarray(axis, dtype=np.float64)
    e = e / np.linalg.norm(e)
    k = np.array([[0.0, -e[2], e[1]], [e[2], 0.0, -e[0]], [-e[1], e[0], 0.0]])
    return np.cos(angle) * np.eye(3) + np.sin(angle) * k + (1.0 - np.cos(angle)) * np.outer(e, e)


def frame_from_axes(z_axis, x_hint=(1.0, 0.0, 0.0)):
    """Rows (x_l, y_l, z_l): z_l along `z_axis`, x_l the projection of x_hint."""
    z = np.asarray(z_axis, dtype=np.float64)
    z = z / np.linalg.norm(z)
    xh = np.asarray(x_hint, dtype=np.float64)
    x = xh - np.dot(xh, z) * z
    if np.linalg.norm(x) < 1e-9:
        xh = np.array([0.0, 1.0, 0.0])
        x = xh - np.dot(xh, z) * z
    x = x / np.linalg.norm(x)
    y = np.cross(z, x)
    return np.stack([x, y, z])


def tilted_frame(Q0, c0, pivot, e1, e2, alpha, beta):
    """Frame of a rigid body rotated about `pivot` by Rot(e2,beta) Rot(e1,alpha)."""
    R = rot(e2, beta) @ rot(e1, alpha)
    Q = np.asarray(Q0) @ R.T
    c = np.asarray(pivot) - R @ (np.asarray(pivot) - np.asarray(c0))
    return Q, c


def new_volume(role, shape, outline=OUTLINE_NONE, Q=None, c=(0, 0, 0), p=(), o=(),
               reflectivity=1.0, n_inside=1.0, shape_param=-1, tilt_param=-1):
    v = np.zeros((), dtype=VOLUME_DTYPE)
    v["role"], v["shape"], v["outline"] = role, shape, outline
    v["shape_param"], v["tilt_param"] = shape_param, tilt_param
    Qm = np.eye(3) if Q is None else np.asarray(Q, dtype=np.float64)
    v["Q"] = Qm.reshape(9)
    v["c"] = c
    pp = np.zeros(16); pp[:len(p)] = p
    oo = np.zeros(4); oo[:len(o)] = o
    v["p"], v["o"] = pp, oo
    v["reflectivity"], v["n_inside"] = reflectivity, n_inside
    v["Q0"], v["c0"] = Qm.reshape(9), c
    return v


@dataclasses.dataclass
class Scene:
    name: str
    volumes: np.ndarray                 # VOLUME_DTYPE[n]
    params: np.ndarray                  # float64[n_params] differentiable parameters
    param_names: List[str]
    precision: int                      # 32 or 64
    max_events: int
    seed: int
    l_ref: float                        # length scale for tolerances
    groups: np.ndarray                  # per-group field / incidence angle (rad)
    ray_maker: Callable = None          # (scene, n_per_group, seed, groups) -> rays
    meta: Dict = dataclasses.field(default_factory=dict)

    @property
    def n_volumes(self):
        return int(self.volumes.shape[0])

    @property
    def n_groups(self):
        return int(len(self.groups))

    def rays(self, n_per_group, seed=None, groups=None):
        """Seeded photon bundle, float64 arrays already rounded to the precision."""
        s = self.seed if seed is None else seed
        g = np.arange(self.n_groups) if groups is None else np.asarray(groups)
        return self.ray_maker(self, int(n_per_group), s, g)


def _finish(name, vols, params, names, precision, max_events, seed, l_ref, groups, ray_maker, **meta):
    arr = np.array(vols, dtype=VOLUME_DTYPE)
    if precision == 32:
        for f in ("Q", "c", "p", "o", "Q0", "c0", "pivot", "e1", "e2"):
            arr[f] = _q(arr[f], 32)
        params = _q(params, 32)
    return Scene(name, arr, np.asarray(params, dtype=np.float64), list(names), precision,
                 max_events, seed, l_ref, np.asarray(groups, dtype=np.float64), ray_maker, dict(meta))


def make_rays(precision, ox, oy, oz, dx, dy, dz, group, lam=400e-9):
    """Photon bundle from explicit arrays (rounded to the precision)."""
    return _pack_rays(precision, ox, oy, oz, dx, dy, dz, group, lam)


def _pack_rays(precision, ox, oy, oz, dx, dy, dz, group, lam=400e-9):
    n = len(ox)
    out = {k: _q(v, precision) for k, v in
           dict(ox=ox, oy=oy, oz=oz, dx=dx, dy=dy, dz=dz).items()}
    out["lam"] = _q(np.full(n, lam), precision)
    out["group"] = np.asarray(group, dtype=np.uint32)
    return out


# ================================================================ C1
def single_mirror(seed=SEED_BASE + 0):
    """Spherical mirror R=16 m, 4 m aperture, focal disc r=0.5 m at z=8 m, FP64.

    The focal disc faces the mirror, so rays at r < 0.5 m meet its back on the
    way in and are absorbed (the camera shadow).  Parameter 0 is the mirror's
    radius of curvature.
    """
    R = 16.0
    vols = [
        new_volume(ROLE_MIRROR, SHAPE_SPHERE, OUTLINE_DISC, p=[1.0 / R], o=[2.0],
                   reflectivity=1.0, shape_param=0),
        new_volume(ROLE_FOCAL, SHAPE_PLANE, OUTLINE_DISC,
                   Q=np.diag([1.0, -1.0, -1.0]), c=(0.0, 0.0, 8.0), o=[0.5]),
    ]

    def rays(scene, n, s, groups):
        rng = np.random.default_rng(s)
        out = []
        for g in groups:
            u1, u2 = rng.random(n), rng.random(n)
            r, ph = 2.0 * np.sqrt(u1), 2.0 * np.pi * u2
            out.append((r * np.cos(ph), r * np.sin(ph), np.full(n, 20.0),
                        np.zeros(n), np.zeros(n), -np.ones(n), np.full(n, g)))
        cols = [np.concatenate(c) for c in zip(*out)]
        return _pack_rays(scene.precision, *cols)

    return _finish("single_mirror", vols, [R], ["R_mirror"], 64, 16, seed, 8.0, [0.0], rays,
                   radius=R, aperture=2.0, focal_z=8.0)


# ================================================================ C2
def _hex_lattice(pitch, rmax):
    """Centres of a hexagonal lattice of pitch `pitch` inside radius rmax,
    origin removed, sorted by (r, phi): tuples (r, phi, x, y)."""
    centres = []
    for i in range(-10, 11):
        for j in range(-10, 11):
            x = pitch * (i + 0.5 * j)
            y = pitch * (math.sqrt(3.0) / 2.0) * j
            r = math.hypot(x, y)
            if r <= rmax and (i, j) != (0, 0):
                centres.append((r, math.atan2(y, x), x, y))
    centres.sort()
    return centres


def _facet_volumes(centres, surface_z, axis_of, radii, tilts, half_flat, reflectivity):
    """Hexagonal spherical facets: facet k centred on the dish surface at
    centre k, with optical axis axis_of(centre), radius radii[k] and a
    hexagonal outline in the plane normal to its axis, tilted by tilts[k]
    about its local x then y axes.  Parameters: radii, then 2 tilts each."""
    nf = len(centres)
    vols, params, names = [], [], []
    params.extend(radii); names.extend([f"facet{k}_R" for k in range(nf)])
    for k in range(nf):
        params.extend(tilts[k]); names.extend([f"facet{k}_tilt_x", f"facet{k}_tilt_y"])
    for k, (r, _, x, y) in enumerate(centres):
        cen = np.array([x, y, surface_z(r)])
        Q0 = frame_from_axes(axis_of(cen))
        e1, e2 = Q0[0].copy(), Q0[1].copy()
        Q, c = tilted_frame(Q0, cen, cen, e1, e2, tilts[k][0], tilts[k][1])
        v = new_volume(ROLE_MIRROR, SHAPE_SPHERE, OUTLINE_HEX, Q=Q, c=c, p=[1.0 / radii[k]],
                       o=[half_flat], reflectivity=reflectivity, shape_param=k, tilt_param=nf + 2 * k)
        v["Q0"], v["c0"], v["pivot"], v["e1"], v["e2"] = Q0.reshape(9), cen, cen, e1, e2
        vols.append(v)
    return vols, params, names


def _dish_camera_and_masts(f, rmax, zrim):
    """A 3 m x 3 m focal plane at z = f facing the dish, closed by 5
    absorbing rectangles (1 m deep), and four absorbing masts (r = 0.1 m)
    from the dish rim at z = zrim to the camera corners."""
    vols = []
    flip = np.diag([1.0, -1.0, -1.0])
    vols.append(new_volume(ROLE_FOCAL, SHAPE_PLANE, OUTLINE_RECT, Q=flip, c=(0, 0, f), o=[1.5, 1.5]))
    vols.append(new_volume(ROLE_OBSCURATION, SHAPE_PLANE, OUTLINE_RECT, c=(0, 0, f + 1.0), o=[1.5, 1.5]))
    for sx in (1.0, -1.0):
        Q = frame_from_axes((sx, 0, 0), x_hint=(0, 0, 1))
        vols.append(new_volume(ROLE_OBSCURATION, SHAPE_PLANE, OUTLINE_RECT, Q=Q,
                               c=(1.5 * sx, 0, f + 0.5), o=[0.5, 1.5]))
    for sy in (1.0, -1.0):
        Q = frame_from_axes((0, sy, 0), x_hint=(0, 0, 1))
        vols.append(new_volume(ROLE_OBSCURATION, SHAPE_PLANE, OUTLINE_RECT, Q=Q,
                               c=(0, 1.5 * sy, f + 0.5), o=[0.5, 1.5]))
    for kk in range(4):
        ph = math.radians(45.0 + 90.0 * kk)
        base = np.array([rmax * math.cos(ph), rmax * math.sin(ph), zrim])
        top = np.array([1.5 * np.sign(math.cos(ph)), 1.5 * np.sign(math.sin(ph)), f])
        ax = top - base
        vols.append(new_volume(ROLE_OBSCURATION, SHAPE_CYLINDER, Q=frame_from_axes(ax), c=base,
                               p=[0.1, float(np.linalg.norm(ax))]))
    return vols


def _dish_rays(r_beam, back):
    """Parallel beams at the groups' field angles (in the x-z plane), uniform
    over a disc of radius r_beam normal to the beam, starting `back` metres
    before the origin."""
    def rays(scene, n, s, gsel):
        rng2 = np.random.default_rng(s)
        out = []
        for g in gsel:
            th = scene.groups[g]
            d = np.array([math.sin(th), 0.0, -math.cos(th)])
            e1v = np.array([math.cos(th), 0.0, math.sin(th)])
            e2v = np.array([0.0, 1.0, 0.0])
            u1, u2 = rng2.random(n), rng2.random(n)
            r, ph = r_beam * np.sqrt(u1), 2.0 * np.pi * u2
            px, py = r * np.cos(ph), r * np.sin(ph)
            o = -back * d[None, :] + px[:, None] * e1v[None, :] + py[:, None] * e2v[None, :]
            out.append((o[:, 0], o[:, 1], o[:, 2], np.full(n, d[0]), np.full(n, d[1]),
                        np.full(n, d[2]), np.full(n, g)))
        cols = [np.concatenate(c) for c in zip(*out)]
        return _pack_rays(scene.precision, *cols)
    return rays


def davies_cotton(seed=SEED_BASE + 1, sigma_tilt=1e-4, fields_deg=(0.0, 0.5, 1.0, 1.5, 2.0),
                  radius_scale=None, tilts=None, precision=32):
    """Davies-Cotton dish, f = 28 m, 198 hexagonal spherical facets.

    Facet centres: hex lattice of pitch 1.55 m (4 cm gaps between 1.51 m
    flat-to-flat facets) inside an 11.5 m circle, origin removed -> 198
    facets on the sphere z = f - sqrt(f^2 - r^2).  Each facet is a sphere of
    radius 2f aimed at (0, 0, 2f), with a hexagonal outline in the plane
    normal to its axis, then tilted by two Gaussian angles (sigma 0.1 mrad)
    about its local x then y axes.  Camera: a 3 m x 3 m focal plane at
    z = f facing the dish, closed by 5 absorbing rectangles (1 m deep).
    Four absorbing masts (r = 0.1 m) from the dish rim to the camera corners.
    Parameters: 198 facet radii, then 2 tilts per facet.
    """
    f, pitch, rmax, half_flat = 28.0, 1.55, 11.5, 0.755
    rng = np.random.default_rng(seed)
    centres = _hex_lattice(pitch, rmax)
    assert len(centres) == 198
    nf = len(centres)
    if tilts is None:
        tilts = rng.normal(0.0, sigma_tilt, size=(nf, 2))
    radii = np.full(nf, 2.0 * f) if radius_scale is None else 2.0 * f * np.asarray(radius_scale)
    vols, params, names = _facet_volumes(centres, lambda r: f - math.sqrt(f * f - r * r),
                                         lambda cen: np.array([0.0, 0.0, 2.0 * f]) - cen, radii, tilts,
                                         half_flat, 0.9)
    vols += _dish_camera_and_masts(f, rmax, f - math.sqrt(f * f - rmax * rmax))
    groups = np.radians(np.asarray(fields_deg, dtype=np.float64))
    return _finish("davies_cotton", vols, params, names, precision, 16, seed, 28.0, groups, _dish_rays(12.0, 40.0),
                   n_facets=nf, focal_length=f, beam=dict(kind="disc_perp", r_in=0.0, r_out=12.0, back=40.0))


def lst_parabolic(seed=SEED_BASE + 8, sigma_tilt=1e-4, fields_deg=(0.0, 0.5, 1.0, 1.5, 2.0),
                  radius_scale=None, tilts=None, precision=32):
    """Segmented parabolic dish (the LST layout: 198 mirrors aligned on a
    parabola), f = 28 m, on the Davies-Cotton lattice and camera.

    Facet centres: the same hexagonal lattice (pitch 1.55 m, 1.51 m flat to
    flat, inside 11.5 m, 198 facets) on the paraboloid z = r^2 / (4 f).
    Each facet is a sphere whose axis is the paraboloid's normal at its
    centre (so on-axis light reflected at the centre goes to the focus
    (0, 0, f)) and whose radius is twice its centre's distance to the focus
    (its focal length equals that distance); hexagonal outline, Gaussian
    tilts (sigma 0.1 mrad) as for the Davies-Cotton dish.  Unlike a
    Davies-Cotton dish, the paraboloid makes every on-axis path from a
    wavefront to the focus equally long (an isochronous dish).  Camera and
    masts as for the Davies-Cotton dish.  Parameters: 198 facet radii, then
    2 tilts per facet.
    """
    f, pitch, rmax, half_flat = 28.0, 1.55, 11.5, 0.755
    rng = np.random.default_rng(seed)
    centres = _hex_lattice(pitch, rmax)
    nf = len(centres)
    if tilts is None:
        tilts = rng.normal(0.0, sigma_tilt, size=(nf, 2))
    foc = np.array([0.0, 0.0, f])

    def surface_z(r):
        return r * r / (4.0 * f)

    def axis_of(cen):
        return np.array([-cen[0] / (2.0 * f), -cen[1] / (2.0 * f), 1.0])

    base = np.array([2.0 * np.linalg.norm(foc - np.array([x, y, surface_z(r)])) for (r, _, x, y) in centres])
    radii = base if radius_scale is None else base * np.asarray(radius_scale)
    vols, params, names = _facet_volumes(centres, surface_z, axis_of, radii, tilts, half_flat, 0.9)
    vols += _dish_camera_and_masts(f, rmax, surface_z(rmax))
    groups = np.radians(np.asarray(fields_deg, dtype=np.float64))
    return _finish("lst_parabolic", vols, params, names, precision, 16, seed, 28.0, groups, _dish_rays(12.0, 40.0),
                   n_facets=nf, focal_length=f, beam=dict(kind="disc_perp", r_in=0.0, r_out=12.0, back=40.0))


# ================================================================ C3
SC_PRIMARY = dict(R=38.0958, k=-1.4980, rn=4.83, r_in=2.19, r_out=4.83, z=0.0)
SC_SECONDARY = dict(R=8.8680, k=-3.1648, rn=2.7, r_in=0.0, r_out=2.7, z=8.4)
SC_FOCAL_Z = 5.3257


def conic_taylor(R, k, rn, n=8):
    """Coefficients b_i of z = sum b_i u^i, u = (r/rn)^2, for the conic (R, k)."""
    c = 1.0 / R
    return np.array([math.comb(2 * i, i) / (4.0 ** i * (2 * i - 1)) * (1.0 + k) ** (i - 1)
                     * c ** (2 * i - 1) * rn ** (2 * i) for i in range(1, n + 1)])


def _ring_panels(r_in, r_out, r_split, n_inner, n_outer):
    out = []
    for (a, b, n) in ((r_in, r_split, n_inner), (r_split, r_out, n_outer)):
        dphi = 2.0 * math.pi / n
        for s in range(n):
            out.append((a, b, s * dphi, (s + 1) * dphi))
    return out


def _sc_two_mirror(name, scale, pan_p, pan_s, tilts, bp, bs, groups, precision, seed, extra_vols=()):
    """The two-mirror Schwarzschild-Couder optics at `scale` times the
    dimensions of SC_PRIMARY / SC_SECONDARY / SC_FOCAL_Z: aspheric mirrors
    cut into the (r_a, r_b, phi_a, phi_b) sectors pan_p / pan_s (radii
    already scaled), each rotated about its sector-centroid point by its
    two tilts (radial, tangential axes), the spherical focal cap, and the
    beam filling the primary's annulus from `12 scale` m above it."""
    pri = dict(SC_PRIMARY, rn=SC_PRIMARY["rn"] * scale, r_in=SC_PRIMARY["r_in"] * scale,
               r_out=SC_PRIMARY["r_out"] * scale, z=SC_PRIMARY["z"] * scale)
    sec = dict(SC_SECONDARY, rn=SC_SECONDARY["rn"] * scale, r_in=SC_SECONDARY["r_in"] * scale,
               r_out=SC_SECONDARY["r_out"] * scale, z=SC_SECONDARY["z"] * scale)
    npan = len(pan_p) + len(pan_s)
    params = list(bp) + list(bs)
    names = [f"primary_b{i}" for i in range(1, 9)] + [f"secondary_b{i}" for i in range(1, 9)]
    for k in range(npan):
        params.extend(tilts[k]); names.extend([f"panel{k}_tilt_r", f"panel{k}_tilt_t"])
    vols = []
    k = 0
    for mirror, pans, b, off, Q0 in ((pri, pan_p, bp, 0, np.eye(3)),
                                     (sec, pan_s, bs, 8, np.diag([1.0, -1.0, -1.0]))):
        c0 = np.array([0.0, 0.0, mirror["z"]])
        for (ra, rb, pa, pb) in pans:
            phm = 0.5 * (pa + pb)
            half = 0.5 * (pb - pa)
            rc = (2.0 / 3.0) * (rb ** 3 - ra ** 3) / (rb ** 2 - ra ** 2) * math.sin(half) / half
            u = (rc / mirror["rn"]) ** 2
            zc = sum(b[i] * u ** (i + 1) for i in range(8))
            piv_l = np.array([rc * math.cos(phm), rc * math.sin(phm), zc])
            pivot = c0 + Q0.T @ piv_l
            e1 = Q0.T @ np.array([math.cos(phm), math.sin(phm), 0.0])
            e2 = Q0.T @ np.array([-math.sin(phm), math.cos(phm), 0.0])
            Q, c = tilted_frame(Q0, c0, pivot, e1, e2, tilts[k][0], tilts[k][1])
            # a one-piece mirror is a disc: 2 pi rounded to FP32 exceeds a sector's range
            whole = ra == 0.0 and pb - pa == 2.0 * math.pi
            v = new_volume(ROLE_MIRROR, SHAPE_ASPHERE, OUTLINE_DISC if whole else OUTLINE_SECTOR, Q=Q, c=c,
                           p=[mirror["rn"]] + list(b), o=[rb] if whole else [ra, rb, pa, pb],
                           reflectivity=1.0, shape_param=off, tilt_param=16 + 2 * k)
            v["Q0"], v["c0"], v["pivot"], v["e1"], v["e2"] = Q0.reshape(9), c0, pivot, e1, e2
            vols.append(v)
            k += 1
    vols.append(new_volume(ROLE_FOCAL, SHAPE_SPHERE, OUTLINE_DISC, c=(0.0, 0.0, SC_FOCAL_Z * scale),
                           p=[-1.0 / scale], o=[0.6 * scale]))
    vols += list(extra_vols)
    back = 12.0 * scale

    def rays(scene, n, s, gsel):
        rng2 = np.random.default_rng(s)
        out = []
        for g in gsel:
            th = scene.groups[g]
            d = np.array([math.sin(th), 0.0, -math.cos(th)])
            u1, u2 = rng2.random(n), rng2.random(n)
            r = np.sqrt(pri["r_in"] ** 2 + u1 * (pri["r_out"] ** 2 - pri["r_in"] ** 2))
            ph = 2.0 * np.pi * u2
            o = np.stack([r * np.cos(ph), r * np.sin(ph), np.zeros(n)], 1) - back * d[None, :]
            out.append((o[:, 0], o[:, 1], o[:, 2], np.full(n, d[0]), np.full(n, d[1]),
                        np.full(n, d[2]), np.full(n, g)))
        cols = [np.concatenate(c) for c in zip(*out)]
        return _pack_rays(scene.precision, *cols)

    return _finish(name, vols, params, names, precision, 16, seed, 5.6 * scale, groups, rays,
                   n_panels=npan, focal_z=SC_FOCAL_Z * scale, scale=scale,
                   beam=dict(kind="annulus_z0", r_in=pri["r_in"], r_out=pri["r_out"], back=back))


def schwarzschild_couder(seed=SEED_BASE + 2, sigma_tilt=5e-5, n_fields=16, max_field_deg=4.0,
                         coeff_scale=None, tilts=None, precision=32, fields_deg=None):
    """Two-mirror Schwarzschild-Couder telescope with segmented aspheric mirrors.

    Sag z = sum_{i=1..8} b_i u^i with u = (r/rn)^2 (normalised form; the
    monomial a_i = b_i / rn^(2i) would span 1e-2 .. 1e-28).  Baseline b_i are
    the Taylor coefficients of the conics (R1 = 38.0958 m, k1 = -1.4980) and
    (R2 = 8.8680 m, k2 = -3.1648), primary vertex at z = 0 concave up,
    secondary vertex at z = 8.4 m concave down.  Panels: primary 16 + 32
    (r 2.19-3.3127-4.83 m), secondary 8 + 16 (r 0-1.5588-2.7 m), each the
    parent surface restricted to its (r, phi) sector and rotated about its
    sector-centroid point by two Gaussian angles (sigma 0.05 mrad) about the
    radial and tangential axes.  Focal surface: a spherical cap of radius
    1 m, vertex at z = 5.3257 m, centre of curvature below, aperture 0.6 m.
    Parameters: 8 primary b_i, 8 secondary b_i, 2 tilts per panel (144).
    Fields: n_fields angles evenly spaced in [0, max_field_deg], or the
    explicit list fields_deg.
    """
    rng = np.random.default_rng(seed)
    pri, sec = SC_PRIMARY, SC_SECONDARY
    bp = conic_taylor(pri["R"], pri["k"], pri["rn"])
    bs = conic_taylor(sec["R"], sec["k"], sec["rn"])
    if coeff_scale is not None:
        cs = np.asarray(coeff_scale)
        bp, bs = bp * cs[:8], bs * cs[8:]
    pan_p = _ring_panels(pri["r_in"], pri["r_out"], 3.3127, 16, 32)
    pan_s = _ring_panels(sec["r_in"], sec["r_out"], 1.5588, 8, 16)
    npan = len(pan_p) + len(pan_s)
    if tilts is None:
        tilts = rng.normal(0.0, sigma_tilt, size=(npan, 2))
    if fields_deg is None:
        groups = np.radians(np.linspace(0.0, max_field_deg, n_fields))
    else:
        groups = np.radians(np.asarray(fields_deg, dtype=np.float64))
    return _sc_two_mirror("schwarzschild_couder", 1.0, pan_p, pan_s, tilts, bp, bs, groups,
                          precision, seed)


GCT_SCALE = 2.283 / 5.6   # effective focal length of the small SC over that of SC_PRIMARY / SC_SECONDARY


def _sc_structure(scale, pri_rim_r, sec_rim_r, sec_z, focal_z, focal_ap):
    """Absorbing telescope structure of the small SC (§3, Figure 1 c, f, i:
    its spot diagram shows mast and truss shadows): four masts (r = 5 cm)
    from outside the primary's rim at z = 0 to just outside and above the
    secondary's rim, a ring of four trusses (r = 3 cm) joining the masts at
    half height, and a camera body (an absorbing box) under the focal cap."""
    vols = []
    r0, z0 = pri_rim_r + 0.13, 0.0
    r1, z1 = sec_rim_r + 0.08, sec_z + 0.1
    mid = []
    for kk in range(4):
        ph = math.radians(45.0 + 90.0 * kk)
        e = np.array([math.cos(ph), math.sin(ph), 0.0])
        base = r0 * e + np.array([0.0, 0.0, z0])
        top = r1 * e + np.array([0.0, 0.0, z1])
        ax = top - base
        vols.append(new_volume(ROLE_OBSCURATION, SHAPE_CYLINDER, Q=frame_from_axes(ax), c=base,
                               p=[0.05, float(np.linalg.norm(ax))]))
        mid.append(0.5 * (base + top))
    for kk in range(4):
        a, b = mid[kk], mid[(kk + 1) % 4]
        ax = b - a
        vols.append(new_volume(ROLE_OBSCURATION, SHAPE_CYLINDER, Q=frame_from_axes(ax), c=a,
                               p=[0.03, float(np.linalg.norm(ax))]))
    # the focal cap reaches down to focal_z - (1 - sqrt(1 - (ap/R)^2)) R, R = scale
    cap_depth = scale * (1.0 - math.sqrt(1.0 - (focal_ap / scale) ** 2))
    top_z = focal_z - cap_depth - 0.02
    vols.append(new_volume(ROLE_OBSCURATION, SHAPE_BOX, c=(0.0, 0.0, top_z - 0.18),
                           p=[focal_ap + 0.015, focal_ap + 0.015, 0.18]))
    return vols


def gct_sc(seed=SEED_BASE + 9, sigma_tilt=5e-5, n_fields=16, max_field_deg=4.4, tilts=None,
           precision=32, fields_deg=None, structure=True):
    """A second Schwarzschild-Couder scale, of the small-sized telescope the
    paper models beside the SCT (§3, Figure 1 c, f, i): the two-mirror
    design of schwarzschild_couder scaled by GCT_SCALE (effective focal
    length 2.283 m; every length, including each sag coefficient b_i of the
    normalised form, times the scale; primary 3.94 m across, secondary
    2.20 m, 3.42 m above it), the primary cut into six petals and the
    secondary in one piece, each rotated about its sector-centroid point by
    two Gaussian angles (sigma_tilt) about the radial and tangential axes,
    plus the absorbing masts, trusses and camera body of _sc_structure
    (structure=False leaves them out).  Parameters: 8 primary b_i, 8
    secondary b_i, 2 tilts per panel (7 panels).  Fields: n_fields angles
    evenly spaced in [0, max_field_deg], or the explicit list fields_deg.
    """
    rng = np.random.default_rng(seed)
    s = GCT_SCALE
    pri, sec = SC_PRIMARY, SC_SECONDARY
    bp = s * conic_taylor(pri["R"], pri["k"], pri["rn"])
    bs = s * conic_taylor(sec["R"], sec["k"], sec["rn"])
    pan_p = [(pri["r_in"] * s, pri["r_out"] * s, k * math.pi / 3.0, (k + 1) * math.pi / 3.0)
             for k in range(6)]
    pan_s = [(0.0, sec["r_out"] * s, 0.0, 2.0 * math.pi)]
    npan = len(pan_p) + len(pan_s)
    if tilts is None:
        tilts = rng.normal(0.0, sigma_tilt, size=(npan, 2))
    if fields_deg is None:
        groups = np.radians(np.linspace(0.0, max_field_deg, n_fields))
    else:
        groups = np.radians(np.asarray(fields_deg, dtype=np.float64))
    extra = []
    if structure:
        extra = _sc_structure(s, pri["r_out"] * s, sec["r_out"] * s, sec["z"] * s, SC_FOCAL_Z * s,
                              0.6 * s)
    sc = _sc_two_mirror("gct_sc", s, pan_p, pan_s, tilts, bp, bs, groups, precision, seed, extra)
    sc.meta["structure"] = list(range(sc.n_volumes - len(extra), sc.n_volumes))
    return sc


# ================================================================ C5
def sweep(seed=SEED_BASE + 5, n_dc=128, n_sc=128, field_deg=1.0, log10_n=(5.0, 7.0), precision=32):
    """Batched design sweep: seeded variants of the Davies-Cotton and
    Schwarzschild-Couder scenes at one field angle.

    Each variant perturbs its family's baseline: facet radii and aspheric
    coefficients times (1 + N(0, 1e-3)), tilts drawn with the family's sigma
    (0.1 mrad DC, 0.05 mrad SC).  Photon counts are round(10^U(lo, hi)).
    Returns (list of Scene, int64 counts); DC variants first.
    """
    rng = np.random.default_rng(seed)
    variants = []
    for v in range(n_dc):
        rs = 1.0 + rng.normal(0.0, 1e-3, 198)
        tl = rng.normal(0.0, 1e-4, (198, 2))
        variants.append(davies_cotton(seed=seed + 1 + v, fields_deg=(field_deg,), radius_scale=rs, tilts=tl,
                                      precision=precision))
    for v in range(n_sc):
        cs = 1.0 + rng.normal(0.0, 1e-3, 16)
        tl = rng.normal(0.0, 5e-5, (72, 2))
        variants.append(schwarzschild_couder(seed=seed + 1 + n_dc + v, fields_deg=(field_deg,), coeff_scale=cs,
                                             tilts=tl, precision=precision))
    counts = np.rint(10.0 ** rng.uniform(log10_n[0], log10_n[1], n_dc + n_sc)).astype(np.int64)
    return variants, counts


def device_rays(scene, n, seed, group=0, device="cuda"):
    """Parallel beam of n photons for one field of a telescope scene,
    generated on the device with torch's seeded generator (the same beam
    geometry as Scene.rays, a different random stream).  Returns a dict of
    device tensors in the scene precision plus int32 groups."""
    import torch
    if "beam" not in scene.meta and "cells" in scene.meta:
        return _device_cone_rays(scene, n, seed, group, device)
    b = scene.meta["beam"]
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    f64 = torch.float64
    u1 = torch.rand(n, generator=gen, device=device, dtype=f64)
    u2 = torch.rand(n, generator=gen, device=device, dtype=f64)
    th = float(scene.groups[group])
    d = (math.sin(th), 0.0, -math.cos(th))
    ph = (2.0 * math.pi) * u2
    if b["kind"] == "disc_perp":
        r = b["r_out"] * torch.sqrt(u1)
        px, py = r * torch.cos(ph), r * torch.sin(ph)
        e1 = (math.cos(th), 0.0, math.sin(th))
        ox = -b["back"] * d[0] + px * e1[0]
        oy = py
        oz = -b["back"] * d[2] + px * e1[2]
    elif b["kind"] == "annulus_z0":
        r = torch.sqrt(b["r_in"] ** 2 + u1 * (b["r_out"] ** 2 - b["r_in"] ** 2))
        ox = r * torch.cos(ph) - b["back"] * d[0]
        oy = r * torch.sin(ph)
        oz = torch.full_like(u1, -b["back"] * d[2])
    else:
        raise ValueError(f"no device beam for {b['kind']}")
    dt = torch.float32 if scene.precision == 32 else torch.float64
    out = dict(ox=ox.to(dt), oy=oy.to(dt), oz=oz.to(dt))
    for k, val in zip(("dx", "dy", "dz"), d):
        out[k] = torch.full((n,), val, dtype=dt, device=device)
    out["group"] = torch.full((n,), int(group), dtype=torch.int32, device=device)
    return out


def _device_cone_rays(scene, n, seed, group, device):
    """The concentrator's photons for one incidence angle on the device: the
    recipe of its host generator (a uniformly chosen cone, a uniform point
    of its entrance hexagon, a uniform azimuth), from torch's seeded
    generator."""
    import torch
    m = scene.meta
    f64 = torch.float64
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    cells = torch.as_tensor(np.asarray(m["cells"]), dtype=f64, device=device)
    a_in, L, zl = float(m["control"][3][0]), float(m["length"]), float(m["z_launch"])
    k = torch.randint(0, len(cells), (n,), generator=gen, device=device)
    half = torch.tensor([a_in, a_in * 2.0 / math.sqrt(3.0)], dtype=f64, device=device)
    pts, need = [], n
    while need > 0:
        c = (torch.rand(int(need * 1.4) + 64, 2, generator=gen, device=device, dtype=f64) * 2.0 - 1.0) * half
        ok = torch.ones(len(c), dtype=torch.bool, device=device)
        for ang in (0.0, math.pi / 3.0, 2.0 * math.pi / 3.0):
            ok &= (c[:, 0] * math.cos(ang) + c[:, 1] * math.sin(ang)).abs() <= a_in
        c = c[ok][:need]
        pts.append(c)
        need -= len(c)
    pts = torch.cat(pts)
    ph = torch.rand(n, generator=gen, device=device, dtype=f64) * (2.0 * math.pi)
    th = float(scene.groups[group])
    dx, dy = math.sin(th) * torch.cos(ph), math.sin(th) * torch.sin(ph)
    dz = torch.full((n,), -math.cos(th), dtype=f64, device=device)
    s = (zl - L) / math.cos(th)
    dt = torch.float32 if scene.precision == 32 else torch.float64
    out = dict(ox=(cells[k, 0] + pts[:, 0] - s * dx).to(dt), oy=(cells[k, 1] + pts[:, 1] - s * dy).to(dt),
               oz=(L - s * dz).to(dt), dx=dx.to(dt), dy=dy.to(dt), dz=dz.to(dt))
    out["group"] = torch.full((n,), int(group), dtype=torch.int32, device=device)
    return out


# ================================================================ C4
def cpc_bezier(a=25.0, theta_c_deg=30.0):
    """Cubic Bezier control points of the compound parabolic concentrator.

    The CPC wall is a parabola with focus at the opposite exit edge and axis
    tilted by the cut-off angle; as a quadratic Bezier its control points are
    the exit edge, the intersection of the end tangents and the entrance
    edge; degree elevation gives the cubic.  Returns [(rho, z)] x 4 (mm).
    """
    th = math.radians(theta_c_deg)
    ap = a * math.sin(th)                       # exit half-width
    L = (a + ap) / math.tan(th)                 # length
    # tangent at the exit edge: direction of the parabola at (ap, 0)
    # parabola in the (rho, z) plane, focus F = (-ap, 0), axis direction
    # w = (sin th, -cos th) (pointing from the vertex away from the opening)
    P0 = np.array([ap, 0.0]); P2 = np.array([a, L])
    F = np.array([-ap, 0.0]); w = np.array([math.sin(th), -math.cos(th)])

    def tangent(P):
        # for a parabola the tangent bisects the focal radius and the axis line
        r = (P - F) / np.linalg.norm(P - F)
        t = r - w
        return t / np.linalg.norm(t)
    t0, t2 = tangent(P0), tangent(P2)
    # P1 = P0 + s t0 = P2 + q t2
    A = np.stack([t0, -t2], 1)
    s, _ = np.linalg.solve(A, P2 - P0)
    P1 = P0 + s * t0
    Q1 = P0 + 2.0 / 3.0 * (P1 - P0)
    Q2 = P2 + 2.0 / 3.0 * (P1 - P2)
    return [tuple(P0), tuple(Q1), tuple(Q2), tuple(P2)], L


def hex_concentrator(seed=SEED_BASE + 3, n_rows=8, n_cols=8, reflectivity=0.92,
                     angles_deg=None, control=None, window=True, precision=32):
    """8 x 8 array of hexagonal cones with a cubic Bezier CPC profile (mm).

    Cone cross-section at height z is a regular hexagon of inradius rho(z):
    12.5 mm at the exit (z = 0), 25 mm at the entrance (z = L = 64.95 mm);
    the baseline profile is the degree-elevated ideal CPC for a 30 deg
    cut-off.  Walls are zero-thickness mirrors (front inside, R = 0.92).
    Cones sit on a hex lattice of 50 mm pitch, alternate rows offset 25 mm.
    A 2 mm PMMA window (n = 1.49) with its bottom 1 mm above the entrance
    covers the array; each exit hexagon is a focal surface and the rest of
    the z = 0 plane absorbs.  Parameters: the interior control points
    (rho1, z1, rho2, z2), shared by every cone.
    """
    ctrl, L = cpc_bezier()
    if control is not None:
        c4 = list(control)
        ctrl = [ctrl[0], (c4[0], c4[1]), (c4[2], c4[3]), ctrl[3]]
    pitch = 50.0
    row = pitch * math.sqrt(3.0) / 2.0
    cells = []
    for j in range(n_rows):
        for i in range(n_cols):
            cells.append((pitch * i + 0.5 * pitch * (j % 2), row * j))
    cells = np.array(cells)
    cells -= cells.mean(axis=0)
    vols = []
    flat_ctrl = [v for pt in ctrl for v in pt]
    for (x, y) in cells:
        vols.append(new_volume(ROLE_MIRROR, SHAPE_HEXCONE, c=(x, y, 0.0), p=flat_ctrl,
                               reflectivity=reflectivity, shape_param=0))
    for (x, y) in cells:
        vols.append(new_volume(ROLE_FOCAL, SHAPE_PLANE, OUTLINE_HEX, c=(x, y, 0.0), o=[ctrl[0][0]]))
    span = float(np.abs(cells).max()) + 2 * pitch
    vols.append(new_volume(ROLE_OBSCURATION, SHAPE_PLANE, OUTLINE_RECT, c=(0.0, 0.0, 0.0),
                           o=[span, span]))
    if window:
        vols.append(new_volume(ROLE_LENS, SHAPE_BOX, c=(0.0, 0.0, L + 2.0), p=[span, span, 1.0],
                               n_inside=1.49))
    params = [ctrl[1][0], ctrl[1][1], ctrl[2][0], ctrl[2][1]]
    names = ["rho1", "z1", "rho2", "z2"]
    if angles_deg is None:
        angles_deg = np.arange(0.0, 45.0 + 1e-9, 0.5)
    groups = np.radians(np.asarray(angles_deg, dtype=np.float64))
    z_launch = L + 8.0
    a_in = ctrl[3][0]

    def rays(scene, n, s, gsel, phi_fixed=None):
        rng2 = np.random.default_rng(s)
        out = []
        for g in gsel:
            th = scene.groups[g]
            k = rng2.integers(0, len(cells), size=n)
            # uniform point in a hexagon of inradius a_in (flats normal to x)
            pts = np.empty((n, 2)); filled = 0
            R = a_in * 2.0 / math.sqrt(3.0)
            while filled < n:
                m = 2 * (n - filled) + 16
                cand = (rng2.random((m, 2)) * 2.0 - 1.0) * np.array([a_in, R])
                ok = np.ones(m, bool)
                for ang in (0.0, math.pi / 3.0, 2.0 * math.pi / 3.0):
                    ok &= np.abs(cand[:, 0] * math.cos(ang) + cand[:, 1] * math.sin(ang)) <= a_in
                cand = cand[ok][: n - filled]
                pts[filled:filled + len(cand)] = cand
                filled += len(cand)
            ph = rng2.random(n) * 2.0 * np.pi if phi_fixed is None else np.full(n, phi_fixed)
            d = np.stack([math.sin(th) * np.cos(ph), math.sin(th) * np.sin(ph),
                          np.full(n, -math.cos(th))], 1)
            P = np.stack([cells[k, 0] + pts[:, 0], cells[k, 1] + pts[:, 1], np.full(n, L)], 1)
            sdist = (z_launch - L) / (-d[:, 2])
            o = P - sdist[:, None] * d
            out.append((o[:, 0], o[:, 1], o[:, 2], d[:, 0], d[:, 1], d[:, 2], np.full(n, g)))
        cols = [np.concatenate(c) for c in zip(*out)]
        return _pack_rays(scene.precision, *cols)

    return _finish("hex_concentrator", vols, params, names, precision, 32, seed, L, groups, rays,
                   n_cones=len(cells), length=L, control=ctrl, cells=cells, z_launch=z_launch)


# ================================================================ small test scenes
def empty_scene(precision=64):
    """No volumes: every photon leaves the scene."""
    def rays(scene, n, s, groups):
        rng = np.random.default_rng(s)
        v = rng.normal(size=(n, 3)); v /= np.linalg.norm(v, axis=1)[:, None]
        return _pack_rays(scene.precision, *rng.normal(size=(3, n)), v[:, 0], v[:, 1], v[:, 2],
                          np.zeros(n))
    return Scene("empty", np.zeros(0, dtype=VOLUME_DTYPE), np.zeros(0), [], precision, 16,
                 SEED_BASE, 1.0, np.array([0.0]), rays)


def window_slab(n_index=1.49, thickness=2.0, precision=64, seed=SEED_BASE + 7, absorption_length=0.0):
    """A lone lens slab with normal-incidence photons (Fresnel statistics;
    bulk absorption with the given absorption length, 0 = none)."""
    vols = [new_volume(ROLE_LENS, SHAPE_BOX, c=(0, 0, 0), p=[100.0, 100.0, thickness / 2],
                       n_inside=n_index)]
    vols[0]["p"][15] = absorption_length

    def rays(scene, n, s, groups):
        rng = np.random.default_rng(s)
        x, y = rng.uniform(-10, 10, size=(2, n))
        return _pack_rays(scene.precision, x, y, np.full(n, 10.0), np.zeros(n), np.zeros(n),
                          -np.ones(n), np.zeros(n))
    return _finish("window_slab", vols, [], [], precision, 64, seed, thickness, [0.0], rays)


# ================================================================ refractive optics
CAUCHY_PMMA = (1.4720, 3.2e-15)   # n(lam) = A + B / lam^2, lam in m: a PMMA-like synthetic law


def cauchy_index(lam, A=CAUCHY_PMMA[0], B=CAUCHY_PMMA[1]):
    """Refractive index of the lens material at wavelength lam (m)."""
    return A + B / (lam * lam)


def _dispersive(v):
    """Give a lens volume the material's dispersion law (p[13] = A,
    p[14] = B of n = A + B / lam^2): photons that carry their own wavelength
    are refracted with n(lam); n_inside stays the index at the scene's
    wavelength for photons that carry none."""
    v["p"][13], v["p"][14] = CAUCHY_PMMA
    return v


def with_wavelengths(scene, rays, lam_min=300e-9, lam_max=600e-9, seed=None):
    """The same photons, each given a wavelength drawn uniformly from
    [lam_min, lam_max] (a continuous spectrum traced in one bundle; rounded
    to the scene precision)."""
    rng = np.random.default_rng(scene.seed + 77 if seed is None else seed)
    out = dict(rays)
    out["lam"] = _q(rng.uniform(lam_min, lam_max, len(rays["ox"])), scene.precision)
    return out


def aspheric_lens(seed=SEED_BASE + 10, lam=400e-9, a=0.25, R=-0.5, k=None, edge=0.01,
                  fields_deg=(0.0, 1.0, 2.0, 3.0), design_lam=400e-9, coeffs=None, precision=32,
                  absorption_length=0.0):
    """A plano-aspheric singlet of the kind used as refracting optics for
    Cherenkov and fluorescence light (§1, §2.1: lenses and refractions), at
    wavelength lam: index cauchy_index(lam); everything else is fixed by the
    design wavelength, so scenes at several wavelengths differ only in the
    index.  Front face: the asphere z = T + S(r), r <= a, with S the Taylor
    coefficients b_1..b_8 (normalised form, rn = a) of the conic of vertex
    radius R (< 0: convex towards the sky) and conic constant
    k = -1/n_design^2 unless given; a refracting lens face whose front side
    (air) faces +z.  Back face: the plane z = 0, r <= a, front side facing
    -z.  Rim: an absorbing cylinder r = a, 0 <= z <= edge.  Centre
    thickness T = edge - S(a).  Focal plane: a disc of radius 0.08 m at the
    paraxial back focus of the design wavelength, z = -(f - T/n) with
    f = |R| / (n - 1).  absorption_length (m, 0 = none): bulk absorption
    of the glass, on both faces.  Parameters: the 8 front-face coefficients.
    Photons: parallel beams at the field angles over a disc of radius a
    normal to the beam, launched 1 m before the origin."""
    n_design = cauchy_index(design_lam)
    if k is None:
        k = -1.0 / n_design ** 2
    b = conic_taylor(R, k, a) if coeffs is None else np.asarray(coeffs, dtype=np.float64)
    T = edge - float(np.sum(b))
    f = abs(R) / (n_design - 1.0)
    z_focal = -(f - T / n_design)
    n = cauchy_index(lam)
    vols = [new_volume(ROLE_LENS, SHAPE_ASPHERE, OUTLINE_DISC, c=(0.0, 0.0, T), p=[a] + list(b), o=[a],
                       n_inside=n, shape_param=0),
            new_volume(ROLE_LENS, SHAPE_PLANE, OUTLINE_DISC, Q=np.diag([1.0, -1.0, -1.0]), c=(0.0, 0.0, 0.0),
                       o=[a], n_inside=n),
            new_volume(ROLE_OBSCURATION, SHAPE_CYLINDER, c=(0.0, 0.0, 0.0), p=[a, edge]),
            new_volume(ROLE_FOCAL, SHAPE_PLANE, OUTLINE_DISC, c=(0.0, 0.0, z_focal), o=[0.08])]
    for v in vols[:2]:
        v["p"][15] = absorption_length
        _dispersive(v)
    names = [f"front_b{i}" for i in range(1, 9)]
    return _finish("aspheric_lens", vols, list(b), names, precision, 16, seed, f,
                   np.radians(np.asarray(fields_deg, dtype=np.float64)), _dish_rays(a, 1.0),
                   lam=lam, n_index=n, thickness=T, design_focus=f, focal_z=z_focal,
                   beam=dict(kind="disc_perp", r_out=a, back=1.0))


def lens_wavelengths(lams=tuple(np.linspace(300e-9, 600e-9, 16)), **kw):
    """The aspheric singlet at each wavelength of lams (one scene per
    wavelength; the same surfaces, the index of that wavelength)."""
    return [aspheric_lens(lam=float(l), **kw) for l in lams]


def fresnel_lens(seed=SEED_BASE + 11, lam=400e-9, a=0.25, n_zones=10, bfl=2.0, t_base=0.01,
                 fields_deg=(0.0, 0.5, 1.0, 1.5), design_lam=400e-9, precision=32, absorption_length=0.0):
    """A flat Fresnel lens of the kind proposed for fluorescence and
    Cherenkov telescopes (§1), at wavelength lam (index cauchy_index(lam);
    the surfaces are fixed by the design wavelength).  Front: the plane
    z = 0, r <= a, refracting, air above.  Back: n_zones annular zones of
    equal width; zone j (r_j <= r <= r_j+1) is a refracting facet starting
    at the groove bottom z = -t_base at r_j and shaped so that light
    parallel to the axis inside the glass meets the focus F = (0, 0, z_F),
    z_F = -t_base - bfl, with one optical path: n (-z) + |P - F| = const_j,
    i.e. the hyperboloid of eccentricity n (k = -n^2) with vertex radius
    (n - 1) w_j, w_j the height of its virtual vertex above F, given as the
    Taylor coefficients b_1..b_8 (normalised form, rn = a) in a frame whose
    +z faces the air below.  Between zones (and at the rim) absorbing
    cylinders close the glass: the risers (draft facets) and the rim.
    Focal plane: a disc of radius 0.08 m at z_F.  absorption_length (m,
    0 = none): bulk absorption of the glass.  Parameters: the 8
    coefficients of each zone."""
    n0 = cauchy_index(design_lam)
    k = -n0 * n0
    z_F = -t_base - bfl
    edges = np.linspace(0.0, a, n_zones + 1)

    def delta(R, r):   # sag of the hyperboloid (k = -n0^2) of vertex radius R, >= 0
        return r * r / (R + math.sqrt(R * R - (1.0 + k) * r * r))

    vols = [new_volume(ROLE_LENS, SHAPE_PLANE, OUTLINE_DISC, c=(0.0, 0.0, 0.0), o=[a],
                       n_inside=cauchy_index(lam))]
    params, names, tops = [], [], []
    for j in range(n_zones):
        r0, r1 = edges[j], edges[j + 1]
        # w: virtual vertex height above F with z_F + w + delta((n0 - 1) w, r0) = -t_base
        w = -t_base - z_F
        for _ in range(200):
            f = z_F + w + delta((n0 - 1.0) * w, r0) + t_base
            h = 1e-7 * w
            fp = (z_F + w + h + delta((n0 - 1.0) * (w + h), r0) + t_base - f) / h
            w_new = w - f / fp
            if abs(w_new - w) < 1e-15 * w:
                w = w_new
                break
            w = w_new
        R = (n0 - 1.0) * w
        b = conic_taylor(-R, k, a)            # sag -delta in the frame facing down
        off = len(params)
        params.extend(b)
        names.extend(f"zone{j}_b{i}" for i in range(1, 9))
        outline, o = (OUTLINE_DISC, [r1]) if r0 == 0.0 else (OUTLINE_ANNULUS, [r0, r1])
        vols.append(new_volume(ROLE_LENS, SHAPE_ASPHERE, outline, Q=np.diag([1.0, -1.0, -1.0]),
                               c=(0.0, 0.0, z_F + w), p=[a] + list(b), o=o, n_inside=cauchy_index(lam),
                               shape_param=off))
        tops.append(z_F + w + delta(R, r1))
    for j in range(n_zones):
        r1 = edges[j + 1]
        top = tops[j] if j < n_zones - 1 else 0.0    # riser up to the zone's outer height; the rim to z = 0
        vols.append(new_volume(ROLE_OBSCURATION, SHAPE_CYLINDER, c=(0.0, 0.0, -t_base), p=[r1, top + t_base]))
    vols.append(new_volume(ROLE_FOCAL, SHAPE_PLANE, OUTLINE_DISC, c=(0.0, 0.0, z_F), o=[0.08]))
    for v in vols:
        if v["role"] == ROLE_LENS:
            v["p"][15] = absorption_length
            _dispersive(v)
    return _finish("fresnel_lens", vols, params, names, precision, 16, seed, bfl,
                   np.radians(np.asarray(fields_deg, dtype=np.float64)), _dish_rays(a, 1.0),
                   lam=lam, n_index=cauchy_index(lam), focal_z=z_F, zone_edges=edges.tolist(),
                   groove_tops=tops, beam=dict(kind="disc_perp", r_out=a, back=1.0))


ALL = {
    "single_mirror": single_mirror,
    "davies_cotton": davies_cotton,
    "schwarzschild_couder": schwarzschild_couder,
    "hex_concentrator": hex_concentrator,
    "lst_parabolic": lst_parabolic,
    "gct_sc": gct_sc,
    "aspheric_lens": aspheric_lens,
    "fresnel_lens": fresnel_lens,
}
