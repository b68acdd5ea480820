"""Pins of the FP64 oracle against values the mathematics fixes.

Each test checks the oracle against something other than itself: published
known-answer vectors, closed forms of textbook optics, invariants, special
cases that reduce to a different formula, and brute force.  Function-level
status:

* Philox4x32-10 .................. pinned (published known-answer vectors)
* sphere cap + plane + reflection  pinned (exact transverse aberration, C1)
* asphere ........................ pinned (conic foci; sphere special case; Newton)
* Fresnel / Snell / TIR .......... pinned (sine/tangent laws, reciprocity, slab)
* Bezier hexagonal cone .......... pinned (ideal 2D CPC acceptance step)
* hex facets, tilts, cylinders ... pinned (Davies-Cotton vertex focusing, occlusion)
* optical path / arrival figures . pinned (ideal paraboloid: stigmatic and isochronous,
                                    path = start height + f; Davies-Cotton spread = the
                                    spread of its sphere's sag over the hit radii)
* non-sequential search .......... pinned (brute force vs culled, symmetry, conservation)
* forced sequences / duals ....... pinned (closed-form derivative of C1; FD vs duals)
* segment outlines, boundary distances, grazing(), the mirror draw, tilted
  geometry(P), gradient_eff_w, the self-hit rule: pinned in
  test_oracle_pins_segments.py
* full-scene figures (DC PSF, SC RMS, cone efficiency curves): parity unpinned
  (the paper prints no values and its figures are not reproducible here).
"""
import math
import os

import numpy as np
import pytest

import scenes

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ Philox
def test_philox_known_answers(orc):
    rows = [l.split() for l in open(os.path.join(GOLD, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(x, 16) for x in r]
        out = orc.philox4x32_10(w[0:4], w[4:6])
        assert [int(x) for x in out] == w[6:10]


def test_philox_uniform_chi2(orc):
    # 2^14 draws into 64 bins; chi2 with 63 dof has mean 63, sd ~11.2
    vals = np.array([orc.draw(12345, i, e) for i in range(4096) for e in range(4)], dtype=np.uint64)
    counts = np.bincount((vals >> np.uint64(26)).astype(np.int64), minlength=64)
    exp = len(vals) / 64.0
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert 20 < chi2 < 120


# ------------------------------------------------------------------ C1: spherical mirror
def aberration(h, R, zf):
    """Exact radial hit coordinate at the plane z = zf of a ray parallel to the axis at height h
    reflected by the sphere of radius R with vertex at z = 0 (law of reflection, sphere geometry)."""
    th = np.arcsin(h / R)
    z1 = R - R * np.cos(th)
    s = (zf - z1) / np.cos(2 * th)
    return h - s * np.sin(2 * th)


def test_c1_exact_transverse_aberration(orc):
    sc = scenes.single_mirror()
    r = sc.rays(20000)
    rec = orc.trace(sc, r)
    h = np.hypot(r["ox"], r["oy"])
    foc = rec["fate"] == scenes.FATE_FOCUSED
    assert foc.sum() > 18000
    ph = np.arctan2(r["oy"], r["ox"])
    radial = rec["pos"][foc, 0] * np.cos(ph[foc]) + rec["pos"][foc, 1] * np.sin(ph[foc])
    expect = aberration(h[foc], 16.0, 8.0)
    assert np.max(np.abs(radial - expect)) <= 1e-12 * sc.l_ref
    assert np.allclose(rec["pos"][foc, 2], 8.0, atol=1e-12)
    # tabulated values of the same closed form (survey appendix A1)
    assert aberration(np.array([0.5, 1.0, 2.0]), 16.0, 8.0) == pytest.approx(
        [-2.4467814577e-4, -1.9704300679e-3, -1.6192533369e-2], rel=1e-9)


def test_c1_shadow_is_exact(orc):
    sc = scenes.single_mirror()
    r = sc.rays(20000)
    rec = orc.trace(sc, r)
    h = np.hypot(r["ox"], r["oy"])
    inner = h < 0.5
    assert np.all(rec["fate"][inner] == scenes.FATE_ABSORBED)
    assert np.all(rec["last_vol"][inner] == 1)
    assert np.all(rec["n_events"][inner] == 1)
    assert np.all(rec["fate"][~inner] == scenes.FATE_FOCUSED)
    assert np.all(rec["n_events"][~inner] == 2)


def test_c1_rms_matches_quadrature(orc):
    from scipy.integrate import quad
    R, a, a0 = 16.0, 2.0, 0.5
    num, _ = quad(lambda h: aberration(np.array(h), R, 8.0) ** 2 * 2 * np.pi * h, a0, a,
                  epsabs=0, epsrel=1e-12)
    exact = math.sqrt(num / (np.pi * (a * a - a0 * a0)))
    assert exact == pytest.approx(8.3019722641e-3, rel=1e-9)
    sc = scenes.single_mirror()
    rec = orc.trace(sc, sc.rays(100000))
    fig = orc.figures(rec, 1)[0]
    # MC sampling spread of the RMS at 1e5 photons is 0.17% (1 sigma)
    assert abs(fig["rms"] / exact - 1.0) < 5 * 0.0017
    assert abs(fig["cx"]) < 1e-4 and abs(fig["cy"]) < 1e-4


def _mirror_only():
    sc = scenes.single_mirror()
    sc.volumes = sc.volumes[:1].copy()
    return sc


def test_c1_paraxial_focus_and_marginal_crossing(orc):
    sc = _mirror_only()
    R = 16.0
    h = np.array([0.01, 0.02, 2.0])
    r = scenes.make_rays(64, h, np.zeros(3), np.full(3, 20.0), np.zeros(3), np.zeros(3),
                         -np.ones(3), np.zeros(3))
    rec = orc.trace(sc, r)
    assert np.all(rec["fate"] == scenes.FATE_EXITED)
    p, d = rec["pos"], rec["dir"]
    # axial crossing of each reflected ray
    s = -p[:, 0] / d[:, 0]
    zc = p[:, 2] + s * d[:, 2]
    th = np.arcsin(h / R)
    assert zc == pytest.approx(R - R / (2 * np.cos(th)), abs=1e-12)
    # paraxial limit: crossing -> R/2, transverse aberration -> -h^3 / (2 R^2)
    assert zc[0] == pytest.approx(R / 2, abs=1e-4)
    x8 = p[:2, 0] + (8.0 - p[:2, 2]) / d[:2, 2] * d[:2, 0]
    assert x8 / (-h[:2] ** 3 / (2 * R * R)) == pytest.approx([1.0, 1.0], abs=1e-5)
    # caustic (nephroid): the reflected ray of the ray at angle theta touches the
    # envelope at (R sin^3 th, R - R cos th (3/2 - cos^2 th))
    th2 = th[2]
    cx, cz = R * np.sin(th2) ** 3, R - R * np.cos(th2) * (1.5 - np.cos(th2) ** 2)
    dist = abs((cx - p[2, 0]) * d[2, 2] - (cz - p[2, 2]) * d[2, 0])
    assert dist < 1e-12


def test_c1_max_events_suspends(orc):
    sc = scenes.single_mirror()
    sc.max_events = 1
    r = sc.rays(2000)
    rec = orc.trace(sc, r)
    h = np.hypot(r["ox"], r["oy"])
    assert np.all(rec["fate"][h < 0.5] == scenes.FATE_ABSORBED)
    assert np.all(rec["fate"][h >= 0.5] == scenes.FATE_SUSPENDED)


def test_empty_scene_and_failed(orc):
    sc = scenes.empty_scene()
    r = sc.rays(100)
    rec = orc.trace(sc, r)
    assert np.all(rec["fate"] == scenes.FATE_EXITED)
    r["dx"][3] = np.nan
    rec = orc.trace(sc, r)
    assert rec["fate"][3] == scenes.FATE_FAILED


def test_non_unit_directions_are_refused(orc):
    """A photon's direction is a unit vector (§2.1): a scaled one is refused
    (FAILED) rather than traced with wrong path lengths; one off by rounding
    is traced as usual."""
    sc = scenes.single_mirror()
    r = sc.rays(200)
    base = orc.trace(sc, r)
    for k in ("dx", "dy", "dz"):
        r[k][7] *= 2.0
        r[k][9] *= 1.0 + 2e-7
    rec = orc.trace(sc, r)
    assert rec["fate"][7] == scenes.FATE_FAILED
    assert rec["fate"][9] == base["fate"][9] != scenes.FATE_FAILED
    keep = np.ones(len(r["ox"]), bool)
    keep[[7, 9]] = False
    assert np.array_equal(rec["fate"][keep], base["fate"][keep])


# ------------------------------------------------------------------ Fresnel / Snell
def test_fresnel_closed_forms(orc):
    n = 1.49
    # normal incidence: ((n-1)/(n+1))^2
    assert orc.fresnel(1.0, 1.0, n) == pytest.approx(((n - 1) / (n + 1)) ** 2, rel=1e-14)
    assert orc.fresnel(1.0, 1.0, n) == pytest.approx(0.038725181852, rel=1e-10)
    # Fresnel's sine and tangent laws (a different form of the same physics)
    for deg in (10.0, 30.0, 50.0, 70.0, 85.0):
        ti = math.radians(deg)
        tt = math.asin(math.sin(ti) / n)
        rs = math.sin(ti - tt) ** 2 / math.sin(ti + tt) ** 2
        rp = math.tan(ti - tt) ** 2 / math.tan(ti + tt) ** 2
        assert orc.fresnel(math.cos(ti), 1.0, n) == pytest.approx(0.5 * (rs + rp), rel=1e-12)
        # reciprocity: same reflectance on the way back
        assert orc.fresnel(math.cos(tt), n, 1.0) == pytest.approx(0.5 * (rs + rp), rel=1e-12)
    assert orc.fresnel(math.cos(math.radians(30.0)), 1.0, n) == pytest.approx(0.040226252, rel=1e-7)
    # Brewster: p-reflectance vanishes, R = Rs/2 = cos^2(2 theta_B)/2
    tb = math.atan(n)
    assert orc.fresnel(math.cos(tb), 1.0, n) == pytest.approx(0.5 * math.cos(2 * tb) ** 2, rel=1e-12)
    assert math.degrees(tb) == pytest.approx(56.132820891, abs=1e-8)
    # total internal reflection beyond the critical angle from inside
    tc = math.asin(1.0 / n)
    assert math.degrees(tc) == pytest.approx(42.155184251, abs=1e-8)
    assert orc.fresnel(math.cos(tc + 1e-6), n, 1.0) == 1.0
    assert orc.fresnel(math.cos(tc - 1e-3), n, 1.0) < 1.0


def test_slab_transmission_statistics(orc):
    sc = scenes.window_slab()
    r = sc.rays(200000)
    rec = orc.trace(sc, r)
    R0 = ((1.49 - 1) / 2.49) ** 2
    T = (1 - R0) / (1 + R0)               # incoherent slab with all internal reflections
    assert T == pytest.approx(0.925437098, rel=1e-8)
    down = rec["dir"][:, 2] < 0
    frac = down.mean()
    sig = math.sqrt(T * (1 - T) / len(down))
    assert abs(frac - T) < 5 * sig
    assert np.all(rec["fate"] == scenes.FATE_EXITED)
    # at normal incidence the direction never changes except in sign
    assert np.allclose(np.abs(rec["dir"][:, 2]), 1.0, atol=1e-15)


@pytest.mark.parametrize("L", [1.0, 4.0])
def test_absorbing_slab_transmission_statistics(orc, L):
    """Slab of thickness d = 2 and absorption length L at normal incidence,
    all internal reflections incoherent: each crossing survives with
    q = exp(-d / L), so transmission (1 - R0)^2 q / (1 - R0^2 q^2),
    reflection R0 + (1 - R0)^2 R0 q^2 / (1 - R0^2 q^2), the rest absorbed."""
    sc = scenes.window_slab(absorption_length=L)
    r = sc.rays(200000)
    rec = orc.trace(sc, r)
    R0 = ((1.49 - 1) / 2.49) ** 2
    q = math.exp(-2.0 / L)
    T = (1 - R0) ** 2 * q / (1 - R0 ** 2 * q ** 2)
    Rf = R0 + (1 - R0) ** 2 * R0 * q ** 2 / (1 - R0 ** 2 * q ** 2)
    n = len(r["ox"])
    ex = rec["fate"] == scenes.FATE_EXITED
    down = ex & (rec["dir"][:, 2] < 0)
    up = ex & (rec["dir"][:, 2] > 0)
    for frac, p in ((down.mean(), T), (up.mean(), Rf), ((rec["fate"] == scenes.FATE_ABSORBED).mean(), 1 - T - Rf)):
        assert abs(frac - p) < 5 * math.sqrt(p * (1 - p) / n), (frac, p)
    assert np.all(ex | (rec["fate"] == scenes.FATE_ABSORBED))


def test_slab_oblique_snell_displacement(orc):
    sc = scenes.window_slab()
    n, half = 1.49, 1.0
    th = np.radians([5.0, 20.0, 40.0, 60.0, 80.0])
    k = len(th)
    r = scenes.make_rays(64, np.zeros(k), np.zeros(k), np.full(k, 10.0), np.sin(th), np.zeros(k),
                         -np.cos(th), np.zeros(k))
    # photon ids 0..k-1: keep only photons transmitted straight through (2 events)
    rec = orc.trace(sc, r, log=True)
    tt = np.arcsin(np.sin(th) / n)
    x1 = (10.0 - half) * np.tan(th)
    through = (rec["n_events"] == 2) & (rec["dir"][:, 2] < 0)
    assert through.sum() >= 3
    assert rec["pos"][through, 0] == pytest.approx(x1[through] + 2 * half * np.tan(tt[through]), abs=1e-12)
    assert rec["dir"][through, 0] == pytest.approx(np.sin(th[through]), abs=1e-14)
    # the refracted direction inside obeys n1 (d x n) = n2 (t x n): sin(t) = sin(i)/n
    assert np.all(rec["log"]["act"][through, :2] == 1)


# ------------------------------------------------------------------ Bezier cone / CPC
def test_cpc_control_points_are_the_parabola():
    ctrl, L = scenes.cpc_bezier()
    th = math.radians(30.0)
    ap = 25.0 * math.sin(th)
    f = ap * (1 + math.sin(th))
    F = np.array([-ap, 0.0])
    w = np.array([math.sin(th), -math.cos(th)])
    P = np.array(ctrl)
    for s in np.linspace(0, 1, 41):
        b = np.array([(1 - s) ** 3, 3 * (1 - s) ** 2 * s, 3 * (1 - s) * s * s, s ** 3])
        X = b @ P
        # focus-directrix property: |X - F| = 2f - (X - F).w, with w the unit
        # axis pointing from the focus away from the vertex side of the opening
        assert np.linalg.norm(X - F) == pytest.approx(2 * f - np.dot(X - F, w), abs=1e-9)
    assert L == pytest.approx(64.9519052838, abs=1e-9)
    assert P[1] == pytest.approx([20.8333333, 14.4337567], abs=1e-6)
    assert P[2] == pytest.approx([25.0, 36.0843918], abs=1e-6)


@pytest.mark.parametrize("deg,expect", [(0.0, 1.0), (10.0, 1.0), (20.0, 1.0), (29.0, 1.0),
                                        (29.9, 1.0), (30.1, 0.0), (31.0, 0.0), (40.0, 0.0)])
def test_ideal_cpc_acceptance_step(orc, deg, expect):
    """In the plane through the axis normal to a pair of flats, the hexagonal cone's
    section is the 2D CPC, which passes every ray below the cut-off and none above."""
    sc = scenes.hex_concentrator(n_rows=1, n_cols=1, reflectivity=1.0, window=False, precision=64)
    sc.volumes["c"][:, :2] = 0.0
    L = sc.meta["length"]
    n = 400
    x = np.linspace(-24.9, 24.9, n)
    th = math.radians(deg)
    d = np.array([math.sin(th), 0.0, -math.cos(th)])
    o = np.stack([x, np.zeros(n), np.full(n, L)], 1) - 5.0 * d
    r = scenes.make_rays(64, o[:, 0], o[:, 1], o[:, 2], np.full(n, d[0]), np.zeros(n),
                         np.full(n, d[2]), np.zeros(n))
    rec = orc.trace(sc, r)
    frac = np.mean(rec["fate"] == scenes.FATE_FOCUSED)
    assert frac == expect


# ------------------------------------------------------------------ asphere
def _asphere_scene(b, rn, r_out, precision=64):
    v = scenes.new_volume(scenes.ROLE_MIRROR, scenes.SHAPE_ASPHERE, scenes.OUTLINE_DISC,
                          p=[rn] + list(b), o=[r_out], reflectivity=1.0)
    sc = scenes.single_mirror()
    sc.volumes = np.array([v], dtype=scenes.VOLUME_DTYPE)
    sc.max_events = 4
    return sc


def test_asphere_conic_foci(orc):
    """Ellipsoidal mirror: a ray from one focus reflects through the other."""
    R, k, rn = 10.0, -0.5, 2.0
    b = scenes.conic_taylor(R, k, rn)
    sc = _asphere_scene(b, rn, 2.0)
    a = R / (1 + k)
    e = math.sqrt(-k)
    f1, f2 = a * (1 - e), a * (1 + e)
    rng = np.random.default_rng(5)
    n = 500
    rr, ph = 1.9 * np.sqrt(rng.random(n)), 2 * np.pi * rng.random(n)
    target = np.stack([rr * np.cos(ph), rr * np.sin(ph), np.zeros(n)], 1)
    o = np.tile([0.0, 0.0, f1], (n, 1))
    d = target - o
    d[:, 2] -= 0.5  # aim below the vertex plane; the mirror is met first on the way
    d /= np.linalg.norm(d, axis=1)[:, None]
    r = scenes.make_rays(64, o[:, 0], o[:, 1], o[:, 2], d[:, 0], d[:, 1], d[:, 2], np.zeros(n))
    rec = orc.trace(sc, r)
    assert np.all(rec["fate"] == scenes.FATE_EXITED) and np.all(rec["n_events"] == 1)
    p, q = rec["pos"], rec["dir"]
    w = np.array([0.0, 0.0, f2]) - p
    miss = np.linalg.norm(np.cross(w, q), axis=1)
    assert miss.max() < 1e-9


def test_asphere_sphere_special_case(orc):
    """With the Taylor coefficients of a sphere, hits equal the exact sphere cap."""
    R, rn = 38.0, 4.8
    b = scenes.conic_taylor(R, 0.0, rn)
    sa = _asphere_scene(b, rn, 4.8)
    ss = _asphere_scene(b, rn, 4.8)
    ss.volumes["shape"] = scenes.SHAPE_SPHERE
    ss.volumes["p"][0, :] = 0.0
    ss.volumes["p"][0, 0] = 1.0 / R
    rng = np.random.default_rng(9)
    n = 2000
    x, y = rng.uniform(-3.3, 3.3, size=(2, n))
    th = rng.uniform(0, 0.3, n); ph = rng.uniform(0, 2 * np.pi, n)
    d = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), -np.cos(th)], 1)
    r = scenes.make_rays(64, x, y, np.full(n, 3.0), d[:, 0], d[:, 1], d[:, 2], np.zeros(n))
    ra, rs = orc.trace(sa, r), orc.trace(ss, r)
    assert np.array_equal(ra["n_events"], rs["n_events"])
    hit = ra["n_events"] >= 1
    assert hit.sum() > 1000
    assert np.max(np.abs(ra["pos"][hit] - rs["pos"][hit])) < 1e-10
    assert np.max(np.abs(ra["dir"][hit] - rs["dir"][hit])) < 1e-10


def test_asphere_root_matches_newton(orc):
    """Root isolation agrees with plain Newton from the vertex-plane guess."""
    sc = scenes.schwarzschild_couder(precision=64, sigma_tilt=0.0)
    b = sc.params[:8]
    rn = 4.83
    one = _asphere_scene(b, rn, 4.83)
    rng = np.random.default_rng(3)
    n = 300
    x, y = rng.uniform(-3.4, 3.4, size=(2, n))
    d = np.stack([rng.normal(0, 0.05, n), rng.normal(0, 0.05, n), -np.ones(n)], 1)
    d /= np.linalg.norm(d, axis=1)[:, None]
    oz = np.full(n, 5.0)
    r = scenes.make_rays(64, x, y, oz, d[:, 0], d[:, 1], d[:, 2], np.zeros(n))
    rec = orc.trace(one, r)
    hit = rec["n_events"] == 1
    t = (oz - 0.0) / -d[:, 2]
    for _ in range(50):
        X = np.stack([x, y, oz], 1) + t[:, None] * d
        u = (X[:, 0] ** 2 + X[:, 1] ** 2) / rn ** 2
        S = sum(b[i] * u ** (i + 1) for i in range(8))
        dS = sum((i + 1) * b[i] * u ** i for i in range(8))
        g = X[:, 2] - S
        gp = d[:, 2] - dS * 2 * (X[:, 0] * d[:, 0] + X[:, 1] * d[:, 1]) / rn ** 2
        t = t - g / gp
    X = np.stack([x, y, oz], 1) + t[:, None] * d
    inside = np.hypot(X[:, 0], X[:, 1]) <= 4.83
    assert np.array_equal(hit, inside)
    assert np.max(np.abs(rec["pos"][hit] - X[hit])) < 1e-11


# ------------------------------------------------------------------ segmented dish, shadowing
def test_dc_vertex_rays_meet_at_focus(orc):
    """Davies-Cotton: facets on the sphere of radius f aimed at 2f send an axial ray
    through each facet vertex exactly to (0, 0, f)."""
    sc = scenes.davies_cotton(sigma_tilt=0.0, precision=64)
    nf = sc.meta["n_facets"]
    c = sc.volumes["c"][:nf]
    n = nf
    r = scenes.make_rays(64, c[:, 0], c[:, 1], np.full(n, 40.0), np.zeros(n), np.zeros(n),
                         -np.ones(n), np.zeros(n))
    rec = orc.trace(sc, r)
    foc = rec["fate"] == scenes.FATE_FOCUSED
    # rays through |x|,|y| <= 1.5 m hit the camera lid first; masts block a few more
    assert foc.sum() > 150
    assert np.max(np.hypot(rec["pos"][foc, 0], rec["pos"][foc, 1])) < 1e-9
    assert np.allclose(rec["pos"][foc, 2], 28.0, atol=1e-12)


def _ray_cyl_first_t(o, d, base, axis, radius, length):
    """Independent ray / finite-cylinder intersection (smallest positive t or inf)."""
    a = axis / np.linalg.norm(axis)
    w = o - base
    dp = d - np.dot(d, a) * a
    wp = w - np.dot(w, a) * a
    A, B, C = dp @ dp, 2 * dp @ wp, wp @ wp - radius ** 2
    disc = B * B - 4 * A * C
    if A == 0 or disc < 0:
        return np.inf
    best = np.inf
    for t in ((-B - math.sqrt(disc)) / (2 * A), (-B + math.sqrt(disc)) / (2 * A)):
        z = np.dot(w + t * d, a)
        if t > 0 and 0 <= z <= length:
            best = min(best, t)
    return best


def test_dc_shadowing_is_exact_occlusion(orc):
    sc = scenes.davies_cotton()
    r = sc.rays(4000, groups=[0])
    rec = orc.trace(sc, r)
    nf = sc.meta["n_facets"]
    lid = nf + 1
    x, y = r["ox"], r["oy"]
    under = (np.abs(x) <= 1.5 - 1e-9) & (np.abs(y) <= 1.5 - 1e-9)
    assert np.all(rec["last_vol"][under] == lid) and np.all(rec["n_events"][under] == 1)
    masts = range(nf + 6, nf + 10)
    for i in np.nonzero(~under)[0]:
        o = np.array([x[i], y[i], r["oz"][i]]); d = np.array([r["dx"][i], r["dy"][i], r["dz"][i]])
        tm = min(_ray_cyl_first_t(o, d, sc.volumes["c"][m], sc.volumes["Q"][m][6:9],
                                  0.1, sc.volumes["p"][m][1]) for m in masts)
        if np.isfinite(tm) and o[2] + tm * d[2] > 3.0:       # above every facet
            assert rec["fate"][i] == scenes.FATE_ABSORBED and rec["n_events"][i] == 1
            assert rec["last_vol"][i] in masts


def test_gct_is_the_sc_design_scaled(orc):
    """Geometric optics has no length scale: the small SC (every length of
    the SC design times s, the primary cut into other panels) with its
    structure removed and no tilts images the launch points s*o exactly
    where the SC images o, times s, with the same exit directions and fates
    (panel boundaries aside, which have measure zero)."""
    s = scenes.GCT_SCALE
    big = scenes.schwarzschild_couder(precision=64, sigma_tilt=0.0)
    small = scenes.gct_sc(precision=64, sigma_tilt=0.0, structure=False)
    r = big.rays(300, groups=[0, 4, 9, 15])
    r2 = {k: (v * s if k in ("ox", "oy", "oz") else v) for k, v in r.items()}
    a, b = orc.trace(big, r), orc.trace(small, r2)
    assert np.array_equal(a["fate"], b["fate"])
    assert np.array_equal(a["n_events"], b["n_events"])
    ok = a["fate"] == scenes.FATE_FOCUSED
    assert ok.sum() > 600
    assert np.abs(b["pos"][ok] - s * a["pos"][ok]).max() < 1e-12 * small.l_ref
    assert np.abs(b["dir"][ok] - a["dir"][ok]).max() < 1e-12
    assert np.abs(b["opl"][ok] - s * a["opl"][ok]).max() < 1e-11 * small.l_ref


def test_gct_structure_shadow_is_exact_occlusion(orc):
    """On-axis photons launched outside the secondary's radius can meet only
    the masts and trusses before the primary: a photon whose line crosses a
    mast or truss (independent ray / cylinder test) is absorbed there at its
    first event, at the nearest one, and no other photon is."""
    sc = scenes.gct_sc(precision=64)
    r = sc.rays(3000, groups=[0])
    rec = orc.trace(sc, r)
    st = sc.meta["structure"]
    cyl = [m for m in st if sc.volumes["shape"][m] == scenes.SHAPE_CYLINDER]
    assert len(cyl) == 8
    sec_r = scenes.SC_SECONDARY["r_out"] * scenes.GCT_SCALE
    rad = np.hypot(r["ox"], r["oy"])
    n_hit = 0
    for i in np.nonzero(rad > sec_r + 1e-6)[0]:
        o = np.array([r["ox"][i], r["oy"][i], r["oz"][i]])
        d = np.array([r["dx"][i], r["dy"][i], r["dz"][i]])
        ts = [_ray_cyl_first_t(o, d, sc.volumes["c"][m], sc.volumes["Q"][m][6:9],
                               sc.volumes["p"][m][0], sc.volumes["p"][m][1]) for m in cyl]
        first_struct = rec["fate"][i] == scenes.FATE_ABSORBED and rec["n_events"][i] == 1 \
            and rec["last_vol"][i] in st
        if np.isfinite(min(ts)):
            n_hit += 1
            assert first_struct and rec["last_vol"][i] == cyl[int(np.argmin(ts))], i
        else:
            assert not first_struct, i
    assert n_hit > 100


@pytest.mark.parametrize("lam", [300e-9, 400e-9, 600e-9])
def test_lens_paraxial_back_focus_is_the_thick_lens_value(orc, lam):
    """Plano-convex thick lens, curved face (vertex radius |R| = 0.5 m)
    towards a beam parallel to the axis: paraxial rays cross the axis at the
    back focal distance f - T/n behind the plane face, f = |R| / (n - 1), with
    n = A + B / lam^2 (A = 1.4720, B = 3.2e-15 m^2).  The crossing of rays at
    heights h and 2h, extrapolated to h = 0 (error O(h^4)), meets it to 1e-9 m;
    the conic constant changes only the higher orders."""
    sc = scenes.aspheric_lens(precision=64, lam=lam)
    T = sc.volumes["c"][0][2]
    n = 1.4720 + 3.2e-15 / lam ** 2
    expect = -(0.5 / (n - 1.0) - T / n)
    zs = []
    for h in (0.002, 0.004):
        m = 16   # the same ray under 16 ids: keep one that Fresnel reflection spared
        r = scenes.make_rays(64, np.full(m, h), np.zeros(m), np.full(m, 1.0), np.zeros(m), np.zeros(m),
                             -np.ones(m), np.zeros(m))
        rec = orc.trace(sc, r)
        ok = np.nonzero((rec["fate"] == scenes.FATE_FOCUSED) & (rec["n_events"] == 3))[0]
        assert len(ok) > 8
        i = ok[0]
        x, z = rec["pos"][i, 0], rec["pos"][i, 2]
        zs.append(z - x * rec["dir"][i, 2] / rec["dir"][i, 0])
    assert abs((4 * zs[0] - zs[1]) / 3 - expect) < 1e-9
    assert abs(zs[0] - expect) > 1e-7          # the extrapolation is needed: aberration is resolved


def test_per_photon_wavelength_back_focus(orc):
    """One bundle, each photon with its own wavelength (300, 400, 600 nm) in
    a singlet built for 500 nm (its fixed index is that of 500 nm): each
    photon crosses the axis at the thick-lens back focus of its own index
    n = A + B / lam^2, not of the scene's, and photons without wavelengths
    use the fixed index."""
    sc = scenes.aspheric_lens(precision=64, lam=500e-9)
    T = sc.volumes["c"][0][2]
    lams = (300e-9, 400e-9, 600e-9)
    m = 16
    zs = {l: [] for l in lams}
    for h in (0.002, 0.004):
        k = m * len(lams)
        r = scenes.make_rays(64, np.full(k, h), np.zeros(k), np.full(k, 1.0), np.zeros(k), np.zeros(k),
                             -np.ones(k), np.zeros(k))
        r["lam"] = np.repeat(lams, m)
        rec = orc.trace(sc, r, wavelengths=True)
        for j, l in enumerate(lams):
            sel = np.arange(j * m, (j + 1) * m)
            ok = sel[(rec["fate"][sel] == scenes.FATE_FOCUSED) & (rec["n_events"][sel] == 3)]
            assert len(ok) > 8
            i = ok[0]
            x, z = rec["pos"][i, 0], rec["pos"][i, 2]
            zs[l].append(z - x * rec["dir"][i, 2] / rec["dir"][i, 0])
    for l in lams:
        n = 1.4720 + 3.2e-15 / l ** 2
        expect = -(0.5 / (n - 1.0) - T / n)
        assert abs((4 * zs[l][0] - zs[l][1]) / 3 - expect) < 1e-9, l
    # without wavelengths every photon sees the scene's fixed (500 nm) index
    r = scenes.make_rays(64, np.full(m, 0.002), np.zeros(m), np.full(m, 1.0), np.zeros(m), np.zeros(m),
                         -np.ones(m), np.zeros(m))
    r["lam"] = np.full(m, 300e-9)
    a, b = orc.trace(sc, r), orc.trace(sc, r, wavelengths=True)
    assert not np.allclose(a["pos"], b["pos"], atol=1e-6)
    c = orc.trace(scenes.aspheric_lens(precision=64, lam=300e-9), r)
    assert np.abs(c["pos"] - b["pos"]).max() < 1e-12


def test_lens_spot_grows_away_from_the_design_wavelength(orc):
    """Longitudinal chromatic aberration of the singlet: the focal plane sits
    at the paraxial focus of 400 nm, and the index rises towards the blue, so
    the focus moves away from the plane and the on-axis spot grows
    monotonically from 400 to 300 nm (the focal shift itself is pinned by the
    paraxial test above)."""
    rms = []
    for lam in (400e-9, 375e-9, 350e-9, 325e-9, 300e-9):
        sc = scenes.aspheric_lens(precision=64, lam=lam, fields_deg=(0.0,))
        r = sc.rays(4000)
        rec = orc.trace(sc, r)
        m = rec["fate"] == scenes.FATE_FOCUSED
        x, y = rec["pos"][m, 0], rec["pos"][m, 1]
        rms.append(np.sqrt(np.mean((x - x.mean()) ** 2 + (y - y.mean()) ** 2)))
    assert all(b > a for a, b in zip(rms, rms[1:])), rms


def test_fresnel_zones_are_stigmatic_and_isochronous(orc):
    """Each zone of the Fresnel lens is a surface of one optical path
    n (-z) + |P - F| from the plane to the focus F, so at the design
    wavelength every on-axis photon that crosses the plane and one facet
    lands on F (to the 8-term Taylor truncation of its hyperboloid, far
    below 1e-9 m here), every zone carries light, and within a zone all such
    paths from the launch plane z = 1 m have one optical length."""
    sc = scenes.fresnel_lens(precision=64, fields_deg=(0.0,))
    r = sc.rays(6000)
    rec = orc.trace(sc, r, log=True)
    ok = (rec["fate"] == scenes.FATE_FOCUSED) & (rec["n_events"] == 3)
    assert ok.mean() > 0.85
    zF = sc.meta["focal_z"]
    assert np.abs(rec["pos"][ok, 0]).max() < 1e-9 and np.abs(rec["pos"][ok, 1]).max() < 1e-9
    assert np.allclose(rec["pos"][ok, 2], zF, atol=1e-12)
    zone = rec["log"]["vol"][ok, 1]
    nz = len(sc.meta["zone_edges"]) - 1
    assert set(np.unique(zone)) == set(range(1, nz + 1))
    opl = rec["opl"][ok]
    means = []
    for j in range(1, nz + 1):
        o = opl[zone == j]
        assert o.max() - o.min() < 1e-9
        means.append(o.mean())
    assert np.ptp(means) > 1e-4          # zones differ: each has its own constant


def test_fresnel_spot_grows_away_from_the_design_wavelength(orc):
    """Off the design wavelength the zones no longer meet one focus: the
    on-axis spot grows monotonically from 400 nm towards the blue."""
    rms = []
    for lam in (400e-9, 375e-9, 350e-9, 325e-9, 300e-9):
        sc = scenes.fresnel_lens(precision=64, lam=lam, fields_deg=(0.0,))
        r = sc.rays(3000)
        rec = orc.trace(sc, r)
        m = rec["fate"] == scenes.FATE_FOCUSED
        x, y = rec["pos"][m, 0], rec["pos"][m, 1]
        rms.append(np.sqrt(np.mean((x - x.mean()) ** 2 + (y - y.mean()) ** 2)))
    assert rms[0] < 1e-8 and all(b > a for a, b in zip(rms, rms[1:])), rms


# ------------------------------------------------------------------ search invariants
@pytest.mark.parametrize("name,n", [("davies_cotton", 300), ("schwarzschild_couder", 100),
                                    ("hex_concentrator", 20), ("lst_parabolic", 300),
                                    ("gct_sc", 200), ("aspheric_lens", 300), ("fresnel_lens", 300)])
def test_brute_force_equals_culled(orc, name, n):
    sc = scenes.ALL[name]()
    r = sc.rays(n)
    a = orc.trace(sc, r, culled=True)
    b = orc.trace(sc, r, culled=False)
    for k in ("fate", "n_events", "last_vol", "seq_hash"):
        assert np.array_equal(a[k], b[k])
    assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["dir"], b["dir"])


@pytest.mark.parametrize("name", ["single_mirror", "davies_cotton", "schwarzschild_couder",
                                  "hex_concentrator", "lst_parabolic", "gct_sc", "aspheric_lens",
                                  "fresnel_lens"])
def test_photon_conservation(orc, name):
    sc = scenes.ALL[name]()
    r = sc.rays(200)
    rec = orc.trace(sc, r)
    c = np.bincount(rec["fate"], minlength=6)
    assert c[0] == 0 and c[1:].sum() == len(r["ox"])
    assert np.all(rec["n_events"] <= sc.max_events)


def test_sc_mirror_symmetry(orc):
    sc = scenes.schwarzschild_couder(precision=64, sigma_tilt=0.0)
    r = sc.rays(300, groups=[8])
    m = dict(r)
    m["oy"] = -r["oy"]; m["dy"] = -r["dy"]
    a, b = orc.trace(sc, r), orc.trace(sc, m)
    assert np.array_equal(a["fate"], b["fate"]) and np.array_equal(a["n_events"], b["n_events"])
    ok = a["fate"] == scenes.FATE_FOCUSED
    assert ok.sum() > 150
    assert np.max(np.abs(a["pos"][ok, 0] - b["pos"][ok, 0])) < 1e-9
    assert np.max(np.abs(a["pos"][ok, 1] + b["pos"][ok, 1])) < 1e-9


def test_sc_plate_scale_first_order():
    """First-order focal length of the two-mirror system from the mirror powers."""
    p1, p2 = 2 / scenes.SC_PRIMARY["R"], 2 / scenes.SC_SECONDARY["R"]
    d = scenes.SC_SECONDARY["z"]
    F = 1 / (p1 + p2 - d * p1 * p2)
    assert F == pytest.approx(5.6, rel=2e-4)


def test_sc_paraxial_plate_scale(orc):
    """Unsegmented two-mirror system, thin ring of rays round the axis at 0.1 deg:
    the image on the paraxial focal plane (z = 8.4 - F (1 - d phi1)) sits at
    F tan(theta), F = 5.6 m, with a correction growing as the ring radius squared."""
    sc = scenes.schwarzschild_couder(precision=64, sigma_tilt=0.0)
    b = sc.params
    vp = scenes.new_volume(scenes.ROLE_MIRROR, scenes.SHAPE_ASPHERE, scenes.OUTLINE_DISC,
                           p=[4.83] + list(b[:8]), o=[4.83])
    vs = scenes.new_volume(scenes.ROLE_MIRROR, scenes.SHAPE_ASPHERE, scenes.OUTLINE_DISC,
                           Q=np.diag([1.0, -1.0, -1.0]), c=(0, 0, 8.4), p=[2.7] + list(b[8:16]),
                           o=[2.7])
    sc.volumes = np.array([vp, vs], dtype=scenes.VOLUME_DTYPE)
    sc.max_events = 2
    p1, p2, dd = 2 / scenes.SC_PRIMARY["R"], 2 / scenes.SC_SECONDARY["R"], 8.4
    F = 1 / (p1 + p2 - dd * p1 * p2)
    z_img = 8.4 - F * (1 - dd * p1)
    th = math.radians(0.1)
    d = np.array([math.sin(th), 0.0, -math.cos(th)])
    rel = []
    for rr in (0.01, 0.02):
        n = 64
        ph = np.arange(n) * 2 * np.pi / n
        P = np.stack([rr * np.cos(ph), rr * np.sin(ph), np.zeros(n)], 1)
        o = P - 7.5 * d
        r = scenes.make_rays(64, o[:, 0], o[:, 1], o[:, 2], np.full(n, d[0]), np.zeros(n),
                             np.full(n, d[2]), np.zeros(n))
        rec = orc.trace(sc, r)
        assert np.all(rec["fate"] == scenes.FATE_SUSPENDED) and np.all(rec["n_events"] == 2)
        p, q = rec["pos"], rec["dir"]
        x = p[:, 0] + (z_img - p[:, 2]) / q[:, 2] * q[:, 0]
        rel.append(x.mean() / (F * math.tan(th)) - 1.0)
    # what is left is third-order distortion (order theta^2 ~ 3e-6) plus the
    # aperture term growing as r^2
    assert abs(rel[0]) < 2e-5
    assert 0.0 < rel[1] - rel[0] < 2e-5


# ------------------------------------------------------------------ forced sequences, duals, FD
def test_c1_dual_derivative_matches_closed_form(orc):
    sc = scenes.single_mirror()
    r = sc.rays(2000)
    rec = orc.trace(sc, r, log=True)
    foc = rec["fate"] == scenes.FATE_FOCUSED
    dpos, _, st = orc.forced_jac(sc, r, rec, sc.params, 0, 1)
    assert np.all(st[foc] == 0)
    h = np.hypot(r["ox"], r["oy"])
    ph = np.arctan2(r["oy"], r["ox"])
    eps = 1e-5
    dx = (aberration(h, 16.0 + eps, 8.0) - aberration(h, 16.0 - eps, 8.0)) / (2 * eps)
    got = dpos[:, 0, 0] * np.cos(ph) + dpos[:, 1, 0] * np.sin(ph)
    assert np.max(np.abs(got[foc] - dx[foc])) < 1e-8 * np.max(np.abs(dx[foc]))
    # forced re-evaluation at the recorded parameters reproduces the trace
    pos, _, st = orc.forced(sc, r, rec, sc.params)
    assert np.max(np.abs(pos[foc] - rec["pos"][foc])) < 1e-12


@pytest.mark.parametrize("name,n,idx", [("schwarzschild_couder", 80, [0, 3, 9, 15, 16, 17, 60, 161]),
                                        ("hex_concentrator", 5, [0, 1, 2, 3]),
                                        ("davies_cotton", 200, [0, 5, 198, 199, 250])])
def test_duals_match_forced_fd(orc, name, n, idx):
    sc = scenes.ALL[name](precision=64) if name != "single_mirror" else scenes.ALL[name]()
    r = sc.rays(n)
    rec = orc.trace(sc, r, log=True)
    foc = rec["fate"] == scenes.FATE_FOCUSED
    idx = [i for i in idx if i < len(sc.params)]
    for j in idx:
        dpos, ddir, st = orc.forced_jac(sc, r, rec, sc.params, j, 1)
        pj = sc.params[j]
        h = 1e-7 if "tilt" in sc.param_names[j] else 1e-6 * max(abs(pj), 1e-3 * sc.l_ref)
        P1, P2 = sc.params.copy(), sc.params.copy()
        P1[j] += h; P2[j] -= h
        a1, b1, s1 = orc.forced(sc, r, rec, P1)
        a2, b2, s2 = orc.forced(sc, r, rec, P2)
        m = foc & (st == 0) & (s1 == 0) & (s2 == 0)
        assert m.sum() > 0.5 * foc.sum()
        fd = (a1 - a2) / (2 * h)
        fdd = (b1 - b2) / (2 * h)
        scale = max(np.max(np.abs(fd[m])), 1e-12)
        assert np.max(np.abs(dpos[m, :, 0] - fd[m])) <= 1e-4 * scale + 1e-9, sc.param_names[j]
        scd = max(np.max(np.abs(fdd[m])), 1e-12)
        assert np.max(np.abs(ddir[m, :, 0] - fdd[m])) <= 1e-4 * scd + 1e-9, sc.param_names[j]


# ------------------------------------------------------------------ optical path, arrival figures
def test_ideal_paraboloid_is_stigmatic_and_isochronous(orc):
    """A paraboloid z = r^2 / (4 f) (an asphere with b1 only) sends every
    on-axis ray to its focus, and every path from the start plane z0 to the
    focus has the length z0 + f (the distance to the focus equals the
    distance to the directrix z = -f)."""
    f, rn, a, z0 = 8.0, 2.0, 2.0, 20.0
    b = np.zeros(8)
    b[0] = rn * rn / (4.0 * f)
    sc = _asphere_scene(b, rn, a)
    foc = scenes.new_volume(scenes.ROLE_FOCAL, scenes.SHAPE_PLANE, scenes.OUTLINE_DISC,
                            Q=np.diag([1.0, -1.0, -1.0]), c=(0.0, 0.0, f), o=[0.05])
    sc.volumes = np.concatenate([sc.volumes, np.array([foc], dtype=scenes.VOLUME_DTYPE)])
    rng = np.random.default_rng(11)
    n = 2000
    r, ph = np.sqrt(0.01 + (a * a - 0.01) * rng.random(n)), 2 * np.pi * rng.random(n)
    rays = scenes.make_rays(64, r * np.cos(ph), r * np.sin(ph), np.full(n, z0), np.zeros(n), np.zeros(n),
                            -np.ones(n), np.zeros(n))
    rec = orc.trace(sc, rays)
    assert np.all(rec["fate"] == scenes.FATE_FOCUSED)
    assert np.abs(rec["pos"][:, :2]).max() < 1e-9
    assert np.abs(rec["opl"] - (z0 + f)).max() < 1e-9
    arr = orc.arrival_figures(rec, 1)[0]
    assert arr["focused"] == n and abs(arr["mean"] - (z0 + f)) < 1e-9 and arr["rms"] < 1e-9


def test_parabolic_dish_is_isochronous_davies_cotton_is_not(orc):
    """On axis, a Davies-Cotton dish (facets on a sphere of radius f about the
    focus) delays a ray at radius r by about the sphere's sag f - sqrt(f^2 -
    r^2) less than the ray at the centre: its arrival spread is the spread of
    that sag over the hit radii.  The segmented paraboloid removes it up to
    the facets' own curvature."""
    f = 28.0
    dc, lst = scenes.davies_cotton(precision=64, sigma_tilt=0.0), scenes.lst_parabolic(precision=64, sigma_tilt=0.0)
    r_dc, r_lst = dc.rays(3000, groups=[0]), lst.rays(3000, groups=[0])
    rd, rl = orc.trace(dc, r_dc), orc.trace(lst, r_lst)
    ad, al = orc.arrival_figures(rd, 1)[0], orc.arrival_figures(rl, 1)[0]
    m = rd["fate"] == scenes.FATE_FOCUSED
    rr = np.hypot(r_dc["ox"][m], r_dc["oy"][m])
    sag = f - np.sqrt(f * f - rr * rr)
    print(f"on-axis arrival spread: DC {ad['rms']:.4e} m (sag spread {sag.std():.4e} m), "
          f"parabolic {al['rms']:.4e} m")
    assert abs(ad["rms"] - sag.std()) < 0.03 * sag.std()
    assert al["rms"] < 0.02 * ad["rms"]
