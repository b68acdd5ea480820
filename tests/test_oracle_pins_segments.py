"""More pins of the FP64 oracle: segment outlines, boundary distances and
the grazing classification, the mirror absorption draw, the tilted
geometry of forced sequences, the derivative of the weighted collection,
and the rule for meeting the face just left.

Each test names the plausible mistake it catches:

* mirror draw ............ absorbed fraction 1 - R (an inverted comparison gives R)
* sector / hex outlines .. membership against independent polar and polygon tests;
                           the SC annulus covered once by its 48 panels; hexagon
                           orientation through the real facet frames; 198 flat hexagons
                           cover 86.4 % of the 12 m disc (apothem / circumradius swap)
* outline_bdist .......... exact boundary distance where the closed form is the
                           distance to a supporting line, a lower bound elsewhere
* grazing() .............. each of its criteria switched on by a constructed photon,
                           and off for a well-conditioned one
* geometry(P) ............ forced sequences at the scene's parameters reproduce the
                           traced tilted DC and SC positions (a wrong rotation order or
                           sign moves them)
* gradient_eff_w ......... central differences of the forced weighted collection
* self-hit rule .......... whispering-gallery bounces inside a spherical bowl (a
                           reflection stays on its side); a refracted photon meets the
                           same spherical face again from the glass side after a chord
                           of length 2 R cos(theta_t)
"""
import math

import numpy as np
import pytest

import scenes

FOC, ABS, EXI = scenes.FATE_FOCUSED, scenes.FATE_ABSORBED, scenes.FATE_EXITED


def _scene(vols, max_events=16, l_ref=1.0, seed=scenes.SEED_BASE + 21):
    sc = scenes.empty_scene(64)
    sc.volumes = np.array(vols, dtype=scenes.VOLUME_DTYPE)
    sc.max_events = max_events
    sc.l_ref = l_ref
    sc.seed = seed
    return sc


def _down(x, y, z, group=None):
    n = len(x)
    return scenes.make_rays(64, x, y, np.full(n, z) if np.isscalar(z) else z, np.zeros(n), np.zeros(n),
                            -np.ones(n), np.zeros(n) if group is None else group)


# ------------------------------------------------------------------ mirror absorption draw
@pytest.mark.parametrize("R", [0.9, 0.3, 1.0, 0.0])
def test_mirror_absorbs_a_fraction_one_minus_R(orc, R):
    """A flat mirror of reflectivity R hit at normal incidence absorbs each
    photon with probability 1 - R (binomial, 5 sigma)."""
    v = scenes.new_volume(scenes.ROLE_MIRROR, scenes.SHAPE_PLANE, scenes.OUTLINE_DISC, o=[2.0], reflectivity=R)
    sc = _scene([v])
    rng = np.random.default_rng(5)
    n = 40000
    r = _down(rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), 1.0)
    rec = orc.trace(sc, r)
    assert np.all(rec["n_events"] == 1)
    absorbed = rec["fate"] == ABS
    assert np.all(absorbed | (rec["fate"] == EXI))
    frac = absorbed.mean()
    sd = math.sqrt(max(R * (1 - R), 1e-12) / n)
    assert abs(frac - (1.0 - R)) <= 5 * sd, (frac, 1 - R)
    # reflected photons leave straight up
    up = ~absorbed
    if up.any():
        assert np.allclose(rec["dir"][up], [0.0, 0.0, 1.0], atol=0)


# ------------------------------------------------------------------ outlines
def _sector_member(x, y, ra, rb, pa, pb):
    r = np.hypot(x, y)
    ph = np.mod(np.arctan2(y, x), 2 * np.pi)
    return (r >= ra) & (r <= rb) & (ph >= pa) & (ph <= pb)


def _hex_vertices(a):
    """Vertices of the hexagon of apothem a whose flats are perpendicular to
    the local x axis (flats at x = +-a): circumradius 2a/sqrt 3 at 30 + 60 k deg."""
    R = 2 * a / math.sqrt(3)
    ang = np.radians(30 + 60 * np.arange(6))
    return np.stack([R * np.cos(ang), R * np.sin(ang)], 1)


def _in_convex(V, x, y):
    inside = np.ones(len(x), bool)
    for k in range(len(V)):
        a, b = V[k], V[(k + 1) % len(V)]
        cr = (b[0] - a[0]) * (y - a[1]) - (b[1] - a[1]) * (x - a[0])
        inside &= cr >= 0
    return inside


def _edge_dist(V, x, y):
    """Distance from (x, y) to the polygon's boundary (min over edge segments)."""
    d = np.full(len(x), np.inf)
    for k in range(len(V)):
        a, b = V[k], V[(k + 1) % len(V)]
        ab = b - a
        t = np.clip(((x - a[0]) * ab[0] + (y - a[1]) * ab[1]) / (ab @ ab), 0, 1)
        d = np.minimum(d, np.hypot(x - (a[0] + t * ab[0]), y - (a[1] + t * ab[1])))
    return d


def test_sc_primary_panels_tile_the_annulus_once(orc):
    """The 48 primary panels (sector outlines, untilted frame) contain a point
    exactly as the polar test r in [ra, rb], phi in [pa, pb] says, and every
    point of the annulus 2.19-4.83 m lies in exactly one of them."""
    sc = scenes.schwarzschild_couder(precision=64, sigma_tilt=0.0)
    npp = 48
    rng = np.random.default_rng(3)
    r = np.sqrt(rng.uniform(2.0 ** 2, 5.0 ** 2, 60000))
    ph = rng.uniform(0, 2 * np.pi, 60000)
    x, y = r * np.cos(ph), r * np.sin(ph)
    count = np.zeros(len(x), int)
    near = np.zeros(len(x), bool)
    for k in range(npp):
        v = sc.volumes[k]
        assert v["outline"] == scenes.OUTLINE_SECTOR
        ra, rb, pa, pb = v["o"]
        got, _ = orc.outline(v, x, y)
        want = _sector_member(x, y, ra, rb, pa, pb)
        # points within 1e-9 of an edge are decided by rounding; skip them
        phm = np.mod(ph, 2 * np.pi)
        edge = (np.abs(r - ra) < 1e-9) | (np.abs(r - rb) < 1e-9) | \
               (np.abs(phm - pa) * r < 1e-9) | (np.abs(phm - pb) * r < 1e-9)
        near |= edge
        assert np.array_equal(got[~edge], want[~edge]), k
        count += got
    inner = (r >= 2.19) & (r <= 4.83) & ~near
    outer = ((r < 2.19) | (r > 4.83)) & ~near
    assert inner.sum() > 40000
    assert np.all(count[inner] == 1)
    assert np.all(count[outer] == 0)


def test_hex_outline_matches_polygon(orc):
    """Hexagonal outline (flats perpendicular to the local x axis): membership
    equals the point-in-polygon test on its six vertices, and a hexagon rotated
    by 30 degrees would fail it."""
    a = 0.755
    v = scenes.new_volume(scenes.ROLE_MIRROR, scenes.SHAPE_PLANE, scenes.OUTLINE_HEX, o=[a])
    rng = np.random.default_rng(4)
    x, y = rng.uniform(-1, 1, (2, 50000))
    V = _hex_vertices(a)
    got, bd = orc.outline(v, x, y)
    want = _in_convex(V, x, y)
    edge = _edge_dist(V, x, y) < 1e-12
    assert np.array_equal(got[~edge], want[~edge])
    # inside a convex polygon the boundary distance is the distance to the nearest supporting line
    ins = want & ~edge
    assert np.max(np.abs(bd[ins] - _edge_dist(V, x[ins], y[ins]))) < 1e-12
    # outside, the supporting-line distance is a lower bound of the true distance
    out = ~want & ~edge
    assert np.all(bd[out] <= _edge_dist(V, x[out], y[out]) + 1e-12)
    rot30 = _in_convex(_hex_vertices(a) @ np.array([[math.cos(0.5236), math.sin(0.5236)],
                                                    [-math.sin(0.5236), math.cos(0.5236)]]), x, y)
    assert not np.array_equal(got, rot30)


def test_dc_facet_hexagons_through_their_frames(orc):
    """Untilted Davies-Cotton facets, each alone: rays along a facet's axis meet
    its spherical cap at the local (x, y) they start from, so a ray is reflected
    iff (x, y) lies in the hexagon of apothem 0.755 m with flats perpendicular to
    the local x axis (the projection of world x)."""
    sc = scenes.davies_cotton(precision=64, sigma_tilt=0.0)
    V = _hex_vertices(0.755)
    rng = np.random.default_rng(6)
    for k in (0, 17, 100, 197):
        vol = sc.volumes[k]
        Q = vol["Q"].reshape(3, 3)
        c = vol["c"]
        xl, yl = rng.uniform(-0.95, 0.95, (2, 3000))
        start = c[None, :] + xl[:, None] * Q[0] + yl[:, None] * Q[1] + 2.0 * Q[2]
        d = -Q[2]
        n = len(xl)
        r = scenes.make_rays(64, start[:, 0], start[:, 1], start[:, 2], np.full(n, d[0]), np.full(n, d[1]),
                             np.full(n, d[2]), np.zeros(n))
        rec = orc.trace(sc, r, volumes=sc.volumes[k:k + 1])
        hit = rec["n_events"] == 1
        want = _in_convex(V, xl, yl)
        edge = _edge_dist(V, xl, yl) < 1e-9
        assert np.array_equal(hit[~edge], want[~edge]), k
        # reflectivity 0.9: hits are reflected or absorbed, misses exit untouched
        assert np.all(rec["fate"][~hit] == EXI)


def test_dc_flat_hexagons_cover_their_area(orc):
    """198 flat hexagons (apothem 0.755 m) at the Davies-Cotton lattice points,
    facing up: rays straight down, uniform over the 12 m disc, land on a
    facet with probability 198 * 2 sqrt(3) a^2 / (pi 12^2) = 0.8643 (5 sigma)."""
    sc = scenes.davies_cotton(precision=64, sigma_tilt=0.0)
    vols = []
    for k in range(198):
        cx, cy = sc.volumes[k]["c"][:2]
        vols.append(scenes.new_volume(scenes.ROLE_OBSCURATION, scenes.SHAPE_PLANE, scenes.OUTLINE_HEX,
                                      c=(cx, cy, 0.0), o=[0.755]))
    flat = _scene(vols, l_ref=28.0)
    rng = np.random.default_rng(8)
    n = 200000
    rr, ph = 12.0 * np.sqrt(rng.random(n)), 2 * np.pi * rng.random(n)
    rec = orc.trace(flat, _down(rr * np.cos(ph), rr * np.sin(ph), 1.0))
    p = 198 * 2 * math.sqrt(3) * 0.755 ** 2 / (math.pi * 144.0)
    assert abs(p - 0.8643) < 1e-4
    frac = (rec["fate"] == ABS).mean()
    assert abs(frac - p) < 5 * math.sqrt(p * (1 - p) / n), frac
    assert np.all(rec["n_events"] <= 1)


@pytest.mark.parametrize("outline,o", [(scenes.OUTLINE_DISC, [1.3]), (scenes.OUTLINE_ANNULUS, [0.4, 1.3]),
                                       (scenes.OUTLINE_RECT, [0.7, 1.1]),
                                       (scenes.OUTLINE_SECTOR, [0.4, 1.3, 0.3, 1.4])])
def test_outline_boundary_distance_closed_forms(orc, outline, o):
    """Boundary distance of disc, annulus, rectangle and annular sector against
    their closed forms: |r - a|; the nearer circle; for a rectangle the nearer
    side inside and the Euclidean distance outside; for a sector the nearer
    circle or radial edge (exact where the perpendicular foot lies on the edge,
    a lower bound elsewhere)."""
    v = scenes.new_volume(scenes.ROLE_MIRROR, scenes.SHAPE_PLANE, outline, o=o)
    rng = np.random.default_rng(9)
    x, y = rng.uniform(-1.6, 1.6, (2, 40000))
    got_in, bd = orc.outline(v, x, y)
    r = np.hypot(x, y)
    if outline == scenes.OUTLINE_DISC:
        exact = np.abs(r - o[0])
        inside = r <= o[0]
    elif outline == scenes.OUTLINE_ANNULUS:
        exact = np.minimum(np.abs(r - o[0]), np.abs(r - o[1]))
        inside = (r >= o[0]) & (r <= o[1])
    elif outline == scenes.OUTLINE_RECT:
        ex, ey = np.abs(x) - o[0], np.abs(y) - o[1]
        inside = (ex <= 0) & (ey <= 0)
        exact = np.where(inside, np.minimum(-ex, -ey), np.hypot(np.maximum(ex, 0), np.maximum(ey, 0)))
    else:
        ra, rb, pa, pb = o
        inside = _sector_member(x, y, ra, rb, pa, pb)
        # radial edges as segments from radius ra to rb
        exact = np.minimum(np.abs(r - ra), np.abs(r - rb))
        foot_ok = np.ones(len(x), bool)
        for p in (pa, pb):
            e = np.array([math.cos(p), math.sin(p)])
            s = x * e[0] + y * e[1]
            perp = np.abs(x * e[1] - y * e[0])
            seg = np.hypot(x - np.clip(s, ra, rb) * e[0], y - np.clip(s, ra, rb) * e[1])
            exact = np.minimum(exact, seg)
            foot_ok &= ~((s < ra) | (s > rb)) | (perp > seg)
        # the arcs are circles in the diagnostic: exact only for points inside
        assert np.all(bd[inside] <= exact[inside] + 1e-12)
        sel = inside & foot_ok
        assert np.max(np.abs(bd[sel] - exact[sel])) < 1e-12
        assert np.array_equal(got_in, inside)
        return
    assert np.array_equal(got_in, inside)
    assert np.max(np.abs(bd - exact)) < 1e-12


# ------------------------------------------------------------------ grazing classification
def test_grazing_criteria(orc):
    """Each criterion of oracle.grazing() switched on by a photon built for it:
    a hit 1e-6 from the outline's rim, a rejected root 1e-6 outside it, a
    glancing hit (|d . n| = 5e-5), a second surface 1e-6 behind the first, a
    draw within the tolerance of the reflectivity; and off for well-conditioned
    photons."""
    m = scenes.new_volume(scenes.ROLE_MIRROR, scenes.SHAPE_PLANE, scenes.OUTLINE_DISC, o=[1.0], reflectivity=1.0)
    sc = _scene([m], l_ref=1.0)
    xs = np.array([1.0 - 1e-6, 1.0 + 1e-6, 0.5, 0.2])
    r = _down(xs, np.zeros(4), 1.0)
    rec = orc.trace(sc, r, log=True)
    assert list(orc.grazing(rec, 1.0)) == [True, True, False, False]
    # glancing incidence
    for sa, want in ((5e-5, True), (1e-3, False)):
        o = np.array([-0.5, 0.0, 0.5 * sa / math.sqrt(1 - sa * sa)])
        d = np.array([math.sqrt(1 - sa * sa), 0.0, -sa])
        rr = scenes.make_rays(64, [o[0]], [o[1]], [o[2]], [d[0]], [d[1]], [d[2]], [0])
        g = orc.trace(sc, rr, log=True)
        assert g["n_events"][0] == 1 and bool(orc.grazing(g, 1.0)[0]) == want
    # two candidate surfaces: an absorbing disc dz above the mirror
    for dz, want in ((1e-6, True), (1e-2, False)):
        ob = scenes.new_volume(scenes.ROLE_OBSCURATION, scenes.SHAPE_PLANE, scenes.OUTLINE_DISC,
                               c=(0.0, 0.0, dz), o=[1.0])
        s2 = _scene([m, ob], l_ref=1.0)
        g = orc.trace(s2, _down(np.array([0.3]), np.zeros(1), 1.0), log=True)
        assert g["last_vol"][0] == 1 and bool(orc.grazing(g, 1.0)[0]) == want
    # draws near the reflectivity threshold
    R = 0.9
    mr = scenes.new_volume(scenes.ROLE_MIRROR, scenes.SHAPE_PLANE, scenes.OUTLINE_DISC, o=[1.0], reflectivity=R)
    s3 = _scene([mr], l_ref=1.0)
    n = 3000
    g = orc.trace(s3, _down(np.zeros(n), np.zeros(n), 1.0), log=True)
    u = np.array([orc.draw(s3.seed, i, 0) for i in range(n)], dtype=np.float64) / 2.0 ** 32
    tol = 1e-2
    flagged = orc.grazing(g, 1.0, tol_draw=tol)
    assert np.array_equal(flagged, np.abs(u - R) < tol)
    assert 20 < flagged.sum() < 200


# ------------------------------------------------------------------ tilted geometry of forced sequences
@pytest.mark.parametrize("name,sigma", [("davies_cotton", 2e-3), ("schwarzschild_couder", 2e-3)])
def test_forced_at_scene_params_reproduces_tilted_trace(orc, name, sigma):
    """The trace reads each tilted frame as the scene builder formed it (numpy);
    forced sequences rebuild it from the tilt parameters (the oracle's
    geometry).  At the scene's own parameters both give the same positions."""
    sc = scenes.ALL[name](precision=64, sigma_tilt=sigma)
    r = sc.rays(200)
    rec = orc.trace(sc, r, log=True)
    foc = rec["fate"] == FOC
    assert foc.sum() > 300
    pos, dirv, st = orc.forced(sc, r, rec, sc.params)
    assert np.all(st[foc] == 0)
    assert np.max(np.abs(pos[foc] - rec["pos"][foc])) < 1e-12 * sc.l_ref
    assert np.max(np.abs(dirv[foc] - rec["dir"][foc])) < 1e-12
    # a tilt changed by 1e-6 rad moves the forced positions of that facet's photons
    k = sc.param_names.index(next(n for n in sc.param_names if "tilt" in n))
    P = sc.params.copy()
    P[k] += 1e-6
    pos2, _, _ = orc.forced(sc, r, rec, P)
    assert np.max(np.abs(pos2[foc] - pos[foc])) > 1e-7 * sc.l_ref


# ------------------------------------------------------------------ weighted collection gradient
def test_gradient_eff_w_matches_central_fd(orc):
    """d/dP of sum_g w_g (1/N_g) sum_FOCUSED |u_z| by the oracle's dual numbers
    against central differences of the same objective over forced sequences."""
    sc = scenes.hex_concentrator(precision=64)
    r = sc.rays(6)
    rec = orc.trace(sc, r, log=True)
    foc = rec["fate"] == FOC
    assert foc.sum() > 100
    rng = np.random.default_rng(12)
    w = rng.uniform(0.5, 1.5, sc.n_groups)
    g = rec["group"].astype(np.int64)
    nl = np.bincount(g, minlength=sc.n_groups).astype(np.float64)

    def objective(P):
        _, dirv, st = orc.forced(sc, r, rec, P)
        ok = foc & (st == 0)
        return np.sum(w[g[ok]] / nl[g[ok]] * np.abs(dirv[ok, 2])), ok

    got = orc.gradient_eff_w(sc, r, rec, w)
    for j in range(len(sc.params)):
        h = 1e-6 * sc.l_ref
        P1, P2 = sc.params.copy(), sc.params.copy()
        P1[j] += h
        P2[j] -= h
        (f1, ok1), (f2, ok2) = objective(P1), objective(P2)
        assert np.array_equal(ok1, ok2)
        fd = (f1 - f2) / (2 * h)
        assert abs(got[j] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.max(np.abs(got))), (j, got[j], fd)


# ------------------------------------------------------------------ meeting the face just left
def test_whispering_gallery_in_a_spherical_bowl(orc):
    """Inside a concave spherical mirror (R = 1, aperture 0.999 R) a ray in a
    meridian plane keeps its distance p from the centre, so successive hits
    advance by the central angle 2 acos(p / R): from a chord between -80 and
    -60 degrees it meets the bowl at -60, -40, ..., 80 degrees (8 events, each
    on the face it just left, from the side it stays on), then leaves."""
    R = 1.0
    bowl = scenes.new_volume(scenes.ROLE_MIRROR, scenes.SHAPE_SPHERE, scenes.OUTLINE_DISC, p=[1.0 / R],
                             o=[0.999 * R])
    sc = _scene([bowl])
    C = np.array([0.0, 0.0, R])

    def P(deg):
        a = math.radians(deg)
        return C + R * np.array([math.sin(a), 0.0, -math.cos(a)])

    a, b = P(-80), P(-60)
    o = 0.5 * (a + b)
    d = (b - a) / np.linalg.norm(b - a)
    r = scenes.make_rays(64, [o[0]], [o[1]], [o[2]], [d[0]], [d[1]], [d[2]], [0])
    rec = orc.trace(sc, r, log=True)
    assert rec["fate"][0] == EXI and rec["n_events"][0] == 8
    assert np.all(rec["log"]["vol"][0, :8] == 0)
    last = P(80)
    out = (P(100) - P(80)) / np.linalg.norm(P(100) - P(80))
    assert np.max(np.abs(rec["pos"][0] - last)) < 1e-12
    assert np.max(np.abs(rec["dir"][0] - out)) < 1e-12
    # chord lengths are all 2 R sin(10 deg)
    assert np.max(np.abs(rec["log"]["t"][0, 1:8] - 2 * R * math.sin(math.radians(10)))) < 1e-12


def test_refracted_photon_meets_the_same_face_from_the_glass_side(orc):
    """A spherical lens face (R = 1, glass inside the ball, aperture 0.999 R):
    a ray entering the ball at incidence theta_i refracts to theta_t
    (sin theta_t = sin theta_i / n) and meets the same face again from inside
    after a chord of length 2 R cos(theta_t), wherever that chord ends on the
    cap."""
    R, nidx = 1.0, 1.5
    cap = scenes.new_volume(scenes.ROLE_LENS, scenes.SHAPE_SPHERE, scenes.OUTLINE_DISC, p=[-1.0 / R],
                            o=[0.999 * R], n_inside=nidx)
    sc = _scene([cap])
    C = np.array([0.0, 0.0, -R])
    # horizontal rays at heights 0.3 R .. 0.95 R above the centre: the chord
    # crosses over the top of the ball and ends on the cap's far side
    d = np.array([-1.0, 0.0, 0.0])
    zs = C[2] + np.linspace(0.3, 0.95, 300) * R
    o = np.stack([np.full(len(zs), 3.0), np.zeros(len(zs)), zs], 1)
    # entry point and incidence angle (ray / sphere), then where the chord ends
    w = o - C
    b = w @ d
    disc = b * b - (np.sum(w * w, 1) - R * R)
    assert np.all(disc > 0)
    P1 = o + (-b - np.sqrt(disc))[:, None] * d
    cos_i = np.abs((P1 - C) @ d) / R
    sin_t = np.sqrt(1 - cos_i ** 2) / nidx
    chord = 2 * R * np.sqrt(1 - sin_t ** 2)
    n = len(zs)
    r = scenes.make_rays(64, o[:, 0], o[:, 1], o[:, 2], np.full(n, d[0]), np.full(n, d[1]), np.full(n, d[2]),
                         np.zeros(n))
    rec = orc.trace(sc, r, log=True)
    lg = rec["log"]
    first_refracts = lg["act"][:, 0] == 1
    assert np.max(np.abs(lg["t"][:, 0] - (-b - np.sqrt(disc)))) < 1e-12
    # the chord ends on the cap (above its rim height) for these rays
    second = first_refracts & (rec["n_events"] >= 2)
    assert first_refracts.sum() > 250
    assert np.array_equal(second, first_refracts)
    assert np.all(lg["vol"][second, 1] == 0)
    assert np.max(np.abs(lg["t"][second, 1] - chord[second])) < 1e-12
