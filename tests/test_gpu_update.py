"""Parameter updates on the device (robast_update_params and its batched
form) against host rebuilds (robast_set_params) and the oracle."""
import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KEYS = ("fate", "n_events", "last_vol", "x", "y", "z", "ux", "uy", "uz", "seq_hash")


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1508_07803_amd as rb
    return rb


def _sc_params(sc, seed):
    """New SC parameters: tilts moved by N(0, 2e-5) rad, coefficients scaled by
    1 + N(0, 1e-4) (a gradient-descent step's size)."""
    rng = np.random.default_rng(seed)
    p = sc.params.copy()
    p[:16] *= 1.0 + rng.normal(0.0, 1e-4, 16)
    p[16:] += rng.normal(0.0, 2e-5, len(p) - 16)
    return p


def _trace(rb, dev, rays, n):
    hits = dev.alloc_hits(n)
    sums = dev.new_sums()
    dev.trace(rays, hits=hits, sums=sums)
    torch.cuda.synchronize()
    return hits, sums


@pytest.mark.parametrize("name,precision", [("schwarzschild_couder", 32), ("schwarzschild_couder", 64),
                                            ("davies_cotton", 32), ("hex_concentrator", 32)])
def test_device_update_matches_host_rebuild_and_oracle(rb, name, precision):
    import oracle
    from test_gpu_parity import compare
    sc = scenes.ALL[name](precision=precision)
    if name == "schwarzschild_couder":
        p1 = _sc_params(sc, 3)
    elif name == "davies_cotton":
        rng = np.random.default_rng(4)
        p1 = sc.params.copy()
        nf = sc.meta["n_facets"]
        p1[:nf] *= 1.0 + rng.normal(0.0, 1e-3, nf)
        p1[nf:] += rng.normal(0.0, 2e-5, len(p1) - nf)
    else:
        p1 = sc.params * (1.0 + np.array([2e-4, -1e-4, 1e-4, 2e-4]))
    if precision == 32:
        p1 = p1.astype(np.float32).astype(np.float64)
    r = sc.rays(600 if name == "hex_concentrator" else 2000)
    n = len(r["ox"])
    dev = rb.Scene(sc)
    rays = dev.upload_rays(r)
    status = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    dev.update_params_device(torch.from_numpy(p1).cuda(), status=status)
    got, sums = _trace(rb, dev, rays, n)
    assert int(status.item()) == 0
    host = rb.Scene(sc)
    host.update_params(p1)
    ref, ref_sums = _trace(rb, host, rays, n)
    # the same geometry: records equal, up to FP32 rounding of rebuilt frames
    same = (got["fate"] == ref["fate"]) & (got["seq_hash"] == ref["seq_hash"])
    assert int((~same).sum()) <= max(3, 1e-5 * n)
    tol = (1e-6 if precision == 32 else 1e-12) * sc.l_ref
    for k in ("x", "y", "z"):
        assert float((got[k][same] - ref[k][same]).abs().max()) <= tol, k
    assert torch.allclose(sums[0::8], ref_sums[0::8])
    # and the oracle, tracing the descriptors with those parameters applied
    # (each body rotated about its own pivot, as the parameters are defined)
    osc = _applied(sc, p1)
    rec = oracle.trace(osc, r, log=True)
    g = {k: v.cpu().numpy() for k, v in got.items()}
    g["seq_hash"] = g["seq_hash"].view(np.uint64)
    g["pos"] = np.stack([g["x"], g["y"], g["z"]], 1).astype(np.float64)
    g["dir"] = np.stack([g["ux"], g["uy"], g["uz"]], 1).astype(np.float64)
    t = 1e-5 if precision == 32 else 1e-9
    nbad, dp, dd, _ = compare(osc, r, g, rec, t * sc.l_ref, t)
    print(f"{name} fp{precision}: device update vs oracle: mismatches {nbad}, max|dpos| {dp:.2e}")


def _applied(sc, P):
    """A copy of the scene whose descriptors carry the parameters P: a tilted
    body's frame is its untilted frame rotated about its pivot by
    Rot(e2, beta) Rot(e1, alpha); a sphere's curvature is 1/R, an asphere's
    sag coefficients and a cone's interior control points are the values."""
    import copy
    out = copy.copy(sc)
    vols = sc.volumes.copy()
    for v in vols:
        if v["tilt_param"] >= 0:
            a, b = P[v["tilt_param"]], P[v["tilt_param"] + 1]
            Q, c = scenes.tilted_frame(v["Q0"].reshape(3, 3), v["c0"], v["pivot"], v["e1"], v["e2"], a, b)
            v["Q"], v["c"] = Q.reshape(9), c
        k = v["shape_param"]
        if k >= 0:
            if v["shape"] == scenes.SHAPE_SPHERE:
                v["p"][0] = 1.0 / P[k]
            elif v["shape"] == scenes.SHAPE_ASPHERE:
                v["p"][1:9] = P[k:k + 8]
            elif v["shape"] == scenes.SHAPE_HEXCONE:
                v["p"][2:6] = P[k:k + 4]
    if sc.precision == 32:
        for f in ("Q", "c", "p"):
            vols[f] = vols[f].astype(np.float32).astype(np.float64)
    out.volumes = vols
    out.params = np.asarray(P, dtype=np.float64)
    return out


def test_device_update_rejections_keep_the_tables(rb):
    """Invalid geometry (a sphere whose aperture reaches its equator) gives
    EINVAL, a tilt that moves panels across their grid cells EUNSUPPORTED;
    either way the scene traces as before, and a valid update then applies."""
    sc = scenes.single_mirror()
    r = sc.rays(3000)
    dev = rb.Scene(sc)
    rays = dev.upload_rays(r)
    n = len(r["ox"])
    before, _ = _trace(rb, dev, rays, n)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    dev.update_params_device(torch.tensor([1.9], dtype=torch.float64, device="cuda"), status=st)
    after, _ = _trace(rb, dev, rays, n)
    assert int(st.item()) == rb.EINVAL
    for k in KEYS:
        assert torch.equal(before[k], after[k]), k
    sc2 = scenes.schwarzschild_couder()
    d2 = rb.Scene(sc2)
    r2 = sc2.rays(500)
    rays2 = d2.upload_rays(r2)
    n2 = len(r2["ox"])
    b2, _ = _trace(rb, d2, rays2, n2)
    p = sc2.params.copy()
    p[16] += 0.3
    d2.update_params_device(torch.from_numpy(p).cuda(), status=st)
    a2, _ = _trace(rb, d2, rays2, n2)
    assert int(st.item()) == rb.EUNSUPPORTED
    for k in KEYS:
        assert torch.equal(b2[k], a2[k]), k
    d2.update_params_device(torch.from_numpy(_sc_params(sc2, 5)).cuda(), status=st)
    c2, _ = _trace(rb, d2, rays2, n2)
    assert int(st.item()) == 0
    assert not torch.equal(c2["x"], b2["x"])


def test_update_and_trace_in_a_graph(rb):
    """A captured graph of (device update from a parameter tensor, trace,
    figures, adjoint) replayed with new parameter values written into the
    tensor between replays: each replay equals eager host-rebuilt scenes at
    those parameters (sums, and gradients to FP32 table rounding)."""
    sc = scenes.schwarzschild_couder()
    r = sc.rays(3000)
    dev = rb.Scene(sc)
    rays = dev.upload_rays(r)
    P = torch.from_numpy(sc.params.copy()).cuda()
    sums = dev.new_sums()
    grad = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
    cot = torch.zeros(sc.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 0] = 1.0 / sc.n_groups
    st = torch.zeros(1, dtype=torch.int32, device="cuda")

    def step(stream=None):
        dev.update_params_device(P, status=st, stream=stream)
        sums.zero_()
        grad.zero_()
        dev.trace(rays, sums=sums, stream=stream, keep_order=True)
        dev.backward(rays, sums, cot, grad, stream=stream)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step(stream=s.cuda_stream)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step(stream=torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        p = _sc_params(sc, 10 + rep).astype(np.float32).astype(np.float64)
        P.copy_(torch.from_numpy(p))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        ref = rb.Scene(sc)
        ref.update_params(p)
        rs = ref.new_sums()
        ref.trace(rays, sums=rs)
        rg = torch.zeros_like(grad)
        ref.backward(rays, rs, cot, rg)
        torch.cuda.synchronize()
        assert torch.equal(sums[0::8], rs[0::8])
        assert float((sums[1::8] - rs[1::8]).abs().sum()) <= 3, rep   # fates: grazing photons aside
        assert torch.allclose(sums[2::8], rs[2::8], rtol=1e-3, atol=1e-3), rep
        assert torch.allclose(grad, rg, rtol=1e-3, atol=1e-3 * float(rg.abs().max())), rep
        _ = (rays["ox"] * 2.0).sum().item()   # eager work between replays


def test_batched_update_equals_per_scene_updates(rb):
    """robast_update_params_batch over a sweep of variants equals each
    variant's own device update (identical photons and sums)."""
    variants, _ = scenes.sweep(n_dc=2, n_sc=2, seed=scenes.SEED_BASE + 61)
    devs = [rb.Scene(v) for v in variants]
    counts = [3000, 2000, 2500, 1500]
    host = [v.rays(c, seed=41 + i) for i, (v, c) in enumerate(zip(variants, counts))]
    rays = {k: torch.cat([d.upload_rays(h)[k] for d, h in zip(devs, host)]) for k in
            ("ox", "oy", "oz", "dx", "dy", "dz", "group")}
    batch = rb.Batch(devs, counts, chunk=1000)
    rng = np.random.default_rng(9)
    newp = []
    for v in variants:
        p = v.params.copy()
        if v.name.startswith("schwarz"):
            p[:16] *= 1.0 + rng.normal(0.0, 1e-4, 16)
            p[16:] += rng.normal(0.0, 2e-5, len(p) - 16)
        else:
            nf = v.meta["n_facets"]
            p[:nf] *= 1.0 + rng.normal(0.0, 1e-3, nf)
            p[nf:] += rng.normal(0.0, 2e-5, len(p) - nf)
        newp.append(p)
    st = torch.full((len(devs),), 7, dtype=torch.int32, device="cuda")
    batch.update_params(torch.from_numpy(np.concatenate(newp)).cuda(), status=st)
    hits = devs[0].alloc_hits(sum(counts))
    sums = batch.new_sums()
    batch.trace(rays, hits=hits, sums=sums)
    torch.cuda.synchronize()
    assert st.tolist() == [0] * len(devs)
    off = 0
    for v, (sc, c) in enumerate(zip(variants, counts)):
        d = rb.Scene(sc)
        d.update_params_device(torch.from_numpy(newp[v]).cuda())
        sub = {k: t[off:off + c] for k, t in rays.items()}
        h1 = d.alloc_hits(c)
        d.trace(sub, hits=h1)
        torch.cuda.synchronize()
        for k in KEYS:
            assert torch.equal(hits[k][off:off + c], h1[k]), (v, k)
        off += c


def test_host_set_params_checks_geometry_first(rb):
    """robast_set_params with parameters that make a surface invalid (the
    sphere's aperture reaching its equator) is rejected before anything
    changes: EINVAL, and the scene traces as before."""
    sc = scenes.single_mirror()
    r = sc.rays(2000)
    dev = rb.Scene(sc)
    rays = dev.upload_rays(r)
    n = len(r["ox"])
    before, _ = _trace(rb, dev, rays, n)
    with pytest.raises(rb.RobastError) as ei:
        dev.update_params([1.9])
    assert ei.value.status == rb.EINVAL and "equator" in str(ei.value)
    assert np.array_equal(dev.params, sc.params)
    after, _ = _trace(rb, dev, rays, n)
    for k in KEYS:
        assert torch.equal(before[k], after[k]), k


def _gd_inputs(sc, seed, scale=1.0):
    """A gradient-like vector and per-parameter steps that move the SC's
    coefficients by ~1e-4 relative and its tilts by ~2e-5 rad (x scale)."""
    rng = np.random.default_rng(seed)
    g = rng.normal(0.0, 1.0, len(sc.params))
    lr = np.where(np.arange(len(sc.params)) < 16, 1e-4 * np.abs(sc.params), 2e-5) * scale
    return g, lr


def test_gd_step_applies_the_step(rb):
    """robast_gd_step: params become p - lr * g (FP64, to rounding), and the
    scene traces exactly as one updated to those parameters; a step that
    would move a panel out of its grid cells is rejected and leaves both
    the parameters and the scene as they were."""
    sc = scenes.schwarzschild_couder()
    r = sc.rays(2000)
    dev = rb.Scene(sc)
    rays = dev.upload_rays(r)
    n = len(r["ox"])
    g, lr = _gd_inputs(sc, 5)
    P = torch.from_numpy(sc.params.copy()).cuda()
    G, LR = torch.from_numpy(g).cuda(), torch.from_numpy(lr).cuda()
    st = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    dev.gd_step(P, G, LR, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    want = sc.params - lr * g
    got = P.cpu().numpy()
    assert np.allclose(got, want, rtol=1e-15, atol=1e-18)
    assert not np.array_equal(got, sc.params)
    h1, s1 = _trace(rb, dev, rays, n)
    ref = rb.Scene(sc)
    ref.update_params_device(P.clone())
    h2, s2 = _trace(rb, ref, rays, n)
    for k in KEYS:
        assert torch.equal(h1[k], h2[k]), k
    assert torch.allclose(s1, s2, rtol=1e-12, atol=1e-12 * float(s2.abs().max()))   # FP64 summation order
    # a step far beyond the grid's margin: rejected, nothing changes
    before = P.clone()
    dev.gd_step(P, G, LR * 1e4, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == rb.EUNSUPPORTED
    assert torch.equal(P, before)
    h3, _ = _trace(rb, dev, rays, n)
    for k in KEYS:
        assert torch.equal(h1[k], h3[k]), k


def test_gd_steps_in_a_graph_equal_eager_steps(rb):
    """One optimisation step -- trace, figures, adjoint of the mean RMS,
    gradient step on the device -- captured once and replayed 3 times
    equals 3 eager steps on a second copy of the scene (parameters to
    FP64 summation order of the gradient, RMS per step)."""
    sc = scenes.schwarzschild_couder()
    r = sc.rays(3000)
    cot = torch.zeros(sc.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 0] = 1.0 / sc.n_groups
    _, lr = _gd_inputs(sc, 6)
    # steps sized from the first gradient so that 3 of them stay in the grid margin
    probe = rb.Scene(sc)
    rays = probe.upload_rays(r)
    s0 = probe.new_sums()
    probe.trace(rays, sums=s0)
    g0 = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
    probe.backward(rays, s0, cot, g0)
    torch.cuda.synchronize()
    g0 = g0.cpu().numpy()
    lr = lr / np.maximum(np.abs(g0), 1e-300 + np.abs(g0).max() * 1e-3)
    LR = torch.from_numpy(lr).cuda()

    def make():
        dev = rb.Scene(sc)
        state = dict(dev=dev, P=torch.from_numpy(sc.params.copy()).cuda(), sums=dev.new_sums(),
                     fig=torch.zeros(sc.n_groups * rb.FIGURE_STRIDE, dtype=torch.float64, device="cuda"),
                     grad=torch.zeros(len(sc.params), dtype=torch.float64, device="cuda"),
                     st=torch.zeros(1, dtype=torch.int32, device="cuda"))
        return state

    def step(S, stream=None):
        S["sums"].zero_()
        S["grad"].zero_()
        S["dev"].trace(rays, sums=S["sums"], stream=stream, keep_order=True)
        S["dev"].figures(S["sums"], fig=S["fig"], stream=stream)
        S["dev"].backward(rays, S["sums"], cot, S["grad"], stream=stream)
        S["dev"].gd_step(S["P"], S["grad"], LR, status=S["st"], stream=stream)

    A, B = make(), make()
    # both copies take their tables from a device update (at the start
    # parameters), so that the two follow one rounding of the FP32 tables
    B["dev"].update_params_device(B["P"])
    # warm A eagerly on a side stream (grows its workspaces), then undo the
    # step it took, and capture
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step(A, stream=s.cuda_stream)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    A["P"].copy_(torch.from_numpy(sc.params.copy()))
    A["dev"].update_params_device(A["P"])
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step(A, stream=torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        step(B)
        torch.cuda.synchronize()
        assert int(A["st"].item()) == 0 and int(B["st"].item()) == 0, rep
        assert torch.equal(A["sums"][0::8], B["sums"][0::8]), rep
        assert torch.allclose(A["fig"][4::8], B["fig"][4::8], rtol=1e-12), rep
        assert torch.allclose(A["P"], B["P"], rtol=1e-12, atol=0.0), rep
        _ = (rays["ox"] * 2.0).sum().item()   # eager work between replays
    assert not torch.equal(A["P"], torch.from_numpy(sc.params).cuda())


def test_batched_gd_step_equals_per_scene_steps(rb):
    """robast_gd_step_batch equals each variant's robast_gd_step (the same
    new parameters bit for bit, the same photons)."""
    variants, _ = scenes.sweep(n_dc=2, n_sc=2, seed=scenes.SEED_BASE + 62)
    devs = [rb.Scene(v) for v in variants]
    counts = [2500, 2000, 1500, 3000]
    host = [v.rays(c, seed=51 + i) for i, (v, c) in enumerate(zip(variants, counts))]
    rays = {k: torch.cat([d.upload_rays(h)[k] for d, h in zip(devs, host)]) for k in
            ("ox", "oy", "oz", "dx", "dy", "dz", "group")}
    batch = rb.Batch(devs, counts, chunk=1000)
    rng = np.random.default_rng(12)
    gs, lrs = [], []
    for v in variants:
        gs.append(rng.normal(0.0, 1.0, len(v.params)))
        if v.name.startswith("schwarz"):
            lrs.append(np.where(np.arange(len(v.params)) < 16, 1e-4 * np.abs(v.params), 2e-5))
        else:
            nf = v.meta["n_facets"]
            lrs.append(np.where(np.arange(len(v.params)) < nf, 1e-3 * np.abs(v.params), 2e-5))
    P = torch.from_numpy(np.concatenate([v.params for v in variants])).cuda()
    G = torch.from_numpy(np.concatenate(gs)).cuda()
    LR = torch.from_numpy(np.concatenate(lrs)).cuda()
    st = torch.full((len(devs),), 7, dtype=torch.int32, device="cuda")
    batch.gd_step(P, G, LR, status=st)
    hits = devs[0].alloc_hits(sum(counts))
    batch.trace(rays, hits=hits)
    torch.cuda.synchronize()
    assert st.tolist() == [0] * len(devs)
    off = poff = 0
    for v, (sc, c) in enumerate(zip(variants, counts)):
        d = rb.Scene(sc)
        p = torch.from_numpy(sc.params.copy()).cuda()
        d.gd_step(p, torch.from_numpy(gs[v]).cuda(), torch.from_numpy(lrs[v]).cuda())
        sub = {k: t[off:off + c] for k, t in rays.items()}
        h1 = d.alloc_hits(c)
        d.trace(sub, hits=h1)
        torch.cuda.synchronize()
        assert torch.equal(P[poff:poff + len(sc.params)], p), v
        for k in KEYS:
            assert torch.equal(hits[k][off:off + c], h1[k]), (v, k)
        off += c
        poff += len(sc.params)


def test_batch_autotune_keeps_results(rb):
    """robast_autotune_batch picks a work-item and workgroup size; photons
    traced with the pick equal those of the default launch bit for bit."""
    variants, _ = scenes.sweep(n_dc=2, n_sc=2, seed=scenes.SEED_BASE + 63)
    devs = [rb.Scene(v) for v in variants]
    counts = [40000, 3000, 60000, 5000]
    host = [v.rays(c // v.n_groups, seed=61 + i) for i, (v, c) in enumerate(zip(variants, counts))]
    counts = [len(h["ox"]) for h in host]
    rays = {k: torch.cat([d.upload_rays(h)[k] for d, h in zip(devs, host)]) for k in
            ("ox", "oy", "oz", "dx", "dy", "dz", "group")}
    batch = rb.Batch(devs, counts, chunk=4096)
    n = sum(counts)
    ref = devs[0].alloc_hits(n)
    rs = batch.new_sums()
    batch.trace(rays, hits=ref, sums=rs)
    best = batch.autotune(rays)
    assert best["chunk"] in (2048, 8192, 32768, 131072) and best["block"] in (128, 256)
    hits = devs[0].alloc_hits(n)
    s = batch.new_sums()
    batch.trace(rays, hits=hits, sums=s)
    torch.cuda.synchronize()
    for k in KEYS:
        assert torch.equal(ref[k], hits[k]), k
    assert torch.allclose(rs, s, rtol=1e-12, atol=1e-12 * float(rs.abs().max()))
