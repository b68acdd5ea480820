"""Batched persistent sweeps against single-scene calls and the oracle.

A batch must give every photon exactly the result of a single-scene call on
its variant (same draws, same search, same arithmetic): fates, event counts,
last volumes, positions and directions are compared bit for bit.  Group sums
and gradients are FP64 sums in another order, compared to 1e-9 relative.
Graph capture: a captured forward + figures + adjoint step replayed several
times, with eager work between replays, equals the eager step each time.
"""
import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1508_07803_amd as rb
    return rb


def small_sweep(n_dc=2, n_sc=3, seed=scenes.SEED_BASE + 55):
    variants, _ = scenes.sweep(seed=seed, n_dc=n_dc, n_sc=n_sc)
    return variants


def concat_rays(rb, devs, counts, seed0=11):
    parts = []
    for v, (d, n) in enumerate(zip(devs, counts)):
        r = d.src.rays(int(n), seed=seed0 + v) if n else None
        parts.append(d.upload_rays(r) if n else None)
    keys = ("ox", "oy", "oz", "dx", "dy", "dz", "group")
    out = {}
    for k in keys:
        ts = [p[k] for p in parts if p is not None]
        out[k] = torch.cat(ts) if ts else torch.zeros(0, device="cuda")
    return out, parts


HIT_KEYS = ("fate", "n_events", "last_vol", "x", "y", "z", "ux", "uy", "uz", "seq_hash")


def as_numpy(hits, sl):
    """Hit tensors (a slice of the concatenated bundle) in the layout of the
    parity tests' compare()."""
    out = {k: hits[k][sl].cpu().numpy() for k in hits}
    out["seq_hash"] = out["seq_hash"].view(np.uint64)
    out["pos"] = np.stack([out["x"], out["y"], out["z"]], 1).astype(np.float64)
    out["dir"] = np.stack([out["ux"], out["uy"], out["uz"]], 1).astype(np.float64)
    return out


# small bundles run unbinned; above 32768 photons the batch bins per variant
COUNTS = {"unbinned": [3001, 0, 1, 2048, 4097], "binned": [40000, 0, 1, 30000, 50001],
          "binned_dirs": [40000, 0, 1, 30000, 50001]}


@pytest.mark.parametrize("kind", sorted(COUNTS))
def test_batch_equals_per_variant_bitwise(rb, kind):
    """Ragged counts (0, 1, chunk multiples and tails), chunk smaller than a
    variant, mixed DC / SC variants, binning by entrance cell or also by
    direction sector: every photon identical to the plain call."""
    variants = small_sweep()
    devs = [rb.Scene(v) for v in variants]
    if kind == "binned_dirs":
        for d in devs:
            d.set_tuning(bin_dirs=16, bin_target=16)
    counts = COUNTS[kind]
    chunk = 1024
    rays, parts = concat_rays(rb, devs, counts)
    batch = rb.Batch(devs, counts, chunk=chunk)
    assert batch.n_photons == sum(counts)
    n = batch.n_photons
    hits = devs[0].alloc_hits(n)
    sums = batch.new_sums()
    batch.trace(rays, hits=hits, sums=sums, id_base=7)
    torch.cuda.synchronize()
    off = 0
    for v, (d, c) in enumerate(zip(devs, counts)):
        if c == 0:
            continue
        h1 = d.alloc_hits(c)
        s1 = d.new_sums()
        d.trace(parts[v], hits=h1, sums=s1, id_base=7)
        torch.cuda.synchronize()
        for k in HIT_KEYS:
            a, b = hits[k][off:off + c], h1[k]
            assert torch.equal(a, b), f"variant {v}: {k} differs at {int((a != b).nonzero()[0])}"
        g = batch.goff[v]
        sb = sums[g * 8:(g + 1) * 8]
        assert torch.allclose(sb, s1, rtol=1e-9, atol=1e-9), (v, sb.tolist(), s1.tolist())
        off += c
    # an empty variant's sums stay zero
    g = batch.goff[1]
    assert torch.count_nonzero(sums[g * 8:(g + 1) * 8]) == 0


@pytest.mark.parametrize("counts,keep", [([5000, 2500, 1, 0, 7000], False), ([40000, 2500, 1, 0, 35000], False),
                                         ([5000, 2500, 1, 0, 7000], True), ([40000, 2500, 1, 0, 35000], True)])
def test_batch_backward_equals_per_variant(rb, counts, keep):
    """Adjoint of the batch against per-variant adjoint calls; also with the
    binned order kept from the forward call."""
    variants = small_sweep(seed=scenes.SEED_BASE + 56)
    devs = [rb.Scene(v) for v in variants]
    rays, parts = concat_rays(rb, devs, counts, seed0=21)
    batch = rb.Batch(devs, counts, chunk=2048)
    sums = batch.new_sums()
    batch.trace(rays, sums=sums, keep_order=keep)
    cot = torch.zeros(batch.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 0] = 1.0
    cot[:, 1] = 0.25
    grad = torch.zeros(batch.n_params, dtype=torch.float64, device="cuda")
    batch.backward(rays, sums, cot, grad)
    torch.cuda.synchronize()
    for v, (d, c) in enumerate(zip(devs, counts)):
        p0, p1 = batch.poff[v], batch.poff[v + 1]
        if c == 0:
            assert torch.count_nonzero(grad[p0:p1]) == 0
            continue
        s1 = d.new_sums()
        d.trace(parts[v], sums=s1)
        g1 = torch.zeros(d.n_params, dtype=torch.float64, device="cuda")
        c1 = cot[batch.goff[v]:batch.goff[v + 1]].contiguous()
        d.backward(parts[v], s1, c1, g1)
        torch.cuda.synchronize()
        scale = float(g1.abs().max())
        assert torch.allclose(grad[p0:p1], g1, rtol=1e-9, atol=1e-12 * max(scale, 1e-300)), v


@pytest.mark.parametrize("n_per", [[30, 200], [400, 2500]])
def test_batch_backward_long_paths(rb, n_per):
    """A batch holding the hex-cone concentrator, whose collected photons
    often take more events than a path record holds: after a forward launch
    that keeps its order, the adjoint replays the short records and searches
    the long ones again; the gradient equals that of per-variant calls that
    search every photon.  Both variants have several groups (n_per photons
    per group; the larger case is binned)."""
    devs = [rb.Scene(scenes.hex_concentrator()), rb.Scene(scenes.schwarzschild_couder())]
    parts = [d.upload_rays(d.src.rays(k, seed=31 + v)) for v, (d, k) in enumerate(zip(devs, n_per))]
    counts = [int(p["ox"].numel()) for p in parts]
    rays = {k: torch.cat([p[k] for p in parts]) for k in parts[0]}
    batch = rb.Batch(devs, counts, chunk=2048)
    cot = torch.zeros(batch.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 0] = 1.0
    cot[:, 1] = 0.5
    grads = []
    for keep in (False, True):
        sums = batch.new_sums()
        batch.trace(rays, sums=sums, keep_order=keep)
        grad = torch.zeros(batch.n_params, dtype=torch.float64, device="cuda")
        batch.backward(rays, sums, cot, grad)
        torch.cuda.synchronize()
        grads.append(grad)
    for v, d in enumerate(devs):
        s1 = d.new_sums()
        d.trace(parts[v], sums=s1)
        g1 = torch.zeros(d.n_params, dtype=torch.float64, device="cuda")
        d.backward(parts[v], s1, cot[batch.goff[v]:batch.goff[v + 1]].contiguous(), g1)
        torch.cuda.synchronize()
        p0, p1 = batch.poff[v], batch.poff[v + 1]
        scale = float(g1.abs().max())
        assert scale > 0
        for keep, grad in zip((False, True), grads):
            err = float((grad[p0:p1] - g1).abs().max()) / scale
            print(f"variant {v} keep={keep}: max diff {err:.2e} of max |g|")
            assert torch.allclose(grad[p0:p1], g1, rtol=1e-9, atol=1e-12 * scale), (v, keep, err)


@pytest.mark.parametrize("n_per", [3000, 12000])
def test_chromatic_batch(rb, n_per):
    """Wavelength as the batch axis: the aspheric singlet at 7 wavelengths
    (same surfaces, the index of each wavelength) in one batch.  Photons are
    bit-identical to per-wavelength calls, gradients agree to FP64 summation
    order, and a sample matches the oracle of its wavelength."""
    import oracle
    from test_gpu_parity import compare
    lams = np.linspace(300e-9, 600e-9, 7)
    variants = scenes.lens_wavelengths(lams)
    devs = [rb.Scene(v) for v in variants]
    host = [v.rays(n_per, seed=41 + i) for i, v in enumerate(variants)]
    parts = [d.upload_rays(r) for d, r in zip(devs, host)]
    counts = [int(p["ox"].numel()) for p in parts]
    rays = {k: torch.cat([p[k] for p in parts]) for k in parts[0]}
    batch = rb.Batch(devs, counts, chunk=2048)
    n = batch.n_photons
    hits = devs[0].alloc_hits(n)
    sums = batch.new_sums()
    batch.trace(rays, hits=hits, sums=sums)
    cot = torch.zeros(batch.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 0] = 1.0
    grad = torch.zeros(batch.n_params, dtype=torch.float64, device="cuda")
    batch.backward(rays, sums, cot, grad)
    fig = batch.figures(sums).cpu().numpy()
    torch.cuda.synchronize()
    off = 0
    for v, (d, c) in enumerate(zip(devs, counts)):
        h1 = d.alloc_hits(c)
        s1 = d.new_sums()
        d.trace(parts[v], hits=h1, sums=s1)
        g1 = torch.zeros(d.n_params, dtype=torch.float64, device="cuda")
        d.backward(parts[v], s1, cot[batch.goff[v]:batch.goff[v + 1]].contiguous(), g1)
        torch.cuda.synchronize()
        for k in HIT_KEYS:
            assert torch.equal(hits[k][off:off + c], h1[k]), (v, k)
        p0, p1 = batch.poff[v], batch.poff[v + 1]
        scale = float(g1.abs().max())
        assert scale > 0
        assert torch.allclose(grad[p0:p1], g1, rtol=1e-9, atol=1e-12 * scale), v
        if v in (0, 6):
            sub = {k: val[:2000] for k, val in host[v].items()}
            got = as_numpy(hits, slice(off, off + 2000))
            ref = oracle.trace(variants[v], sub, log=True)
            compare(variants[v], sub, got, ref, 1e-5 * variants[v].l_ref, 1e-5)
        off += c
    # the plane sits at the 400 nm paraxial focus; spherical aberration puts
    # the best focus inside it, where longer wavelengths focus: the blue end
    # is the worst and the sharpest spot lies between the ends
    rms0 = fig.reshape(-1, 8)[[batch.goff[v] for v in range(7)], 4]
    assert np.argmax(rms0) == 0 and 0 < np.argmin(rms0) < 6, rms0


def test_batch_photons_match_oracle(rb):
    """Direct parity of batched photons with the FP64 oracle."""
    import oracle
    from test_gpu_parity import compare
    variants = small_sweep(n_dc=1, n_sc=1, seed=scenes.SEED_BASE + 57)
    devs = [rb.Scene(v) for v in variants]
    counts = [6000, 6000]
    host = [v.rays(c, seed=31 + i) for i, (v, c) in enumerate(zip(variants, counts))]
    rays = {k: torch.cat([d.upload_rays(h)[k] for d, h in zip(devs, host)]) for k in
            ("ox", "oy", "oz", "dx", "dy", "dz", "group")}
    batch = rb.Batch(devs, counts, chunk=1000)
    hits = devs[0].alloc_hits(sum(counts))
    batch.trace(rays, hits=hits)
    torch.cuda.synchronize()
    off = 0
    for v, (sc, c) in enumerate(zip(variants, counts)):
        rec = oracle.trace(sc, host[v], log=True)
        nbad, dp, dd, _ = compare(sc, host[v], as_numpy(hits, slice(off, off + c)), rec, 1e-5 * sc.l_ref, 1e-5)
        print(f"{sc.name}: N={c} mismatches={nbad} max|dpos|={dp:.3e} max|ddir|={dd:.3e}")
        off += c


@pytest.mark.parametrize("counts", [[4000, 3000, 5000], [40000, 3000, 50000]])
def test_batch_graph_capture_replays(rb, counts):
    """Captured step (zero sums, trace, figures, adjoint) replayed 3 times with
    eager work and a parameter update in between; each replay equals eager.
    The second case bins (the binning kernels are part of the graph)."""
    variants = small_sweep(n_dc=1, n_sc=2, seed=scenes.SEED_BASE + 58)
    devs = [rb.Scene(v) for v in variants]
    rays, _ = concat_rays(rb, devs, counts, seed0=41)
    batch = rb.Batch(devs, counts, chunk=1024)
    sums = batch.new_sums()
    fig = torch.zeros(batch.n_groups * 8, dtype=torch.float64, device="cuda")
    cot = torch.zeros(batch.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 0] = 1.0
    grad = torch.zeros(batch.n_params, dtype=torch.float64, device="cuda")

    def step(stream=None):
        sums.zero_()
        grad.zero_()
        batch.trace(rays, sums=sums, stream=stream, keep_order=True)
        batch.figures(sums, fig=fig, stream=stream)
        batch.backward(rays, sums, cot, grad, stream=stream)

    step()
    torch.cuda.synchronize()
    ref = (sums.clone(), fig.clone(), grad.clone())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()   # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step(stream=torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        sums.fill_(-1.0)
        grad.fill_(123.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.allclose(sums, ref[0], rtol=1e-12, atol=1e-9), rep
        assert torch.allclose(fig, ref[1], rtol=1e-12, atol=1e-12), rep
        assert torch.allclose(grad, ref[2], rtol=1e-9, atol=1e-12 * float(ref[2].abs().max())), rep
        _ = (rays["ox"] * 2.0).sum().item()   # eager work between replays
    # a parameter update of a member scene is seen by the next replay
    p = devs[1].params.copy()
    p[:16] *= 1.0 + 1e-3
    devs[1].update_params(p)
    step()
    torch.cuda.synchronize()
    eager = (sums.clone(), grad.clone())
    assert not torch.allclose(eager[1], ref[2])
    g.replay()
    torch.cuda.synchronize()
    assert torch.allclose(sums, eager[0], rtol=1e-12, atol=1e-9)
    assert torch.allclose(grad, eager[1], rtol=1e-9, atol=1e-12 * float(eager[1].abs().max()))


def test_full_size_variants_sampled_against_oracle(rb):
    """Two variants at the sweep's largest size (1e7 photons each, device-side
    rays) in the bench's launch configuration (chunk 8192): three blocks of
    1000 consecutive photons per variant (start, middle, end) are recomputed
    by the oracle with their photon ids, and each variant's launched count in
    the group sums is exact."""
    import oracle
    from test_gpu_parity import compare
    variants = small_sweep(n_dc=1, n_sc=1, seed=scenes.SEED_BASE + 59)
    devs = [rb.Scene(v) for v in variants]
    counts = [10_000_000, 10_000_000]
    parts = [scenes.device_rays(v, c, seed=91 + i) for i, (v, c) in enumerate(zip(variants, counts))]
    rays = {k: torch.cat([p[k] for p in parts]) for k in parts[0]}
    del parts
    n = sum(counts)
    batch = rb.Batch(devs, counts, chunk=8192)
    hits = {k: torch.empty(n, dtype=devs[0].dtype, device="cuda") for k in ("x", "y", "z", "ux", "uy", "uz")}
    hits["fate"] = torch.empty(n, dtype=torch.uint8, device="cuda")
    hits["n_events"] = torch.empty(n, dtype=torch.uint8, device="cuda")
    hits["last_vol"] = torch.empty(n, dtype=torch.int32, device="cuda")
    hits["seq_hash"] = torch.empty(n, dtype=torch.int64, device="cuda")
    sums = batch.new_sums()
    batch.trace(rays, hits=hits, sums=sums)
    torch.cuda.synchronize()
    off = 0
    for v, (sc, c) in enumerate(zip(variants, counts)):
        for start in (0, c // 2, c - 1000):
            sl = slice(off + start, off + start + 1000)
            host = {k: rays[k][sl].double().cpu().numpy() for k in ("ox", "oy", "oz", "dx", "dy", "dz")}
            host["group"] = rays["group"][sl].cpu().numpy().astype(np.uint32)
            rec = oracle.trace(sc, host, id_base=start, log=True)
            compare(sc, host, as_numpy(hits, sl), rec, 1e-5 * sc.l_ref, 1e-5, id_base=start)
        assert float(sums[batch.goff[v] * 8]) == c
        off += c
