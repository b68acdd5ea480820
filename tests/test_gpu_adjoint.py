"""Reverse-mode gradients of the HIP library against the FP64 oracle.

The oracle's gradient is the pathwise (fixed-sequence) derivative by dual
numbers along each photon's recorded surface sequence; its dual numbers are
themselves pinned to central finite differences of forced sequences and to a
closed-form derivative (tests/test_oracle_pins.py).  Bar per component:
|g_gpu - g_ref| <= 1e-3 * max(|g_ref|, floor * max|g_ref|), with floor 1e-3
for FP64 scenes and 1e-2 for FP32 scenes, whose focal positions carry FP32
rounding into the centroid-subtracted cotangents of small components; FP32
components down to 1e-3 of the largest are held to 3e-3 relative as well
(measured worst: 1.4e-3, a primary coefficient of the small SC).
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


def gpu_grad(rb, sc, r, w_rms=None, w_eff=None, id_base=0):
    """Gradient by both backward modes: after a plain trace (sequences found
    again by a search) and after a trace that keeps its order (sequences
    replayed from the path records).  They must agree to FP64 summation
    order; the path-record gradient is returned."""
    dev = rb.Scene(sc)
    rays = dev.upload_rays(r)
    cot = torch.zeros(sc.n_groups, 2, dtype=torch.float64, device="cuda")
    if w_rms is not None:
        cot[:, 0] = torch.as_tensor(w_rms, dtype=torch.float64)
    if w_eff is not None:
        cot[:, 1] = torch.as_tensor(w_eff, dtype=torch.float64)
    out = []
    for keep in (False, True):
        sums = dev.new_sums()
        dev.trace(rays, sums=sums, id_base=id_base, keep_order=keep)
        grad = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
        dev.backward(rays, sums, cot, grad, id_base=id_base)
        torch.cuda.synchronize()
        out.append(grad.cpu().numpy())
    dev.close()
    scale = np.abs(out[0]).max()
    assert np.allclose(out[1], out[0], rtol=1e-9, atol=1e-12 * scale), np.abs(out[1] - out[0]).max() / scale
    return out[1]


def check(g, ref, floor, names):
    scale = np.abs(ref).max()
    assert scale > 0
    err = np.abs(g - ref) / np.maximum(np.abs(ref), floor * scale)
    worst = int(np.argmax(err))
    assert err.max() <= 1e-3, f"{names[worst]}: gpu {g[worst]:.6e} ref {ref[worst]:.6e} (rel {err.max():.2e})"
    if floor > 1e-3:
        # the smaller components of FP32 scenes, to a wider bar
        err2 = np.abs(g - ref) / np.maximum(np.abs(ref), 1e-3 * scale)
        w2 = int(np.argmax(err2))
        assert err2.max() <= 3e-3, f"{names[w2]}: gpu {g[w2]:.6e} ref {ref[w2]:.6e} (rel {err2.max():.2e})"
    return err.max()


def test_single_mirror_radius_fp64(rb):
    import oracle
    sc = scenes.single_mirror()
    r = sc.rays(50000)
    g = gpu_grad(rb, sc, r, w_rms=[1.0])
    rec = oracle.trace(sc, r, log=True)
    ref = oracle.gradient_rms(sc, r, rec, [1.0])
    assert abs(g[0] - ref[0]) <= 1e-9 * abs(ref[0])


@pytest.mark.parametrize("precision,n_per,floor", [(32, 3000, 1e-2), (64, 1000, 1e-3)])
def test_sc_rms_gradient(rb, precision, n_per, floor):
    import oracle
    sc = scenes.schwarzschild_couder(precision=precision)
    r = sc.rays(n_per)
    w = np.full(sc.n_groups, 1.0 / sc.n_groups)
    g = gpu_grad(rb, sc, r, w_rms=w)
    rec = oracle.trace(sc, r, log=True)
    ref = oracle.gradient_rms(sc, r, rec, w)
    e = check(g, ref, floor, sc.param_names)
    print(f"SC fp{precision}: 160 params, worst rel {e:.2e}")


@pytest.mark.parametrize("precision,n_per,floor", [(32, 10000, 1e-2), (64, 2000, 1e-3)])
def test_dc_rms_gradient(rb, precision, n_per, floor):
    import oracle
    sc = scenes.davies_cotton(precision=precision)
    r = sc.rays(n_per)
    w = np.full(sc.n_groups, 1.0 / sc.n_groups)
    g = gpu_grad(rb, sc, r, w_rms=w)
    rec = oracle.trace(sc, r, log=True)
    ref = oracle.gradient_rms(sc, r, rec, w)
    e = check(g, ref, floor, sc.param_names)
    print(f"DC fp{precision}: 594 params, worst rel {e:.2e}")


@pytest.mark.parametrize("precision,n_per,floor", [(32, 10000, 1e-2), (64, 2000, 1e-3)])
def test_lst_rms_gradient(rb, precision, n_per, floor):
    """The segmented parabolic dish: facet radii and tilts."""
    import oracle
    sc = scenes.lst_parabolic(precision=precision)
    r = sc.rays(n_per)
    w = np.full(sc.n_groups, 1.0 / sc.n_groups)
    g = gpu_grad(rb, sc, r, w_rms=w)
    rec = oracle.trace(sc, r, log=True)
    ref = oracle.gradient_rms(sc, r, rec, w)
    e = check(g, ref, floor, sc.param_names)
    print(f"LST fp{precision}: 594 params, worst rel {e:.2e}")


@pytest.mark.parametrize("precision,n_per,floor", [(32, 5000, 1e-2), (64, 1000, 1e-3)])
def test_small_sc_rms_gradient(rb, precision, n_per, floor):
    """The small SC: petal and secondary coefficients and tilts, with the
    structure's shadows removing photons from the figures."""
    import oracle
    sc = scenes.gct_sc(precision=precision)
    r = sc.rays(n_per)
    w = np.full(sc.n_groups, 1.0 / sc.n_groups)
    g = gpu_grad(rb, sc, r, w_rms=w)
    rec = oracle.trace(sc, r, log=True)
    ref = oracle.gradient_rms(sc, r, rec, w)
    e = check(g, ref, floor, sc.param_names)
    print(f"GCT fp{precision}: 30 params, worst rel {e:.2e}")


@pytest.mark.parametrize("precision,n_per,floor,lam", [(32, 20000, 1e-2, 400e-9), (64, 3000, 1e-3, 400e-9),
                                                      (64, 3000, 1e-3, 300e-9)])
def test_lens_rms_gradient(rb, precision, n_per, floor, lam):
    """The aspheric singlet: d(mean RMS)/d(front-face coefficients) through
    two refractions of a curved face (normal and Hessian terms)."""
    import oracle
    sc = scenes.aspheric_lens(precision=precision, lam=lam)
    r = sc.rays(n_per)
    w = np.full(sc.n_groups, 1.0 / sc.n_groups)
    g = gpu_grad(rb, sc, r, w_rms=w)
    rec = oracle.trace(sc, r, log=True)
    ref = oracle.gradient_rms(sc, r, rec, w)
    e = check(g, ref, floor, sc.param_names)
    print(f"lens fp{precision} {lam * 1e9:.0f} nm: 8 params, worst rel {e:.2e}")


@pytest.mark.parametrize("precision,n_per,floor", [(32, 20000, 1e-2), (64, 3000, 1e-3)])
def test_fresnel_rms_gradient(rb, precision, n_per, floor):
    """The Fresnel lens at 350 nm (off its design wavelength): d(mean RMS)
    / d(the 8 coefficients of each of its 10 zones)."""
    import oracle
    sc = scenes.fresnel_lens(precision=precision, lam=350e-9)
    r = sc.rays(n_per)
    w = np.full(sc.n_groups, 1.0 / sc.n_groups)
    g = gpu_grad(rb, sc, r, w_rms=w)
    rec = oracle.trace(sc, r, log=True)
    ref = oracle.gradient_rms(sc, r, rec, w)
    e = check(g, ref, floor, sc.param_names)
    print(f"fresnel fp{precision}: 80 params, worst rel {e:.2e}")


@pytest.mark.parametrize("precision", [32, 64])
def test_concentrator_weighted_collection_gradient(rb, precision):
    import oracle
    sc = scenes.hex_concentrator(precision=precision)
    r = sc.rays(300)
    w = np.full(sc.n_groups, 1.0 / sc.n_groups)
    g = gpu_grad(rb, sc, r, w_eff=w)
    rec = oracle.trace(sc, r, log=True)
    ref = oracle.gradient_eff_w(sc, r, rec, w)
    e = check(g, ref, 1e-3, sc.param_names)
    print(f"cone fp{precision}: 4 control scalars, worst rel {e:.2e}")


def test_gradient_matches_central_fd_of_forced_sequences(rb):
    """GPU adjoint vs central finite differences of the oracle's forced
    sequences (same photons, fates frozen) for a sample of parameters."""
    import oracle
    sc = scenes.schwarzschild_couder(precision=64)
    r = sc.rays(500)
    w = np.full(sc.n_groups, 1.0 / sc.n_groups)
    g = gpu_grad(rb, sc, r, w_rms=w)
    rec = oracle.trace(sc, r, log=True)
    foc = rec["fate"] == scenes.FATE_FOCUSED
    grp = rec["group"].astype(int)

    def loss(P):
        pos, _, st = oracle.forced(sc, r, rec, P)
        tot = 0.0
        for k in range(sc.n_groups):
            m = foc & (grp == k)
            x, y = pos[m, 0], pos[m, 1]
            tot += w[k] * np.sqrt(np.mean((x - x.mean()) ** 2 + (y - y.mean()) ** 2))
        return tot

    for j in (0, 2, 8, 11, 16, 40, 100, 159):
        h = 1e-7 if "tilt" in sc.param_names[j] else 1e-6 * abs(sc.params[j])
        P1, P2 = sc.params.copy(), sc.params.copy()
        P1[j] += h; P2[j] -= h
        fd = (loss(P1) - loss(P2)) / (2 * h)
        assert abs(g[j] - fd) <= 1e-3 * max(abs(fd), 1e-3 * np.abs(g).max()), sc.param_names[j]


def test_backward_split_launches_add_up(rb):
    """Gradients accumulate (+=): two launches over halves equal one launch."""
    sc = scenes.schwarzschild_couder()
    r = sc.rays(2000)
    dev = rb.Scene(sc)
    rays = dev.upload_rays(r)
    n = len(r["ox"])
    sums = dev.new_sums()
    dev.trace(rays, sums=sums)
    cot = torch.zeros(sc.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 0] = 1.0 / sc.n_groups
    g1 = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
    dev.backward(rays, sums, cot, g1)
    g2 = torch.zeros_like(g1)
    h = n // 3
    dev.backward({k: v[:h] for k, v in rays.items()}, sums, cot, g2, n=h)
    dev.backward({k: v[h:] for k, v in rays.items()}, sums, cot, g2, n=n - h, id_base=h)
    torch.cuda.synchronize()
    assert torch.allclose(g1, g2, rtol=1e-9, atol=1e-12 * float(g1.abs().max()))


def test_autograd_function(rb):
    """torch.autograd through RobastTrace: d(mean RMS)/d(params)."""
    sc = scenes.schwarzschild_couder()
    r = sc.rays(1000)
    dev = rb.Scene(sc)
    rays = dev.upload_rays(r)
    params = torch.tensor(sc.params, dtype=torch.float64, requires_grad=True)
    fig = rb.RobastTrace.apply(params, dev, rays)
    loss = fig[:, 4].mean()
    loss.backward()
    ref = gpu_grad(rb, sc, r, w_rms=np.full(sc.n_groups, 1.0 / sc.n_groups))
    assert np.allclose(params.grad.numpy(), ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())


def test_autograd_two_forwards_then_backward_and_cuda_params(rb):
    """backward of the first of two forward calls with different parameters
    is the gradient at the first call's parameters; CUDA params get a CUDA
    gradient of their own dtype."""
    sc = scenes.schwarzschild_couder()
    r = sc.rays(800)
    dev = rb.Scene(sc)
    rays = dev.upload_rays(r)
    p1 = torch.tensor(sc.params, dtype=torch.float64, device="cuda", requires_grad=True)
    p2 = (p1.detach() * (1 + 1e-3)).requires_grad_(True)
    loss1 = rb.RobastTrace.apply(p1, dev, rays)[:, 4].mean()
    loss2 = rb.RobastTrace.apply(p2, dev, rays)[:, 4].mean()
    loss1.backward()
    assert p1.grad.device.type == "cuda" and p1.grad.dtype == torch.float64
    loss2.backward()
    ref = gpu_grad(rb, sc, r, w_rms=np.full(sc.n_groups, 1.0 / sc.n_groups))
    # the scene restored to p1 rebuilds its frames from the tilt parameters,
    # which round to FP32 tables a little differently from the scene built
    # from the descriptors: agreement to FP32 table rounding, and far closer
    # than the gradient at p2
    e1 = np.abs(p1.grad.cpu().numpy() - ref).max()
    e2 = np.abs(p2.grad.cpu().numpy() - ref).max()
    assert e1 <= 1e-3 * np.abs(ref).max(), e1
    assert e1 < 0.1 * e2, (e1, e2)


@pytest.mark.parametrize("name,precision,n_per,tol", [("schwarzschild_couder", 64, 300, 1e-9),
                                                      ("schwarzschild_couder", 32, 1500, 1e-3),
                                                      ("hex_concentrator", 64, 8, 1e-9)])
def test_photon_cotangent_gradient(rb, name, precision, n_per, tol):
    """A per-photon loss sum_p c_p . (exit x, y, z, ux, uy, uz) of the FOCUSED
    photons, c_p random: the gradient against the oracle's dual numbers along
    the same sequences."""
    import oracle
    sc = scenes.ALL[name](precision=precision)
    r = sc.rays(n_per)
    n = len(r["ox"])
    rng = np.random.default_rng(17)
    c = rng.normal(size=(n, 6))
    dev = rb.Scene(sc)
    rays = dev.upload_rays(r)
    rec = oracle.trace(sc, r, log=True)
    # photons whose fate or sequence differ from the oracle's (grazing an
    # edge: at most the parity tests' rate) carry no cotangent, so both
    # sides sum over the same photons
    hits = dev.alloc_hits(n)
    dev.trace(rays, hits=hits)
    torch.cuda.synchronize()
    same = (hits["fate"].cpu().numpy() == rec["fate"]) & \
        (hits["seq_hash"].cpu().numpy().view(np.uint64) == rec["seq_hash"])
    assert same.sum() >= n - max(3, 1e-5 * n)
    c[~same] = 0.0
    pc = torch.from_numpy(c).cuda()
    for keep in (False, True):
        dev.trace(rays, sums=dev.new_sums(), keep_order=keep)
        g = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
        dev.backward(rays, None, None, g, photon_cot=pc)
        torch.cuda.synchronize()
        g = g.cpu().numpy()
        if keep:
            assert np.allclose(g, g_search, rtol=1e-9, atol=1e-12 * np.abs(g).max())
        g_search = g
    foc = rec["fate"] == scenes.FATE_FOCUSED
    ref = np.zeros(len(sc.params))
    for p0 in range(0, len(sc.params), 8):
        cnt = min(8, len(sc.params) - p0)
        dpos, ddir, st = oracle.forced_jac(sc, r, rec, sc.params, p0, cnt)
        m = foc & (st == 0)
        ref[p0:p0 + cnt] = np.einsum("nk,nkj->j", c[m, :3], dpos[m]) + np.einsum("nk,nkj->j", c[m, 3:], ddir[m])
    scale = np.abs(ref).max()
    err = np.abs(g - ref) / np.maximum(np.abs(ref), 1e-2 * scale)
    print(f"{name} fp{precision}: per-photon cotangent gradient, worst rel {err.max():.2e}")
    assert err.max() <= tol


def test_backward_sequence_check(rb):
    """The debug check: sequences re-derived by the backward pass equal the
    forward ones (OK); a forward hash changed by hand is reported
    (EMISMATCH), the gradient still accumulated."""
    sc = scenes.hex_concentrator()
    r = sc.rays(60)
    dev = rb.Scene(sc)
    rays = dev.upload_rays(r)
    n = len(r["ox"])
    hits = dev.alloc_hits(n)
    sums = dev.new_sums()
    dev.trace(rays, hits=hits, sums=sums)
    cot = torch.zeros(sc.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 1] = 1.0
    g1 = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
    dev.backward(rays, sums, cot, g1, fwd_hash=hits["seq_hash"], check=True)
    g0 = torch.zeros_like(g1)
    dev.backward(rays, sums, cot, g0)
    torch.cuda.synchronize()
    assert torch.allclose(g1, g0, rtol=1e-9, atol=0)
    bad = hits["seq_hash"].clone()
    bad[[3, 77]] ^= 1
    g2 = torch.zeros_like(g1)
    with pytest.raises(rb.RobastError) as ei:
        dev.backward(rays, sums, cot, g2, fwd_hash=bad, check=True)
    assert ei.value.status == rb.EMISMATCH and "2 photons" in str(ei.value)
    assert torch.allclose(g2, g0, rtol=1e-9, atol=0)


@pytest.mark.parametrize("name,n_per", [("hex_concentrator", 30), ("davies_cotton", 2000)])
def test_sequence_log_matches_oracle(rb, name, n_per):
    """seq_log holds each photon's event codes (volume << 8 | face << 4 |
    action): equal to the oracle's log wherever the fates agree."""
    import oracle
    sc = scenes.ALL[name]()
    r = sc.rays(n_per)
    n = len(r["ox"])
    dev = rb.Scene(sc)
    rays = dev.upload_rays(r)
    hits = dev.alloc_hits(n)
    hits["seq_log"] = torch.full((n * sc.max_events,), 0x7fffffff, dtype=torch.int32, device="cuda")
    dev.trace(rays, hits=hits)
    torch.cuda.synchronize()
    log = hits["seq_log"].cpu().numpy().view(np.uint32).reshape(n, sc.max_events)
    rec = oracle.trace(sc, r, log=True)
    same = (hits["seq_hash"].cpu().numpy().view(np.uint64) == rec["seq_hash"])
    assert same.mean() > 0.999
    lg = rec["log"]
    codes = (lg["vol"].astype(np.int64) << 8) | (lg["face"].astype(np.int64) << 4) | lg["act"].astype(np.int64)
    ne = rec["n_events"].astype(np.int64)
    k = np.arange(sc.max_events)[None, :]
    live = k < ne[:, None]
    assert np.array_equal(log[same][live[same]], codes[same][live[same]].astype(np.uint32))
    assert np.all(log[~live] == 0x7fffffff)


@pytest.mark.parametrize("precision,n_per,floor", [(32, 10000, 1e-2), (64, 2000, 1e-3)])
def test_lens_rms_gradient_with_wavelengths(rb, precision, n_per, floor):
    """The singlet traced over a spectrum (a wavelength per photon): the RMS
    gradient against the oracle's dual numbers along the same sequences,
    with each photon's own index."""
    import oracle
    sc = scenes.aspheric_lens(precision=precision)
    r = scenes.with_wavelengths(sc, sc.rays(n_per))
    dev = rb.Scene(sc)
    rays = dev.upload_rays(r, wavelengths=True)
    w = np.full(sc.n_groups, 1.0 / sc.n_groups)
    cot = torch.zeros(sc.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 0] = torch.as_tensor(w)
    out = []
    for keep in (False, True):
        sums = dev.new_sums()
        dev.trace(rays, sums=sums, keep_order=keep)
        g = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
        dev.backward(rays, sums, cot, g)
        torch.cuda.synchronize()
        out.append(g.cpu().numpy())
    assert np.allclose(out[1], out[0], rtol=1e-9, atol=1e-12 * np.abs(out[0]).max())
    rec = oracle.trace(sc, r, log=True, wavelengths=True)
    ref = oracle.gradient_rms(sc, r, rec, w)
    e = check(out[1], ref, floor, sc.param_names)
    print(f"lens spectrum fp{precision}: {len(sc.params)} params, worst rel {e:.2e}")
