"""Launch tuning never changes a photon's result.

Photon binning (counting sort by entrance cell, optionally by direction
sector), the cell size, the grid size and the workgroup size only change which lane traces which photon and
in which order: every per-photon record must be bit-identical across tunings, group
sums and gradients equal up to FP64 summation order (1e-12 / 1e-9
relative).  The binned path is also what the parity tests against the
oracle exercise (their bundles exceed the binning threshold).
"""
import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TUNINGS = [dict(bin_photons=0, waves_mult=1),
           dict(bin_photons=1, waves_mult=1),
           dict(bin_photons=1, waves_mult=2, bin_target=512),
           dict(bin_photons=1, waves_mult=1, bin_target=16),
           dict(bin_photons=1, waves_mult=16),
           dict(bin_photons=1, waves_mult=4, block=64),
           dict(bin_photons=0, waves_mult=2, block=128),
           dict(bin_photons=1, waves_mult=4, bin_target=32, bin_dirs=16),
           dict(bin_photons=1, waves_mult=4, bin_target=8, bin_dirs=64),
           dict(bin_photons=1, waves_mult=4, bin_dirs=4),]


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1508_07803_amd as rb
    return rb


@pytest.mark.parametrize("name,n_per", [("schwarzschild_couder", 2500), ("davies_cotton", 8000),
                                        ("hex_concentrator", 400)])
def test_tunings_give_identical_photons(rb, name, n_per):
    sc = getattr(scenes, name)()
    r = sc.rays(n_per)
    dev = rb.Scene(sc)
    rays = dev.upload_rays(r)
    n = int(rays["ox"].numel())
    assert n >= 32768   # above the binning threshold
    runs = []
    for t in TUNINGS:
        dev.set_tuning(**t)
        hits = dev.alloc_hits(n)
        sums = dev.new_sums()
        dev.trace(rays, hits=hits, sums=sums, id_base=5)
        torch.cuda.synchronize()
        runs.append((hits, sums))
    h0, s0 = runs[0]
    for t, (h, s) in zip(TUNINGS[1:], runs[1:]):
        for k in h0:
            assert torch.equal(h0[k], h[k]), f"{t}: {k} differs"
        assert torch.allclose(s0, s, rtol=1e-12, atol=1e-12 * float(s0.abs().max())), t


def test_tunings_give_identical_gradients(rb):
    sc = scenes.schwarzschild_couder()
    r = sc.rays(2500)
    dev = rb.Scene(sc)
    rays = dev.upload_rays(r)
    cot = torch.zeros(sc.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 0] = 1.0 / sc.n_groups
    grads = []
    for t in TUNINGS[:3]:
        dev.set_tuning(**t)
        sums = dev.new_sums()
        dev.trace(rays, sums=sums)
        g = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
        dev.backward(rays, sums, cot, g)
        torch.cuda.synchronize()
        grads.append(g)
    for g in grads[1:]:
        assert torch.allclose(grads[0], g, rtol=1e-9, atol=1e-12 * float(grads[0].abs().max()))


def test_autotune_keeps_results(rb):
    sc = scenes.davies_cotton()
    r = sc.rays(10000)
    dev = rb.Scene(sc)
    rays = dev.upload_rays(r)
    n = int(rays["ox"].numel())
    ref = dev.alloc_hits(n)
    dev.trace(rays, hits=ref)
    best = dev.autotune(rays)
    assert best == dev.tuning
    assert best["bin_target"] >= 1 and best["waves_mult"] >= 1
    hits = dev.alloc_hits(n)
    dev.trace(rays, hits=hits)
    torch.cuda.synchronize()
    for k in ref:
        assert torch.equal(ref[k], hits[k]), k


def test_tuning_rejects_out_of_range(rb):
    dev = rb.Scene(scenes.single_mirror())
    for bad in (dict(bin_target=1 << 20), dict(waves_mult=0), dict(waves_mult=65), dict(bin_target=0),
                dict(block=96), dict(block=512), dict(bin_dirs=2), dict(bin_dirs=128)):
        with pytest.raises(rb.RobastError):
            dev.set_tuning(**bad)
    assert dev.tuning == dict(bin_photons=1, bin_target=128, waves_mult=4, block=256, bin_dirs=1)


def test_kept_order_reused_by_backward(rb):
    """trace(keep_order) + backward, and bin_photons + trace + backward, give
    the photons and gradients of independent calls."""
    sc = scenes.schwarzschild_couder()
    r = sc.rays(2500)
    dev = rb.Scene(sc)
    rays = dev.upload_rays(r)
    n = int(rays["ox"].numel())
    cot = torch.zeros(sc.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 0] = 1.0 / sc.n_groups

    def run(mode):
        hits = dev.alloc_hits(n)
        sums = dev.new_sums()
        if mode == "bin_first":
            dev.bin_photons(rays)
        dev.trace(rays, hits=hits, sums=sums, keep_order=(mode != "plain"))
        g = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
        dev.backward(rays, sums, cot, g)
        torch.cuda.synchronize()
        return hits, sums, g

    ref = run("plain")
    for mode in ("keep", "bin_first"):
        hits, sums, g = run(mode)
        for k in ref[0]:
            assert torch.equal(ref[0][k], hits[k]), (mode, k)
        assert torch.allclose(ref[1], sums, rtol=1e-12, atol=1e-12 * float(ref[1].abs().max()))
        assert torch.allclose(ref[2], g, rtol=1e-9, atol=1e-12 * float(ref[2].abs().max())), mode
    # a kept order is not used for other photon arrays
    dev.trace(rays, sums=dev.new_sums(), keep_order=True)
    other = {k: v.clone() for k, v in rays.items()}
    other["ox"] += 0.01
    g1 = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
    s1 = dev.new_sums()
    dev.trace(other, sums=s1)
    dev.backward(other, s1, cot, g1)
    dev.set_tuning(bin_photons=0)
    g2 = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
    s2 = dev.new_sums()
    dev.trace(other, sums=s2)
    dev.backward(other, s2, cot, g2)
    torch.cuda.synchronize()
    assert torch.allclose(g1, g2, rtol=1e-9, atol=1e-12 * float(g2.abs().max()))


def test_path_records_dropped_when_stale(rb):
    """The path records of a trace that kept its order are used only by the
    next backward call on the same photons and scene; a parameter update, a
    different count or id_base, or an intervening call makes the backward
    call search again, with the gradient of an independent computation."""
    sc = scenes.schwarzschild_couder()
    r = sc.rays(2500)
    rays_host = r
    cot = torch.zeros(sc.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 0] = 1.0 / sc.n_groups

    def fresh(params, n=None, id_base=0):
        d = rb.Scene(sc)
        d.update_params(params)
        rays = d.upload_rays(rays_host)
        s = d.new_sums()
        d.trace(rays, sums=s, n=n, id_base=id_base)
        g = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
        d.backward(rays, s, cot, g, n=n, id_base=id_base)
        torch.cuda.synchronize()
        return s, g

    def close(a, b):
        return torch.allclose(a, b, rtol=1e-9, atol=1e-12 * float(b.abs().max()))

    dev = rb.Scene(sc)
    rays = dev.upload_rays(r)
    n = int(rays["ox"].numel())
    # parameter update between the trace and the backward call
    p2 = np.array(sc.params) * (1 + 1e-4)
    s = dev.new_sums()
    dev.trace(rays, sums=s, keep_order=True)
    dev.update_params(p2)
    s2 = dev.new_sums()
    dev.trace(rays, sums=s2)                 # sums of the updated scene, order not kept
    g = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
    dev.backward(rays, s2, cot, g)
    torch.cuda.synchronize()
    ref_s, ref_g = fresh(p2)
    assert close(s2, ref_s) and close(g, ref_g)
    # a backward call on fewer photons than the kept trace (another binned
    # order): it must search, as after a trace that kept nothing
    m = n - 777
    s = dev.new_sums()
    dev.trace(rays, sums=s, keep_order=True)
    ga = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
    dev.backward(rays, s, cot, ga, n=m)
    sp = dev.new_sums()
    dev.trace(rays, sums=sp)
    gb = torch.zeros_like(ga)
    dev.backward(rays, sp, cot, gb, n=m)
    torch.cuda.synchronize()
    assert close(s, sp) and close(ga, gb)
    # the records are one-shot: a second backward call searches again
    s = dev.new_sums()
    dev.trace(rays, sums=s, keep_order=True)
    g1 = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
    g2 = torch.zeros_like(g1)
    dev.backward(rays, s, cot, g1)
    dev.backward(rays, s, cot, g2)
    torch.cuda.synchronize()
    assert close(g1, g2)
