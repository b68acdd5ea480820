"""robast_trace_static (the trace for callers that cannot allocate) against
robast_trace, through the C ABI: identical per-photon records and equal
group sums on two calls in a row, the second with fewer photons, and a
clear EINVAL for a bundle whose binning outgrows the fixed workspace."""
import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KEYS = ("fate", "n_events", "last_vol", "x", "y", "z", "ux", "uy", "uz", "opl", "seq_hash")


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1508_07803_amd as rb
    return rb


def _both(rb, dev, sc, rays, n):
    h1, h2 = dev.alloc_hits(n), dev.alloc_hits(n)
    s1, s2 = dev.new_sums(), dev.new_sums()
    dev.trace(rays, n=n, hits=h1, sums=s1)
    dev.trace_static(rays, n=n, hits=h2, sums=s2)
    torch.cuda.synchronize()
    for k in KEYS:
        assert torch.equal(h1[k], h2[k]), k
    a, b = s1.cpu().numpy(), s2.cpu().numpy()
    assert np.allclose(a, b, rtol=1e-12, atol=0), np.abs(a - b).max()
    assert a.reshape(-1, 8)[:, 0].sum() == n
    return h2


@pytest.mark.parametrize("name", ["schwarzschild_couder", "hex_concentrator"])
def test_static_trace_equals_trace(rb, name):
    sc = scenes.ALL[name]()
    dev = rb.Scene(sc)
    assert dev.tuning["bin_photons"] == 1
    # first call: binned (above the 32768 threshold), 1/3 of the workspace
    n1 = 300_000
    rays = dev.upload_rays(sc.rays((n1 + sc.n_groups - 1) // sc.n_groups, seed=7))
    _both(rb, dev, sc, rays, n1)
    # second call, smaller and ragged, reusing the workspace
    n2 = 40_001
    rays2 = dev.upload_rays(sc.rays((n2 + sc.n_groups - 1) // sc.n_groups, seed=8))
    _both(rb, dev, sc, rays2, n2)
    # below the binning threshold (no workspace used)
    _both(rb, dev, sc, rays2, 1000)


def test_static_trace_rejects_oversize(rb):
    sc = scenes.schwarzschild_couder()
    dev = rb.Scene(sc)
    n = 1_200_000
    parts = [scenes.device_rays(sc, n // 4, seed=9 + g, group=g) for g in (0, 5, 10, 15)]
    rays = {k: torch.cat([p[k] for p in parts]) for k in parts[0]}
    hits = dev.alloc_hits(n)
    with pytest.raises(rb.RobastError) as ei:
        dev.trace_static(rays, n=n, hits=hits)
    assert ei.value.status == rb.EINVAL and "static workspace" in str(ei.value)
    # with binning off the same bundle is traced, equal to robast_trace
    dev.set_tuning(bin_photons=0)
    _both(rb, dev, sc, rays, n)
