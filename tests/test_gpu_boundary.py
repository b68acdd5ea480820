"""Boundary (fate-flip) gradient of the concentrator's collection efficiency
(robast_boundary_grad, edge sampling) against central finite differences
of the oracle's collection efficiency with common random numbers: the same
photons, ids and draws traced by the FP64 reference tracer at p +- h.

The comparison is statistical.  The edge-sampling estimate is averaged over
independent photon batches on the GPU (its standard error from their
spread); the finite difference's standard error follows from the number of
photons whose fate differs between p + h and p - h.  The design is the
8x8 array at 10-20 deg (below the cut-off, where the efficiency is a smooth
function of the control points) with the second interior control point
moved inward from the entrance radius, so that neighbouring walls do not
meet tangentially below the rim (there the efficiency has a kink).
"""
import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ANGLES = [10.0, 15.0, 20.0]
BASE = np.array([20.83333333, 14.43375673, 24.5, 36.08439182])


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1508_07803_amd as rb
    return rb


def _edge_sampling(rb, sc, npf, batches, band):
    dev = rb.Scene(sc)
    cot = torch.full((sc.n_groups,), 1.0 / sc.n_groups, dtype=torch.float64, device="cuda")
    est = []
    for b in range(batches):
        parts = [scenes.device_rays(sc, npf, seed=sc.seed + 7919 * b + 1000 * g, group=g) for g in range(sc.n_groups)]
        rays = {k: torch.cat([p[k] for p in parts]) for k in parts[0]}
        sums = dev.new_sums()
        dev.trace(rays, sums=sums)
        g = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
        dev.boundary_grad(rays, sums, cot, g, band=band)
        torch.cuda.synchronize()
        est.append(g.cpu().numpy())
    est = np.array(est)
    return est.mean(0), est.std(0, ddof=1) / np.sqrt(batches)


def _oracle_fd(sc, n_per, h):
    import oracle
    r = sc.rays(n_per, seed=sc.seed + 4242)
    n = len(r["ox"])
    g = np.asarray(r["group"]).astype(int)
    fd, se = [], []
    for k in range(len(sc.params)):
        foc = []
        for sgn in (1.0, -1.0):
            p = BASE.copy()
            p[k] += sgn * h
            s2 = scenes.hex_concentrator(angles_deg=ANGLES, control=p)
            foc.append(oracle.trace(s2, r)["fate"] == 1)
        eta = [np.mean([f[g == j].mean() for j in range(sc.n_groups)]) for f in foc]
        fd.append((eta[0] - eta[1]) / (2 * h))
        se.append(np.sqrt((foc[0] != foc[1]).sum()) / (2 * h * n))
    return np.array(fd), np.array(se)


def test_boundary_gradient_matches_oracle_finite_differences(rb):
    sc = scenes.hex_concentrator(angles_deg=ANGLES, control=BASE)
    es, es_se = _edge_sampling(rb, sc, 2_000_000, 6, band=0.01)
    fd, fd_se = _oracle_fd(sc, 200_000, h=0.25)
    print("edge sampling", es, "+-", es_se)
    print("oracle FD    ", fd, "+-", fd_se)
    sig = np.sqrt(es_se ** 2 + fd_se ** 2)
    assert np.all(np.abs(es - fd) < 4.0 * sig + 1e-5), (es, fd, sig)
    # the two largest components, rho1 and rho2, to 25 %
    for k in (0, 2):
        assert abs(es[k] - fd[k]) < 0.25 * abs(fd[k]), (k, es[k], fd[k])
    # not trivially zero
    assert abs(fd[2]) > 5 * fd_se[2]


def test_boundary_gradient_is_zero_where_nothing_flips(rb):
    """Far beyond the cut-off no photon is collected, and none is near
    being collected: the estimate is zero up to its own noise."""
    sc = scenes.hex_concentrator(angles_deg=[44.0, 45.0], control=BASE)
    es, es_se = _edge_sampling(rb, sc, 1_000_000, 4, band=0.01)
    assert np.all(np.abs(es) < 4.0 * es_se + 2e-5), (es, es_se)


def test_boundary_gradient_arguments(rb):
    sc = scenes.hex_concentrator(angles_deg=ANGLES, control=BASE)
    dev = rb.Scene(sc)
    rays = dev.upload_rays(sc.rays(100))
    sums = dev.new_sums()
    dev.trace(rays, sums=sums)
    cot = torch.ones(sc.n_groups, dtype=torch.float64, device="cuda")
    g = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
    for band in (0.0, 1.0, -0.1):
        with pytest.raises(rb.RobastError):
            dev.boundary_grad(rays, sums, cot, g, band=band)
    lam = torch.full_like(rays["ox"], 400e-9)
    with pytest.raises(rb.RobastError):
        dev.boundary_grad(dict(rays, lam=lam), sums, cot, g)


def test_boundary_gradient_binned_and_interleaved_with_backward(rb):
    """The boundary gradient over the binned order equals the one over the
    caller's order (up to FP64 summation order), and calling it between a
    trace that keeps its order and the backward call, with the same photons
    or with other ones, leaves the backward's gradient unchanged."""
    sc = scenes.hex_concentrator(angles_deg=ANGLES, control=BASE)
    dev = rb.Scene(sc)
    parts = [scenes.device_rays(sc, 40_000, seed=sc.seed + 1000 * g, group=g) for g in range(sc.n_groups)]
    rays = {k: torch.cat([p[k] for p in parts]) for k in parts[0]}
    other = {k: v.flip(0).contiguous() for k, v in rays.items()}
    ceta = torch.full((sc.n_groups,), 1.0 / sc.n_groups, dtype=torch.float64, device="cuda")
    cot = torch.zeros(sc.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 1] = 1.0 / sc.n_groups
    P = len(sc.params)

    def boundary(tuning):
        dev.set_tuning(**tuning)
        sums = dev.new_sums()
        dev.trace(rays, sums=sums)
        g = torch.zeros(P, dtype=torch.float64, device="cuda")
        dev.boundary_grad(rays, sums, ceta, g, band=0.02)
        return g

    g_plain = boundary(dict(bin_photons=0))
    for t in (dict(bin_photons=1, bin_dirs=1), dict(bin_photons=1, bin_dirs=16, bin_target=16)):
        g = boundary(t)
        assert torch.allclose(g, g_plain, rtol=1e-9, atol=1e-12 * float(g_plain.abs().max())), t
    assert float(g_plain.abs().max()) > 0

    dev.set_tuning(bin_photons=1, bin_dirs=1)
    grads = []
    for between in (None, rays, other):
        sums = dev.new_sums()
        dev.trace(rays, sums=sums, keep_order=True)
        if between is not None:
            s2 = dev.new_sums()
            if between is other:
                dev.trace(other, sums=s2)
            else:
                s2 = sums
            gb = torch.zeros(P, dtype=torch.float64, device="cuda")
            dev.boundary_grad(between, s2, ceta, gb, band=0.02)
        g = torch.zeros(P, dtype=torch.float64, device="cuda")
        dev.backward(rays, sums, cot, g)
        torch.cuda.synchronize()
        grads.append(g)
    for g in grads[1:]:
        assert torch.allclose(g, grads[0], rtol=1e-9, atol=1e-12 * float(grads[0].abs().max()))
