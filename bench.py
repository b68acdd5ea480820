"""Benchmark: traced photons/s on the two-mirror Schwarzschild-Couder telescope,
and the batched forward + adjoint design sweep against plain per-variant calls.

Workload (one step): 16 field angles (0..4 deg) x 1e7 photons = 1.6e8 photons,
FP32, synthetic seeded scene and photon bundles generated on the device before
timing starts.  A step is the whole hot path: photon binning, forward trace
with per-field figure sums, the figures (centroid, RMS spot radius,
efficiency), and the reverse-mode gradient of the mean RMS with respect to the
160 scene parameters (16 aspheric coefficients, 144 panel tilts).

Prints one JSON line.  Besides the contract fields:
  kernels       per-launch durations (HIP events on the launch stream) of
                the binning, trace and adjoint phases of the step;
  roofline      the dominant kernel's algorithmic VALU operations per second
                against the MI355X VALU issue rate (256 CU x 64 lanes x
                2.4 GHz); roofline_kernels gives it for both kernels;
  sweep         256 Davies-Cotton / Schwarzschild-Couder variants with
                log-uniform photon counts, 20 gradient-descent steps: the
                batched step (forward + adjoint + device update, one HIP
                graph) against plain per-variant calls from the same start;
  cpu_baseline  the FP64 reference tracer on a bounded sample on the host.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

VALU_PEAK_OPS = 256 * 64 * 2.4e9        # lane-operations per second (non-packed)

# Algorithmic VALU cost per interaction, in lane-op slots (quarter-rate ops --
# sqrt, reciprocal, 32-bit integer multiply -- count 4; FP64 ops count 1, the
# MI355X FP64 vector rate equals its non-packed FP32 rate): the exact
# intersection of the surface that is hit, its normal and the interaction.
# Acceleration-structure overhead (box tests of other candidates, grid walk)
# is not counted, so the figure is a lower bound of the work done.
COST = {
    "frame": 21,          # x_l = Q (x - c), d_l = Q d
    "plane": 10,
    "sphere": 60,         # stable quadratic, hemisphere + outline test
    "asphere": 230,       # z-slab and aperture bracket, 4 safeguarded Newton steps on the 8-term sag
    "cylinder": 40,
    "box": 45,            # six slabs, bounds
    "hexcone": 720,       # six walls: Bernstein cubic, critical points, ~6 Newton steps each
    "normal": 35,         # gradient, world normal, normalisation (rsqrt)
    "reflect": 10,
    "refract": 40,        # Fresnel (two divisions), Snell (sqrt)
    "draw": 90,           # Philox4x32-10: 20 32-bit multiplies (x4) + xors/adds
    "hash": 20,
}
# Reverse sweep, per event of a FOCUSED photon (FP64): pull-back through the
# interaction, the normal (with the surface Hessian), the hit point and the
# implicit root to the shape and tilt parameters.
PULLBACK = {"plane": 150, "sphere": 300, "asphere": 420, "cylinder": 250, "box": 200, "hexcone": 600}
SHAPE_NAME = {1: "plane", 2: "sphere", 3: "asphere", 4: "cylinder", 5: "box", 6: "hexcone"}

# sources each kernel is built from, and the scene compiler that lays out
# its tables (its counters go stale when any of them changes)
KERNEL_SOURCES = {
    "k_trace": ["device_trace.hpp", "kernels.hip", "kernels.hpp", "scene_layout.hpp", "abi.cpp"],
    "k_backward_path": ["device_trace.hpp", "adjoint_device.hpp", "adjoint.hip", "kernels.hpp", "scene_layout.hpp",
                        "abi.cpp"],
}
TRAFFIC_SUMMARY = os.path.join("profiles", "k_trace_k_backward_sc_16x1e7_hbm_traffic.md")


def event_cost(scene, v, a):
    """Forward cost of events at volumes v with actions a (arrays)."""
    shapes = scene.volumes["shape"][v]
    roles = scene.volumes["role"][v]
    refl = scene.volumes["reflectivity"][v]
    c = np.zeros(len(v))
    for sh, name in SHAPE_NAME.items():
        c += (shapes == sh) * (COST["frame"] + COST[name] + COST["normal"] + COST["hash"])
    c += COST["reflect"] * (a == 0) + COST["refract"] * (a == 1)
    c += COST["draw"] * (((roles == 1) & (refl < 1.0)) | (roles == 2))
    return c


def ops_per_photon(scene, rec):
    """Algorithmic VALU ops per photon of the forward trace and of the adjoint,
    from the reference tracer's event log."""
    lg = rec["log"]
    vol, act = lg["vol"], lg["act"]
    n = len(rec["fate"])
    fwd = np.zeros(n)
    per_event = np.zeros(vol.shape)
    for k in range(vol.shape[1]):
        m = vol[:, k] >= 0
        if m.any():
            per_event[m, k] = event_cost(scene, vol[m, k], act[m, k])
    fwd = per_event.sum(axis=1) + COST["frame"] * (rec["fate"] == 3)
    # adjoint along the recorded sequence of a FOCUSED photon: each event's
    # exact intersection, normal and interaction once (the state entering
    # it) and its pull-back; other photons need nothing
    adj = np.zeros(n)
    foc = rec["fate"] == 1
    shapes = scene.volumes["shape"]
    for e in range(vol.shape[1]):
        m = foc & (vol[:, e] >= 0)
        if not m.any():
            continue
        adj[m] += per_event[m, e]
        for sh, name in SHAPE_NAME.items():
            adj[m] += PULLBACK[name] * (shapes[vol[m, e]] == sh)
    return float(fwd.mean()), float(adj.mean())


def sources_digest(names):
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(ROOT, "paper_1508_07803_amd", "csrc", nm), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """Calibrated HBM bytes per launch of `kernel` from the committed counter
    summary, if its sources are the ones the counters were taken on."""
    path = os.path.join(ROOT, TRAFFIC_SUMMARY)
    if not os.path.exists(path):
        return None
    m = re.search(kernel + r"\s+traffic_bytes_per_launch:\s*([0-9.eE+]+)\s+sources_sha256_16:\s*([0-9a-f]{16})",
                  open(path).read())
    if not m or m.group(2) != sources_digest(KERNEL_SOURCES[kernel]):
        return None
    return float(m.group(1))


def ev(torch):
    return torch.cuda.Event(enable_timing=True)


def host_cores():
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return min(cores, 16)


def c3_bundle(scenes, torch, sc, npf):
    """16 fields x npf photons, generated on the device, field-major."""
    parts = [scenes.device_rays(sc, npf, seed=sc.seed + 1000 * g, group=g) for g in range(sc.n_groups)]
    rays = {k: torch.cat([p[k] for p in parts]) for k in parts[0]}
    return rays


def run_sweep(args, torch, rb, scenes):
    """The design sweep as an optimisation: 256 variants, each step a
    forward trace + figures + adjoint of each variant's RMS + a gradient
    step on the device.  Batched (one forward, one adjoint and one update
    launch, the whole step replayed from a HIP graph, launch shape from the
    batch autotuner) against plain per-variant calls, each over the same
    number of steps from the same start."""
    t0 = time.time()
    variants, counts = scenes.sweep()
    devs = [rb.Scene(v) for v in variants]
    parts = [scenes.device_rays(v, int(c), seed=v.seed + 17, group=0) for v, c in zip(variants, counts)]
    rays = {k: torch.cat([p[k] for p in parts]) for k in parts[0]}
    del parts
    n = int(counts.sum())
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    batch = rb.Batch(devs, counts, chunk=args.sweep_chunk)
    tuned = batch.autotune(rays)
    sums = batch.new_sums()
    fig = torch.zeros(batch.n_groups * rb.FIGURE_STRIDE, dtype=torch.float64, device="cuda")
    cot = torch.zeros(batch.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 0] = 1.0                                    # each variant: its own RMS at 1 deg
    grad = torch.zeros(batch.n_params, dtype=torch.float64, device="cuda")
    go, po = batch.goff, batch.poff
    P0 = torch.from_numpy(np.concatenate([d.params for d in devs])).cuda()
    P = P0.clone()
    status = torch.zeros(len(devs), dtype=torch.int32, device="cuda")
    sub = [{k: t[offs[v]:offs[v + 1]] for k, t in rays.items()} for v in range(len(devs))]
    print(f"[bench] sweep: {len(devs)} variants, {n:.3e} photons, ready in {time.time() - t0:.1f}s; "
          f"autotuned {tuned}", file=sys.stderr, flush=True)

    def batched_fb():
        sums.zero_()
        grad.zero_()
        batch.trace(rays, sums=sums, keep_order=True)
        batch.figures(sums, fig=fig)
        batch.backward(rays, sums, cot, grad)

    def plain_fb():
        sums.zero_()
        grad.zero_()
        for v, d in enumerate(devs):
            s_v = sums[go[v] * 8:go[v + 1] * 8]
            d.trace(sub[v], sums=s_v, keep_order=True)
            d.figures(s_v, fig=fig[go[v] * 8:go[v + 1] * 8])
            d.backward(sub[v], s_v, cot[go[v]:go[v + 1]], grad[po[v]:po[v + 1]])

    # the same photons and parameters through both paths give the same sums
    # and gradients (up to FP64 summation order)
    batched_fb()
    torch.cuda.synchronize()
    sums_b, grad_b = sums.clone(), grad.clone()
    plain_fb()
    torch.cuda.synchronize()
    rel_s = float(((sums - sums_b).abs() / sums_b.abs().clamp_min(1e-300)).max())
    rel_g = float((grad - grad_b).abs().max() / grad_b.abs().max().clamp_min(1e-300))
    # fixed GD step per family and parameter class, set from the first gradient
    g = grad_b.cpu().numpy()
    lr = []
    for v, d in enumerate(devs):
        gv = g[po[v]:po[v + 1]]
        tilt = np.array(["tilt" in nm for nm in d.src.param_names])
        sig = 1e-4 if d.src.name == "davies_cotton" else 5e-5
        lt = 0.2 * sig / max(np.abs(gv[tilt]).max(), 1e-300)
        ls = 2e-4 * np.abs(d.params[~tilt]).max() / max(np.abs(gv[~tilt]).max(), 1e-300)
        lr.append(np.where(tilt, lt, ls))
    LR = torch.from_numpy(np.concatenate(lr)).cuda()

    def plain_step():
        plain_fb()
        for v, d in enumerate(devs):
            d.gd_step(P[po[v]:po[v + 1]], grad[po[v]:po[v + 1]], LR[po[v]:po[v + 1]], status=status[v:v + 1])

    def batched_step():
        batched_fb()
        batch.gd_step(P, grad, LR, status=status)

    def run(step_fn):
        times, losses, rejected = [], [], 0
        for k in range(args.sweep_steps):
            a, b = ev(torch), ev(torch)
            a.record()
            step_fn()
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
            losses.append(float(fig.view(-1, rb.FIGURE_STRIDE)[:, 4].mean()))
            rejected += int((status != 0).sum())
        return times, losses, rejected

    # plain trajectory from the start parameters
    plain_step()                                   # warm-up step, then back to the start
    P.copy_(P0)
    batch.update_params(P)
    torch.cuda.synchronize()
    t_p, loss_p, rej_p = run(plain_step)
    P_plain = P.clone()
    # batched trajectory from the same start, the whole step from a HIP graph
    P.copy_(P0)
    batch.update_params(P)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batched_step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    P.copy_(P0)
    batch.update_params(P)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batched_step()
    torch.cuda.synchronize()
    t_b, loss_b, rej_b = run(graph.replay)
    dp = float(((P - P_plain).abs() / P_plain.abs().clamp_min(1e-300)).max())
    dl = max(abs(a - b) / abs(b) for a, b in zip(loss_b, loss_p))
    tb, tp = float(np.mean(t_b)), float(np.mean(t_p))
    print(f"[bench] sweep: {args.sweep_steps} GD steps, batched {tb:.1f} ms, plain {tp:.1f} ms per step; "
          f"mean RMS {loss_b[0] * 1e3:.4f} -> {loss_b[-1] * 1e3:.4f} mm; rejected updates {rej_b}/{rej_p}",
          file=sys.stderr, flush=True)
    return {
        "workload": "256 variants (128 Davies-Cotton, 128 Schwarzschild-Couder) at 1 deg, perturbed radii / "
                    "coefficients / tilts, photons per variant round(10^U(5,7)); one step = forward trace + "
                    "figures + adjoint of each variant's RMS + a gradient-descent update on the device",
        "photons_per_step": n, "variants": len(devs), "steps": args.sweep_steps, "tuning": tuned,
        "batched_ms_per_step": tb, "plain_ms_per_step": tp, "speedup": tp / tb,
        "batched_photons_per_s": n / (tb / 1e3), "plain_photons_per_s": n / (tp / 1e3),
        "batched": "one binning + forward launch, one adjoint launch and one update launch per step, "
                   "replayed from a HIP graph",
        "plain": f"{len(devs)} x (binning + trace + figures + coefficients + adjoint + update) launches",
        "max_rel_diff_batched_vs_plain": max(rel_s, rel_g),
        "trajectory_max_rel_diff": {"params": dp, "mean_rms": dl},
        "rejected_updates": {"batched": rej_b, "plain": rej_p},
        "mean_rms_m_per_step": loss_b,
    }


def cpu_baseline(scenes, sc, per_group, what):
    """The reference tracer on a bounded sample of a config's photons, on the
    host's cores (at most 16 threads, the host share of one GPU)."""
    import oracle
    cores = host_cores()
    sample = sc.rays(per_group, seed=sc.seed + 99)
    rec, dt = oracle.timed_trace(sc, sample, nthreads=cores)
    ncpu = len(sample["ox"])
    print(f"[bench] cpu baseline {sc.name}: {ncpu / dt:.3e} photons/s on {cores} threads ({ncpu} photons, "
          f"{dt:.1f} s)", file=sys.stderr, flush=True)
    return {"value": ncpu / dt, "unit": "photons/s", "cores": cores, "kind": "oracle",
            "sample": f"{ncpu} photons ({per_group} per group x {sc.n_groups} groups) of the same scene, "
                      f"{what}, FP64 brute-force search, {dt:.1f} s"}


def roofline(ops, n, ms, traffic=None):
    achieved = ops * n / (ms / 1e3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_OPS / 1e12, "unit": "Tops/s",
            "frac": achieved * 1e12 / VALU_PEAK_OPS, "traffic": traffic, "ops_per_photon": ops,
            "kernel_ms": ms}


def run_config(args, torch, rb, scenes, sc, npf, objective, cpu_per_group, describe):
    """One config's step on the device: binning + forward trace with group
    sums + figures + adjoint of the objective (objective: "rms" or "eff",
    the mean over the groups), under the launch tuning the autotuner picks
    on every 4th group of the bundle, per-phase times from HIP events, the roofline
    of both kernels from the reference tracer's event log, and the CPU
    baseline."""
    import oracle
    dev = rb.Scene(sc)
    t0 = time.time()
    parts = [scenes.device_rays(sc, npf, seed=sc.seed + 1000 * g, group=g) for g in range(sc.n_groups)]
    rays = {k: torch.cat([p[k] for p in parts]) for k in parts[0]}
    del parts
    n = int(rays["ox"].numel())
    torch.cuda.synchronize()
    print(f"[bench] {sc.name}: {n:.3e} photons generated on the device in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    # launch tuning from the autotuner on every photon of every 4th group
    # (each group at its full density, so the binning grid is the same)
    t0 = time.time()
    if args.config_tuning:
        tuning = dev.set_tuning(**json.loads(args.config_tuning))
    else:
        sample = (rays["group"] % 4) == 0
        tuning = dev.autotune({k: v[sample].contiguous() for k, v in rays.items()})
    print(f"[bench] {sc.name}: autotuned {tuning} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    sums = dev.new_sums()
    fig = torch.zeros(sc.n_groups * rb.FIGURE_STRIDE, dtype=torch.float64, device="cuda")
    grad = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
    cot = torch.zeros(sc.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 0 if objective == "rms" else 1] = 1.0 / sc.n_groups
    evs = [ev(torch) for _ in range(5)]
    t = {"binning": [], "trace": [], "adjoint": [], "step": []}
    for rep in range(args.config_steps + 1):
        sums.zero_()
        grad.zero_()
        evs[0].record()
        dev.bin_photons(rays)
        evs[1].record()
        dev.trace(rays, sums=sums, keep_order=True)
        evs[2].record()
        dev.figures(sums, fig=fig)
        evs[3].record()
        dev.backward(rays, sums, cot, grad)
        evs[4].record()
        torch.cuda.synchronize()
        if rep:   # the first step warms up
            t["binning"].append(evs[0].elapsed_time(evs[1]))
            t["trace"].append(evs[1].elapsed_time(evs[2]))
            t["adjoint"].append(evs[3].elapsed_time(evs[4]))
            t["step"].append(evs[0].elapsed_time(evs[4]))
    ms = {k: float(np.mean(v)) for k, v in t.items()}
    figs = fig.view(sc.n_groups, rb.FIGURE_STRIDE).cpu().numpy()
    boundary = None
    if objective == "eff":
        # the boundary (fate-flip) gradient of the mean collection efficiency,
        # edge sampling in a band of 0.01, on the same photons
        gb = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
        ceta = torch.full((sc.n_groups,), 1.0 / sc.n_groups, dtype=torch.float64, device="cuda")
        a, b = ev(torch), ev(torch)
        a.record()
        dev.boundary_grad(rays, sums, ceta, gb, band=0.01)
        b.record()
        torch.cuda.synchronize()
        boundary = {"ms": a.elapsed_time(b), "band": 0.01, "gradient": gb.cpu().numpy().tolist(),
                    "params": list(sc.param_names)}
        print(f"[bench] {sc.name}: boundary gradient {boundary['ms']:.1f} ms", file=sys.stderr, flush=True)
    tally = oracle.trace(sc, sc.rays(max(1, 40000 // sc.n_groups), seed=sc.seed + 77), log=True)
    ops_fwd, ops_adj = ops_per_photon(sc, tally)
    rk = {"k_trace": roofline(ops_fwd, n, ms["trace"]), "k_backward_path": roofline(ops_adj, n, ms["adjoint"])}
    dominant = "k_backward_path" if ms["adjoint"] > ms["trace"] else "k_trace"
    cpu = None if args.no_cpu_baseline else cpu_baseline(scenes, sc, cpu_per_group, "forward trace only")
    print(f"[bench] {sc.name}: step {ms['step']:.2f} ms (binning {ms['binning']:.2f}, trace {ms['trace']:.2f}, "
          f"adjoint {ms['adjoint']:.2f}); {n / (ms['step'] / 1e3):.3e} photons/s; trace frac "
          f"{rk['k_trace']['frac']:.3f}", file=sys.stderr, flush=True)
    col = 4 if objective == "rms" else 5
    return {"workload": describe, "photons": n, "ms_per_step": ms["step"],
            "photons_per_s": n / (ms["step"] / 1e3), "binning_ms": ms["binning"], "trace_ms": ms["trace"],
            "adjoint_ms": ms["adjoint"], "trace_photons_per_s": n / (ms["trace"] / 1e3), "tuning": tuning,
            "roofline": dict(rk[dominant], kernel=dominant), "roofline_kernels": rk, "cpu_baseline": cpu,
            ("rms_spot" if objective == "rms" else "efficiency"): figs[:, col].tolist(),
            "gradient_norm": float(grad.norm()), "boundary_gradient": boundary}


def run_single_mirror(args, torch, rb, scenes):
    """The single spherical mirror (FP64, 1e5 on-axis photons): trace with
    per-photon hit records and the RMS spot; launch-bound at this size."""
    sc = scenes.single_mirror()
    dev = rb.Scene(sc)
    rays = dev.upload_rays(sc.rays(100000))
    n = int(rays["ox"].numel())
    hits = {"fate": torch.empty(n, dtype=torch.uint8, device="cuda"),
            "x": torch.empty(n, dtype=torch.float64, device="cuda"),
            "y": torch.empty(n, dtype=torch.float64, device="cuda"),
            "z": torch.empty(n, dtype=torch.float64, device="cuda")}
    sums = dev.new_sums()
    fig = torch.zeros(sc.n_groups * rb.FIGURE_STRIDE, dtype=torch.float64, device="cuda")
    ts = []
    for rep in range(6):
        sums.zero_()
        a, b = ev(torch), ev(torch)
        a.record()
        dev.trace(rays, hits=hits, sums=sums)
        dev.figures(sums, fig=fig)
        b.record()
        torch.cuda.synchronize()
        if rep:
            ts.append(a.elapsed_time(b))
    ms = float(np.mean(ts))
    cpu = None if args.no_cpu_baseline else cpu_baseline(scenes, sc, 1_000_000, "forward trace only")
    print(f"[bench] single_mirror: {ms:.3f} ms per trace + figures ({n / (ms / 1e3):.3e} photons/s)",
          file=sys.stderr, flush=True)
    return {"workload": "single_mirror: R = 16 m, 4 m aperture, 1e5 on-axis photons, FP64; trace writing fate "
                        "and focal-plane hits + RMS spot", "photons": n, "ms_per_step": ms,
            "photons_per_s": n / (ms / 1e3), "rms_spot_m": float(fig[4].item()), "cpu_baseline": cpu}


def run_lst(args, torch, rb, scenes):
    """The segmented parabolic dish (198 facets on a parabola, 5 fields x
    1e7 photons): a binned trace writing fates and optical paths, then the
    arrival-time spread figures from those records."""
    sc = scenes.lst_parabolic()
    dev = rb.Scene(sc)
    npf = args.lst_photons_per_field
    parts = [scenes.device_rays(sc, npf, seed=sc.seed + 1000 * g, group=g) for g in range(sc.n_groups)]
    rays = {k: torch.cat([p[k] for p in parts]) for k in parts[0]}
    del parts
    n = int(rays["ox"].numel())
    hits = {"fate": torch.empty(n, dtype=torch.uint8, device="cuda"),
            "opl": torch.empty(n, dtype=torch.float32, device="cuda")}
    sums = dev.new_sums()
    out = torch.zeros(sc.n_groups * 4, dtype=torch.float64, device="cuda")
    t_tr, t_ar = [], []
    for rep in range(4):
        sums.zero_()
        e = [ev(torch) for _ in range(3)]
        e[0].record()
        dev.trace(rays, hits=hits, sums=sums)
        e[1].record()
        dev.arrival_figures(rays, hits, out=out)
        e[2].record()
        torch.cuda.synchronize()
        if rep:
            t_tr.append(e[0].elapsed_time(e[1]))
            t_ar.append(e[1].elapsed_time(e[2]))
    fig = dev.figures(sums).cpu().numpy()
    arr = out.view(sc.n_groups, 4).cpu().numpy()
    tt, ta = float(np.mean(t_tr)), float(np.mean(t_ar))
    print(f"[bench] lst: trace {tt:.2f} ms ({n / (tt / 1e3):.3e} photons/s), arrival figures {ta:.3f} ms",
          file=sys.stderr, flush=True)
    return {"workload": f"lst_parabolic: {sc.n_groups} fields (0-2 deg) x {npf:.0e} photons, 198 spherical facets on "
                        "a parabola; binning + trace writing fate and optical path, then arrival-time figures",
            "photons": n, "trace_ms": tt, "trace_photons_per_s": n / (tt / 1e3), "arrival_figures_ms": ta,
            "rms_spot_m": fig[:, 4].tolist(), "arrival_rms_path_m": arr[:, 2].tolist()}


def run_gct(args, torch, rb, scenes):
    """The small Schwarzschild-Couder telescope (6-petal primary, monolithic
    secondary, masts, trusses and camera body; 16 fields x 1e7 photons): the
    step of the main workload (binning + trace + figures + adjoint of the
    mean RMS over the 30 mirror parameters), then one trace writing fates and
    last volumes for the fraction of photons the structure absorbs."""
    sc = scenes.gct_sc()
    dev = rb.Scene(sc)
    npf = args.gct_photons_per_field
    parts = [scenes.device_rays(sc, npf, seed=sc.seed + 1000 * g, group=g) for g in range(sc.n_groups)]
    rays = {k: torch.cat([p[k] for p in parts]) for k in parts[0]}
    del parts
    n = int(rays["ox"].numel())
    cot = torch.zeros(sc.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 0] = 1.0 / sc.n_groups
    grad = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
    t = {"binning": [], "trace": [], "adjoint": []}
    for rep in range(4):
        sums = dev.new_sums()
        grad.zero_()
        e = [ev(torch) for _ in range(4)]
        e[0].record()
        dev.bin_photons(rays)
        e[1].record()
        dev.trace(rays, sums=sums, keep_order=True)
        e[2].record()
        dev.backward(rays, sums, cot, grad)
        e[3].record()
        torch.cuda.synchronize()
        if rep:
            for k, (a, b) in zip(t, ((0, 1), (1, 2), (2, 3))):
                t[k].append(e[a].elapsed_time(e[b]))
    fig = dev.figures(sums).cpu().numpy()
    hits = {"fate": torch.empty(n, dtype=torch.uint8, device="cuda"),
            "last_vol": torch.empty(n, dtype=torch.int32, device="cuda")}
    dev.trace(rays, hits=hits)
    st = torch.tensor(sc.meta["structure"], dtype=torch.int32, device="cuda")
    shadow = (hits["fate"] == scenes.FATE_ABSORBED) & torch.isin(hits["last_vol"], st)
    per_field = shadow.view(sc.n_groups, npf).double().mean(1).cpu().numpy()
    ms = {k: float(np.mean(v)) for k, v in t.items()}
    tot = sum(ms.values())
    print(f"[bench] gct: step {tot:.2f} ms (binning {ms['binning']:.2f}, trace {ms['trace']:.2f}, "
          f"adjoint {ms['adjoint']:.2f}; {n / (tot / 1e3):.3e} photons/s), structure shadow "
          f"{per_field.mean():.4f}", file=sys.stderr, flush=True)
    return {"workload": f"gct_sc: {sc.n_groups} fields (0-4.4 deg) x {npf:.0e} photons, small SC (6 aspheric "
                        "petals, monolithic aspheric secondary, 4 masts, 4 trusses, camera body); binning + "
                        f"trace + figures + adjoint ({len(sc.params)} params)",
            "photons": n, "ms_per_step": tot, "photons_per_s": n / (tot / 1e3),
            "binning_ms": ms["binning"], "trace_ms": ms["trace"], "adjoint_ms": ms["adjoint"],
            "rms_spot_m": fig[:, 4].tolist(), "structure_shadow_fraction": per_field.tolist()}


def run_chromatic(args, torch, rb, scenes, name="aspheric_lens"):
    """Wavelength as the batch axis: a refracting lens (the aspheric singlet
    or the Fresnel lens) at 16 wavelengths (300-600 nm; the same surfaces,
    the index of each wavelength), 4 fields x 2.5e6 photons each, with the
    launch tuning the autotuner picks.  One step = binning (if kept) +
    forward + figures + adjoint of every wavelength's RMS, batched (one
    forward and one adjoint launch) against per-wavelength calls."""
    lams = np.linspace(300e-9, 600e-9, 16)
    variants = [scenes.ALL[name](lam=float(l)) for l in lams]
    devs = [rb.Scene(v) for v in variants]
    npf = args.chromatic_photons_per_field
    parts = [scenes.device_rays(v, npf, seed=v.seed + 100 * i + g, group=g)
             for i, v in enumerate(variants) for g in range(v.n_groups)]
    rays = {k: torch.cat([p[k] for p in parts]) for k in parts[0]}
    del parts
    counts = [npf * v.n_groups for v in variants]
    n = int(sum(counts))
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    # launch tuning from the autotuner on the first wavelength's photons (the
    # surfaces are the same at every wavelength), applied to every variant
    # and so to both the batched and the plain path
    tuning = devs[0].autotune({k: t[offs[0]:offs[1]] for k, t in rays.items()})
    for d in devs:
        d.set_tuning(**tuning)
    batch = rb.Batch(devs, counts, chunk=args.sweep_chunk)
    sums = batch.new_sums()
    fig = torch.zeros(batch.n_groups * rb.FIGURE_STRIDE, dtype=torch.float64, device="cuda")
    cot = torch.zeros(batch.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 0] = 1.0
    grad = torch.zeros(batch.n_params, dtype=torch.float64, device="cuda")
    go, po = batch.goff, batch.poff
    sub = [{k: t[offs[v]:offs[v + 1]] for k, t in rays.items()} for v in range(len(devs))]

    def batched_step():
        sums.zero_()
        grad.zero_()
        batch.trace(rays, sums=sums, keep_order=True)
        batch.figures(sums, fig=fig)
        batch.backward(rays, sums, cot, grad)

    def plain_step():
        sums.zero_()
        grad.zero_()
        for v, d in enumerate(devs):
            s_v = sums[go[v] * 8:go[v + 1] * 8]
            d.trace(sub[v], sums=s_v, keep_order=True)
            d.figures(s_v, fig=fig[go[v] * 8:go[v + 1] * 8])
            d.backward(sub[v], s_v, cot[go[v]:go[v + 1]], grad[po[v]:po[v + 1]])

    t_b, t_p = [], []
    for rep in range(4):
        for step, out in ((batched_step, t_b), (plain_step, t_p)):
            a, b = ev(torch), ev(torch)
            a.record()
            step()
            b.record()
            torch.cuda.synchronize()
            if rep:
                out.append(a.elapsed_time(b))
    batched_step()
    rms = fig.view(-1, rb.FIGURE_STRIDE)[:, 4].cpu().numpy()
    on_axis = [float(rms[go[v]]) for v in range(len(devs))]
    tb, tp = float(np.mean(t_b)), float(np.mean(t_p))
    print(f"[bench] chromatic {name} ({tuning}): batched {tb:.2f} ms, plain {tp:.2f} ms ({n / (tb / 1e3):.3e} photons/s); "
          f"on-axis RMS {min(on_axis) * 1e3:.2f}-{max(on_axis) * 1e3:.2f} mm", file=sys.stderr, flush=True)
    fields = ", ".join(f"{np.degrees(g):g}" for g in variants[0].groups)
    return {"workload": f"{name} at 16 wavelengths (300-600 nm, Cauchy index) x 4 fields ({fields} deg) x "
                        f"{npf:.1e} photons; one step = binning + forward + figures + adjoint "
                        f"({len(variants[0].params)} surface coefficients per wavelength)",
            "photons_per_step": n, "batched_ms_per_step": tb, "plain_ms_per_step": tp,
            "batched_photons_per_s": n / (tb / 1e3), "speedup": tp / tb, "tuning": tuning,
            "wavelengths_nm": (lams * 1e9).tolist(), "on_axis_rms_m": on_axis}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--photons-per-field", type=int, default=10_000_000)
    ap.add_argument("--cpu-sample-per-field", type=int, default=62_500)
    ap.add_argument("--config-steps", type=int, default=3)
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the single-mirror, Davies-Cotton and concentrator sections")
    ap.add_argument("--configs", default="single_mirror,davies_cotton,hex_concentrator",
                    help="which of those sections to run (comma-separated)")
    ap.add_argument("--config-tuning", default=None,
                    help="JSON launch tuning for the config sections instead of the autotuner's "
                         "(for profiling runs), e.g. '{\"bin_target\": 32, \"bin_dirs\": 4}'")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--sweep-steps", type=int, default=20)
    ap.add_argument("--sweep-chunk", type=int, default=8192)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--lst-photons-per-field", type=int, default=10_000_000)
    ap.add_argument("--no-lst", action="store_true")
    ap.add_argument("--gct-photons-per-field", type=int, default=10_000_000)
    ap.add_argument("--no-gct", action="store_true")
    ap.add_argument("--chromatic-photons-per-field", type=int, default=2_500_000)
    ap.add_argument("--no-chromatic", action="store_true")
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="copy this many GiB device to device first (a known-size kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_1508_07803_amd as rb
    import scenes

    assert torch.cuda.is_available(), "needs a HIP device"
    if args.calibrate_copy_gib > 0:
        nel = int(args.calibrate_copy_gib * (1 << 30)) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {nel * 4} bytes done", file=sys.stderr, flush=True)
        del src, dst
    sc = scenes.schwarzschild_couder()
    dev = rb.Scene(sc)
    npf = args.photons_per_field
    n = npf * sc.n_groups
    t0 = time.time()
    rays = c3_bundle(scenes, torch, sc, npf)
    torch.cuda.synchronize()
    print(f"[bench] {n:.3e} photons generated on the device in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)

    sums = dev.new_sums()
    fig = torch.zeros(sc.n_groups * rb.FIGURE_STRIDE, dtype=torch.float64, device="cuda")
    grad = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
    cot = torch.zeros(sc.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 0] = 1.0 / sc.n_groups                    # L = mean RMS over the fields
    do_bwd = not args.no_backward
    stream = torch.cuda.current_stream()
    evs = [ev(torch) for _ in range(5)]

    def step():
        sums.zero_()
        evs[0].record(stream)
        dev.bin_photons(rays)                         # counting sort by entrance cell
        evs[1].record(stream)
        dev.trace(rays, sums=sums, keep_order=do_bwd)    # + path records for the adjoint
        evs[2].record(stream)
        dev.figures(sums, fig=fig)
        grad.zero_()
        evs[3].record(stream)
        if do_bwd:
            dev.backward(rays, sums, cot, grad)      # binned order and paths of the trace
        evs[4].record(stream)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"[bench] warmup {i} done", file=sys.stderr, flush=True)
    k_bin, k_trace, k_bwd = [], [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step()
        evs[4].synchronize()
        k_bin.append(evs[0].elapsed_time(evs[1]))
        k_trace.append(evs[1].elapsed_time(evs[2]))
        k_bwd.append(evs[3].elapsed_time(evs[4]))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_per_step = 1e3 * t_total / args.steps
    figs = fig.view(sc.n_groups, rb.FIGURE_STRIDE).cpu().numpy()
    print(f"[bench] {args.steps} steps in {t_total:.3f}s; binning {np.mean(k_bin):.2f} ms, trace "
          f"{np.mean(k_trace):.2f} ms, adjoint {np.mean(k_bwd):.2f} ms per step", file=sys.stderr, flush=True)

    sweep = None if args.no_sweep else run_sweep(args, torch, rb, scenes)
    lst = None if args.no_lst else run_lst(args, torch, rb, scenes)
    gct = None if args.no_gct else run_gct(args, torch, rb, scenes)
    chromatic = None if args.no_chromatic else {
        nm: run_chromatic(args, torch, rb, scenes, nm) for nm in ("aspheric_lens", "fresnel_lens")}
    configs = None
    if not args.no_configs:
        want = set(args.configs.split(","))
        runs = {
            "single_mirror": lambda: run_single_mirror(args, torch, rb, scenes),
            "davies_cotton": lambda: run_config(
                args, torch, rb, scenes, scenes.davies_cotton(), 10_000_000, "rms", 1_000_000,
                "davies_cotton: 5 fields (0-2 deg) x 1e7 photons, 198 spherical facets, camera box and masts; "
                "binning + trace + figures + adjoint of the mean RMS (594 params: radii, tilts)"),
            "hex_concentrator": lambda: run_config(
                args, torch, rb, scenes, scenes.hex_concentrator(), 1_000_000, "eff", 11_000,
                "hex_concentrator: 91 incidence angles (0-45 deg) x 1e6 photons, 8x8 Bezier hex cones under a "
                "PMMA window, up to 32 events; binning + trace + figures + adjoint of the mean weighted "
                "collection efficiency (4 control-point coordinates), and the boundary gradient of the "
                "mean collection efficiency"),
        }
        configs = {k: f() for k, f in runs.items() if k in want}

    # algorithmic op tallies from the reference tracer's event log
    import oracle
    tally = oracle.trace(sc, sc.rays(400, seed=sc.seed + 77), log=True)
    ops_fwd, ops_adj = ops_per_photon(sc, tally)
    cpu = None if args.no_cpu_baseline else cpu_baseline(scenes, sc, args.cpu_sample_per_field,
                                                          "forward trace only")

    t_trace, t_bwd = float(np.mean(k_trace)), float(np.mean(k_bwd))
    rk = {"k_trace": roofline(ops_fwd, n, t_trace, measured_traffic("k_trace"))}
    if do_bwd:
        rk["k_backward_path"] = roofline(ops_adj, n, t_bwd, measured_traffic("k_backward_path"))
    dominant = "k_backward_path" if do_bwd and t_bwd > t_trace else "k_trace"
    out = {
        "metric": "traced photons/s (2-mirror SC, 1e7 rays); batched fwd+adjoint vs plain, 1 GPU",
        "value": n / (ms_per_step / 1e3),
        "unit": "photons/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "schwarzschild_couder: 16 fields (0-4 deg) x 1e7 photons, 72 aspheric panels, "
                               "binning + forward + figures" + (" + adjoint (160 params)" if do_bwd else ""),
                   "photons_per_step": n, "fields": sc.n_groups, "precision": 32},
        "kernels": {"binning_ms": float(np.mean(k_bin)), "trace_ms": t_trace, "adjoint_ms": t_bwd,
                    "trace_photons_per_s": n / (t_trace / 1e3)},
        "roofline": dict(rk[dominant], kernel=dominant),
        "roofline_kernels": rk,
        "sweep": sweep,
        "lst": lst,
        "gct": gct,
        "chromatic": chromatic,
        "configs": configs,
        "cpu_baseline": cpu,
        "figures": {"rms_mean_m": float(np.mean(figs[:, 4])), "efficiency_mean": float(np.mean(figs[:, 5]))},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
