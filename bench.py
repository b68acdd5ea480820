"""Benchmark: traced photons/s on the two-mirror Schwarzschild-Couder telescope.

Workload: 16 field angles (0..4 deg) x 1e7 photons = 1.6e8 photons per step,
FP32, synthetic scene and photon bundles (seeded), inputs resident in HBM
before timing starts.  One step is the whole hot path: forward trace with
per-field figure sums, the figures (centroid, RMS spot radius, efficiency),
and the reverse-mode gradient of the mean RMS with respect to the 160 scene
parameters (16 aspheric coefficients, 144 panel tilts).

Prints one JSON line (rank 0).  Also reported:
  roofline      the trace kernel's algorithmic VALU operations per second
                against the MI355X VALU issue rate (256 CU x 64 lanes x 2.4 GHz);
  cpu_baseline  the FP64 reference tracer on a bounded sample on the host.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

VALU_PEAK_OPS = 256 * 64 * 2.4e9        # lane-operations per second (non-packed)

# Algorithmic VALU cost per interaction, in lane-op slots (quarter-rate ops --
# sqrt, reciprocal, 32-bit integer multiply -- count 4): the exact
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
SHAPE_NAME = {1: "plane", 2: "sphere", 3: "asphere", 4: "cylinder", 5: "box", 6: "hexcone"}


def ops_per_photon(scene, rec):
    """Algorithmic VALU ops per photon from the reference tracer's event log."""
    lg = rec["log"]
    vol, act = lg["vol"], lg["act"]
    n = len(rec["fate"])
    total = 0.0
    shapes = scene.volumes["shape"]
    roles = scene.volumes["role"]
    refl = scene.volumes["reflectivity"]
    for k in range(vol.shape[1]):
        m = vol[:, k] >= 0
        if not m.any():
            continue
        v = vol[m, k]
        a = act[m, k]
        for sh in np.unique(shapes[v]):
            total += (COST["frame"] + COST[SHAPE_NAME[int(sh)]] + COST["normal"] + COST["hash"]) * \
                np.count_nonzero(shapes[v] == sh)
        total += COST["reflect"] * np.count_nonzero(a == 0) + COST["refract"] * np.count_nonzero(a == 1)
        lens = roles[v] == 2
        total += COST["draw"] * np.count_nonzero(((roles[v] == 1) & (refl[v] < 1.0)) | lens)
    # the final search that finds nothing (EXITED) still costs one frame test
    total += COST["frame"] * np.count_nonzero(rec["fate"] == 3)
    return total / n


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--photons-per-field", type=int, default=10_000_000)
    ap.add_argument("--cpu-sample-per-field", type=int, default=20_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_1508_07803_amd as rb
    import scenes

    assert torch.cuda.is_available(), "needs a HIP device"
    sc = scenes.schwarzschild_couder()
    dev = rb.Scene(sc)
    npf = args.photons_per_field
    n = npf * sc.n_groups
    # photon bundle, generated per field on the host and uploaded (untimed)
    rays = {k: torch.empty(n, dtype=torch.float32, device="cuda") for k in ("ox", "oy", "oz", "dx", "dy", "dz")}
    rays["group"] = torch.empty(n, dtype=torch.int32, device="cuda")
    t0 = time.time()
    for g in range(sc.n_groups):
        r = sc.rays(npf, seed=sc.seed + 1000 * g, groups=[g])
        for k in ("ox", "oy", "oz", "dx", "dy", "dz"):
            rays[k][g * npf:(g + 1) * npf].copy_(torch.from_numpy(r[k].astype(np.float32)))
        rays["group"][g * npf:(g + 1) * npf].copy_(torch.from_numpy(r["group"].astype(np.int32)))
        print(f"[bench] field {g}: {npf} photons uploaded", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    print(f"[bench] inputs ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    sums = dev.new_sums()
    grad = torch.zeros(len(sc.params), dtype=torch.float64, device="cuda")
    cot = torch.zeros(sc.n_groups, 2, dtype=torch.float64, device="cuda")
    cot[:, 0] = 1.0 / sc.n_groups                    # L = mean RMS over the fields
    do_bwd = not args.no_backward
    if do_bwd:
        try:
            dev.backward({k: v[:1] for k, v in rays.items()}, sums, cot, grad, n=1)
        except rb.RobastError as e:
            print(f"[bench] backward unavailable: {e}", file=sys.stderr, flush=True)
            do_bwd = False
    stream = torch.cuda.current_stream()
    ev_tr0, ev_tr1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def step(record):
        sums.zero_()
        if record:
            ev_tr0.record(stream)
        dev.trace(rays, sums=sums)
        if record:
            ev_tr1.record(stream)
        fig = dev.figures(sums)
        if do_bwd:
            grad.zero_()
            dev.backward(rays, sums, cot, grad)
        return fig

    for i in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i} done", file=sys.stderr, flush=True)
    trace_ms = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        fig = step(True)
        # per-launch duration of the trace kernel, measured on its own stream
        ev_tr1.synchronize()
        trace_ms.append(ev_tr0.elapsed_time(ev_tr1))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_per_step = 1e3 * t_total / args.steps
    figs = fig.cpu().numpy()
    print(f"[bench] {args.steps} steps in {t_total:.3f}s; trace kernel {np.mean(trace_ms):.3f} ms avg",
          file=sys.stderr, flush=True)

    # CPU baseline (reference tracer) on a bounded sample + op tallies
    cpu = None
    ops = None
    import oracle
    tally_rays = sc.rays(400, seed=sc.seed + 77)
    tally = oracle.trace(sc, tally_rays, log=True)
    ops = ops_per_photon(sc, tally)
    if not args.no_cpu_baseline:
        cores = os.cpu_count() or 1
        try:
            cores = len(os.sched_getaffinity(0))
        except AttributeError:
            pass
        cores = min(cores, 16)
        sample = sc.rays(args.cpu_sample_per_field, seed=sc.seed + 99)
        rec, dt = oracle.timed_trace(sc, sample, nthreads=cores)
        ncpu = len(sample["ox"])
        cpu = {"value": ncpu / dt, "unit": "photons/s", "cores": cores, "kind": "oracle",
               "sample": f"{ncpu} photons ({args.cpu_sample_per_field} per field x {sc.n_groups} fields) "
                         f"of the same scene, FP64 brute-force search, {dt:.1f}s"}
        print(f"[bench] cpu baseline {ncpu / dt:.3e} photons/s on {cores} threads", file=sys.stderr,
              flush=True)

    trace_s = np.mean(trace_ms) / 1e3
    achieved = ops * n / trace_s / 1e12
    out = {
        "metric": "traced photons/s (2-mirror SC, 1e7 rays per field)",
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
        "config": {"workload": "schwarzschild_couder: 16 fields x 1e7 photons, 72 aspheric panels, "
                               "forward + figures" + (" + adjoint (160 params)" if do_bwd else ""),
                   "photons_per_step": n, "fields": sc.n_groups, "precision": 32},
        "trace_kernel_ms": float(np.mean(trace_ms)),
        "trace_photons_per_s": n / trace_s,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "Tops/s", "frac": achieved * 1e12 / VALU_PEAK_OPS, "traffic": None,
                     "ops_per_photon": ops},
        "cpu_baseline": cpu,
        "figures": {"rms_mean_m": float(np.mean(figs[:, 4])), "efficiency_mean": float(np.mean(figs[:, 5]))},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
