#!/usr/bin/env python3
"""Benchmark: histories/s on the ~20k-facet synthetic HPGe detector.

Workload: p-type coaxial HPGe detector (crystal r 32 mm, h 60 mm, 5 mm bore,
0.7 mm dead layer, Al cup / end-cap / window), 20236 facets, in an air box;
isotropic point source 250 mm above the end-cap; 12 log-spaced energies
40-2000 keV; per energy N_e = max(1e8, histories for a 0.5 % FEPE relative
standard error, from a 1e7-history pilot).  One step = one persistent
launch transporting all 12 x N_e histories (inputs already resident on the
GPU).  Also reported: the same step with score-function gradients for the
five detector density groups (fwd+grad / fwd cost), the ALU roofline of the
transport kernel and the CPU oracle on a bounded sample.

python bench.py [--gpus 1] [--steps K] [--warmup W]
python bench.py --workload {c2near,c3,c4,c5,build} [--steps K] [--warmup W]
    secondary workloads (one JSON line each, not the metric): the same detector
    with the source at 100 mm; 64 bottle jobs batched against one launch per job;
    volume source with gradients; the ~1M-facet Marinelli stress case; mesh
    preparation times.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic VALU lane-operations per event of the method, counted from its
# arithmetic (one FP32/INT32 operation = 1; a transcendental, which issues at
# quarter rate on the vector ALU, = 4).  The derivation of each figure is given
# with the roofline discussion of the design notes.
OPS_PER_EVENT = {
    "rng_calls": 116,    # Philox4x32-10: 10 x (2 mul_lo + 2 mul_hi + 4 xor + 2 add), + 4 uniforms
    "emissions": 35,     # isotropic direction, -ln u, energy-grid index
    "segments": 76,      # 3 log-log partials (3 exp), 1/mu, ray set-up (3 rcp, shear), move
    "node_visits": 36,   # two slab tests (12 FMA, 12 min/max) + near/far order + stack
    "tri_tests": 40,     # watertight test: 9 sub, 6 shear FMA, 3 edge fns, signs, det, T
    "photo": 8,
    "compton": 100,      # Butcher-Messel sampling (~1.3 trials), deposit, rotation, re-index
    "coherent": 70,      # Cardano inverse of the Thomson CDF, rotation
    "crossings": 10,     # region update, tau update, bookkeeping
    "locates": 40,       # probe-ray set-up (its traversal is in node_visits/tri_tests)
    "plane_tests": 13,   # exit plane: two 3-term dot products, reciprocal, product, min
    "box_tests": 30,     # screened history: ray set-up (3 rcp, 3 products) + one slab test
    "cone_tests": 5,     # screened history: direction against the cone around the inner box
    "pair": 40,          # pair event: deposit, annihilation axis (sqrt, sin, cos), LDS store
}
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz one-lane-op slots per second
PEAK_SCLK_MHZ = 2400.0
PEAK_LANE_OPS = 256 * 4 * 16 * PEAK_SCLK_MHZ * 1e6

# HBM bytes per timed launch of this workload, from FETCH_SIZE / WRITE_SIZE counter
# runs scaled by a copy probe (profiles/transport_hpge20k_counters.md), valid only
# for the kernel sources they were taken with (SHA-256 of the files below).
KERNEL_SOURCES = ["paper_2605_25963_amd/csrc/transport.hip",
                  "paper_2605_25963_amd/csrc/transport_common.h",
                  "paper_2605_25963_amd/csrc/device_common.h",
                  "paper_2605_25963_amd/csrc/gadep_internal.h",
                  "paper_2605_25963_amd/csrc/runtime.cpp",
                  "paper_2605_25963_amd/csrc/mesh_prep.cpp"]
MEASURED_TRAFFIC = {"sources_sha256": "5326819c08314fe5d5b4bf7ba552d5e70791894386ea2ab9d3bb5dcc0c158e8f",
                    "bytes_per_launch": 6.133e+07}


def measured_traffic():
    """Counter-measured HBM bytes per launch, or None once the kernel has changed."""
    import hashlib
    h = hashlib.sha256()
    try:
        for f in KERNEL_SOURCES:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
    except OSError:
        return None
    if h.hexdigest() != MEASURED_TRAFFIC["sources_sha256"]:
        return None
    return MEASURED_TRAFFIC["bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--min-histories", type=float, default=1e8, help="per energy")
    ap.add_argument("--pilot", type=float, default=1e7)
    ap.add_argument("--cpu-seconds", type=float, default=60.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the one-step summaries of the C3, C4 and C5 workloads on the metric line")
    ap.add_argument("--guide", type=int, default=None,
                    help="ablation: GADEP_OPT_GUIDE for the metric workload (0 = fixed claims)")
    ap.add_argument("--claim", type=int, default=None, help="ablation: GADEP_OPT_CLAIM")
    ap.add_argument("--split-pct", type=int, default=None,
                    help="ablation: GADEP_OPT_SPLIT_PCT (transport BVH split budget, %%)")
    ap.add_argument("--quick", action="store_true",
                    help="profiling run: 1e7 histories per energy, no grad, no CPU baseline")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device-to-device three times (scales HBM byte counters)")
    ap.add_argument("--workload", default="c2",
                    choices=["c2", "c2near", "c3", "c4", "c5", "build"],
                    help="c2: the metric (default); c2near: same at 100 mm; c3: 64 bottle jobs "
                         "batched vs one launch each; c4: volume source, fwd+grad/fwd; c5: "
                         "~1M facets, Marinelli, 16 matrices, lines, spectra; build: mesh "
                         "preparation + upload times")
    a = ap.parse_args()
    if a.quick:
        a.min_histories, a.pilot, a.no_grad, a.no_cpu_baseline = 1e7, 1e6, True, True
        a.no_secondary = True
    return a


def cpu_baseline(w, target_s):
    """The oracle on the host cores, on a bounded sample of the same workload:
    rounds over all energies (disjoint history ranges) until target_s has
    passed."""
    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    s = oracle.scene_from_workload(w)
    # calibrate the size of one round (about a fifth of the target)
    t0 = time.perf_counter()
    for k, E in enumerate(w.energies):
        s.run(w.source, E, 50_000, 2002, unit=k, threads=threads)
    t_cal = time.perf_counter() - t0
    per_e = max(50_000, int(50_000 * 0.2 * target_s / max(t_cal, 1e-3)))
    t0 = time.perf_counter()
    n = 0
    rounds = 0
    while True:
        for k, E in enumerate(w.energies):
            r = s.run(w.source, E, per_e, 2002, unit=k, first=(rounds + 1) * per_e, threads=threads)
            n += r.tally.n_histories
        rounds += 1
        if time.perf_counter() - t0 >= target_s:
            break
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "histories/s", "cores": threads, "kind": "oracle",
            "per_core": n / dt / threads,
            "sample": f"{rounds} rounds of {per_e} histories at each of the {len(w.energies)} energies "
                      f"({n} total, {dt:.1f} s), same detector and source",
            "host": host_cpu()}


def host_cpu():
    """Model name of the host CPU and the number of logical CPUs the OS reports."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{name}, {os.cpu_count()} logical CPUs"


def copy_probe():
    """A plain copy of known size: its FETCH_SIZE / WRITE_SIZE per dispatch give the
    factor that turns those counters into bytes."""
    import torch
    n = 1 << 30
    x = torch.empty(n, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n, "dispatches": 3}), flush=True)


def main():
    a = parse()
    if a.copy_probe:
        copy_probe()
        return
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {a.gpus}); the transport "
              "shards over independent histories, see the design notes", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2605_25963_amd import gadep
    from workloads import configs as C

    if a.workload not in ("c2", "c2near"):
        print(json.dumps(OTHER[a.workload](a, torch, gadep, C)), flush=True)
        return
    distance = 250.0 if a.workload == "c2" else 100.0
    stream = torch.cuda.current_stream()
    ctx = _ablate(gadep.Context(0, stream if stream.cuda_stream else None), a, gadep)
    m = measure(a, torch, gadep, C, ctx, distance, a.steps, a.warmup, full=True)
    near = None
    if a.workload == "c2" and not a.quick:
        # the same detector with the source at 100 mm, where more histories enter it
        mn = measure(a, torch, gadep, C, ctx, 100.0, min(a.steps, 5), 1, full=False)
        near = {"value": mn["total"] / mn["dt"], "unit": "histories/s", "ms_per_step": mn["dt"] * 1e3,
                "histories_per_step": mn["total"], "max_fepe_rse": float(mn["rse"].max()),
                "frac": mn["roof"]["frac"], "kernel_ms": mn["roof"]["kernel_ms"],
                "active_lanes": mn["roof"]["active_lanes"]}
    cone = None
    if a.workload == "c2" and not a.quick:
        cone = measure_cone(a, torch, gadep, C, ctx, min(a.steps, 5))
    secondary = None
    if a.workload == "c2" and not a.no_secondary:
        # one warm-up and one timed step of each secondary workload, so that
        # the metric's own run reports them too
        secondary = {}
        sa = argparse.Namespace(**vars(a))
        sa.steps, sa.warmup = 1, 1
        skip = ("metric", "n_gpus", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline",
                "dtype", "data")
        for name in ("c3", "c4", "c5"):
            try:
                r = OTHER[name](sa, torch, gadep, C)
                secondary[name] = {k: v for k, v in r.items() if k not in skip}
            except Exception as e:  # a failure here must not cost the metric line
                secondary[name] = {"error": repr(e)}
            print(f"bench: secondary workload {name} done", file=sys.stderr, flush=True)
    w = m["w"]
    base = None if a.no_cpu_baseline else cpu_baseline(w, a.cpu_seconds)
    if base:
        base["gpu_over_oracle"] = m["total"] / m["dt"] / base["value"]
    line = {
        "metric": "histories/s on 20k-tri HPGe mesh at <=0.5% FEPE RSE; fwd+grad/fwd cost",
        "value": m["total"] / m["dt"],
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": m["dt"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"hpge_coaxial_20236_facets_point_{distance:.0f}mm_12_energies",
                   "n_facets": int(len(w.scene.tri)), "energies_keV": [round(e, 3) for e in w.energies],
                   "histories_per_energy": [int(x) for x in m["n_e"]], "histories_per_step": m["total"],
                   "max_fepe_rse": float(m["rse"].max()),
                   **({"ablation": {"guide": a.guide, "claim": a.claim, "split_pct": a.split_pct}}
                      if (a.guide, a.claim, a.split_pct) != (None, None, None) else {})},
        "fwd_grad_over_fwd": m["fwd_grad_ratio"],
        "batched_grad_vs_single_job": m["batched_vs_single"],
        "fepe": [float(x) for x in m["fepe"]],
        "rates": m["rates"],
        "roofline": m["roof"],
        "c2_source_100mm": near,
        "cone_emission": cone,
        "secondary_workloads": secondary,
        "cpu_baseline": base,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def measure_cone(a, torch, gadep, C, ctx, steps):
    """The metric's detector and source with cone emission (variance reduction,
    not the metric): histories start only towards the detector and carry the
    weight Omega/4pi.  N per energy is sized for the same 0.5 % FEPE RSE; the
    analog-equivalent rate counts the analog histories that RSE would take."""
    w = C.c2_hpge(n_histories=0)
    gadep.load_workload(ctx, w)
    src = C.Source(C.KIND_CONE, pos=w.source.pos)

    def jobs(n_per_e):
        return [dict(source=src, energies=[E], n_histories=int(n_per_e[k]), stream=k)
                for k, E in enumerate(w.energies)]

    pilot = ctx.run_batch(jobs([1e6] * len(w.energies)), 998)
    wt = pilot.weights()
    q0 = np.maximum(pilot.fepe() / wt, 1e-12)  # FEP probability per cone history
    q = np.maximum(q0 - 3.0 * np.sqrt(q0 * (1 - q0) / 1e6), 0.5 * q0)
    n_c = np.maximum(1e6, np.ceil((1 - q) / (q * 0.005 ** 2))).astype(np.int64)
    J = jobs(n_c)
    ctx.run_batch(J, 1002)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = ctx.run_batch(J, 1002)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    p = r.fepe()
    rse = r.fepe_sigma() / np.maximum(p, 1e-300)
    n_analog = np.sum((1 - p) / (np.maximum(p, 1e-300) * rse ** 2))
    return {"value": float(n_c.sum()) / dt, "unit": "histories/s", "weight": float(wt[0]),
            "histories_per_energy": [int(x) for x in n_c], "ms_per_step": dt * 1e3,
            "max_fepe_rse": float(rse.max()),
            "analog_equivalent_histories_per_s": float(n_analog) / dt,
            "fepe": [float(x) for x in p]}


def measure(a, torch, gadep, C, ctx, distance, steps, warmup, full):
    """One distance of the metric's detector: pilot-sized N_e, timed steps, event
    counts and roofline; with full=True also the gradient run and the batched+grad
    against single-job comparison."""
    w = C.c2_hpge(n_histories=0, distance=distance)
    gadep.load_workload(ctx, w)
    n_groups = len(w.groups)

    def jobs(n_per_e, grad=False):
        return [dict(source=w.source, energies=[E], n_histories=int(n_per_e[k]), stream=k,
                     scales=[1.0] * n_groups if grad else None) for k, E in enumerate(w.energies)]

    # pilot: FEPE estimate per energy to size N_e for 0.5 % RSE
    pilot = ctx.run_batch(jobs([a.pilot] * len(w.energies)), 999)
    # the pilot's estimate lowered by three of its standard errors, so that the
    # run's own estimate (another draw) still meets the target
    p0 = np.maximum(pilot.fepe(), 1e-12)
    p = np.maximum(p0 - 3.0 * np.sqrt(p0 * (1 - p0) / a.pilot), 0.5 * p0)
    need = np.ceil((1 - p) / (p * 0.005 ** 2))
    n_e = (np.maximum(a.min_histories, need) if not a.quick else
           np.full(len(p), a.min_histories)).astype(np.int64)
    total = int(n_e.sum())
    J = jobs(n_e)
    JG = jobs(n_e, True)

    def step(grad=False, seed=1002):
        if grad:
            return ctx.run_batch(JG, seed, grad=True)
        return ctx.run_batch(J, seed)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    kernel_ms = []
    sclks = []
    res = None
    t0 = time.perf_counter()
    for _ in range(steps):
        res = step()
        kernel_ms.append(ctx.get_last_launch_ms())
        sclks.append(ctx.get_last_clock_mhz())
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # the shader clock the timed launches ran at (in-kernel clock counters)
    sclk = float(np.mean(sclks))
    fepe = res.fepe()
    rse = np.sqrt((1 - fepe) / (n_e * np.maximum(fepe, 1e-300)))

    fwd_grad_ratio = None
    batched_vs_single = None
    if full and not a.no_grad:
        step(grad=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            rg = step(grad=True)
        torch.cuda.synchronize()
        dtg = (time.perf_counter() - t1) / steps
        fwd_grad_ratio = dtg / dt
        # the plain single-job kernel: one forward gadep_run launch per energy,
        # the same histories (each meets the same RSE)
        for k, E in enumerate(w.energies):
            ctx.run(w.source, [E], int(n_e[k]), 1002)
        torch.cuda.synchronize()
        reps = max(1, min(steps, 3))
        t2 = time.perf_counter()
        for _ in range(reps):
            for k, E in enumerate(w.energies):
                ctx.run(w.source, [E], int(n_e[k]), 1002)
        torch.cuda.synchronize()
        dts = (time.perf_counter() - t2) / reps
        gf = rg.fepe()
        batched_vs_single = {
            "batched_grad_histories_per_s": total / dtg,
            "single_job_histories_per_s": total / dts,
            "batched_grad_over_single_job": dts / dtg,
            "max_fepe_rse": float(np.sqrt((1 - gf) / (n_e * np.maximum(gf, 1e-300))).max()),
            "batched_grad": f"one gadep_run_batch launch over the {len(w.energies)} energies with "
                            f"dFEPE/ds for {n_groups} density groups",
            "single_job": f"{len(w.energies)} gadep_run launches, one per energy, no gradients"}

    # event counts of the same histories (deterministic) for the op model
    ctx.set_option(gadep.OPT_COUNTERS, 1)
    step()
    ev = ctx.get_counters()
    count_ms, count_sclk = ctx.get_last_launch_ms(), ctx.get_last_clock_mhz()
    ctx.set_option(gadep.OPT_COUNTERS, 0)
    ops = sum(OPS_PER_EVENT[k] * ev[k] for k in OPS_PER_EVENT)
    # lanes busy per wavefront step: node visits per iteration with a node
    # step, facet tests per iteration with a facet test
    lanes = {"node": ev["node_visits"] / max(ev["iterations_node"], 1),
             "facet": ev["tri_tests"] / max(ev["iterations_facet"], 1),
             "iterations_per_pass": ev["iterations"] / max(ev["passes"], 1)}
    # where the wavefronts' time goes (counting variant, shader-clock cycles)
    cyc = {k[7:]: ev[k] for k in ev if k.startswith("cycles_")}
    cyc_total = max(sum(cyc.values()), 1)
    lanes["time_share"] = {k: v / cyc_total for k, v in cyc.items()}
    # share of the counting launch the grid was busy: summed wavefront
    # lifetimes over wavefronts x launch duration (the rest is the tail)
    lanes["grid_busy"] = ev["wave_cycles"] / max(ev["wavefronts"] * count_ms * 1e-3 * count_sclk * 1e6, 1.0)
    k_ms = float(np.mean(kernel_ms))
    achieved = ops / (k_ms * 1e-3)
    peak = PEAK_LANE_OPS * (sclk / PEAK_SCLK_MHZ if sclk else 1.0)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
            "unit": "T lane-op/s", "frac": achieved / peak,
            "traffic": (measured_traffic() if distance == 250.0 and
                        (a.guide, a.claim, a.split_pct) == (None, None, None) else None),
            "kernel_ms": k_ms, "measured_sclk_mhz": sclk,
            "peak_at_2400_mhz": PEAK_LANE_OPS / 1e12, "ops_per_history": ops / total,
            "events_per_history": {k: ev[k] / total for k in ev
                                   if not k.startswith("cycles_") and k not in ("wavefronts", "wave_cycles")},
            "active_lanes": lanes}
    s = k_ms * 1e-3
    rates = {"node_visits_per_s": ev["node_visits"] / s, "facet_tests_per_s": ev["tri_tests"] / s,
             "interactions_per_s": (ev["photo"] + ev["compton"] + ev["coherent"] + ev["pair"]) / s,
             "segments_per_s": ev["segments"] / s}
    return {"w": w, "n_e": n_e, "total": total, "dt": dt, "fepe": fepe, "rse": rse, "roof": roof,
            "rates": rates, "fwd_grad_ratio": fwd_grad_ratio, "batched_vs_single": batched_vs_single}


# ---------------------------------------------------------------------------
# secondary workloads (one JSON line each; not the metric)

def _ablate(ctx, a, gadep):
    """The ablation options of the command line, set on a new context."""
    for opt, v in ((gadep.OPT_GUIDE, a.guide), (gadep.OPT_CLAIM, a.claim), (gadep.OPT_SPLIT_PCT, a.split_pct)):
        if v is not None:
            ctx.set_option(opt, v)
    return ctx


def _timed(ctx, torch, fn, steps, warmup):
    for i in range(warmup):
        fn()
        print(f"bench: warm-up step {i + 1} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ks = []
    for i in range(steps):
        fn()
        ks.append(ctx.get_last_launch_ms())
        print(f"bench: step {i + 1} done ({ks[-1]:.1f} ms)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, float(np.mean(ks)) if ks else None


def _line(metric, value, unit, a, dt, workload, extra, higher=True):
    d = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": a.steps,
         "warmup": a.warmup, "ms_per_step": dt * 1e3, "higher_is_better": higher,
         "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
         "config": {"workload": workload}}
    d.update(extra)
    return d


def _rates(ctx, gadep, run, k_ms):
    """Event counts of one run (counting variant) as rates over the timed launch."""
    ctx.set_option(gadep.OPT_COUNTERS, 1)
    run()
    ev = ctx.get_counters()
    ctx.set_option(gadep.OPT_COUNTERS, 0)
    s = k_ms * 1e-3
    return {"node_visits_per_s": ev["node_visits"] / s, "facet_tests_per_s": ev["tri_tests"] / s,
            "interactions_per_s": (ev["photo"] + ev["compton"] + ev["coherent"]) / s,
            "segments_per_s": ev["segments"] / s}


def bench_c3(a, torch, gadep, C):
    """64 bottle jobs on the 256-facet crystal: one detector scene and 64
    overlays (two-level geometry), batched in one launch against one launch
    per job; autotuned block size, park threshold and claim."""
    jobs = C.c3_jobs(64)
    ws = [C.c3_job_workload(j) for j in jobs]
    ctx = _ablate(gadep.Context(0), a, gadep)
    w0 = ws[0]
    for m, tab in w0.tables.items():
        ctx.set_xs(m, w0.grid, *tab)
    base = C.bare_crystal(64).build()
    mat, rho, grp, act = C.Workload("base", base, w0.materials, w0.tables, w0.grid, w0.source,
                                    [], 0, 0).region_arrays()
    torch.cuda.synchronize()
    f0 = torch.cuda.mem_get_info()[0]
    ctx.load_scene(0, base.xyz, base.tri, base.tri_region,
                   [(int(mat[r]), float(rho[r]), int(grp[r]), gadep.ACTIVE if act[r] else 0)
                    for r in range(len(mat))])
    for k, j in enumerate(jobs):
        ov = C.bottle_overlay(j["r"], j["h"], 2.0, j["matrix"], j["density"], group=1)
        ctx.load_overlay(1 + k, 0, 0, ov.xyz, ov.tri, ov.tri_region, C.overlay_regions(ov, w0.materials))
    torch.cuda.synchronize()
    geometry_mb = (f0 - torch.cuda.mem_get_info()[0]) / 1e6
    spec = [dict(source=w.source, energies=w.energies, n_histories=max(1, j["n_total"] // len(w.energies)),
                 scene=1 + k, stream=k) for k, (j, w) in enumerate(zip(jobs, ws))]
    total = sum(s["n_histories"] * len(s["energies"]) for s in spec)
    tuned = ctx.autotune(spec, 20_000_000)
    dt, k_ms = _timed(ctx, torch, lambda: ctx.run_batch(spec, 1003), a.steps, a.warmup)
    singles = 0.0
    for s1 in spec:
        ctx.run_batch([s1], 1003)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.run_batch([s1], 1003)
        torch.cuda.synchronize()
        singles += time.perf_counter() - t0
    rates = _rates(ctx, gadep, lambda: ctx.run_batch(spec, 1003), k_ms)
    ctx.close()
    return _line("histories/s, 64 bottle jobs x 20 energies in one launch", total / dt, "histories/s",
                 a, dt, "c3_64_bottle_overlays_on_256_facet_crystal_20_energies",
                 {"histories_per_step": total, "kernel_ms": k_ms, "sum_of_single_job_launches_s": singles,
                  "batched_over_single_speedup": singles / dt,
                  "autotuned_block_period_claim": list(tuned),
                  "geometry_device_mb_detector_plus_64_overlays": geometry_mb,
                  "rates": rates,
                  "hpge20k_64_overlays": _c3_on_detector(a, torch, gadep, C, jobs)})


def _c3_on_detector(a, torch, gadep, C, jobs):
    """The same 64 bottle jobs (a tenth of their histories) as overlays above the
    end-cap of the 20236-facet detector: one copy of the detector BVH, one
    batched launch against one launch per job."""
    det = C.c2_hpge(n_histories=1).scene
    mats = ["vacuum", "air", "Al", "Ge", "Cu", "PP", "water", "soil"]
    tables, grid = C._tables_for(mats, coherent=False)
    ctx = _ablate(gadep.Context(0), a, gadep)
    for m, tab in tables.items():
        ctx.set_xs(m, grid, *tab)
    host = det.region_id("air")
    regions = [(mats.index(r["material"]), float(r["density"]), int(r["group"]),
                gadep.ACTIVE if r["active"] else 0) for r in det.regions]
    torch.cuda.synchronize()
    f0 = torch.cuda.mem_get_info()[0]
    ctx.load_scene(0, det.xyz, det.tri, det.tri_region, regions)
    torch.cuda.synchronize()
    f1 = torch.cuda.mem_get_info()[0]
    z0 = 5.5 + 2.0  # 2 mm above the end-cap
    energies = C.log_energies(20)
    spec = []
    for k, j in enumerate(jobs):
        ov = C.bottle_overlay(j["r"], j["h"], z0, j["matrix"], j["density"], group=len(C.HPGE_GROUPS))
        ctx.load_overlay(1 + k, 0, host, ov.xyz, ov.tri, ov.tri_region, C.overlay_regions(ov, mats))
        src = C.Source(C.KIND_CYL, pos=(0.0, 0.0, z0 + 1.5), r_in=0.0, r_out=j["r"], h=j["h"],
                       region=det.n_regions + 1)
        spec.append(dict(source=src, energies=energies, n_histories=max(1, j["n_total"] // 10 // len(energies)),
                         scene=1 + k, stream=k))
    torch.cuda.synchronize()
    f2 = torch.cuda.mem_get_info()[0]
    total = sum(s["n_histories"] * len(s["energies"]) for s in spec)
    tuned = ctx.autotune(spec, 20_000_000)
    dt, k_ms = _timed(ctx, torch, lambda: ctx.run_batch(spec, 1007), a.steps, a.warmup)
    singles = 0.0
    for s1 in spec:
        ctx.run_batch([s1], 1007)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.run_batch([s1], 1007)
        torch.cuda.synchronize()
        singles += time.perf_counter() - t0
    ctx.close()
    return {"value": total / dt, "unit": "histories/s", "histories_per_step": total, "ms_per_step": dt * 1e3,
            "kernel_ms": k_ms, "sum_of_single_job_launches_s": singles,
            "batched_over_single_speedup": singles / dt, "autotuned_block_period_claim": list(tuned),
            "geometry_device_mb_detector": (f0 - f1) / 1e6,
            "geometry_device_mb_64_overlays": (f1 - f2) / 1e6}


def bench_c4(a, torch, gadep, C):
    w = C.c4_grad()
    ctx = _ablate(gadep.Context(0), a, gadep)
    gadep.load_workload(ctx, w)
    ng = len(w.groups)
    J = [dict(source=w.source, energies=w.energies, n_histories=w.n_histories, stream=0)]
    JG = [dict(J[0], scales=[1.0] * ng)]
    total = w.n_histories * len(w.energies)
    dt, k_ms = _timed(ctx, torch, lambda: ctx.run_batch(J, 1004), a.steps, a.warmup)
    dtg, kg_ms = _timed(ctx, torch, lambda: ctx.run_batch(JG, 1004, grad=True), a.steps, a.warmup)
    return _line("histories/s, 20236-facet HPGe detector + water sample, volume source, 20 energies",
                 total / dt, "histories/s", a, dt, "c4_hpge_water_sample_volume_source_20_energies",
                 {"histories_per_step": total, "kernel_ms": k_ms, "grad_kernel_ms": kg_ms,
                  "fwd_grad_over_fwd": dtg / dt,
                  "rates": _rates(ctx, gadep, lambda: ctx.run_batch(J, 1004), k_ms)})


def bench_c5(a, torch, gadep, C):
    t0 = time.perf_counter()
    w = C.c5_stress()
    t_gen = time.perf_counter() - t0
    ctx = _ablate(gadep.Context(0), a, gadep)
    print(f"bench: {len(w.scene.tri)} facets generated", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    gadep.load_workload(ctx, w)
    t_load = time.perf_counter() - t0
    print(f"bench: mesh loaded in {t_load:.1f} s", file=sys.stderr, flush=True)
    rng = np.random.default_rng(3005)
    mat, rho, grp, act = w.region_arrays()
    m = w.scene.region_id("matrix")
    ng = len(w.groups)
    n_job = w.n_histories  # 2e9 histories over 16 matrices
    jobs = []
    for j in range(16):
        mo, do = mat.copy(), rho.copy()
        mo[m] = w.materials.index("water" if j % 2 == 0 else "soil")
        do[m] = float(rng.uniform(0.8, 1.6))
        jobs.append(dict(source=w.source, energies=None, n_histories=n_job, stream=j,
                         scales=[1.0] * ng, material_override=mo, density_override=do))
    total = n_job * 16
    nch, width = 8192, 0.25
    holder = {}

    def run():
        holder["r"] = ctx.run_batch(jobs, 1005, grad=True, spectrum=(nch, width))

    dt, k_ms = _timed(ctx, torch, run, a.steps, a.warmup)
    spec = torch.tensor(holder["r"].spectra.astype(np.float64), device="cuda")
    out = torch.empty_like(spec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.broaden_dev(spec.data_ptr(), out.data_ptr(), 16, nch, width, 0.64, 0.0018)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    return _line("histories/s, ~1M-facet detector + Marinelli, 16 matrices, lines, spectra, gradients",
                 total / dt, "histories/s", a, dt, "c5_marinelli_962572_facets_16_matrices_13_lines",
                 {"histories_per_step": total, "kernel_ms": k_ms, "n_facets": int(len(w.scene.tri)),
                  "mesh_generation_s": t_gen, "load_mesh_s": t_load, "broadening_16x8192_ms": t_b * 1e3})


def bench_build(a, torch, gadep, C):
    ctx = _ablate(gadep.Context(0), a, gadep)
    out = {}
    for name, make in (("c1_256", lambda: C.c1_bare()), ("c2_20236", lambda: C.c2_hpge(n_histories=1)),
                       ("c5_962572", lambda: C.c5_stress(n_histories=1))):
        w = make()
        mat, rho, grp, act = w.region_arrays()
        regions = [(int(mat[r]), float(rho[r]), int(grp[r]), gadep.ACTIVE if act[r] else 0)
                   for r in range(len(mat))]
        t0 = time.perf_counter()
        ctx.load_scene(0, w.scene.xyz, w.scene.tri, w.scene.tri_region, regions)
        torch.cuda.synchronize()
        out[name] = {"facets": int(len(w.scene.tri)), "seconds": time.perf_counter() - t0}
        print(f"bench: {name} loaded", file=sys.stderr, flush=True)
    tot = sum(v["seconds"] for v in out.values())
    return _line("seconds to validate, derive topology, build both BVHs and upload a mesh",
                 tot, "s", a, tot, "load_mesh_256_20236_962572_facets", {"per_mesh": out},
                 higher=False)


OTHER = {"c3": bench_c3, "c4": bench_c4, "c5": bench_c5, "build": bench_build}


if __name__ == "__main__":
    main()
