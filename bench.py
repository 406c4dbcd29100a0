"""Benchmark of the FSLBM step with the enhanced bubble model on one MI355X.

Default workload: 256^3 periodic box with 16 gas threads (radius 8, 0.1 R
sinusoidal radius perturbation of wavelength 72, 1e-3 fill-level noise),
tau = 0.55, sigma = 5e-3, FP32 storage and arithmetic.  The threads
rupture (Rayleigh-Plateau) between steps 1128 and 1192 into about three
bubbles each.  The benchmark first evolves the scene to step 1120, then
runs the warm-up and the timed window (default 5 + 80 steps), so that the
window holds the bubble splits and their labelling runs whatever the
warm-up and window lengths.

Prints one JSON line (rank 0, N = 1) with the whole-step throughput in
MLUPS, the HBM roofline of the dominant kernel (liquid-cell stream-collide)
measured with HIP events on the library's stream over the timed window,
the achievable bandwidth of a plain streaming copy, and the CPU oracle
timed on a bounded sample of the same workload (all host threads of this
job and one thread).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s
# The 16 threads of the 256^3 workload rupture between steps 1128 and 1192
# (51 bubble merges and splits, FP32); starting the warm-up at step 1120
# puts them in the timed window.
RUPTURE_START = 1120
METRIC = "FSLBM MLUPS and % of HBM roofline; served p50/p99 latency vs plain"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bulk_bytes_per_launch(counts: dict, store_bytes: int) -> float:
    """Algorithmic bytes of one launch of the stream-collide kernel, which
    writes every row of the new lattice whole: a liquid cell pulls 19 PDFs,
    writes 19 PDFs and reads and writes its flag byte (38 S + 2); an
    interface cell reads its flag and list slot (1 + 4), copies the 19
    post-collision values and the new flag left at its slot into the
    lattice (38 S + 2); a gas, wall or inlet cell reads and writes its flag
    byte (2).  The zeros stored for gas cells next to fluid cells (a layout
    choice that keeps cache lines whole) are not counted."""
    S = store_bytes
    return counts["liq"] * (38 * S + 2) + counts["iface"] * (38 * S + 7) + counts["other"] * 2


def count_types(t) -> dict:
    import numpy as np

    b = np.bincount(t, minlength=5)
    return dict(gas=int(b[0]), iface=int(b[1]), liq=int(b[2]), other=int(b[0] + b[3] + b[4]))


def host_threads() -> int:
    """Host threads this job may use: the OpenMP setting of the host (the
    host may give each GPU a share of its cores), else the CPUs of this
    process's affinity mask."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(scene, seconds: float, threads: int, max_steps: int):
    import oracle

    oracle.set_threads(threads)
    o = oracle.Oracle.from_scene(scene)
    steps, t0 = 0, time.perf_counter()
    while True:
        o.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= max_steps:
            break
    del o
    return scene.n * steps / el / 1e6, steps, el


def cpu_baseline(scene, seconds: float, threads: int, single: bool) -> dict:
    """The oracle as it stands, on the host cores, on whole steps of the same
    workload from its initial state until about `seconds` have passed:
    once with `threads` OpenMP threads and, if `single`, once with one
    thread (at least one whole step)."""
    import oracle

    oracle.build(force=False)
    mlups, steps, el = _oracle_rate(scene, seconds, threads, 50)
    out = {"value": round(mlups, 4), "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"{scene.name} {scene.nx}x{scene.ny}x{scene.nz}, FP64 oracle, first {steps} "
                     f"step(s) from the initial state, {el:.1f} s wall on {threads} threads",
           "cpu_model": cpu_model()}
    if single:
        m1, s1, e1 = _oracle_rate(scene, 1.0, 1, 1)
        out["single_thread"] = {"value": round(m1, 4), "unit": "MLUPS", "cores": 1,
                                "sample": f"first {s1} step(s), {e1:.1f} s wall"}
    oracle.set_threads(1)
    return out


def copy_bandwidth_context(mib: int = 1024, reps: int = 10) -> dict:
    """Achievable HBM bandwidth: the library's streaming copy kernel over
    two buffers of `mib` MiB."""
    import torch

    import paper_1604_01632_amd as F

    n = mib * (1 << 20)
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    gbs = F.fslbm_copy_bandwidth(dst, src, reps)
    del src, dst
    torch.cuda.empty_cache()
    return {"GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "kernel": "fslbm_copy_bandwidth (16-byte non-temporal loads and stores)",
            "bytes_each_way": n, "reps": reps}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_bulk_p1_256cubed_fp32_hbm_traffic.md")
CSRC = os.path.join(ROOT, "paper_1604_01632_amd", "csrc")


# What each timed phase of one domain's step holds (passes that touch
# disjoint data share a launch, so a phase can hold part of another's work).
PHASE_PASSES = {
    "bulk_ms": "stream-collide",
    "iface_ms": "geometry, interface update",
    "convert_ms": "new cell types, new interface cells",
    "excess_ms": "excess mass and topology trigger; tile counts of the next interface list",
    "gather_ms": "tile-count scan and labelled set; list fill and unions; excess gather, "
                 "volume sums and roots",
    "label_ms": "assign and per-bubble volumes; new components' sums",
    "bubbles_ms": "install, injection, pressure",
}


def kernel_source_hash() -> str:
    """SHA-256 over the HIP sources of the library (sorted by name): the
    recorded HBM traffic is valid only for the kernels it was measured on."""
    import hashlib

    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(CSRC, name), "rb") as fh:
                h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def recorded_traffic(precision: str, workload: str):
    """HBM bytes per launch of the liquid-cell kernel from the two rocprofv3
    counter passes (FETCH_SIZE, WRITE_SIZE) recorded under profiles/, scaled
    by the copy-kernel factor recorded there; None when the file is missing,
    is for another workload, or the kernel sources changed since."""
    if not os.path.exists(TRAFFIC_FILE) or (precision, workload) != ("fp32", "p1"):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_probe(mib: int, reps: int) -> int:
    """A plain device-to-device copy of known size, for scaling the HBM byte
    counters (run under rocprofv3 --pmc)."""
    import torch

    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                      "reps": reps}), flush=True)
    return 0


def bench_batched(args) -> int:
    """Batched form: 256 walled domains of uneven sizes advanced together
    (one graph launch per step) against the plain loop that steps each
    domain on its own with the same kernels."""
    import tempfile

    import torch

    import paper_1604_01632_amd as F
    import scenes

    torch.cuda.set_device(0)
    t = time.perf_counter()
    scs = scenes.batch_domains(count=args.domains, seed=4)
    log(f"[bench] {len(scs)} domains built in {time.perf_counter() - t:.1f} s")
    doms = [F.Domain.from_scene(sc, args.precision) for sc in scs]
    cells = sum(d.N for d in doms)
    cache = os.path.join(tempfile.gettempdir(), "fslbm_batch_tuning.txt")
    b = F.Batch(doms, tuning_cache_path=cache)
    info = b.info()
    log(f"[bench] batch of {len(doms)} domains, {cells} cells; tuning {info}")
    steps = args.steps if args.steps_given else 2000
    b.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    batched = cells * steps / t_batch / 1e6
    plain_steps = max(1, min(steps, args.plain_steps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d in doms:
        d.step(plain_steps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    plain = cells * plain_steps / t_plain / 1e6
    reads = [d.read(("cell_type",)) for d in doms]
    s = [r["scalars"] for r in reads]
    bad = sum(1 for x in s if not np.isfinite(x["total_mass"]))
    # whole-step algorithmic traffic of all domains: fluid cells move the
    # PDFs read and written plus flags, fill level, mass and IDs of the
    # interface layer (2 * 19 S + 8 bytes), gas and wall cells their flag
    store_bytes = {"fp64": 8, "fp32": 4, "fp16dev": 2}[args.precision]
    n_fluid = sum(int(np.count_nonzero((r["cell_type"] == 1) | (r["cell_type"] == 2))) for r in reads)
    b_alg = 2 * 19 * store_bytes + 8
    whole_gbs = (n_fluid * b_alg + (cells - n_fluid)) / (t_batch / steps) / 1e9
    log(f"[bench] batched {batched:.1f} MLUPS ({t_batch / steps * 1e3:.3f} ms/step, "
        f"{whole_gbs:.0f} GB/s algorithmic), plain loop {plain:.1f} MLUPS "
        f"({t_plain / plain_steps * 1e3:.3f} ms/step); non-finite domains {bad}")
    out = {
        "metric": METRIC, "value": round(batched, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(t_batch / steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16dev": "f16-storage/f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"batched: {len(doms)} walled domains, extents 32..96 per axis, 1..8 "
                               "gas spheres R 4..12 in Laplace equilibrium, g 1e-5, tau 0.55..0.8, "
                               f"sigma 2e-3, {args.precision}, one graph launch per step",
                   "cells": cells, "plain_loop_mlups": round(plain, 1),
                   "plain_loop_steps": plain_steps, "speedup_vs_plain": round(batched / plain, 2),
                   "tuning": info},
        "roofline": {"kernel": "whole batched step (all kernels of all domains)", "bound": "hbm",
                     "achieved": round(whole_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(whole_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_step": int(n_fluid * b_alg + (cells - n_fluid))},
        "cpu_baseline": None,
    }
    b.close()
    print(json.dumps(out), flush=True)
    return 0


def _bubble_errors(sc, ref, got) -> dict:
    """Bubble count of `got` against `ref` and the largest relative volume
    error, bubbles paired by centroid (the ID sequences of the forms differ
    when they see different numbers of merges and splits)."""
    from tests.parity import match_by_centroid

    rb, gb = ref[0], got[0]
    out = {"bubbles": int(len(gb["id"])), "bubbles_fp64": int(len(rb["id"])),
           "same_ids": rb["id"].tolist() == gb["id"].tolist(), "max_rel_volume_error": None}
    if len(rb["id"]) == len(gb["id"]):
        m = match_by_centroid(ref[2], got[2], (sc.nz, sc.ny, sc.nx))
        if m is not None:
            err = np.abs(gb["volume"][m] - rb["volume"]) / rb["volume"]
            out["max_rel_volume_error"] = float(err.max()) if len(err) else 0.0
    out["total_volume_rel_error"] = float(abs(gb["volume"].sum() - rb["volume"].sum())
                                          / max(rb["volume"].sum(), 1e-300))
    return out


def bench_forms(args) -> int:
    """Precision forms against the plain FP64 form on the same GPU: the
    256^3 thread workload stepped in FP64, FP32 and FP16-deviation storage
    (MLUPS of each), and the accuracy of FP32 and FP16-deviation against
    FP64 at the horizons of the thread-rupture (C2, 20000 steps) and orifice
    (C3, 50000 steps) scenes: bubble count, per-bubble volume, total-mass
    drift.  The FP64 path reproduces the oracle bit for bit on the parity
    cases; at these horizons it stands in for the oracle, whose CPU run
    would take hours."""
    import torch

    import paper_1604_01632_amd as F
    import scenes

    torch.cuda.set_device(0)
    forms = ("fp64", "fp32", "fp16dev")
    sc = scenes.config("p1")
    start = args.start_step if args.start_step >= 0 else RUPTURE_START
    speed = {}
    for prec in forms:
        dom = F.Domain.from_scene(sc, prec)
        if start:
            dom.step(start)  # into the rupture epoch, as the default line
        dom.step(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dom.step(args.steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        speed[prec] = {"mlups": round(sc.n * args.steps / dt / 1e6, 1),
                       "ms_per_step": round(dt / args.steps * 1e3, 4)}
        log(f"[bench] p1 {prec}: {speed[prec]}")
        dom.close()
        del dom
        torch.cuda.empty_cache()
    from tests.parity import centroids

    accuracy = {}
    for name, horizon in (("c2", args.c2_steps), ("c3", args.c3_steps), ("c3d", args.c3d_steps)):
        cs = scenes.config(name)
        res = {}
        for prec in forms:
            dom = F.Domain.from_scene(cs, prec)
            m0 = dom.read(("cell_type",))["scalars"]["total_mass"]
            done = 0
            while done < horizon:
                n = min(5000, horizon - done)
                dom.step(n)
                dom.sync()
                done += n
                log(f"[bench] {name} {prec}: {done}/{horizon} steps")
            r = dom.read(("bubble_id",))
            s = r["scalars"]
            b = dom.bubbles()
            res[prec] = (b, abs(s["total_mass"] - m0) / m0,
                         centroids(r["bubble_id"], b["id"], (cs.nz, cs.ny, cs.nx)),
                         int(s["n_topology"]))
            dom.close()
            del dom
            torch.cuda.empty_cache()
        accuracy[name] = {"horizon": horizon, "fp64_mass_drift": res["fp64"][1],
                          "fp64_bubbles": int(len(res["fp64"][0]["id"])),
                          "fp64_merges_splits": res["fp64"][3]}
        for prec in ("fp32", "fp16dev"):
            e = _bubble_errors(cs, res["fp64"], res[prec])
            e["mass_drift"] = res[prec][1]
            e["merges_splits"] = res[prec][3]
            accuracy[name][prec] = e
        log(f"[bench] {name}: {accuracy[name]}")
    out = {
        "metric": METRIC, "value": speed["fp32"]["mlups"], "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": speed["fp32"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "precision forms: p1 256^3 thread rupture in fp64, fp32 and "
                               f"fp16-deviation storage, window after step {start} + "
                               f"{args.warmup} (value: fp32); accuracy of fp32 and "
                               "fp16dev against fp64 at the c2, c3 and c3d (detaching orifice) "
                               "horizons, bubbles paired by centroid",
                   "p1": speed,
                   "speedup_vs_fp64": {p: round(speed[p]["mlups"] / speed["fp64"]["mlups"], 2)
                                       for p in forms},
                   "accuracy": accuracy},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


# Detachment volumes of Sec. 3.2 (Table tab:detRad), mm^3: the paper's own
# FSLBM runs and the two comparison results it quotes, at 1 ml/min (the
# analytic one for a vanishing flow rate).  Context for the trend only: the
# runs here use a similarity mapping, not the paper's time step.
PORE_TABLE = {70.0: {"paper_fslbm": 38.0, "vof_2d": 39.0, "analytic_q0": 33.0},
              90.0: {"paper_fslbm": 51.0, "vof_2d": 69.0, "analytic_q0": 69.0}}


def first_detachment(sc, precision, max_steps, check_every, log_every=20):
    """Step a pore scene until the first bubble without inlet or atmosphere
    flag appears (a bubble pinched off the pore); returns (steps, its volume
    in cells, seconds of device time, detached before max_steps)."""
    import torch

    import paper_1604_01632_amd as F

    dom = F.Domain.from_scene(sc, precision)
    done, vol, found = 0, 0.0, False
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k = 0
    while done < max_steps and not found:
        dom.step(check_every)
        done += check_every
        b = dom.bubbles()
        free = [v for f, v in zip(b["flags"], b["volume"]) if int(f) == 0]
        if free:
            found, vol = True, float(max(free))
        k += 1
        if k % log_every == 0:
            inlet = [round(float(v), 1) for f, v in zip(b["flags"], b["volume"]) if int(f) & 1]
            log(f"[bench] pore theta={sc.contact_angle:g} q={sc.meta['q_ml_min']:g}: {done} steps, "
                f"inlet bubble {inlet} cells")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    dom.close()
    del dom
    torch.cuda.empty_cache()
    return done, vol, dt, found


def bench_pore(args) -> int:
    """The pore case of Sec. 3.2: gas blown through a pore of radius r in
    the bottom wall into liquid under gravity, with an open top (atmosphere
    bubble at p0) and a static contact angle at the walls.  For contact
    angles 70 and 90 degrees and flow rates 1 and 10 ml/min, the first
    detached bubble's volume in mm^3, by the similarity mapping (Bond number
    of water-air at the 1 mm orifice, flow rate per capillary time), next to
    the paper's table."""
    import torch

    import scenes

    torch.cuda.set_device(0)
    r = args.pore_radius
    units = scenes.pore_units_similar(r)
    runs, cells_steps, secs = [], 0.0, 0.0
    rates = tuple(float(q) for q in args.pore_rates.split(","))
    angles = tuple(float(a) for a in args.pore_angles.split(","))
    for theta in angles:
        for q in rates:
            sc = scenes.pore(r=r, theta=theta, q_ml_min=q, tau=0.6, units=units)
            # volume flow per step in cells: detachment below 200 r^3
            max_steps = int(200 * r ** 3 / sc.inject_rate)
            steps, vol, dt, found = first_detachment(sc, args.precision, max_steps, 1000)
            cells_steps += sc.n * steps
            secs += dt
            row = {"theta": theta, "q_ml_min": q, "detached": found, "steps": steps,
                   "v_d_cells": round(vol, 1), "v_d_mm3": round(vol * units["mm3_per_cell"], 2),
                   "t_d_ms": round(steps * units["dt"] * 1e3, 1),
                   "mlups": round(sc.n * steps / dt / 1e6, 1)}
            runs.append(row)
            log(f"[bench] pore: {row}")
    v = {(row["theta"], row["q_ml_min"]): row["v_d_mm3"] for row in runs}
    out = {
        "metric": METRIC, "value": round(cells_steps / secs / 1e6, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": int(sum(row["steps"] for row in runs)), "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16dev": "f16dev"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"pore detachment (Sec. 3.2): {sc.nx}x{sc.ny}x{sc.nz} walled box, "
                               f"pore r = {r} cells (1 mm), open top (atmosphere at p0), "
                               f"contact angle {args.pore_angles} deg, {args.pore_rates} ml/min, Bond number "
                               f"{units['bond']:.4f} and flow per capillary time of water-air, "
                               f"sigma {units['sigma']}, tau 0.6, {args.precision}; each run to "
                               "its first detachment",
                   "runs": runs,
                   "trend_70_below_90": (all(v[(70.0, q)] < v[(90.0, q)] for q in rates)
                                         if {70.0, 90.0} <= set(angles) else None),
                   "trend_rate_increases_volume": (all(v[(t, min(rates))] < v[(t, max(rates))]
                                                       for t in angles)
                                                   if len(rates) > 1 else None),
                   "paper_table_mm3": {str(int(t)): row for t, row in PORE_TABLE.items()},
                   "units": {k: units[k] for k in ("dx", "dt", "g", "sigma", "bond",
                                                   "capillary_time_steps", "mm3_per_cell")}},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_served(args) -> int:
    """Served form: a Poisson stream of foam requests at 80 % of the measured
    capacity, continuous batching against the plain first-come-first-served
    loop on the same arrival trace."""
    import torch

    import paper_1604_01632_amd as F
    from paper_1604_01632_amd import serve
    import scenes

    torch.cuda.set_device(0)
    descs = scenes.serve_requests(count=args.requests, seed=5)
    work = np.array([d["edge"] ** 3 * d["horizon"] for d in descs], dtype=np.float64)
    # the scenes stand for what clients send: built before the clock starts
    # (in host processes), so that latency measures the serving system
    import concurrent.futures as cf
    t = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=max(1, min(16, host_threads()))) as ex:
        built = list(ex.map(scenes.request_scene, descs, chunksize=4))
    log(f"[bench] served: {len(built)} request scenes built in {time.perf_counter() - t:.1f} s")
    # capacity: aggregate rate of a full batch of sample requests
    sample = built[:min(12, len(built))]
    doms = [F.Domain.from_scene(sc, "fp32") for sc in sample]
    b = F.Batch(doms, tuning_cache_path="")
    b.step(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(60)
    torch.cuda.synchronize()
    cap_mlups = sum(d.N for d in doms) * 60 / (time.perf_counter() - t0) / 1e6
    b.close()
    for d in doms:
        d.close()
    del doms, b
    rate = 0.8 * cap_mlups * 1e6 / work.mean()
    rng = np.random.Generator(np.random.PCG64(55))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(descs)))
    arrivals -= arrivals[0]
    reqs = [serve.Request(d["id"], float(a), d["horizon"], (lambda k=k: built[k]))
            for k, (d, a) in enumerate(zip(descs, arrivals))]
    log(f"[bench] served: {len(reqs)} requests, capacity {cap_mlups:.0f} MLUPS, rate {rate:.3f}/s")
    def progress(tag):
        n = [0]

        def f(msg):
            n[0] += 1
            if n[0] % 32 == 0:
                log(f"[bench] {tag}: {n[0]} requests done")
        return f

    srv = serve.Server("fp32", max_active=args.max_active, quantum=args.quantum)
    t0 = time.perf_counter()
    res = srv.run(reqs, log=progress("continuous batching"))
    s_srv = serve.summary(res, time.perf_counter() - t0)
    log(f"[bench] continuous batching: {s_srv}")
    t0 = time.perf_counter()
    res_fifo = serve.run_fifo(reqs, "fp32", log=progress("plain loop"))
    s_fifo = serve.summary(res_fifo, time.perf_counter() - t0)
    log(f"[bench] plain loop: {s_fifo}")
    by = {r.id: r for r in res_fifo}
    same = all(np.array_equal(r.bubbles["volume"], by[r.id].bubbles["volume"])
               and r.scalars == by[r.id].scalars for r in res if not r.error)
    out = {
        "metric": METRIC, "value": round(s_srv["mlups"], 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": int(sum(d["horizon"] for d in descs)), "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"served: {len(reqs)} foam requests, cubic edges 32..192 "
                               "(log-uniform, multiples of 16), 1..64 spheres R 3..10, horizons "
                               "500..5000, Poisson arrivals at 80 % of capacity, fp32",
                   "p50_latency_s": round(s_srv["p50_s"], 3), "p99_latency_s": round(s_srv["p99_s"], 3),
                   "plain_p50_latency_s": round(s_fifo["p50_s"], 3),
                   "plain_p99_latency_s": round(s_fifo["p99_s"], 3),
                   "plain_mlups": round(s_fifo["mlups"], 1), "capacity_mlups": round(cap_mlups, 1),
                   "aggregate_vs_capacity": round(s_srv["mlups"] / cap_mlups, 3),
                   "rejected": s_srv["rejected"],
                   "arrival_rate_per_s": round(rate, 4), "results_same_alone_and_mixed": bool(same)},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--start-step", type=int, default=-1,
                    help="steps run before the warm-up (default: the rupture epoch of p1, "
                         f"step {RUPTURE_START}; 0 for other workloads)")
    ap.add_argument("--workload", default="p1",
                    help="p1 (default: 256^3 thread rupture), c1/c2/c3, batched, served, forms, "
                         "pore")
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "fp16dev"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-single-thread", action="store_true",
                    help="skip the single-threaded oracle sample")
    ap.add_argument("--no-phase-timing", action="store_true",
                    help="time the window without events around the stream-collide kernel "
                         "(no roofline figure)")
    ap.add_argument("--no-phase-breakdown", dest="phase_breakdown", action="store_false",
                    help="skip the rerun of the window with every phase timed")
    ap.add_argument("--no-trigger-compare", dest="trigger_compare", action="store_false",
                    help="skip the rerun of the window with the anti-parallel-normals trigger")
    ap.add_argument("--no-copy-probe", action="store_true",
                    help="skip the achievable-bandwidth copy probe")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain copy of MIB MiB (counter scaling) and exit")
    ap.add_argument("--domains", type=int, default=256, help="batched workload: domains")
    ap.add_argument("--pore-radius", type=int, default=10, help="pore workload: pore radius in cells")
    ap.add_argument("--pore-rates", default="1,10", help="pore workload: flow rates in ml/min")
    ap.add_argument("--pore-angles", default="70,90", help="pore workload: contact angles in degrees")
    ap.add_argument("--plain-steps", type=int, default=50,
                    help="batched workload: steps of the plain per-domain loop")
    ap.add_argument("--requests", type=int, default=512, help="served workload: requests")
    ap.add_argument("--max-active", type=int, default=64, help="served workload: slots")
    ap.add_argument("--quantum", type=int, default=100, help="served workload: steps per decision")
    ap.add_argument("--c2-steps", type=int, default=20000, help="forms workload: c2 horizon")
    ap.add_argument("--c3-steps", type=int, default=50000, help="forms workload: c3 horizon")
    ap.add_argument("--c3d-steps", type=int, default=7000,
                    help="forms workload: horizon of the detaching orifice variant")
    args = ap.parse_args()
    args.steps_given = args.steps is not None
    if args.steps is None:
        args.steps = 80
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        return 2

    if args.copy_probe:
        return copy_probe(args.copy_probe, 5)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "served":
        return bench_served(args)
    if args.workload == "forms":
        return bench_forms(args)
    if args.workload == "pore":
        return bench_pore(args)

    import numpy as np
    import torch

    import paper_1604_01632_amd as F
    import scenes

    torch.cuda.set_device(0)
    sc = scenes.config(args.workload)
    prec = F.PRECISIONS[args.precision]
    store_bytes = {0: 8, 1: 4, 2: 2}[prec]
    start = args.start_step if args.start_step >= 0 else (RUPTURE_START if args.workload == "p1" else 0)
    N = sc.n

    def run_window(phases, period, **over):
        """Evolve a fresh domain to `start`, warm up, then time the window;
        returns the measurements and the domain."""
        dom = F.Domain.from_scene(sc, args.precision, **over)
        if start:
            dom.step(start)
        dom.step(args.warmup)
        torch.cuda.synchronize()
        r0 = dom.read(("cell_type",))
        b0 = dom.bubbles()
        F.fslbm_set_timing(dom.handle, period, phases)
        stream = torch.cuda.current_stream()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        dom.step(args.steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        T = F.fslbm_get_timing(dom.handle)
        F.fslbm_set_timing(dom.handle, 0)
        r1 = dom.read(("cell_type", "bubble_id"))
        end_ids = r1.pop("bubble_id")
        return dict(gpu_ms=ev0.elapsed_time(ev1), wall=wall, T=T, r0=r0, r1=r1, b0=b0,
                    b1=dom.bubbles(), end_ids=end_ids), dom

    log(f"[bench] {sc.name}: {sc.nx}x{sc.ny}x{sc.nz} ({N} cells) {args.precision}; evolve to step "
        f"{start}, warm-up {args.warmup}, timed {args.steps}")
    # the timed window: events only around the stream-collide kernel, on
    # about ten of its steps (each event pair delays the stream by ~10 us)
    period = 0 if args.no_phase_timing else max(1, args.steps // 10)
    m, dom = run_window(["bulk"], period)
    dom.close()
    del dom
    torch.cuda.empty_cache()
    T = m["T"]
    c0, c1 = count_types(m["r0"]["cell_type"]), count_types(m["r1"]["cell_type"])
    s0, s1 = m["r0"]["scalars"], m["r1"]["scalars"]
    ms_per_step = max(m["gpu_ms"], m["wall"] * 1e3) / args.steps
    mlups = N / (ms_per_step * 1e-3) / 1e6
    counts = {k: 0.5 * (c0[k] + c1[k]) for k in c0}
    bytes_bulk = bulk_bytes_per_launch(counts, store_bytes)
    bulk_avg_ms = T["bulk_ms"] / max(1, T["steps"])
    achieved = bytes_bulk / (bulk_avg_ms * 1e-3) / 1e9 if T["steps"] else 0.0
    topo = int(s1["n_topology"] - s0["n_topology"])
    # whole-step algorithmic traffic: fluid cells move B bytes (PDFs read and
    # written, flags, fill level, mass and bubble IDs of the thin interface
    # layer amortised), gas, wall and inlet cells their flag byte
    b_alg = 2 * 19 * store_bytes + 8
    n_fluid = counts["liq"] + counts["iface"]
    whole_gbs = (n_fluid * b_alg + (N - n_fluid) * 1) / (ms_per_step * 1e-3) / 1e9
    log(f"[bench] window: {ms_per_step:.4f} ms/step, {mlups:.1f} MLUPS, topology changes {topo}, "
        f"bubbles {len(m['b0']['id'])} -> {len(m['b1']['id'])}, mass drift "
        f"{abs(s1['total_mass'] - s0['total_mass']) / s0['total_mass']:.2e}, cells {c1}")
    if topo == 0:
        log("[bench] WARNING: no bubble merge or split in the timed window: this is not the "
            "breakup-active case")
    phases = None
    if args.phase_breakdown:
        # the same window again (the run is deterministic), every phase timed
        # on every step: where the time of a step goes
        mp, dom = run_window(None, 1)
        dom.close()
        del dom
        torch.cuda.empty_cache()
        phases = {k: round(mp["T"][k] / max(1, mp["T"]["steps"]) * 1e3, 2) for k in
                  ("bulk_ms", "iface_ms", "convert_ms", "excess_ms", "gather_ms", "label_ms",
                   "bubbles_ms")}
        log(f"[bench] per-step phase times (us, same window rerun, every phase timed): {phases}")
    triggers = None
    if args.trigger_compare:
        # the same window with the paper's split trigger (anti-parallel
        # normals, Sec. 2.3.2) instead of the exact one: how often each
        # starts a labelling run, and whether the normals trigger left a
        # split undetected (fewer bubbles, or a different state at the end)
        mn, dom = run_window(None, 0, split_trigger=F.TRIGGER_NORMALS, trigger_cos=-0.5)
        end_n = dom.read(("cell_type", "bubble_id"))
        dom.close()
        del dom
        torch.cuda.empty_cache()
        runs_e = int(s1["n_label_runs"] - s0["n_label_runs"])
        runs_n = int(mn["r1"]["scalars"]["n_label_runs"] - mn["r0"]["scalars"]["n_label_runs"])
        same = bool(np.array_equal(end_n["cell_type"], m["r1"]["cell_type"])
                    and np.array_equal(end_n["bubble_id"], m["end_ids"]))
        triggers = {
            "exact": {"label_runs": runs_e, "per_1000_steps": round(1000.0 * runs_e / args.steps, 1),
                      "bubbles_end": int(len(m["b1"]["id"])), "ms_per_step": round(ms_per_step, 4)},
            "normals": {"label_runs": runs_n, "per_1000_steps": round(1000.0 * runs_n / args.steps, 1),
                        "bubbles_end": int(len(mn["b1"]["id"])),
                        "ms_per_step": round(max(mn["gpu_ms"], mn["wall"] * 1e3) / args.steps, 4),
                        "trigger_cos": -0.5},
            "same_state_at_end": same,
        }
        log(f"[bench] triggers over the window: {triggers}")
    copy = copy_bandwidth_context() if not args.no_copy_probe else None
    if copy:
        log(f"[bench] streaming copy: {copy['GBs']} GB/s ({copy['frac_of_peak']} of peak)")
    desc = {"p1": "16 gas threads R=8 (0.1R sinusoidal perturbation, wavelength 72, 1e-3 noise), "
                  "tau=0.55, sigma=0.005"}.get(args.workload, f"tau={sc.tau}, sigma={sc.sigma}")
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16dev": "f16-storage/f32"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": f"{sc.name}: {sc.nx}x{sc.ny}x{sc.nz} "
                        f"{'periodic' if all(sc.periodic) else 'walled'} D3Q19 FSLBM + bubble "
                        f"model, {desc}, {args.precision}; window = steps "
                        f"{start + args.warmup + 1}..{start + args.warmup + args.steps}",
            "cells": N,
            "precision": args.precision,
            "start_step": start,
            "topology_changes_in_window": topo,
            "breakup_active": topo > 0,
            "bubbles_start_end": [int(len(m["b0"]["id"])), int(len(m["b1"]["id"]))],
            "whole_step_alg_GBs": round(whole_gbs, 1),
            "whole_step_frac": round(whole_gbs / HBM_PEAK_GBS, 4),
            "whole_step_bytes_per_fluid_cell": b_alg,
            "bulk_sampled_steps": int(T["steps"]),
            "phase_us": phases,
            "phase_passes": PHASE_PASSES if phases else None,
            "split_triggers": triggers,
            "achievable_copy": copy,
        },
        "roofline": {
            "kernel": "k_bulk (liquid-cell stream-collide)",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": recorded_traffic(args.precision, args.workload),
            "bytes_per_launch": int(bytes_bulk),
            "avg_launch_us": round(bulk_avg_ms * 1e3, 2),
        },
    }
    if not args.no_cpu_baseline:
        threads = host_threads()
        log(f"[bench] cpu baseline: oracle on {threads} threads (~{args.cpu_seconds} s), then on "
            "one thread (one step)")
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_seconds, threads, not args.no_single_thread)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
