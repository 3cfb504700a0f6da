"""Benchmark: photon cell-crossings per second of the whole transport step.

One step is the full hot path over one batch of synthetic input already
resident in HBM: pack the fields (kappa_c, velocity, emission weight),
allocate the packets to cells, walk every packet (emission, drift, deposits,
escape), finish the tallies (conservation check) and compute the
recombination feed. Workload: the 256^3 k^2 Gaussian field of rms contrast 2
(clipped to 1e-2..1e2) with its curl-free flow at z = 1100, 2^28 packets (the
largest single-box workload; --config c2 runs the 128^3 box with 1e7 packets).

Prints one JSON line (rank 0). The dominant kernel's roofline uses the walk
kernel's duration measured with HIP events on the library's stream and the
algorithmic bytes per crossing (one 16-byte cell record read, one 8-byte
tally update). The CPU baseline is the FP64 oracle on a bounded sample.
"""
import argparse
import csv
import hashlib
import dataclasses
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_CROSSING_VEL = 16 + 8      # float4 record (kappa, U) + int64 tally update
BYTES_PER_CROSSING_NOVEL = 4 + 8     # float record (kappa) + int64 tally update
HBM_PEAK_GBS = 8000.0
# the sources of the dominant kernel (the tiled walk): stored byte counters are
# only reported while these are unchanged
WALK_SOURCES = ("paper_2312_11448_amd/csrc/walk_core.hpp", "paper_2312_11448_amd/csrc/kernels_tiled.hip",
                "paper_2312_11448_amd/csrc/common.hpp")
# the walk's launches: tile generations and the tail walk (its one-block
# prefix kernel is timed with it and counted in its bytes, not as a launch)
WALK_KERNEL = "tile_walk_kernel"
WALK_LAUNCH_KERNELS = ("tile_walk_kernel", "tail_walk_kernel")
WALK_BYTE_KERNELS = ("tile_walk_kernel", "tail_walk_kernel", "tail_prefix_kernel")


_COMMENT = re.compile(r"//[^\n]*|/\*.*?\*/", re.S)


def source_hash(paths):
    """SHA-256 of the code of the given sources, with comments and whitespace
    runs removed: a stored counter figure stays valid across comment edits
    and goes stale when the code changes. (The sources hold no string literal
    with a comment marker.)"""
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel)) as fh:
            code = _COMMENT.sub(" ", fh.read())
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()


def walk_source_hash():
    return source_hash(WALK_SOURCES)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "batch", "surrogate", "scatter"],
                    help="c3: the 256^3 workload, 2^28 packets (default); c2: the 128^3 box, 1e7 packets; "
                         "batch: 64 uneven boxes in one context; "
                         "surrogate: train the mixing-correction network on Monte-Carlo boxes, evaluate it "
                         "on held-out boxes and time its inference on the 256^3 box")
    ap.add_argument("--profile", default="doppler", choices=["doppler", "voigt"],
                    help="line profile of every box (voigt: Eq. (MC) with its damping wing)")
    ap.add_argument("--train-steps", type=int, default=6000)
    ap.add_argument("--ref-runs", type=int, default=8,
                    help="surrogate: transports of 128 packets per cell averaged into each reference")
    ap.add_argument("--photons", type=int, default=1 << 20, help="scatter: photons per step")
    ap.add_argument("--zeta", type=float, default=1e4,
                    help="scatter: expansion-rate factor of the App. A test problem (1e4: tau_S = 6e4, "
                         "about 7e4 scatterings per photon)")
    ap.add_argument("--graph", type=int, choices=[0, 1], default=None,
                    help="replay each transport as a captured HIP graph (default 0)")
    ap.add_argument("--tail", type=int, default=None, metavar="PPM",
                    help="MC_LYA_OPT_TAIL: the tail walk takes over below this many millionths of the packets in "
                         "flight (default: the library's 2 % for a single box, 20 % for the batch, whose last "
                         "generations are held by a few crowded tiles of its low-redshift boxes)")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the walk options on the first emission, before the warm-up")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="budget of the oracle's CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic", default=None,
                    help="measured HBM bytes per launch of the walk kernel (rocprofv3 counters); default "
                         "profiles/walk_traffic.json, or walk_traffic_voigt.json with --profile voigt")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain elementwise copy of MIB MiB (float32 negation, "
                         "reads and writes MIB MiB) five times, to scale byte counters")
    ap.add_argument("--probe-bandwidth", action="store_true",
                    help="only measure the achievable read bandwidth by working-set size (L2, MALL, HBM) and "
                         "the streaming copy's")
    ap.add_argument("--summarize-counters", nargs=4, metavar=("FETCH", "WRITE", "CAL_FETCH", "CAL_WRITE"),
                    help="only turn four rocprofv3 counter_collection.csv files (FETCH_SIZE and WRITE_SIZE "
                         "of the benchmark, then of --calibrate-copy) into the walk's HBM bytes per launch, "
                         "written to --traffic")
    ap.add_argument("--valu", default=None,
                    help="measured VALU instructions per crossing of the walk (rocprofv3 counters); default "
                         "profiles/walk_valu.json, or walk_valu_voigt.json with --profile voigt")
    ap.add_argument("--calibration-mib", type=int, default=1024)
    ap.add_argument("--summarize-valu", nargs=3, metavar=("CSV", "LOG", "OUT"),
                    help="only turn a rocprofv3 counter_collection.csv with SQ_INSTS_VALU / SQ_INSTS_SALU of "
                         "a benchmark run, and that run's JSON line (LOG), into wave instructions per crossing "
                         "(walk) or per scattering (--config scatter), written to OUT")
    a = ap.parse_args()
    suffix = "_voigt" if a.profile == "voigt" else ""
    if a.traffic is None:
        a.traffic = os.path.join(ROOT, "profiles", f"walk_traffic{suffix}.json")
    if a.valu is None:
        a.valu = os.path.join(ROOT, "profiles", f"walk_valu{suffix}.json")
    return a


def _counter_rows(path, counter):
    with open(path, newline="") as fh:
        return [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]


def _first_generation(name):
    """True for a dispatch of the first tile generation, tile_walk_kernel<VEL,
    GEN0 = true, VOIGT>."""
    if WALK_KERNEL + "<" not in name:
        return False
    args = name.split(WALK_KERNEL + "<", 1)[1].split(">", 1)[0].split(",")
    return len(args) == 3 and args[1].strip() == "true"


def summarize_counters(a):
    """HBM bytes per walk (one transport) from FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch), each scaled by what the same counter reads for a copy of known
    size. Transports are counted by their first tile generation (one per
    single-batch transport); the benchmark divides by its own launch count,
    since the number of (empty) generation launches after the tail walk
    varies from run to run."""
    f_csv, w_csv, cf_csv, cw_csv = a.summarize_counters
    known = a.calibration_mib * (1 << 20)
    scale = {}
    for name, path, counter in (("fetch", cf_csv, "FETCH_SIZE"), ("write", cw_csv, "WRITE_SIZE")):
        vals = [float(r["Counter_Value"]) * 1024.0 for r in _counter_rows(path, counter)
                if "neg_kernel" in r["Kernel_Name"]]
        if not vals:
            raise SystemExit(f"no copy-kernel rows in {path}")
        scale[name] = known / (sum(vals) / len(vals))
    per = {}
    launches = {}
    for name, path, counter in (("fetch", f_csv, "FETCH_SIZE"), ("write", w_csv, "WRITE_SIZE")):
        rows = _counter_rows(path, counter)
        vals = [float(r["Counter_Value"]) * 1024.0 for r in rows
                if any(k in r["Kernel_Name"] for k in WALK_BYTE_KERNELS)]
        n = sum(1 for r in rows if any(k in r["Kernel_Name"] for k in WALK_LAUNCH_KERNELS))
        walks = sum(1 for r in rows if _first_generation(r["Kernel_Name"]))
        if not vals or not n or not walks:
            raise SystemExit(f"no walk rows in {path}")
        per[name] = scale[name] * sum(vals) / walks
        launches[name] = {"launches": n, "walks": walks}
    out = {"config": a.config, "profile": a.profile, "kernel": " + ".join(WALK_BYTE_KERNELS), "counted": launches,
           "fetch_scale": scale["fetch"], "write_scale": scale["write"],
           "fetch_bytes_per_walk": per["fetch"], "write_bytes_per_walk": per["write"],
           "bytes_per_walk": per["fetch"] + per["write"], "source_sha256": walk_source_hash()}
    with open(a.traffic, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out), flush=True)


def summarize_valu(a):
    """Vector and scalar wave instructions per unit of work of the dominant
    kernel, from SQ_INSTS_VALU / SQ_INSTS_SALU summed over its dispatches of a
    profiled benchmark run, divided by the work that run did (its warm-up
    and timed steps, from its JSON line)."""
    csv_path, log_path, out_path = a.summarize_valu
    with open(log_path) as fh:
        line = [json.loads(t) for t in fh if t.startswith("{")][-1]
    runs = line["steps"] + line["warmup"]
    scatter = line["metric"].startswith("resonant")
    kernels = ("scatter_kernel",) if scatter else WALK_BYTE_KERNELS
    units = runs * (line["config"]["scatterings_per_step"] if scatter else line["config"]["crossings_per_step"])
    tot = {}
    for name in ("SQ_INSTS_VALU", "SQ_INSTS_SALU"):
        rows = [r for r in _counter_rows(csv_path, name) if any(k in r["Kernel_Name"] for k in kernels)]
        if not rows:
            raise SystemExit(f"no {name} rows of {kernels} in {csv_path}")
        tot[name] = sum(float(r["Counter_Value"]) for r in rows)
    unit = "scattering" if scatter else "crossing"
    out = {"kernel": " + ".join(kernels), "workload": line["config"]["workload"], "unit": unit,
           f"valu_wave_instr_per_{unit}": tot["SQ_INSTS_VALU"] / units,
           f"salu_wave_instr_per_{unit}": tot["SQ_INSTS_SALU"] / units,
           "source_sha256": scatter_source_hash() if scatter else walk_source_hash()}
    if scatter:
        out.update(photons=line["config"]["photons"], zeta=a.zeta)
    else:
        out.update(config=a.config, profile=a.profile)
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out), flush=True)


def calibrate_copy(mib):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "neg", "bytes_read": n * 4, "bytes_written": n * 4,
                      "launches": 5}), flush=True)


def probe_bandwidth():
    """Achievable read bandwidth by working-set size: the library's read probe
    (mc_lya_probe_read: one launch reads the buffer many times over, each
    thread the same positions every pass) from a few MiB (served by the
    XCDs' L2 caches) through the 256 MB last-level cache (MALL) to GiB sizes
    (HBM), timed with events on the current stream, plus the streaming copy
    (torch's negation: one read and one write per element) at HBM sizes.
    Prints one JSON line per measurement."""
    import torch
    import paper_2312_11448_amd as M
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    sink = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    for mib in (4, 16, 32, 64, 128, 192, 256, 512, 1024, 4096):
        nbytes = mib << 20
        buf = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        passes = max(2, min(4096, (16 << 30) // nbytes))
        grid = cus * 8
        M.mc_lya_probe_read(buf.data_ptr(), nbytes, 1, grid, sink.data_ptr())
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        M.mc_lya_probe_read(buf.data_ptr(), nbytes, passes, grid, sink.data_ptr())
        t1.record()
        t1.synchronize()
        s = t0.elapsed_time(t1) / 1e3
        print(json.dumps({"probe": "read", "working_set_mib": mib, "passes": passes,
                          "GB_per_s": nbytes * passes / s / 1e9}), flush=True)
        del buf
    for mib in (1024, 4096):
        n = mib * (1 << 20) // 8           # two buffers of mib / 2 MiB each
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        reps = max(20, min(2000, (8 << 30) // (8 * n)))
        for _ in range(5):
            torch.neg(src, out=dst)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            torch.neg(src, out=dst)
        t1.record()
        t1.synchronize()
        s = t0.elapsed_time(t1) / 1e3
        print(json.dumps({"probe": "neg", "working_set_mib": mib, "reps": reps,
                          "GB_per_s": 8.0 * n * reps / s / 1e9}), flush=True)
        del src, dst


def workload_name(config, specs):
    voigt = ", Voigt profile" if getattr(specs[0], "profile", "doppler") == "voigt" else ""
    if config == "batch":
        return (f"batch of {len(specs)} boxes, N ~ U{{16..96}}, z ~ U[800, 1400], k^2 GRF rms ~ U[0.2, 2] "
                f"+ curl-free flow (rms 0.1 v_th), T = T0 (1+z), x_e = 0.1, "
                f"{specs[0].n_packets:.0e} packets per box{voigt}")
    return specs[0].name + voigt


def cpu_baseline(specs, budget_s):
    """The oracle as it is, on the host's cores, over packet blocks of the same
    workload (one fiftieth of a box's packets per block, boxes in turn) until
    the time budget of oracle transport is spent."""
    from oracle import walker
    threads = int(os.environ.get("OMP_NUM_THREADS", 0) or os.cpu_count() or 1)
    preps = [None] * len(specs)
    done = [0] * len(specs)
    cross, spent, blocks = 0, 0.0, 0
    while spent < budget_s and any(d < s.n_packets for d, s in zip(done, specs)):
        for i, spec in enumerate(specs):
            n = spec.n_packets
            if done[i] >= n or spent >= budget_s:
                continue
            if preps[i] is None:
                preps[i] = walker.Prepared(spec)
            block = max(1, n // 50)
            t0 = time.perf_counter()
            r = preps[i].transport(done[i], min(n, done[i] + block), nthreads=threads)
            spent += time.perf_counter() - t0
            cross += r["crossings"]
            done[i] = min(n, done[i] + block)
            blocks += 1
    walked = sum(done)
    total = sum(s.n_packets for s in specs)
    where = (f"packets [0, {done[0]}) of {total}" if len(specs) == 1 else
             f"{blocks} blocks of 1/50 of a box's packets over {sum(d > 0 for d in done)} of "
             f"{len(specs)} boxes ({walked} of {total} packets)")
    return {"value": cross / spent, "unit": "crossings/s", "cores": threads, "kind": "oracle",
            "sample": f"{where} of the same workload ({cross} crossings in {spent:.1f} s of oracle "
                      f"transport, FP64 C + OpenMP)"}


# VALU issue peak of the chip in wave instructions: 256 compute units x 4
# SIMDs, one wave64 instruction per SIMD every 4 cycles at 2.4 GHz.
VALU_PEAK_GINSTR = 256 * 4 * 2.4e9 / 4 / 1e9
SCATTER_SOURCES = ("paper_2312_11448_amd/csrc/kernels_scatter.hip", "paper_2312_11448_amd/csrc/walk_core.hpp",
                   "paper_2312_11448_amd/csrc/dawson.hpp", "paper_2312_11448_amd/csrc/common.hpp")


def scatter_source_hash():
    return source_hash(SCATTER_SOURCES)


def bench_scatter(a):
    """Resonant-scattering Monte Carlo (App. A): scatterings per second of
    whole steps (emit, scatter, tally, feed) over a photon batch of the 32^3
    lognormal box at z = 1100 with the Voigt profile and the physical p_ab,
    with the expansion rate scaled by zeta as in the App. A test problem (at
    zeta = 1 a photon scatters ~3e6 times and the slowest of a batch sets the
    step time)."""
    import torch
    import workloads as W
    import paper_2312_11448_amd as M
    spec = W.make_box("c1", n_packets=a.photons, profile="voigt", zeta=a.zeta)
    dev = torch.device("cuda:0")
    sim = M.Simulation([spec], device=dev)
    sim.set_option(M.MC_LYA_OPT_TIMING, 1)

    def step():
        sim.emit()
        sim.scatter()
        t = sim.tally(want_emitted=False)
        f = sim.feed()
        return t, f

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize(dev)
    sim.kernel_time()
    t0 = time.perf_counter()
    nscat = cross = 0
    for _ in range(a.steps):
        t, f = step()
        st = t["stats"][0]
        if st.conserved != 1 or st.capped_packets:
            raise SystemExit("conservation identity failed")
        nscat += st.scatterings
        cross += st.crossings
    torch.cuda.synchronize(dev)
    dt = time.perf_counter() - t0
    kms, launches = sim.kernel_time()
    sim.close()
    rate = nscat / dt
    valu = None
    path = os.path.join(ROOT, "profiles", "scatter_valu.json")
    if os.path.exists(path):
        with open(path) as fh:
            pr = json.load(fh)
        if (pr.get("source_sha256") == scatter_source_hash() and pr.get("photons") == a.photons
                and pr.get("zeta") == a.zeta):
            valu = pr["valu_wave_instr_per_scattering"]
    achieved = None if valu is None else valu * (nscat / (kms / 1e3)) / 1e9
    fs = f["stats"][0]
    out = {
        "metric": "resonant scatterings/s", "value": rate, "unit": "scatterings/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": dt * 1e3 / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"App. A scattering Monte Carlo: {a.photons} photons of the 32^3 lognormal "
                               f"(ln-sigma 0.3) box, z=1100, T=3000K, x_e=0.1, zeta={a.zeta:g}, Voigt profile, "
                               f"physical p_ab, lost below x=-300",
                   "photons": a.photons, "scatterings_per_step": nscat / a.steps,
                   "scatterings_per_photon": nscat / a.steps / a.photons,
                   "crossings_per_step": cross / a.steps, "kernel_ms_per_step": kms / a.steps,
                   "c_mc": fs.c_mc, "f_escape": fs.f_escape, "f_absorbed": fs.f_absorbed, "f_wing": fs.f_wing},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_GINSTR,
                     "unit": "G wave-instr/s (VALU issue)",
                     "frac": None if achieved is None else achieved / VALU_PEAK_GINSTR, "traffic": None},
    }
    print(json.dumps(out), flush=True)


def bench_surrogate(a):
    """Surrogate cells per second (features + inference over the 256^3 box),
    with its accuracy against a high-statistics Monte-Carlo reference of
    held-out 256^3 boxes. Training: 200 field seeds of the three single-box
    workloads (each box's own Monte Carlo, 2^17 cells kept per box)."""
    import numpy as np
    import torch
    import workloads as W
    from workloads import surrogate as WS
    import paper_2312_11448_amd as M
    from paper_2312_11448_amd import surrogate as SG

    t_start = time.perf_counter()
    parts = []
    boxes = WS.training_boxes()
    t_fields = 0.0
    sims = {}            # one context per workload family; each new box's fields are loaded into it
    for i, (key, fseed, ppc, pseed) in enumerate(boxes):
        t0 = time.perf_counter()
        spec = WS.family_box(key, fseed, ppc, pseed, device="cuda")
        t_fields += time.perf_counter() - t0
        if key not in sims:
            for k in list(sims):
                sims.pop(k).close()
            sims[key] = M.Simulation(spec, max_packets=spec.n_packets,
                                     batch_packets=min(spec.n_packets, SG.BATCH))
        parts.append(SG.mc_cells([spec], keep=1 << 17, pick_seed=i, sim=sims[key]))
        del spec
        if i % 10 == 9 or i == len(boxes) - 1:
            print(f"surrogate: training box {i + 1}/{len(boxes)} ({key}), {time.perf_counter() - t_start:.0f} s",
                  flush=True)
    for k in list(sims):
        sims.pop(k).close()
    data = SG.concat(parts)
    del parts
    n_train = int(data["features"].shape[0])
    with M.Mlp(WS.initial_params(1)) as mlp:
        t0 = time.perf_counter()
        losses = SG.train(mlp, data, steps=a.train_steps, log_every=max(1, a.train_steps // 10))
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        lo, hi = SG.envelope(data["features"][data["w"] > 0])
        mlp.set_envelope(lo, hi)
        del data
        print(f"surrogate: trained {a.train_steps} steps in {t_train:.1f} s", flush=True)
        eval_specs = [WS.family_box(k, fs, 16, ps, device="cuda") for k, fs, ps in WS.evaluation_boxes()]
        ref = SG.reference(eval_specs, runs=a.ref_runs, packets_per_cell=128, seed0=5000)
        print(f"surrogate: reference 1 done, {time.perf_counter() - t_start:.0f} s", flush=True)
        ref2 = SG.reference(eval_specs, runs=a.ref_runs, packets_per_cell=128, seed0=6000)
        print(f"surrogate: reference 2 done, {time.perf_counter() - t_start:.0f} s", flush=True)
        pred = SG.predict(mlp, eval_specs)
        acc = SG.evaluate(pred["M"], ref, ref2)
        n_out = pred["n_outside"]
        del ref, ref2, pred
        big = W.make_box("c3")
        with M.Simulation(big) as sim:
            t_all, t_inf, n, _ = SG.time_inference(mlp, sim)
            # the Monte Carlo of the same box and packet count, timed after a
            # first transport
            sim.emit()
            sim.transport()
            sim.emit()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.transport()
            st = sim.tally(want_emitted=False)["stats"][0]
            torch.cuda.synchronize()
            t_mc = time.perf_counter() - t0
            feats = sim.features()
            sample = feats[:: max(1, n // (1 << 18))][: 1 << 18].cpu().numpy().astype(np.float64)
        params = np.array(mlp.params(), dtype=np.float64)
    flops = SG.forward_flops_per_cell() * n
    achieved = flops / t_inf / 1e12
    out = {
        "metric": "surrogate cells/s", "value": n / t_all, "unit": "cells/s", "n_gpus": 1,
        "steps": 5, "warmup": 2, "ms_per_step": t_all * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "8-64-64-1 ReLU network on the 256^3 k^2 field (features + inference); "
                               "trained on 200 field seeds of the 32^3, 128^3 and 256^3 workloads "
                               "(512, 128 and 64 packets per cell), evaluated on 3 held-out 256^3 seeds "
                               f"against the mean of {a.ref_runs} transports of 128 packets per cell",
                   "cells": n, "inference_ms": t_inf * 1e3, "features_ms": (t_all - t_inf) * 1e3,
                   "mc_transport_s_same_box": t_mc, "mc_crossings": st.crossings,
                   "speedup_vs_mc": t_mc / t_all, "train_steps": a.train_steps, "train_cells": n_train,
                   "train_s": t_train, "field_generation_s": t_fields,
                   "train_loss": losses, "eval_cells_outside_envelope": n_out,
                   "accuracy_vs_reference_mc": acc, "wall_s": time.perf_counter() - t_start},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": achieved / 2500.0, "traffic": None},
    }
    if not a.no_cpu_baseline:
        from oracle import surrogate as OS
        threads = int(os.environ.get("OMP_NUM_THREADS", 0) or os.cpu_count() or 1)
        t0 = time.perf_counter()
        OS.forward(params, sample)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": sample.shape[0] / dt, "unit": "cells/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{sample.shape[0]} cells of the 256^3 box through the FP64 "
                                         f"numpy network ({dt:.2f} s)"}
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.calibrate_copy:
        calibrate_copy(a.calibrate_copy)
        return
    if a.probe_bandwidth:
        probe_bandwidth()
        return
    if a.summarize_counters:
        summarize_counters(a)
        return
    if a.summarize_valu:
        summarize_valu(a)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import workloads as W
    import paper_2312_11448_amd as M
    if a.config == "surrogate":
        return bench_surrogate(a)
    if a.config == "scatter":
        return bench_scatter(a)

    specs = W.batch_specs() if a.config == "batch" else [W.make_box(a.config)]
    if a.profile != "doppler":
        specs = [dataclasses.replace(sp, profile=a.profile) for sp in specs]
    dev = torch.device("cuda:0")
    sim = M.Simulation(specs, device=dev)
    # one event pair around each transport's walk, its launches counted: the
    # launches run back to back, as they do untimed
    sim.set_option(M.MC_LYA_OPT_TIMING, 2)
    graph = a.graph if a.graph is not None else 0
    sim.set_option(M.MC_LYA_OPT_GRAPH, graph)
    tail = a.tail if a.tail is not None else (200000 if a.config == "batch" else None)
    if tail is not None:
        sim.set_option(M.MC_LYA_OPT_TAIL, tail)
    seeds, npk = [s.seed for s in specs], [s.n_packets for s in specs]
    tuned = None
    if a.autotune:
        sim.emit(seeds, npk)
        r = sim.autotune(1)
        tuned = {"kernel": r.kernel, "tile_share": r.tile_share, "block": r.block,
                 "waves_per_cu": r.waves_per_cu, "chunk": r.chunk, "refill": r.refill,
                 "tile_chunk": r.tile_chunk, "tile_refill": r.tile_refill,
                 "transport_ms": r.best_ms, "default_ms": r.start_ms}

    def step():
        sim.refresh()
        sim.emit(seeds, npk)
        sim.transport()
        t = sim.tally(want_emitted=False)
        f = sim.feed()
        return t, f

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize(dev)
    sim.kernel_time()                      # drop the warm-up launches
    t0 = time.perf_counter()
    cross = 0
    for _ in range(a.steps):
        t, f = step()
        for st in t["stats"]:
            if st.conserved != 1 or st.capped_packets:
                raise SystemExit("conservation identity failed")
            cross += st.crossings
    torch.cuda.synchronize(dev)
    dt = time.perf_counter() - t0
    kms, launches = sim.kernel_time()
    # the walk of one step may be several launches (one per tile generation):
    # time and bytes are both taken per step
    walk_s = kms / 1e3 / a.steps
    cross_per_step = cross / a.steps
    bpc = BYTES_PER_CROSSING_VEL if specs[0].velocity is not None else BYTES_PER_CROSSING_NOVEL
    achieved = bpc * cross_per_step / walk_s / 1e9
    traffic = None
    if os.path.exists(a.traffic):
        with open(a.traffic) as fh:
            tr = json.load(fh)
        if (tr.get("config") == a.config and tr.get("profile", "doppler") == a.profile
                and tr.get("source_sha256") == walk_source_hash()):
            traffic = tr.get("bytes_per_walk")     # per launch below, with this run's launch count
    # the walk's issue rate: measured VALU instructions per crossing (rocprofv3
    # SQ_INSTS_VALU over the same workload and sources) times this run's rate
    valu = None
    if os.path.exists(a.valu):
        with open(a.valu) as fh:
            pv = json.load(fh)
        if (pv.get("config") == a.config and pv.get("profile") == a.profile
                and pv.get("source_sha256") == walk_source_hash()):
            valu = pv["valu_wave_instr_per_crossing"] * cross_per_step / walk_s / 1e9
    out = {
        "metric": "photon cell-crossings/s",
        "value": cross / dt,
        "unit": "crossings/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload_name(a.config, specs), "cells": sum(x.ncells for x in specs),
                   "packets": sum(npk), "graph": graph, "tail_ppm": tail, "autotuned": tuned,
                   "crossings_per_step": cross_per_step,
                   "packets_per_s": sum(npk) * a.steps / dt,
                   "walk_ms": walk_s * 1e3,
                   "walk_launches_per_step": launches / a.steps,
                   "walk_launch_avg_us": kms * 1e3 / max(1, launches),
                   "walk_alg_bytes_per_launch": bpc * cross / max(1, launches),
                   "walk_crossings_per_s": cross_per_step / walk_s,
                   "f_absorbed": f["stats"][0].f_absorbed, "c_mc": f["stats"][0].c_mc},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if traffic is None else traffic * a.steps / max(1, launches)},
        "roofline_valu": {"bound": "alu", "achieved": valu, "peak": VALU_PEAK_GINSTR,
                          "unit": "G wave-instr/s (VALU issue)",
                          "frac": None if valu is None else valu / VALU_PEAK_GINSTR},
    }
    sim.close()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(specs, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
