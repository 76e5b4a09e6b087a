"""Throughput of the axisymmetric cascaded LB time step on one MI355X.

Workload: the 1024 x 2048 rotating-lid cylinder with buoyancy (Re = 1000,
Ri = 0.5, Pr = 1), FP32 arithmetic and storage, in the faster (by a short
trial) of the single-buffer layout (AA, one step per launch) and the
two-buffer layout with two steps per launch (AB2), steps replayed as
captured HIP graphs.  A step is one update of every node's 19 populations
(D2Q9 + 2 x D2Q5).  Prints one JSON line.

The dominant (only) kernel is the fused step kernel (k_step, or k_step_two
for two steps); its algorithmic traffic is 152 B per node update (19
populations x 4 B, read and written once), so achieved GB/s = 152 * nodes /
average step time.  Beside
the headline the line carries: the same step on a lattice too large for the
Infinity Cache, the error of every storage type against the FP64 oracle,
the batched and served workloads, and the oracle's own speed on the host.
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS (D2Q9+2×D2Q5 node updates/s), % HBM roofline; batched solves/s, p99 latency"
PEAK_HBM_GBS = 8000.0
BYTES_PER_UPDATE = {"f32": 152, "f16": 76, "bf16": 76}


STEP_SOURCES = ["paper_1806_10241_amd/csrc/axlb_node.h", "paper_1806_10241_amd/csrc/axlb_kernels.hip",
                "paper_1806_10241_amd/csrc/axlb_device.h", "paper_1806_10241_amd/csrc/axlb_twostep.hip"]


def code_text(source: bytes) -> bytes:
    """A C++ source without its comments and with whitespace runs collapsed,
    so that edits to comments alone keep a counter summary valid."""
    import re
    text = source.decode()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split()).encode()


def step_kernel_hash() -> str:
    """sha256 of the code (comments excluded) of the step-kernel sources."""
    import hashlib
    h = hashlib.sha256()
    for rel in STEP_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(code_text(f.read()))
    return h.hexdigest()


def profile_path(storage: str, Nr: int, Nz: int, layout: str) -> str:
    suffix = "" if layout == "aa" else "_" + layout
    return os.path.join(ROOT, "profiles", "step_kernel_%dx%d_%s%s.md" % (Nr, Nz, storage, suffix))


def measured_traffic(storage: str, Nr: int, Nz: int, layout: str = "aa"):
    """HBM bytes per launch of the dominant step kernel from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of
    known size); None unless that summary was taken on the current
    step-kernel sources and on this workload."""
    path = profile_path(storage, Nr, Nz, layout)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != step_kernel_hash():
        return None
    try:
        return int(float(vals["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def step_working_set(Nr: int, Nz: int, storage: str, layout: str) -> int:
    """Bytes a step touches: the population buffer(s) and both time levels of
    the lagged fields (FP32 velocities with FP32 storage, binary16 with
    16-bit storage; T in FP32), rows padded to 64 nodes."""
    plane = Nz * ((Nr + 63) // 64 * 64)
    es = 4 if storage == "f32" else 2
    pops = 19 * es * plane * (1 if layout == "aa" else 2)
    return pops + 2 * (3 * es + 4) * plane


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    """Threads this process may use: the OpenMP setting if there is one,
    else the CPUs in its affinity mask."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


ACCURACY_CASE = dict(Nr=128, Nz=256, Re=1000.0, Ri=0.5, u_noise=1e-4)
ACCURACY_STEPS = 1000


def accuracy_runs():
    """The benchmark's physics at reduced resolution (rotating-lid cylinder
    128 x 256, same Re, Ri, Pr and seeded noise) after 1000 steps with each
    storage type on the GPU: fields and wall Nusselt numbers."""
    from paper_1806_10241_amd import axlb
    from paper_1806_10241_amd import inputs as I
    c = I.rotating_lid_cylinder(**ACCURACY_CASE)
    out = {}
    for st in ("f32", "f16", "bf16"):
        lat = axlb.Lattice(c, storage=st)
        lat.step(ACCURACY_STEPS)
        out[st] = (lat.fields(), lat.nusselt())
        lat.close()
    return out


def rel_errors(F, R):
    """Relative L2 errors after the parity tests' convention: rho - 1 and T
    against their own norms, velocity components against the speed norm;
    plus the largest Nusselt error."""
    speed = np.linalg.norm(np.sqrt(R["ur"] ** 2 + R["uz"] ** 2 + R["uth"] ** 2))
    e = {}
    for k in ("ur", "uz", "uth"):
        e[k] = float(np.linalg.norm(F[k] - R[k]) / speed)
    e["T"] = float(np.linalg.norm(F["T"] - R["T"]) / np.linalg.norm(R["T"]))
    e["rho-1"] = float(np.linalg.norm(F["rho"] - R["rho"]) / np.linalg.norm(R["rho"] - 1.0))
    return e


def cpu_leg(case, single_steps: int, multi_steps: int, gpu_accuracy):
    """The FP64 oracle on this host: built for this CPU (-march=native), timed
    on the first steps of the benchmark workload with one thread and with
    every core this process may use; and, as the reference of the accuracy
    report, run on the reduced-resolution case that accuracy_runs() ran."""
    import tempfile

    import oracle
    from paper_1806_10241_amd import inputs as I
    with tempfile.TemporaryDirectory() as d:
        lib = oracle._load(oracle.build_native(os.path.join(d, "liboracle_native.so")))
        cores = host_cores()
        timings = []
        for threads, steps in ((1, single_steps), (cores, multi_steps)):
            lib.orc_set_threads(threads)
            L = oracle.Lattice(case, deriv_mode=oracle.DERIV_PREVIOUS, fields=case["fields"](),
                               lib=lib)
            t0 = time.perf_counter()
            L.step(steps)
            dt = time.perf_counter() - t0
            timings.append((case["Nr"] * case["Nz"] * steps / dt / 1e6, steps, dt))
            del L
        accuracy = None
        if gpu_accuracy is not None:
            c = I.rotating_lid_cylinder(**ACCURACY_CASE)
            R = oracle.Lattice(c, deriv_mode=oracle.DERIV_PREVIOUS, fields=c["fields"](), lib=lib)
            R.step(ACCURACY_STEPS)
            Rf, Rnu = R.fields(), R.nusselt()
            del R
            accuracy = {"case": "rotating-lid cylinder %dx%d, Re=%g, Ri=%g, %d steps"
                                % (c["Nr"], c["Nz"], c["Re"], c["Ri"], ACCURACY_STEPS),
                        "bars": {"f32": 1e-5, "f16": 2e-3, "bf16": 2e-3, "nusselt": 5e-3}}
            for st, (F, nu) in gpu_accuracy.items():
                e = rel_errors(F, Rf)
                e["nusselt"] = float(max(abs(a - b) / abs(b) for a, b in zip(nu, Rnu)))
                accuracy[st] = {k: float("%.3g" % v) for k, v in e.items()}
    (v1, s1, dt1), (vn, sn, dtn) = timings
    base = {"value": round(vn, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": "%d steps of the %dx%d workload, FP64, %d threads (%.1f s); "
                      "built -O3 -march=native on %s" % (sn, case["Nr"], case["Nz"], cores, dtn,
                                                         cpu_model()),
            "single_thread": {"value": round(v1, 3), "unit": "MLUPS", "cores": 1,
                              "sample": "%d steps (%.1f s)" % (s1, dt1)},
            "cpu_model": cpu_model()}
    return base, accuracy


def bench_small_members(n, steps, warmup):
    """A batch of many small annuli (Nr ~ U{16..64}, Nz ~ U{16..128}, AA
    members), stepped with every member on the work-list (autotuned tile and
    schedule) and with each member whole in one workgroup (a bundle per
    launch)."""
    from paper_1806_10241_amd import axlb
    from paper_1806_10241_amd import inputs as I

    cases = I.batched_annuli(n=n, seed=7, nr=(16, 64), nz=(16, 128))
    nodes = sum(c["Nr"] * c["Nz"] for c in cases)
    lats = [axlb.Lattice(c) for c in cases]
    b = axlb.Batch(lats)
    tile, blocks, _ = b.autotune(steps_per_trial=20)
    picked = b.whole()[0]
    out = {"instances": n, "nodes": nodes, "steps": steps,
           "work_list_schedule": {"tile": "%dx%d" % axlb.tile_shape(tile), "blocks": blocks},
           "autotuner_picked_whole": picked > 0}
    for name, limit in (("work_list", 0), ("whole_members", axlb.WHOLE_MAX_NODES)):
        b.set_whole(limit)
        b.step(warmup)
        b.sync()
        t0 = time.perf_counter()
        b.step(steps)
        b.sync()
        dt = time.perf_counter() - t0
        out[name] = {"mlups": round(nodes * steps / dt / 1e6, 1), "ms_per_step": round(dt / steps * 1e3, 4)}
    b.close()
    for lat in lats:
        lat.close()
    out["speedup_whole"] = round(out["whole_members"]["mlups"] / out["work_list"]["mlups"], 2)
    return out


def bench_batched(n, steps, warmup, baseline_steps):
    """256-way batch of uneven annulus-convection instances (seeded), two
    ways: single-buffer (AA) members in fused one-step launches with an
    autotuned schedule and cache-sized groups, and two-buffer members in
    fused two-step launches (AB2); both with 100-step graph bundles, against
    the same instances stepped by one launch per instance per step."""
    from paper_1806_10241_amd import axlb
    from paper_1806_10241_amd import inputs as I

    cases = I.batched_annuli(n=n, seed=4)
    nodes = sum(c["Nr"] * c["Nz"] for c in cases)
    runs = {}
    for layout in ("aa", "ab2"):
        lats = [axlb.Lattice(c, layout=layout) for c in cases]
        b = axlb.Batch(lats)
        sched = None
        if layout == "aa":
            tile, blocks, _ = b.autotune(steps_per_trial=20)
            sched = {"tile": "%dx%d" % axlb.tile_shape(tile), "blocks": blocks,
                     "whole_members": b.whole()[1]}
        b.step(warmup)
        b.sync()
        t0 = time.perf_counter()
        b.step(steps)
        b.sync()
        dt = time.perf_counter() - t0
        b.close()
        nonfinite = 0
        for lat in lats:
            try:
                lat.residual()
            except axlb.AxlbError:
                nonfinite += 1
        runs[layout] = {"mlups": round(nodes * steps / dt / 1e6, 1),
                        "solves_per_s": round(n / (dt * 1e4 / steps), 3),
                        "nonfinite_instances": nonfinite}
        if sched:
            runs[layout]["schedule"] = sched
        if layout == "aa":
            # the loop of single launches on the same (AA) instances
            axlb.step_each(lats, 2)
            for lat in lats:
                lat.sync()
            t1 = time.perf_counter()
            axlb.step_each(lats, baseline_steps)
            for lat in lats:
                lat.sync()
            dt_loop = time.perf_counter() - t1
            loop = {"steps": baseline_steps,
                    "mlups": round(nodes * baseline_steps / dt_loop / 1e6, 1)}
        for lat in lats:
            lat.close()
        del lats
    best = max(runs, key=lambda k: runs[k]["mlups"])
    return {"instances": n, "nodes": nodes, "steps": steps, "layout": best,
            "mlups": runs[best]["mlups"], "solves_per_s": runs[best]["solves_per_s"],
            "solve": "1e4 steps of one instance", "by_layout": runs,
            "loop_of_single_launches": loop,
            "speedup_vs_loop": round(runs[best]["mlups"] / loop["mlups"], 2),
            "nonfinite_instances": runs[best]["nonfinite_instances"]}


def bench_served(n, rate, tol, max_steps, budget_gib, max_nr_log2, max_nz_log2, order, window,
                 baseline=True):
    """Poisson arrivals of mixed solve requests (seeded trace) served by the
    continuous-batching pool, against serving the same trace one request at
    a time with plain single-lattice runs.  Latency = arrival to result."""
    from paper_1806_10241_amd import axlb
    from paper_1806_10241_amd import inputs as I

    trace = I.serving_trace(n=n, rate=rate, seed=5, max_nr_log2=max_nr_log2,
                            max_nz_log2=max_nz_log2)
    pool = axlb.Pool(budget_bytes=int(budget_gib * (1 << 30)), order=order, node_window=window)
    arrival, done, steps_of = {}, {}, {}
    pending = list(trace)
    t0 = time.perf_counter()
    reported = 0.0
    while pending or len(done) < len(arrival):
        now = time.perf_counter() - t0
        if now - reported >= 30.0:  # progress of a long trace
            reported = now
            print("bench: served %d of %d requests (%d arrived) after %.0f s"
                  % (len(done), n, len(arrival), now), file=sys.stderr, flush=True)
        while pending and pending[0][0] <= now:
            at, case, st = pending.pop(0)
            rid = pool.submit(case, st, tol=tol, max_steps=max_steps)
            arrival[rid] = at
        if len(done) < len(arrival):
            pool.tick()
            now = time.perf_counter() - t0
            for rid in arrival:
                if rid not in done:
                    state, steps, _ = pool.status(rid)
                    if state in (axlb.REQ_DONE, axlb.REQ_FAILED):
                        done[rid] = now
                        steps_of[rid] = steps
        elif pending:
            time.sleep(max(0.0, pending[0][0] - (time.perf_counter() - t0)))
    makespan = time.perf_counter() - t0
    _, node_updates = pool.usage()
    lat_s = np.array([done[r] - arrival[r] for r in arrival])
    pool.close()
    out = {"requests": n, "rate_per_s": rate, "arrival_span_s": round(trace[-1][0], 3),
           "tol": tol, "max_steps": max_steps,
           "budget_gib": budget_gib, "admission": order, "node_window": window,
           "grid": "Nr 64..%d x Nz 64..%d" % (2 ** max_nr_log2, 2 ** max_nz_log2),
           "p50_s": round(float(np.percentile(lat_s, 50)), 4),
           "p99_s": round(float(np.percentile(lat_s, 99)), 4),
           "solves_per_s": round(n / makespan, 3),
           "aggregate_mlups": round(node_updates / makespan / 1e6, 1)}
    if not baseline:
        return out
    # one request at a time: each case alone in the pool's layout for its
    # storage, same stop rule, FIFO queue
    finish = 0.0
    lat1 = []
    for at, case, st in trace:
        lat = axlb.Lattice(case, storage=st, layout="ab2" if st == "f32" else "aa")
        t1 = time.perf_counter()
        lat.residual()
        while lat.steps < max_steps:
            lat.step(100)
            if lat.residual() < tol:
                break
        service = time.perf_counter() - t1
        lat.close()
        finish = max(finish, at) + service
        lat1.append(finish - at)
    lat1 = np.array(lat1)
    out["one_at_a_time"] = {"p50_s": round(float(np.percentile(lat1, 50)), 4),
                            "p99_s": round(float(np.percentile(lat1, 99)), 4),
                            "solves_per_s": round(n / finish, 3)}
    return out


def layout_trial(case, storage: str, steps: int = 60):
    """ms per step of the single-buffer layout (256 x 1 tile) and of two steps
    per launch on two buffers, on the workload, graph replays."""
    import torch

    from paper_1806_10241_amd import axlb
    out = {}
    for layout in ("aa", "ab2"):
        stream = torch.cuda.Stream()
        lat = axlb.Lattice(case, layout=layout, storage=storage, stream=stream)
        if layout == "aa":
            lat.set_tile(axlb_default_tile())
        lat.step(20)
        lat.prepare_steps(steps)
        lat.sync()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        lat.step(steps)
        b.record(stream)
        b.synchronize()
        out[layout] = a.elapsed_time(b) / steps
        lat.close()
        del lat
        torch.cuda.empty_cache()
    return out


def headline(args, case, stream):
    """The timed run: warmup, then exactly args.steps steps replayed as
    graphs captured beforehand, bracketed by HIP events on the lattice's
    stream."""
    import torch

    from paper_1806_10241_amd import axlb
    nodes = case["Nr"] * case["Nz"]
    lat = axlb.Lattice(case, storage=args.storage, layout=args.layout, stream=stream,
                       deriv=args.deriv)
    print("bench: %dx%d %s %s, warmup %d" % (args.Nr, args.Nz, args.storage, args.layout,
                                             args.warmup), file=sys.stderr, flush=True)
    if args.tile >= 0:
        lat.set_tile(args.tile)
        tune = None
    elif args.layout == "ab2":
        tune = None  # the two-step launches have one tile; the single-step one is unused
    else:
        best, ms = lat.autotune(steps_per_trial=40)
        tune = {"%dx%d" % axlb.tile_shape(t): round(m * 1e3, 2) for t, m in enumerate(ms)}
        print("bench: autotune us/step per tile %s" % tune, file=sys.stderr, flush=True)
    _, tile_rz = lat.tile()
    tile = "%dx%d" % tile_rz if args.layout != "ab2" else "30x22 (two-step launch)"
    if args.single_launches:
        lat.set_graphs(False)
    lat.step(args.warmup)
    if not args.single_launches:
        lat.prepare_steps(args.steps)
    lat.sync()
    torch.cuda.synchronize()

    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    lat.step(args.steps)
    end.record(stream)
    end.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end)
    r = lat.residual()
    lat.close()
    ms_per_step = ms / args.steps
    if args.single_launches:
        launch = ("one two-step kernel launch per pair of steps" if args.layout == "ab2"
                  else "one kernel launch per step")
    else:
        bundles, tail = divmod(args.steps, 100)
        parts = (["%d replays of a 100-step graph" % bundles] if bundles else []) + \
            (["one %d-step graph" % tail] if tail >= 2 else []) + \
            (["one single launch"] if tail == 1 else [])
        launch = ", then ".join(parts) + " (captured before the timed region)"
    print("bench: timed %d steps in %.3f s (events %.4f ms/step)" % (args.steps, wall, ms_per_step),
          file=sys.stderr, flush=True)
    return {"ms_per_step": ms_per_step, "mlups": nodes * args.steps / (ms / 1e3) / 1e6,
            "launch": launch, "tile": tile, "autotune_us_per_step": tune,
            "finite": bool(r == r)}


def out_of_cache(Nr, Nz, steps, storage="f32"):
    """The same workload on a lattice whose state exceeds the 256 MB Infinity
    Cache (so HBM carries every byte), single-buffer (AA) and two steps per
    launch on two buffers (AB2); graph replays, HIP events."""
    import torch

    from paper_1806_10241_amd import axlb
    from paper_1806_10241_amd import inputs as I
    case = I.rotating_lid_cylinder(Nr=Nr, Nz=Nz, Re=1000.0, Ri=0.5, u_noise=1e-4)
    nodes = Nr * Nz
    out = {"Nr": Nr, "Nz": Nz, "storage": storage, "steps": steps}
    for layout in ("aa", "ab2"):
        stream = torch.cuda.Stream()
        lat = axlb.Lattice(case, storage=storage, layout=layout, stream=stream)
        if layout == "aa":
            lat.set_tile(axlb_default_tile())
        lat.step(20)
        lat.prepare_steps(steps)
        lat.sync()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        lat.step(steps)
        b.record(stream)
        b.synchronize()
        ms = a.elapsed_time(b) / steps
        state = step_working_set(Nr, Nz, storage, layout)
        lat.close()
        del lat
        torch.cuda.empty_cache()
        achieved = BYTES_PER_UPDATE[storage] * nodes / (ms / 1e3) / 1e9
        out[layout] = {"mlups": round(nodes / (ms / 1e3) / 1e6, 1), "ms_per_step": round(ms, 4),
                       "working_set_bytes": state, "achieved_gbs": round(achieved, 1),
                       "frac": round(achieved / PEAK_HBM_GBS, 4)}
    return out


def storage_variants(Nr, Nz, steps):
    """The headline workload with 16-bit population storage (binary16, and
    bfloat16 stored relative to its writer's linear equilibrium; FP32
    arithmetic), single-buffer (AA) and two steps per launch (AB2): graph
    replays timed with HIP events on the lattice's stream.  Their accuracy
    against the oracle is in `accuracy`."""
    import torch

    from paper_1806_10241_amd import axlb
    from paper_1806_10241_amd import inputs as I
    case = I.rotating_lid_cylinder(Nr=Nr, Nz=Nz, Re=1000.0, Ri=0.5, u_noise=1e-4)
    nodes = Nr * Nz
    out = {"Nr": Nr, "Nz": Nz, "steps": steps, "bytes_per_node_update": 76}
    for storage in ("f16", "bf16"):
        out[storage] = {}
        for layout in ("aa", "ab2"):
            stream = torch.cuda.Stream()
            lat = axlb.Lattice(case, storage=storage, layout=layout, stream=stream)
            if layout == "aa":
                lat.set_tile(axlb_default_tile())
            lat.step(20)
            lat.prepare_steps(steps)
            lat.sync()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            lat.step(steps)
            b.record(stream)
            b.synchronize()
            ms = a.elapsed_time(b) / steps
            lat.close()
            del lat
            torch.cuda.empty_cache()
            achieved = BYTES_PER_UPDATE[storage] * nodes / (ms / 1e3) / 1e9
            out[storage][layout] = {"mlups": round(nodes / (ms / 1e3) / 1e6, 1),
                                    "ms_per_step": round(ms, 4),
                                    "frac": round(achieved / PEAK_HBM_GBS, 4)}
    return out


def axlb_default_tile():
    """The 256 x 1 tile (the autotuner's usual choice at these widths)."""
    from paper_1806_10241_amd import axlb
    for t in range(axlb.NTILES):
        if axlb.tile_shape(t) == (256, 1):
            return t
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--layout", default="auto", choices=["auto", "aa", "ab", "ab2"],
                    help="streaming layout; auto: the faster of aa and ab2 on the workload")
    ap.add_argument("--deriv", default="lagged", choices=["lagged", "current"],
                    help="time level of the source-term derivatives (current needs --layout ab)")
    ap.add_argument("--Nr", type=int, default=1024)
    ap.add_argument("--Nz", type=int, default=2048)
    ap.add_argument("--cpu-steps", type=int, default=20,
                    help="steps of the oracle on one thread on the benchmark lattice")
    ap.add_argument("--cpu-steps-all", type=int, default=300,
                    help="steps of the oracle on every core on the benchmark lattice")
    ap.add_argument("--u-noise", type=float, default=1e-4,
                    help="seeded velocity noise of the initial state (0: at rest, so that "
                         "the swirl populations stay exactly zero away from the lid)")
    ap.add_argument("--tile", type=int, default=-1,
                    help="step-kernel tile shape; -1: autotune on the workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the 16-bit storage step rates")
    ap.add_argument("--ooc-Nr", type=int, default=2048,
                    help="width of the out-of-cache lattice (0: skip that measurement)")
    ap.add_argument("--ooc-Nz", type=int, default=4096)
    ap.add_argument("--ooc-steps", type=int, default=200)
    ap.add_argument("--batch-n", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=10000)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--small-n", type=int, default=1024,
                    help="members of the small-member batch")
    ap.add_argument("--serve-n", type=int, default=64)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-tol", type=float, default=1e-7)
    ap.add_argument("--serve-max-steps", type=int, default=100000)
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-max-nr-log2", type=float, default=10.0)
    ap.add_argument("--serve-max-nz-log2", type=float, default=11.0)
    ap.add_argument("--serve-order", default="smallest", choices=["smallest", "fifo"])
    ap.add_argument("--serve-window", type=int, default=4 << 20,
                    help="cap on resident fluid nodes in the pool (0: none)")
    ap.add_argument("--serve-below-n", type=int, default=24,
                    help="requests of the run at 0.7 x the measured saturation rate (0: skip)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-baseline", action="store_true",
                    help="also serve the trace one request at a time")
    ap.add_argument("--single-launches", action="store_true",
                    help="one kernel launch per step instead of graph replays")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB five times "
                         "(reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the time step runs on one GPU; a slab decomposition across GPUs "
              "is not implemented, so only --gpus 1 is measured", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n,
                          "launches": 5}), flush=True)
        return

    from paper_1806_10241_amd import axlb
    from paper_1806_10241_amd import inputs as I

    case = I.rotating_lid_cylinder(Nr=args.Nr, Nz=args.Nz, Re=1000.0, Ri=0.5,
                                   u_noise=args.u_noise)
    nodes = case["Nr"] * case["Nz"]
    trials = None
    if args.layout == "auto":
        if args.deriv != "lagged":
            args.layout = "ab"
        else:
            trials = layout_trial(case, args.storage)
            args.layout = min(trials, key=trials.get)
            print("bench: layout trials (ms/step) %s -> %s" % (trials, args.layout),
                  file=sys.stderr, flush=True)
    h = headline(args, case, torch.cuda.Stream())
    ms_per_step = h["ms_per_step"]
    achieved = BYTES_PER_UPDATE[args.storage] * nodes / (ms_per_step / 1e3) / 1e9
    working_set = step_working_set(args.Nr, args.Nz, args.storage, args.layout)

    out = {
        "metric": METRIC,
        "value": round(h["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "f32" else "f32-compute/%s-storage" % args.storage,
        "data": "synthetic",
        "config": {"workload": "rotating-lid cylinder with buoyancy, Re=1000, Ri=0.5, Pr=1",
                   "initial_noise": {"T": 1e-4, "u": args.u_noise},
                   "Nr": args.Nr, "Nz": args.Nz, "storage": args.storage,
                   "layout": args.layout, "derivatives": args.deriv,
                   "layout_trials_ms_per_step": ({k: round(v, 5) for k, v in trials.items()}
                                                 if trials else None),
                   "lag_storage": ("u_z, u_r, u_theta, T - T_ref as FP32: 16 B per node "
                                   "written and read per step" if args.storage == "f32" else
                                   "u_z, u_r, u_theta as binary16 (x 2^10), T - T_ref as FP32: "
                                   "10 B per node written and read per step"),
                   "launch": h["launch"],
                   "tile": h["tile"], "autotune_us_per_step": h["autotune_us_per_step"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": (measured_traffic(args.storage, args.Nr, args.Nz, args.layout)
                                 if args.layout in ("aa", "ab2") and args.deriv == "lagged"
                                 else None),
                     "kernel": ("k_step_two (two steps per launch; achieved and traffic are per "
                                "launch, algorithmic bytes 2 x %d B per node)"
                                % BYTES_PER_UPDATE[args.storage] if args.layout == "ab2" else
                                "k_step (one step per launch, %d B per node)"
                                % BYTES_PER_UPDATE[args.storage]),
                     "working_set_bytes": working_set,
                     "cache_resident": working_set < 256e6,
                     "note": "algorithmic bytes (%d B per node update) over the measured step "
                             "time; the state plus lagged fields %s the 256 MB Infinity Cache, "
                             "see out_of_cache for a lattice that does not fit"
                             % (BYTES_PER_UPDATE[args.storage],
                                "fit in" if working_set < 256e6 else "exceed")},
        "finite": h["finite"],
    }
    if args.ooc_Nr > 0:
        print("bench: out-of-cache %dx%d" % (args.ooc_Nr, args.ooc_Nz), file=sys.stderr,
              flush=True)
        out["out_of_cache"] = out_of_cache(args.ooc_Nr, args.ooc_Nz, args.ooc_steps, args.storage)
    if args.storage == "f32" and not args.no_variants:
        print("bench: 16-bit storage variants", file=sys.stderr, flush=True)
        out["storage_variants"] = storage_variants(args.Nr, args.Nz, 1000)
    gpu_accuracy = None
    if not args.no_accuracy:
        print("bench: accuracy runs", file=sys.stderr, flush=True)
        gpu_accuracy = accuracy_runs()
    if not args.no_batch:
        print("bench: batched, %d instances" % args.batch_n, file=sys.stderr, flush=True)
        out["batched"] = bench_batched(args.batch_n, args.batch_steps, 200, args.batch_steps)
        print("bench: batched, %d small instances" % args.small_n, file=sys.stderr, flush=True)
        out["batched_small"] = bench_small_members(args.small_n, 2000, 200)
    if not args.no_serve:
        print("bench: served, %d requests" % args.serve_n, file=sys.stderr, flush=True)
        served = bench_served(args.serve_n, args.serve_rate, args.serve_tol,
                              args.serve_max_steps, args.serve_budget_gib,
                              args.serve_max_nr_log2, args.serve_max_nz_log2,
                              args.serve_order, args.serve_window,
                              baseline=args.serve_baseline)
        served["note"] = ("queue-dominated: all %d requests arrive within %.2f s, far faster "
                          "than they can be served" % (args.serve_n, served["arrival_span_s"]))
        if args.serve_below_n > 0:
            rate = 0.7 * served["solves_per_s"]
            print("bench: served below saturation, %d requests at %.3f/s"
                  % (args.serve_below_n, rate), file=sys.stderr, flush=True)
            served["below_saturation"] = bench_served(
                args.serve_below_n, rate, args.serve_tol, args.serve_max_steps,
                args.serve_budget_gib, args.serve_max_nr_log2, args.serve_max_nz_log2,
                args.serve_order, args.serve_window, baseline=False)
        out["served"] = served
    if not args.no_cpu_baseline or gpu_accuracy is not None:
        print("bench: oracle on the host", file=sys.stderr, flush=True)
        base, acc = cpu_leg(case, args.cpu_steps, args.cpu_steps_all, gpu_accuracy)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = base
        if acc is not None:
            out["accuracy"] = acc
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
