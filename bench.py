"""Throughput of the axisymmetric cascaded LB time step on one MI355X.

Workload: the 1024 x 2048 rotating-lid cylinder with buoyancy (Re = 1000,
Ri = 0.5, Pr = 1), FP32 arithmetic and storage, single-buffer (AA) layout,
100-step HIP graph bundles.  A step is one update of every node's 19
populations (D2Q9 + 2 x D2Q5).  Prints one JSON line.

The dominant (only) kernel per step is the fused step kernel; its
algorithmic traffic is 152 B per node update (19 populations x 4 B, read and
written once), so achieved GB/s = 152 * nodes / average step time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS (D2Q9+2×D2Q5 node updates/s), % HBM roofline; batched solves/s, p99 latency"
PEAK_HBM_GBS = 8000.0
BYTES_PER_UPDATE = {"f32": 152, "f16": 76, "bf16": 76}


def cpu_baseline(case, steps: int):
    """The FP64 oracle, single-threaded, on the first `steps` steps of the
    same workload; MLUPS over the stepping only."""
    import oracle
    L = oracle.Lattice(case, deriv_mode=oracle.DERIV_PREVIOUS, fields=case["fields"]())
    t0 = time.perf_counter()
    L.step(steps)
    dt = time.perf_counter() - t0
    mlups = case["Nr"] * case["Nz"] * steps / dt / 1e6
    return {"value": round(mlups, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": "%d steps of the %dx%d workload, FP64, one thread (%.1f s)"
                      % (steps, case["Nr"], case["Nz"], dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--layout", default="aa", choices=["aa", "ab"])
    ap.add_argument("--Nr", type=int, default=1024)
    ap.add_argument("--Nz", type=int, default=2048)
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--single-launches", action="store_true",
                    help="one kernel launch per step instead of 100-step graphs")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB five times "
                         "(reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; the path is single-GPU "
              "(multi-GPU sharding is a design note only)", file=sys.stderr)
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

    case = I.rotating_lid_cylinder(Nr=args.Nr, Nz=args.Nz, Re=1000.0, Ri=0.5)
    nodes = case["Nr"] * case["Nz"]
    stream = torch.cuda.Stream()
    lat = axlb.Lattice(case, storage=args.storage, layout=args.layout, stream=stream)
    print("bench: %dx%d %s %s, warmup %d" % (args.Nr, args.Nz, args.storage, args.layout,
                                             args.warmup), file=sys.stderr, flush=True)
    lat.step(args.warmup)
    lat.sync()
    torch.cuda.synchronize()

    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    if args.single_launches:
        for _ in range(args.steps):
            lat.step(1)
    else:
        lat.step(args.steps)
    end.record(stream)
    end.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end)
    ms_per_step = ms / args.steps
    mlups = nodes * args.steps / (ms / 1e3) / 1e6
    achieved = BYTES_PER_UPDATE[args.storage] * nodes / (ms_per_step / 1e3) / 1e9
    r = lat.residual()
    print("bench: timed %d steps in %.3f s (events %.3f ms/step)" % (args.steps, wall, ms_per_step),
          file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
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
                   "Nr": args.Nr, "Nz": args.Nz, "storage": args.storage,
                   "layout": args.layout,
                   "graph_bundle": 0 if args.single_launches else 100},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": None},
        "finite": bool(r == r),
    }
    lat.close()
    if not args.no_cpu_baseline:
        print("bench: oracle CPU baseline, %d steps" % args.cpu_steps, file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
