"""Throughput of the MI355X EM-shower transport loop.

One step = one pass of the whole hot path over one batch: reset tallies,
enqueue all primaries, step the population to extinction, read the per-slab
deposits back to the host.  Workload: 10^4 events of one 10 GeV electron
(Gaussian 1 mrad slope smear) in the 50-layer Pb/lAr calorimeter, FP64.

Prints one JSON line with the throughput (primaries/s), the roofline of the
dominant kernel (the step kernel: algorithmic track-record bytes per launch
over its measured average launch duration, HBM bound) and the oracle timed on
the host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "primaries/sec (10 GeV e-, 50-layer Pb/lAr) FP64 vs mixed; offload p99 ms"
HBM_PEAK_GBS = 8000.0
TRACK_BYTES = 76  # FP64 SoA record: pos 24, dir 24, E 8, id 8, event 4, step 4, slab 4


def cpu_baseline(geo, cfg, prim, n_events, threads):
    """The oracle as it stands, P worker threads over disjoint events."""
    import oracle
    o = oracle.Oracle(geo, cfg)
    sample = prim[:n_events]
    chunks = np.array_split(np.arange(n_events), threads)
    errors = []

    def work(idx):
        try:
            p = sample[idx].copy()
            p["event"] = np.arange(len(idx))
            o.run(p, n_events=len(idx), event_keys=idx.astype(np.uint32))
        except Exception as exc:  # pragma: no cover
            errors.append(exc)

    t0 = time.perf_counter()
    ts = [threading.Thread(target=work, args=(c,)) for c in chunks if len(c)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    dt = time.perf_counter() - t0
    if errors:
        raise errors[0]
    return dict(value=n_events / dt, unit="primaries/s", cores=len(ts), kind="oracle",
                sample=f"first {n_events} events of the workload, {len(ts)} threads, {dt:.1f} s wall")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cal_10GeV_e-_x10k")
    ap.add_argument("--capacity", type=int, default=8 << 20)
    ap.add_argument("--blocks", type=int, default=0)
    ap.add_argument("--steps-per-launch", type=int, default=16)
    ap.add_argument("--steps-per-visit", type=int, default=16)
    ap.add_argument("--refill-below", type=int, default=8)
    ap.add_argument("--cpu-events", type=int, default=640)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run one device-to-device copy of this many bytes (calibrates HBM counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); events shard across GPUs with no "
              "exchange during transport, so the one-GPU figure is the per-GPU throughput", file=sys.stderr)
        sys.exit(2)

    import torch

    import ems_inputs as I
    import paper_2209_15445_amd as E

    geo, cfg, prim = I.workload(args.workload)
    n = len(prim)
    c = E.make_config(cfg, n, track_capacity=args.capacity, steps_per_launch=args.steps_per_launch,
                      launch_blocks=args.blocks, steps_per_visit=args.steps_per_visit,
                      refill_below=args.refill_below)
    eng = E.Transport(c, geo)

    def one_step():
        eng.reset()
        eng.enqueue(prim)
        eng.run()
        return eng.edep()

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    kernel_ms = 0.0
    launches = 0
    steps = [0, 0, 0]
    created = [0, 0, 0]
    visits = [0, 0, 0]
    t0 = time.perf_counter()
    for _ in range(args.steps):
        edep = one_step()
        s = eng.stats()
        kernel_ms += s["step_kernel_ms"]
        launches += s["launches"]
        steps = [a + b for a, b in zip(steps, s["steps"])]
        created = [a + b for a, b in zip(created, s["created"])]
        visits = [a + b for a, b in zip(visits, s["visits"])]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    eng.close()

    value = n * args.steps / dt
    # each visit reads one track record and writes at most one (survivor or
    # carried track); each secondary record is written once
    alg_bytes = TRACK_BYTES * (2 * sum(visits) + sum(created))
    per_launch = alg_bytes / max(launches, 1)
    avg_launch_s = kernel_ms / 1e3 / max(launches, 1)
    achieved = per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "primaries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "events": n, "primary": "e-", "energy_MeV": float(prim["ekin"][0]),
                   "geometry": "50 x (2.3 mm Pb + 5.7 mm lAr), 40x40 cm", "bz_tesla": cfg.bz_tesla,
                   "precision": "fp64", "track_steps_per_step": sum(steps) // args.steps,
                   "visits_per_step": sum(visits) // args.steps,
                   "steps_per_visit": args.steps_per_visit, "refill_below": args.refill_below},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_visit (photon + e-/e+ launch per iteration)", "bytes_per_launch": per_launch,
                     "avg_launch_us": avg_launch_s * 1e6,
                     "launches": launches},
    }
    if not args.no_cpu:
        threads = max(1, min(16, os.cpu_count() or 1))
        out["cpu_baseline"] = cpu_baseline(geo, cfg, prim, min(args.cpu_events, n), threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
