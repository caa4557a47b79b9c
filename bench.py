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
TRACK_BYTES_MIXED = 64  # mixed form: direction in FP32


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
    # one core: the first events on a single thread
    n1 = max(1, min(n_events, 128))
    t1 = time.perf_counter()
    work(np.arange(n1))
    dt1 = time.perf_counter() - t1
    if errors:
        raise errors[0]
    return dict(value=n_events / dt, unit="primaries/s", cores=len(ts), kind="oracle", value_1core=n1 / dt1,
                sample=f"first {n_events} events of the workload, {len(ts)} threads, {dt:.1f} s wall; "
                       f"1 core: first {n1} events, {dt1:.1f} s")


def serving(E, I, args, precision):
    """Offload-server leg.  Requests: U{1..200} e-/e+/gamma tracks, total
    energy lognormal(ln 5 GeV, 1) clamped to [10 MeV, 2 TeV], Bz 3.8 T, from
    P producer threads (native threads of ems_server_drive, so the load is
    not limited by the interpreter; a pool of distinct requests per
    producer, reused with fresh event keys).  First the saturated closed
    loop (each producer keeps a window of requests outstanding; latency
    from submission), then Poisson arrivals at 80% of that request rate from
    a schedule fixed in advance, latency counted from each request's
    scheduled arrival, so a producer running late adds its delay to the
    latency instead of hiding it.  The first 10% of the completions of each
    leg are dropped from its statistics."""
    geo = I.calorimeter()
    cfg = I.RunConfig(seed=5, bz_tesla=3.8)
    P = args.serve_producers
    pools = []
    for p in range(P):
        rng = np.random.Generator(np.random.Philox(5 + p))
        pools.append([I.serving_request(rng) for _ in range(args.serve_pool)])
    c = E.make_config(cfg, args.serve_slots, track_capacity=args.serve_capacity,
                      steps_per_launch=args.serve_steps_per_launch, steps_per_visit=args.serve_steps_per_visit,
                      refill_below=args.refill_below, interact_min=args.interact_min, short_electron_MeV=args.short_mev, precision=precision,
                      photon_steps_per_visit=args.serve_photon_steps_per_visit,
                      photon_refill_below=args.serve_photon_refill_below)
    srv = E.Server(c, geo, admit_cap_bytes=args.serve_admit_gib << 30)
    n_each = max(1, args.serve_requests // P)
    total = n_each * P

    def req(p, i):
        return pools[p][i % len(pools[p])]

    def drop_warmup(target, stop):
        # clear the statistics once the first 10% of the requests are done
        while srv.stats()["completed"] < target and not stop.is_set():
            time.sleep(0.002)
        srv.reset_stats()

    def run_leg(producers, window):
        srv.reset_stats()
        stop = threading.Event()
        mon = threading.Thread(target=drop_warmup, args=(total // 10, stop))
        mon.start()
        t0 = time.monotonic_ns()
        try:
            lag, last = srv.drive(producers, window)
        finally:
            stop.set()
            mon.join()
        return lag, last, t0, time.monotonic_ns()

    prims = sum(len(req(p, i)) for p in range(P) for i in range(n_each))
    closed = [[(req(p, i), p * 1_000_000 + i, 0) for i in range(n_each)] for p in range(P)]
    _, _, t0, t1 = run_leg(closed, args.serve_window)
    wall = (t1 - t0) / 1e9
    sat = srv.stats()
    sat_rps = total / wall
    res = {"workload": "serving: requests of U{1..200} e-/e+/gamma tracks, lognormal(ln 5 GeV, 1) total, Bz 3.8 T",
           "precision": "fp64" if precision == E.FP64 else "mixed",
           "producers": f"{P} native threads (ems_server_drive)",
           "slots": args.serve_slots, "window": args.serve_window,
           "iterations_per_poll": args.serve_steps_per_launch, "steps_per_visit": args.serve_steps_per_visit,
           "interact_min": args.interact_min, "photon_steps_per_visit": args.serve_photon_steps_per_visit,
           "photon_refill_below": args.serve_photon_refill_below,
           "admit_cap_bytes": args.serve_admit_gib << 30,
           "saturated": {"requests": total, "primaries_per_s": prims / wall, "requests_per_s": sat_rps,
                         "p50_ms": sat["p50_ms"], "p99_ms": sat["p99_ms"],
                         "peak_admitted_bytes": sat["peak_admitted_bytes"]}}
    rate = 0.8 * sat_rps / P
    # each producer's arrivals are fixed in advance: a Poisson process of
    # rate/P from a seeded generator
    t_start = time.monotonic_ns() + 100_000_000
    sched = [t_start + np.cumsum(np.random.default_rng(100 + p).exponential(1e9 / rate, n_each)).astype(np.int64)
             for p in range(P)]
    opened = [[(req(p, i), 500_000 + p * 1_000_000 + i, int(sched[p][i])) for i in range(n_each)]
              for p in range(P)]
    lag, last, _, t_end = run_leg(opened, 1)
    po = srv.stats()
    srv.close()
    span = (max(int(a[-1]) for a in sched) - t_start) / 1e9  # the schedule's length
    sub = (last - t_start) / 1e9                              # submissions took
    wall = (t_end - t_start) / 1e9                            # to the last result
    # the schedule offers `total` requests over `span` (its producers run at
    # rate/P each, so its own length exceeds the mean by the spread of the
    # slowest producer's last arrival); achieved: the same requests over the
    # time their submission actually took
    offered = total / span
    achieved = total / max(sub, span)
    res["poisson_80pct"] = {"requests": total, "target_requests_per_s": rate * P,
                            "offered_requests_per_s": offered,
                            "achieved_requests_per_s": achieved,
                            "achieved_over_offered": achieved / offered,
                            "below_95pct_of_offered": achieved < 0.95 * offered,
                            "max_submission_lag_ms": lag,
                            "latency_from": "scheduled arrival",
                            "p50_ms": po["p50_ms"], "p99_ms": po["p99_ms"], "mean_ms": po["mean_ms"],
                            "max_ms": po["max_ms"], "primaries_per_s": prims / wall,
                            "dropped_warmup_requests": total // 10}
    return res


# the photon kernel's visit length and refill threshold per geometry kind
# (measured best): slab stacks favour long visits and an early refill, box
# geometries, whose photon steps wait on box records, the opposite
PHOTON_LAUNCH = {"slab": (32, 24), "boxes": (16, 40)}
# short-electron threshold (MeV) per workload and form where the launch of
# its own pays off (measured: the 10^5-event beam in the mixed form gains 3%;
# 10^4-event workloads and the FP64 form lose 1-7%, small batches 13%)
SHORT_MEV = {("cal_10GeV_e-_x100k", 1): 0.5}


def photon_launch(args, geo):
    kind = "boxes" if hasattr(geo, "world_lo") else "slab"
    pv, pr = PHOTON_LAUNCH[kind]
    return (pv if args.photon_steps_per_visit is None else args.photon_steps_per_visit,
            pr if args.photon_refill_below is None else args.photon_refill_below)


def transport_leg(E, I, workload, precision, capacity, args):
    """W warm-up steps, then K timed steps of one workload in one form."""
    import torch
    geo, cfg, prim = I.workload(workload)
    n = len(prim)
    visit = args.steps_per_visit if precision == E.FP64 else args.steps_per_visit_mixed
    pvisit, prefill = photon_launch(args, geo)
    short_mev = SHORT_MEV.get((workload, precision), 0.0) if args.short_mev is None else args.short_mev
    c = E.make_config(cfg, n, track_capacity=capacity, steps_per_launch=args.steps_per_launch,
                      launch_blocks=args.blocks, steps_per_visit=visit, refill_below=args.refill_below,
                      interact_min=args.interact_min, short_electron_MeV=short_mev, photon_steps_per_visit=pvisit,
                      photon_refill_below=prefill, precision=precision, flags=E.F_KERNEL_TIMING)
    eng = E.Transport(c, geo)
    # the job's inputs resident in HBM before the timed region; the tallies
    # stay there (the rate with host memory on both sides follows below)
    prim_dev = torch.from_numpy(np.ascontiguousarray(prim).view(np.uint8)).to("cuda")
    out_dev = torch.empty((c.max_events, eng.n_slabs), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    def one_step():
        eng.reset()
        eng.enqueue_device(prim_dev)
        eng.run()
        eng.edep_device(out_dev)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    kms = [0.0, 0.0, 0.0]
    launches = 0
    short_steps = 0
    steps = [0, 0, 0]
    made_by = [0, 0]
    visits = [0, 0, 0]
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step()
        s = eng.stats()
        kms = [a + b for a, b in zip(kms, s["kernel_ms"])]
        launches += s["launches"]
        short_steps += s["short_steps"]
        steps = [a + b for a, b in zip(steps, s["steps"])]
        made_by = [a + b for a, b in zip(made_by, s["made_by"])]
        visits = [a + b for a, b in zip(visits, s["visits"])]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    edep = out_dev.cpu().numpy()
    # the same steps with the primaries taken from host memory and the
    # tallies copied to host memory (both over PCIe): a few steps after one
    # untimed one
    host_steps = max(1, min(args.steps, 5))
    eng.reset()
    eng.enqueue(prim)
    eng.run()
    eng.edep()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(host_steps):
        eng.reset()
        eng.enqueue(prim)
        eng.run()
        eng.edep()
    torch.cuda.synchronize()
    value_host_io = n * host_steps / (time.perf_counter() - t1)
    eng.close()
    tb = TRACK_BYTES if precision == E.FP64 else TRACK_BYTES_MIXED
    # algorithmic bytes of the method: every track-step reads the track's
    # record and writes the survivor (2 records), every secondary adds one
    # record.  Multi-step visits move fewer: one read and at most one write
    # per visit ("record_bytes_per_launch").
    # The short-electron launch takes one step of each short e- (its share
    # of the e- steps is counted apart: short_steps).
    names = ["k_visit<photons>", "k_visit<e-/e+>", "k_short<e->"]
    alg = [tb * (2 * steps[0] + made_by[0]), tb * (2 * (steps[1] + steps[2] - short_steps) + made_by[1]),
           tb * 2 * short_steps]
    rec = [tb * (2 * visits[0] + made_by[0]), tb * (2 * (visits[1] + visits[2] - short_steps) + made_by[1]),
           tb * 2 * short_steps]
    kern = {}
    for i in range(3 if kms[2] > 0 else 2):
        per_launch = alg[i] / max(launches, 1)
        avg_s = kms[i] / 1e3 / max(launches, 1)
        ach = per_launch / avg_s / 1e9 if avg_s > 0 else 0.0
        kern[names[i]] = {"achieved": ach, "frac": ach / HBM_PEAK_GBS, "bytes_per_launch": per_launch,
                          "record_bytes_per_launch": rec[i] / max(launches, 1),
                          "avg_launch_us": avg_s * 1e6, "launches": launches, "share_of_kernel_time":
                          kms[i] / max(sum(kms), 1e-12)}
    dom = names[1] if kms[1] >= kms[0] else names[0]
    d = kern[dom]
    key = counter_key(workload, precision == E.FP64, visit, args.refill_below, args.interact_min,
                      pvisit, prefill, c.short_electron_MeV)
    roof = {"bound": "hbm", "achieved": d["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": d["frac"], "traffic": traffic_for(dom, key),
            "kernel": dom, "bytes_per_launch": d["bytes_per_launch"], "avg_launch_us": d["avg_launch_us"],
            "launches": launches, "kernels": kern}
    # the whole step against the same peak: the method's bytes of both
    # kernels over the wall time of a step (enqueue to tallies in device memory)
    run_b = sum(alg) / args.steps
    roof["run"] = {"bytes_per_step": run_b, "GB_per_s": run_b / (dt / args.steps) / 1e9,
                   "frac": run_b / (dt / args.steps) / 1e9 / HBM_PEAK_GBS}
    # the same steps replayed from captured graphs (no per-kernel events)
    value_graph = None
    if args.graph_check:
        cg = E.make_config(cfg, n, track_capacity=capacity, steps_per_launch=args.steps_per_launch,
                           launch_blocks=args.blocks, steps_per_visit=visit, refill_below=args.refill_below,
                           interact_min=args.interact_min, short_electron_MeV=short_mev, photon_steps_per_visit=pvisit,
                           photon_refill_below=prefill, precision=precision)
        eng = E.Transport(cg, geo)
        one_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            one_step()
        torch.cuda.synchronize()
        value_graph = n * args.steps / (time.perf_counter() - t0)
        assert eng.stats()["graph_launches"] > 0
        eng.close()
    return dict(geo=geo, cfg=cfg, prim=prim, key=key, photon_launch=[pvisit, prefill], short_mev=c.short_electron_MeV,
                value=n * args.steps / dt, ms_per_step=dt / args.steps * 1e3,
                value_graph=value_graph, value_host_io=value_host_io,
                track_steps=sum(steps) // args.steps, visits=sum(visits) // args.steps, roofline=roof, edep=edep,
                deferred=s["deferred"], peak_live=s["peak_live"], iterations=s["iterations"])


def copy_bandwidth(n_bytes=1 << 31, reps=5):
    """Achievable HBM bandwidth of a device-to-device copy (read + write
    bytes over the copy time), GB/s."""
    import torch
    a = torch.empty(n_bytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * n_bytes / (ms / 1e3) / 1e9


def atomic_probe(E, n_cells, n_ops=1 << 28, reps=3):
    """Ceiling of the tallies' FP64 atomic rate: the library's probe (the
    deposit instruction, uniform over as many cells as the run's tallies),
    best of a few repetitions, in G atomics/s."""
    import torch
    cells = torch.zeros(n_cells, dtype=torch.float64, device="cuda")
    best = min(E.probe_atomics(cells, n_ops) for _ in range(reps))
    assert float(cells.sum().item()) == float(n_ops)  # every add landed
    return n_ops / (best / 1e3) / 1e9


def atomics_report(leg, workload, peak):
    """Atomic rate of each visit kernel against the probe: atomic requests
    per launch counted by rocprofv3 (TCC_ATOMIC_sum, committed in
    profiles/atomics.txt with the digest of the kernels measured) over the
    kernel's live average launch time; null while the kernels differ from
    the measured ones."""
    kern = leg["roofline"]["kernels"]
    out = {"unit": "G atomics/s", "probe_peak": peak,
           "probe": "2^28 FP64 atomic adds, uniform over the run's [events][columns] tally cells"}
    for k, v in kern.items():
        n = counted_for(k, workload, "atomics.txt")
        ach = n / (v["avg_launch_us"] * 1e-6) / 1e9 if n is not None and v["avg_launch_us"] > 0 else None
        out[k] = {"atomic_requests_per_launch": n, "achieved": ach,
                  "frac": ach / peak if ach is not None and peak else None}
    return out


def kernel_source_digest(csrc=None):
    """SHA-256 over the sources the visit kernels are built from
    (ems_kernels.hip, ems_kernels_slab_f32.hip and the headers they include,
    directly or through other headers) with their comments and blank space
    removed, and over the compiler flags of the FP32 slab-stack kernels:
    counter figures are valid only for the code they were measured on, and
    neither a comment nor a host-only file changes that code."""
    import hashlib
    import re
    from paper_2209_15445_amd import build as ems_build
    h = hashlib.sha256()
    csrc = csrc or os.path.join(ROOT, "paper_2209_15445_amd", "csrc")
    h.update(" ".join(ems_build.SLAB_F32_FLAGS).encode() + b"\0")
    used, todo = set(), ["ems_kernels.hip", ems_build.SLAB_F32_SOURCE]
    while todo:
        name = todo.pop()
        if name in used or not os.path.exists(os.path.join(csrc, name)):
            continue
        used.add(name)
        src = open(os.path.join(csrc, name), encoding="utf-8").read()
        todo += re.findall(r'^\s*#include\s+"([^"/]+)"', src, re.M)
    for name in sorted(used):
        text = open(os.path.join(csrc, name), encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(" ".join(line.split()) for line in text.splitlines() if line.strip())
        h.update(name.encode() + b"\0" + code.encode() + b"\0")
    return h.hexdigest()


def counter_key(workload, fp64, visit, refill, interact_min, photon_visit, photon_refill, short_mev=0.0):
    """Rows of the counter tables are keyed by workload, form and the launch
    parameters that shape a launch's batches (and the short-electron
    threshold, when there is one)."""
    return (f"{workload}/{'fp64' if fp64 else 'mixed'}/v{visit}r{refill}i{interact_min}"
            f"pv{photon_visit}pr{photon_refill}" + (f"s{short_mev:g}" if short_mev > 0 else ""))


def counted_for(kernel, workload, name="traffic.txt"):
    """A counter-measured per-launch figure of a kernel on a workload from a
    committed profile table (profiles/traffic.txt: HBM bytes from
    FETCH_SIZE + WRITE_SIZE scaled by a plain-copy calibration;
    profiles/atomics.txt: TCC atomic requests), or None when the kernels
    changed since it was measured."""
    if workload is None:
        return None
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        parts = line.split()
        if len(parts) == 4 and not line.startswith("#"):
            rec[(parts[0], parts[1])] = (parts[2], float(parts[3]))
    hit = rec.get((kernel, workload))
    if hit is None or hit[0] != kernel_source_digest():
        return None
    return hit[1]


def traffic_for(kernel, workload):
    return counted_for(kernel, workload, "traffic.txt")


def with_traffic_rate(roof, copy_gbs):
    """Counter-measured HBM bytes over the live launch time, against the
    peak and against an achievable copy."""
    roof["copy_GB_per_s"] = copy_gbs
    if roof["traffic"] is not None:
        tg = roof["traffic"] / (roof["avg_launch_us"] * 1e-6) / 1e9
        roof["traffic_GB_per_s"] = tg
        roof["traffic_frac"] = tg / HBM_PEAK_GBS
        roof["traffic_frac_of_copy"] = tg / copy_gbs


def layer_error(leg, n_events):
    """Per-layer mean deposit of the mixed form against the FP64 oracle on the
    first n_events events of the same workload (same event keys, so the pair
    is correlated): relative error per layer, its RMS and maximum over the
    layers holding >= 0.1% of the peak, with the statistical error."""
    import oracle
    geo, cfg, prim = leg["geo"], leg["cfg"], leg["prim"]
    k = min(n_events, len(prim))
    idx = np.arange(k)
    threads = cpu_threads()[0]
    o = oracle.Oracle(geo, cfg)
    parts = np.array_split(idx, threads)
    res = [None] * len(parts)

    def work(j):
        p = prim[parts[j]].copy()
        p["event"] = np.arange(len(parts[j]))
        res[j] = o.run(p, n_events=len(parts[j]), event_keys=parts[j].astype(np.uint32))["edep"]

    ts = [threading.Thread(target=work, args=(j,)) for j in range(len(parts)) if len(parts[j])]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    ref = np.concatenate([r for r in res if r is not None])
    nl = geo.n_slabs // 2
    lo = ref.reshape(k, nl, 2).sum(axis=2)
    lm = leg["edep"][:k].reshape(k, nl, 2).sum(axis=2)
    mo, mm = lo.mean(axis=0), lm.mean(axis=0)
    live = mo > 1e-3 * mo.max()
    rel = (mm - mo)[live] / mo[live]
    stat = np.sqrt(lo.var(axis=0) / k)[live] / mo[live]
    return {"events": int(k), "layers": int(live.sum()), "rms_rel": float(np.sqrt(np.mean(rel ** 2))),
            "max_abs_rel": float(np.abs(rel).max()), "mean_stat_rel": float(stat.mean()),
            "total_rel": float((lm.sum() - lo.sum()) / lo.sum())}


def geometry_label(geo):
    """what a workload's geometry is, with its sizes"""
    if hasattr(geo, "world_lo"):
        w = np.subtract(geo.world_hi, geo.world_lo)
        return f"{geo.n_boxes} boxes in a {w[0]:g} x {w[1]:g} x {w[2]:g} mm world (BVH)"
    z = np.asarray(geo.z_mm)
    return f"{len(z) - 1} slabs over {z[-1] - z[0]:g} mm, {2 * geo.half_xy_mm:g} mm square"


def leg_summary(leg):
    """Throughput and the roofline of the dominant kernel of one leg (the
    same quantities as the headline line's, per workload and form)."""
    r = leg["roofline"]
    return {"value": leg["value"], "unit": "primaries/s", "ms_per_step": leg["ms_per_step"],
            "value_host_io": leg["value_host_io"], "geometry": geometry_label(leg["geo"]),
            "photon_launch": leg["photon_launch"], "track_steps_per_step": leg["track_steps"],
            "iterations": leg["iterations"],
            "roofline": {"bound": r["bound"], "kernel": r["kernel"], "achieved": r["achieved"], "peak": r["peak"],
                         "unit": r["unit"], "frac": r["frac"], "bytes_per_launch": r["bytes_per_launch"],
                         "avg_launch_us": r["avg_launch_us"], "run_frac": r["run"]["frac"]},
            "kernel_avg_launch_us": {k: v["avg_launch_us"] for k, v in r["kernels"].items()}}


def cpu_threads():
    """Worker threads for the oracle: the CPUs this process may run on,
    capped by the job's CPU share where the environment states one
    (OMP_NUM_THREADS); also returns the machine's and the affinity's CPU
    counts for the record."""
    machine = os.cpu_count() or 1
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = machine
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    threads = min(affinity, share) if share > 0 else affinity
    return max(1, threads), machine, affinity, share or None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cal_10GeV_e-_x10k")
    ap.add_argument("--capacity", type=int, default=1 << 25)
    ap.add_argument("--blocks", type=int, default=0)
    ap.add_argument("--steps-per-launch", type=int, default=16)
    ap.add_argument("--steps-per-visit", type=int, default=16, help="FP64 legs")
    ap.add_argument("--steps-per-visit-mixed", type=int, default=32, help="mixed legs")
    ap.add_argument("--refill-below", type=int, default=32)
    ap.add_argument("--short-mev", type=float, default=None,
                    help="e- secondaries below this energy take their first step in the short-electron launch "
                         "(0: off; default: SHORT_MEV per workload and form)")
    ap.add_argument("--interact-min", type=int, default=24,
                    help="e-/e+ batches sample interactions once this many lanes wait for one")
    ap.add_argument("--photon-steps-per-visit", type=int, default=None,
                    help="photon kernel, both forms (default: per geometry kind, PHOTON_LAUNCH)")
    ap.add_argument("--photon-refill-below", type=int, default=None,
                    help="photon kernel, both forms (default: per geometry kind, PHOTON_LAUNCH)")
    ap.add_argument("--cpu-events", type=int, default=2048, help="events of the timed oracle sample")
    ap.add_argument("--error-events", type=int, default=10000,
                    help="events of the mixed form compared with the FP64 oracle per layer")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--graph-check", type=int, default=1,
                    help="also time the same steps replayed from captured graphs (no per-kernel events)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--mixed-workload", default="cal_10GeV_e-_x100k")
    ap.add_argument("--mixed-capacity", type=int, default=1 << 28)
    ap.add_argument("--extra-capacity", type=int, default=1 << 26)
    ap.add_argument("--small-workload", default="cal_1GeV_e-_x32",
                    help="also time this small batch in both forms ('' to skip)")
    ap.add_argument("--extra-workload",
                    default="cal_mixed_1-100GeV_bz3.8_x10k,calPbWO4_10GeV_e-_x10k,cal_10GeV_e-_x10k_msc_fluct,"
                            "towers_10GeV_e-_x10k",
                    help="also time these workloads (comma-separated) in both forms ('' to skip)")
    ap.add_argument("--serve-slots", type=int, default=16384)
    ap.add_argument("--serve-producers", type=int, default=64)
    ap.add_argument("--serve-window", type=int, default=64, help="outstanding requests per producer (closed loop)")
    ap.add_argument("--serve-pool", type=int, default=64, help="distinct requests per producer (reused, new keys)")
    ap.add_argument("--serve-requests", type=int, default=40960)
    ap.add_argument("--serve-capacity", type=int, default=1 << 24)
    ap.add_argument("--serve-admit-gib", type=int, default=8)
    ap.add_argument("--serve-steps-per-launch", type=int, default=1, help="iterations between host polls")
    ap.add_argument("--serve-steps-per-visit", type=int, default=12)
    ap.add_argument("--serve-photon-steps-per-visit", type=int, default=32)
    ap.add_argument("--serve-photon-refill-below", type=int, default=24)
    ap.add_argument("--no-fp64-serve", action="store_true")
    ap.add_argument("--atomic-probe", type=int, default=0,
                    help="only run the library's FP64 atomic probe with this many adds (calibrates atomic counters)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run one device-to-device copy of this many bytes (calibrates HBM counters)")
    args = ap.parse_args()
    if args.atomic_probe:
        import torch

        import paper_2209_15445_amd as E
        cells = torch.zeros(10**6, dtype=torch.float64, device="cuda")
        ms = E.probe_atomics(cells, args.atomic_probe)
        print(json.dumps({"atomic_probe_ops": args.atomic_probe, "ms": ms}), flush=True)
        return
    if args.copy_probe:
        import torch
        # the source is never written on the device, so none of it sits in a
        # cache when the copy reads it; the copy is the probe's only kernel
        a = torch.empty(args.copy_probe, dtype=torch.uint8, device="cuda")
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

    fp = transport_leg(E, I, args.workload, E.FP64, args.capacity, args)
    geo, cfg, prim = fp["geo"], fp["cfg"], fp["prim"]
    n = len(prim)
    out = {
        "metric": METRIC,
        "value": fp["value"],
        "unit": "primaries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "events": n, "primary": "e-", "energy_MeV": float(prim["ekin"][0]),
                   "geometry": geometry_label(geo), "bz_tesla": cfg.bz_tesla,
                   "precision": "fp64", "track_steps_per_step": fp["track_steps"],
                   "visits_per_step": fp["visits"], "iterations": fp["iterations"],
                   "peak_live": fp["peak_live"], "deferred_steps": fp["deferred"], "capacity": args.capacity,
                   "steps_per_visit": args.steps_per_visit, "refill_below": args.refill_below,
                   "interact_min": args.interact_min, "photon_steps_per_visit": fp["photon_launch"][0],
                   "photon_refill_below": fp["photon_launch"][1], "short_electron_MeV": fp["short_mev"]},
        "roofline": fp["roofline"],
        "value_graph_replay": fp["value_graph"],
        "inputs": "primaries resident in device memory, deposits left there (ems_enqueue_device, "
                  "ems_read_edep_device); value_host_io: primaries from and deposits to host memory",
        "value_host_io": fp["value_host_io"],
    }
    out["atomics"] = atomics_report(fp, fp["key"], atomic_probe(E, n * geo.n_cols))
    copy_gbs = copy_bandwidth()
    with_traffic_rate(out["roofline"], copy_gbs)
    if not args.no_mixed:
        mx = transport_leg(E, I, args.mixed_workload, E.MIXED, args.mixed_capacity, args)
        out["mixed"] = {"workload": args.mixed_workload, "events": len(mx["prim"]), "value": mx["value"],
                        "unit": "primaries/s", "ms_per_step": mx["ms_per_step"], "dtype": "f32 physics / f64 state",
                        "value_graph_replay": mx["value_graph"], "value_host_io": mx["value_host_io"],
                        "track_steps_per_step": mx["track_steps"], "iterations": mx["iterations"],
                        "peak_live": mx["peak_live"], "deferred_steps": mx["deferred"],
                        "capacity": args.mixed_capacity, "steps_per_visit": args.steps_per_visit_mixed,
                        "short_electron_MeV": mx["short_mev"],
                        "roofline": mx["roofline"],
                        "atomics": atomics_report(mx, mx["key"], atomic_probe(E, len(mx["prim"]) * mx["geo"].n_cols))}
        with_traffic_rate(out["mixed"]["roofline"], copy_gbs)
        if not args.no_cpu:
            out["mixed"]["per_layer_error_vs_fp64_oracle"] = layer_error(mx, args.error_events)
    if args.small_workload:
        # the small-batch regime (32 showers: too few tracks to fill the
        # device for most of the run), both forms
        out["small_batch"] = {}
        for prec, tag in ((E.FP64, "fp64"), (E.MIXED, "mixed")):
            leg = transport_leg(E, I, args.small_workload, prec, 1 << 22, args)
            out["small_batch"][f"{args.small_workload}/{tag}"] = leg_summary(leg)
    if args.extra_workload:
        out["other_workloads"] = {}
    for wl in filter(None, args.extra_workload.split(",")):
        for prec, tag in ((E.FP64, "fp64"), (E.MIXED, "mixed")):
            leg = transport_leg(E, I, wl, prec, args.extra_capacity, args)
            out["other_workloads"][f"{wl}/{tag}"] = leg_summary(leg)
    if not args.no_serve and not args.no_fp64_serve:
        out["serving"] = serving(E, I, args, E.FP64)
    if not args.no_serve:
        if not args.no_mixed:
            out["serving_mixed"] = serving(E, I, args, E.MIXED)
    if not args.no_cpu:
        threads, machine, affinity, share = cpu_threads()
        out["cpu_baseline"] = cpu_baseline(geo, cfg, prim, min(args.cpu_events, n), threads)
        out["cpu_baseline"].update(machine_cpus=machine, affinity_cpus=affinity, cpu_share=share)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
