"""GPU tests of the continuous-batching offload server: a request's result is
the same alone and mixed with concurrent requests from many producer threads,
equals the oracle's for the same tracks and event key, conserves energy, and
the server drains (Flush) and respects its admission budget."""
import threading

import numpy as np
import pytest

import ems_inputs as I
from parity_util import ME

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_15445_amd as E
    E.lib()
    return E


def make_server(E, slots=64, cap_bytes=1 << 30, capacity=1 << 20, bz=3.8):
    geo = I.calorimeter()
    cfg = I.RunConfig(seed=5, bz_tesla=bz)
    c = E.make_config(cfg, slots, track_capacity=capacity, steps_per_launch=4)
    return geo, cfg, E.Server(c, geo, cap_bytes)


def residual(edep, led, tracks):
    out = edep.sum() + led["escaped"].sum() + led["killed"] + 2 * ME * (int(led["n_pair"]) - int(led["n_annih"]))
    return abs(out - tracks["ekin"].sum()) / tracks["ekin"].sum()


def test_same_result_alone_and_in_the_mix(E, oracle_mod):
    print("alone vs mix", flush=True)
    rng = np.random.Generator(np.random.Philox(55))
    probe = I.serving_request(rng, e_median_MeV=2000.0, max_tracks=30)
    key = 777
    geo, cfg, srv = make_server(E)
    alone_edep, alone_led = srv.wait(srv.submit(probe, key), timeout_s=120)
    srv.close()

    geo, cfg, srv = make_server(E, slots=24)
    results = {}
    reqs = {}

    def producer(p):
        r = np.random.Generator(np.random.Philox(1000 + p))
        mine = []
        for i in range(12):
            tr = I.serving_request(r, e_median_MeV=1000.0, max_tracks=40)
            k = p * 1000 + i
            mine.append((srv.submit(tr, k), tr, k))
            if p == 3 and i == 5:
                mine.append((srv.submit(probe, key), probe, key))
        for t, tr, k in mine:
            results[t] = srv.wait(t, timeout_s=300)
            reqs[t] = (tr, k)

    ths = [threading.Thread(target=producer, args=(p,)) for p in range(8)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    st = srv.stats()
    srv.close()
    assert len(results) == 8 * 12 + 1 and st["completed"] == len(results)
    probe_t = [t for t, (tr, k) in reqs.items() if k == key][0]
    mix_edep, mix_led = results[probe_t]
    assert np.allclose(mix_edep, alone_edep, rtol=1e-12, atol=1e-12)
    for f in ("n_pair", "n_annih"):
        assert mix_led[f] == alone_led[f]
    for t, (edep, led) in results.items():
        assert residual(edep, led, reqs[t][0]) < 1e-9
    # the oracle, given the same tracks and event key, gives the same deposits
    p = probe.copy()
    p["event"] = 0
    r = oracle_mod.Oracle(geo, cfg).run(p, n_events=1, event_keys=[key])
    assert np.allclose(alone_edep, r["edep"][0], rtol=1e-8, atol=1e-8)


def test_flush_admission_and_errors(E):
    print("flush / admission", flush=True)
    cap = 40 << 20
    geo, cfg, srv = make_server(E, slots=16, cap_bytes=cap)
    rng = np.random.Generator(np.random.Philox(9))
    tickets = [srv.submit(I.serving_request(rng, e_median_MeV=3000.0, max_tracks=50), k) for k in range(60)]
    srv.flush()
    assert all(srv.poll(t) for t in tickets)
    st = srv.stats()
    assert st["completed"] == 60 and st["in_flight"] == 0 and st["queued"] == 0
    assert st["peak_admitted_bytes"] <= cap
    bad = I.serving_request(rng)
    bad["ekin"][0] = -1.0
    with pytest.raises(E.EmsError) as ei:
        srv.submit(bad, 1)
    assert ei.value.code == E.E_INVALID
    with pytest.raises(E.EmsError):
        srv.wait(123456789, timeout_s=0.1)
    srv.close()


def test_latency_counts_from_the_given_arrival(E):
    # a request handed over with an arrival 200 ms in the past reports at
    # least those 200 ms; an arrival in the future counts from the call
    import time
    print("latency from arrival", flush=True)
    geo, cfg, srv = make_server(E, slots=8)
    rng = np.random.Generator(np.random.Philox(21))
    tr = I.serving_request(rng, e_median_MeV=500.0, max_tracks=10)
    srv.reset_stats()
    srv.wait(srv.submit(tr, 1, arrival_ns=time.monotonic_ns() - 200_000_000), timeout_s=60)
    st = srv.stats()
    assert st["completed"] == 1 and st["max_ms"] >= 200.0, st
    srv.reset_stats()
    srv.wait(srv.submit(tr, 2, arrival_ns=time.monotonic_ns() + 10_000_000_000), timeout_s=60)
    st = srv.stats()
    assert st["completed"] == 1 and 0.0 <= st["max_ms"] < 5000.0, st
    srv.close()


def test_native_producers_drive_the_server(E):
    # ems_server_drive: closed loop (window 3) and scheduled arrivals from 6
    # native threads; every request completes, lateness is reported and the
    # latency of scheduled requests counts from their arrival
    import time
    print("native producers", flush=True)
    geo, cfg, srv = make_server(E, slots=16)
    rng = np.random.Generator(np.random.Philox(31))
    reqs = [[(I.serving_request(rng, e_median_MeV=300.0, max_tracks=8), p * 100 + i, 0) for i in range(10)]
            for p in range(6)]
    srv.reset_stats()
    lag, last = srv.drive(reqs, window=3)
    st = srv.stats()
    assert st["completed"] == 60 and st["in_flight"] == 0 and lag == 0.0 and last > 0
    t0 = time.monotonic_ns() + 20_000_000
    timed = [[(tr, 5000 + k, t0 + 2_000_000 * i) for i, (tr, k, _) in enumerate(r)] for r in reqs]
    srv.reset_stats()
    lag, last = srv.drive(timed, window=1)
    st = srv.stats()
    assert st["completed"] == 60 and last >= t0 + 18_000_000 and lag >= 0.0
    # a request scheduled in the past reports at least its age
    srv.reset_stats()
    srv.drive([[(reqs[0][0][0], 9999, time.monotonic_ns() - 100_000_000)]], window=1)
    assert srv.stats()["max_ms"] >= 100.0
    srv.close()


def test_server_returns_outgoing_tracks(E, oracle_mod):
    """A request's outgoing tracks come back with its deposits and equal the
    oracle's for the same tracks and event key."""
    from parity_util import compare_exits
    print("server exits", flush=True)
    geo = I.calorimeter()
    cfg = I.RunConfig(seed=5, bz_tesla=3.8)
    c = E.make_config(cfg, 32, track_capacity=1 << 20, steps_per_launch=2, exit_capacity=1 << 16)
    srv = E.Server(c, geo, 1 << 30)
    rng = np.random.Generator(np.random.Philox(77))
    reqs = [I.serving_request(rng, e_median_MeV=800.0, max_tracks=20) for _ in range(6)]
    tickets = [srv.submit(r, 300 + i) for i, r in enumerate(reqs)]
    got = [srv.wait(tk, timeout_s=120, exits=True) for tk in tickets]
    srv.close()
    for i, (edep, led, ex) in enumerate(got):
        p = reqs[i].copy()
        p["event"] = 0
        r = oracle_mod.Oracle(geo, cfg).run(p, n_events=1, event_keys=[300 + i], exit_cap=1 << 16)
        compare_exits(ex, r["exits"])
        assert abs(ex["ekin"].sum() - led["escaped"].sum()) <= 1e-9 * max(1.0, led["escaped"].sum())


def test_server_with_box_geometry(E, oracle_mod):
    """the server over a box geometry (towers with cracks, no field): a
    request gives the same deposits per volume alone, in a mix of producers,
    and from the oracle with the same tracks and key"""
    print("server with boxes", flush=True)
    geo = I.towers(cells=5, n_layers=20)
    cfg = I.RunConfig(seed=6)
    c = E.make_config(cfg, 16, track_capacity=1 << 20, steps_per_launch=4)
    rng = np.random.Generator(np.random.Philox(77))
    probe = I.serving_request(rng, e_median_MeV=500.0, max_tracks=20, half_xy_mm=80.0)
    probe["pos"][:, 2] = 0.0
    srv = E.Server(c, geo, 1 << 30)
    alone = srv.wait(srv.submit(probe, 4242), timeout_s=120)
    tickets = []
    for i in range(24):
        tr = I.serving_request(rng, e_median_MeV=500.0, max_tracks=20, half_xy_mm=80.0)
        tr["pos"][:, 2] = 0.0
        tickets.append((srv.submit(tr, i), tr))
        if i == 11:
            tickets.append((srv.submit(probe, 4242), probe))
    res = [(srv.wait(t, timeout_s=300), tr) for t, tr in tickets]
    srv.close()
    (mix_edep, mix_led) = res[12][0]
    assert mix_edep.shape == (geo.n_cols,)
    assert np.allclose(mix_edep, alone[0], rtol=1e-12, atol=1e-12)
    for (edep, led), tr in res:
        assert residual(edep, led, tr) < 1e-9
    p = probe.copy()
    p["event"] = 0
    r = oracle_mod.Oracle(geo, cfg).run(p, n_events=1, event_keys=np.array([4242], dtype=np.uint32))
    assert np.allclose(r["edep"][0], alone[0], rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_same_result_alone_and_in_the_64_producer_mix(E, oracle_mod, precision):
    """The serving recipe at its producer count: 64 host threads each submit
    requests of U{1..200} e-/e+/gamma tracks with lognormal(ln 5 GeV, 1)
    total energy in Bz = 3.8 T, with four probe requests submitted from
    different producers in the middle of the mix.  Each probe gives the
    same deposits per slab (1e-12) and the same counts as when it ran alone
    on an empty server, in both forms; every request conserves energy (1e-9
    FP64, 1e-5 mixed); the FP64 probes equal the oracle's (1e-8)."""
    print(f"64-producer mix, {precision}", flush=True)
    prec = E.FP64 if precision == "fp64" else E.MIXED
    geo = I.calorimeter()
    cfg = I.RunConfig(seed=5, bz_tesla=3.8)
    c = E.make_config(cfg, 512, track_capacity=1 << 22, steps_per_launch=1, precision=prec,
                      flags=E.F_FULL_LEDGER, photon_steps_per_visit=32, photon_refill_below=24)
    prng = np.random.Generator(np.random.Philox(4321))
    probes = [(I.serving_request(prng), 900_000 + i) for i in range(4)]
    srv = E.Server(c, geo, 8 << 30)
    alone = [srv.wait(srv.submit(tr, k), timeout_s=120) for tr, k in probes]
    srv.close()

    srv = E.Server(c, geo, 8 << 30)
    results, reqs = {}, {}
    lock = threading.Lock()
    per_producer = 6

    def producer(p):
        rng = np.random.Generator(np.random.Philox(5 + p))
        mine = []
        for i in range(per_producer):
            tr = I.serving_request(rng)
            mine.append((srv.submit(tr, p * 1000 + i), tr, p * 1000 + i))
            if p % 16 == 3 and i == per_producer // 2:
                tr, k = probes[p // 16]
                mine.append((srv.submit(tr, k), tr, k))
        for t, tr, k in mine:
            r = srv.wait(t, timeout_s=300)
            with lock:
                results[t] = r
                reqs[t] = (tr, k)

    ths = [threading.Thread(target=producer, args=(p,)) for p in range(64)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    st = srv.stats()
    srv.close()
    assert len(results) == 64 * per_producer + 4 and st["completed"] == len(results)
    print("peak admitted bytes", st["peak_admitted_bytes"], "chunks", st["chunks"], flush=True)
    by_key = {k: results[t] for t, (tr, k) in reqs.items()}
    worst = 0.0
    for (tr, k), (a_edep, a_led) in zip(probes, alone):
        m_edep, m_led = by_key[k]
        scale = max(1.0, float(np.abs(a_edep).max()))
        worst = max(worst, float(np.abs(m_edep - a_edep).max()) / scale)
        for f in ("n_steps", "n_created", "n_null", "n_pair", "n_annih"):
            assert np.array_equal(m_led[f], a_led[f]), (k, f)
    print("largest alone-vs-mix deposit difference (relative)", worst, flush=True)
    assert worst <= 1e-12
    tol = 1e-9 if prec == E.FP64 else 1e-5
    for t, (edep, led) in results.items():
        assert residual(edep, led, reqs[t][0]) < tol
    if prec == E.FP64:
        o = oracle_mod.Oracle(geo, cfg)
        for (tr, k), (a_edep, a_led) in zip(probes, alone):
            p = tr.copy()
            p["event"] = 0
            r = o.run(p, n_events=1, event_keys=np.array([k], dtype=np.uint32))
            assert np.allclose(a_edep, r["edep"][0], rtol=1e-8, atol=1e-8)
            assert int(a_led["n_steps"]) == int(r["ledger"]["n_steps"][0])
