"""Primaries in and deposits out through device memory (ems_enqueue_device,
ems_read_edep_device): the device computes the checks, normalisation,
volume location and per-row ids that the host path computes, so the same
records give the same step records bit for bit (and tallies equal up to
the order of their atomic sums); deposits copied to device memory equal
those copied to the host.  Also: several groups of 1024
records with rows spread over them, two enqueues in a row, invalid records
(all or nothing), an empty batch, a batch mixing host and device primaries,
pointers that are not device memory."""
import ctypes as C

import numpy as np
import pytest

import ems_inputs as I
from parity_util import sort_log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_15445_amd as E
    E.lib()
    return E


def on_device(p):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(p).view(np.uint8)).to("cuda")
    torch.cuda.synchronize()
    return t


def scrambled(p, seed):
    """rows interleaved, directions of random length, some primaries on a
    plane or face moving backwards"""
    rng = np.random.default_rng(seed)
    q = p[rng.permutation(len(p))].copy()
    q["dir"] *= rng.uniform(0.2, 7.0, size=(len(q), 1))
    return q


def run_both(E, geo, cfg, parts, n_events, precision=0, log_cap=400000, flags=0):
    """the same primaries (a list of enqueue batches) through the host and
    the device path; returns (host, device) results"""
    import torch
    out = []
    for dev in (False, True):
        c = E.make_config(cfg, n_events, track_capacity=1 << 20, precision=precision,
                          flags=flags | E.F_STEPLOG | E.F_FULL_LEDGER, steplog_capacity=log_cap)
        t = E.Transport(c, geo)
        for p in parts:
            if dev:
                t.enqueue_device(on_device(p))
            else:
                t.enqueue(p)
        t.run()
        r = dict(edep=t.edep(), ledger=t.ledger(), stats=t.stats())
        r["log"], r["n_log"] = t.steplog()
        if dev:
            d = torch.empty((n_events, t.n_slabs), dtype=torch.float64, device="cuda")
            t.edep_device(d)
            torch.cuda.synchronize()
            r["edep_dev"] = d.cpu().numpy()
        t.close()
        out.append(r)
    return out


def assert_identical(h, d):
    """every step record equal bit for bit (logs in any order); tallies
    summed by atomics in run-dependent order: equal to 1e-12"""
    n = h["n_log"]
    assert n == d["n_log"] and n > 0
    a, b = sort_log(h["log"][:n]), sort_log(d["log"][:n])
    diff = {}
    for f in a.dtype.names:
        bad = np.nonzero(np.any((a[f] != b[f]).reshape(n, -1), axis=1))[0]
        if len(bad):
            dv = np.abs(a[f][bad].astype(np.float64) - b[f][bad].astype(np.float64)).max()
            diff[f] = (len(bad), int(bad[0]), float(dv))
    assert not diff, f"step records differ (field: count, first sorted index, largest difference): {diff}"
    assert np.array_equal(d["edep"], d["edep_dev"])
    assert np.allclose(h["edep"], d["edep"], rtol=1e-12, atol=1e-12)
    for f in ("n_steps", "n_created", "n_null", "n_pair", "n_annih"):
        assert np.array_equal(h["ledger"][f], d["ledger"][f]), f
    for f in ("edep", "escaped", "killed", "charged_len"):
        assert np.allclose(h["ledger"][f], d["ledger"][f], rtol=1e-12, atol=1e-12), f


@pytest.mark.parametrize("precision", [0, 1])
def test_slab_stack_device_primaries_give_the_host_histories(E, precision):
    print(f"device primaries, slab stack, precision {precision}", flush=True)
    geo = I.calorimeter()
    cfg = I.RunConfig(seed=5, bz_tesla=3.8)
    p = scrambled(I.random_tracks(600, 20, geo, 1e-3, 50.0, seed=8), 1)
    # on planes, moving backwards and forwards
    p["pos"][:40, 2] = np.asarray(geo.z_mm)[np.arange(40) % len(geo.z_mm)]
    p["dir"][:20, 2] = -np.abs(p["dir"][:20, 2])
    h, d = run_both(E, geo, cfg, [p], 20, precision=precision)
    assert_identical(h, d)


def test_box_geometry_device_primaries_give_the_host_histories(E):
    print("device primaries, towers", flush=True)
    geo = I.towers(cells=5, n_layers=6)
    cfg = I.RunConfig(seed=3)
    rng = np.random.default_rng(4)
    n = 400
    p = I.primaries(n)
    p["event"] = rng.integers(0, 16, n)
    p["species"] = rng.integers(0, 3, n)
    p["ekin"] = rng.uniform(0.05, 30.0, n)
    wl, wh = np.array(geo.world_lo), np.array(geo.world_hi)
    p["pos"] = rng.uniform(wl + 1e-3, wh - 1e-3, size=(n, 3))
    # a quarter exactly on box faces
    k = rng.integers(0, geo.n_boxes, n // 4)
    ax = rng.integers(0, 3, n // 4)
    p["pos"][np.arange(n // 4), ax] = np.where(rng.integers(0, 2, n // 4) == 1, geo.hi[k, ax], geo.lo[k, ax])
    p["dir"] = rng.normal(size=(n, 3)) * rng.uniform(0.1, 5.0, size=(n, 1))
    # on a face of the world: moving inwards (outwards the point is outside)
    for j in range(3):
        p["dir"][p["pos"][:, j] == wl[j], j] = np.abs(p["dir"][p["pos"][:, j] == wl[j], j]) + 0.1
        p["dir"][p["pos"][:, j] == wh[j], j] = -np.abs(p["dir"][p["pos"][:, j] == wh[j], j]) - 0.1
    h, d = run_both(E, geo, cfg, [p], 16)
    assert_identical(h, d)


def test_rows_spread_over_several_groups_and_two_enqueues(E):
    """5000 low-energy primaries over 7 rows in random order (ids run across
    the device's groups of 1024), enqueued in two batches of 3100 and 1900"""
    print("device primaries, 5000 over 7 rows", flush=True)
    geo = I.calorimeter()
    cfg = I.RunConfig(seed=9)
    rng = np.random.default_rng(12)
    n = 5000
    p = I.primaries(n)
    p["event"] = rng.integers(0, 7, n)
    p["species"] = rng.integers(0, 3, n)
    p["ekin"] = rng.uniform(0.02, 2.0, n)
    p["pos"] = np.column_stack([rng.uniform(-50, 50, n), rng.uniform(-50, 50, n), rng.uniform(0.0, 40.0, n)])
    p["dir"] = rng.normal(size=(n, 3))
    h, d = run_both(E, geo, cfg, [p[:3100], p[3100:]], 7, log_cap=2000000)
    assert_identical(h, d)


def test_invalid_device_primaries_are_all_or_nothing(E):
    import torch
    print("device primaries, invalid", flush=True)
    geo, cfg, prim = I.workload("cal_1GeV_e-_x32")
    c = E.make_config(cfg, 32, track_capacity=1 << 16)
    t = E.Transport(c, geo)
    bad = prim.copy()
    bad["ekin"][19] = np.nan
    bad["dir"][25] = 0.0
    with pytest.raises(E.EmsError) as ei:
        t.enqueue_device(on_device(bad))
    assert ei.value.code == E.E_INVALID and "#19" in str(ei.value)
    outside = prim.copy()
    outside["pos"][3, 2] = -1.0
    with pytest.raises(E.EmsError) as ei:
        t.enqueue_device(on_device(outside))
    assert ei.value.code == E.E_INVALID and "#3" in str(ei.value)
    too_many = I.beam(1 << 17, I.ELECTRON, 10.0)
    too_many["event"] = 0
    with pytest.raises(E.EmsError) as ei:
        t.enqueue_device(on_device(too_many))
    assert ei.value.code == E.E_CAPACITY
    # not device memory, and more records than the allocation holds
    host = np.ascontiguousarray(prim)
    assert E.lib().ems_enqueue_device(t._h, host.ctypes.data_as(C.c_void_p), len(host)) == E.E_INVALID
    d = on_device(prim)
    assert E.lib().ems_enqueue_device(t._h, C.c_void_p(d.data_ptr()), 1 << 39) == E.E_INVALID
    out = np.zeros((32, t.n_slabs))
    assert E.lib().ems_read_edep_device(t._h, 0, 32, out.ctypes.data_as(C.c_void_p)) == E.E_INVALID
    # an empty batch is accepted and adds nothing
    t.enqueue_device(on_device(prim[:0]))
    # nothing of the refused calls reached the queues
    t.enqueue_device(d)
    t.run()
    got = torch.zeros((32, t.n_slabs), dtype=torch.float64, device="cuda")
    t.edep_device(got)
    t.edep_device(torch.zeros((0, t.n_slabs), dtype=torch.float64, device="cuda"), first=32)
    got = got.cpu().numpy()
    t.close()
    c2 = E.make_config(cfg, 32, track_capacity=1 << 16)
    t2 = E.Transport(c2, geo)
    t2.enqueue(prim)
    t2.run()
    want = t2.edep()
    t2.close()
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12)


def test_a_batch_takes_primaries_from_one_side(E):
    print("device primaries, host/device mix refused", flush=True)
    geo, cfg, prim = I.workload("cal_1GeV_e-_x32")
    c = E.make_config(cfg, 32, track_capacity=1 << 16)
    t = E.Transport(c, geo)
    t.enqueue_device(on_device(prim[:4]))
    with pytest.raises(E.EmsError) as ei:
        t.enqueue(prim[4:8])
    assert ei.value.code == E.E_STATE
    t.run()
    first = t.edep()
    t.reset()
    t.enqueue(prim[:4])
    with pytest.raises(E.EmsError) as ei:
        t.enqueue_device(on_device(prim[4:8]))
    assert ei.value.code == E.E_STATE
    t.run()
    second = t.edep()
    t.reset()
    # after a reset the device path starts its ids at 0 again
    t.enqueue_device(on_device(prim[:4]))
    t.run()
    third = t.edep()
    t.close()
    assert np.allclose(first, second, rtol=1e-12, atol=1e-12)
    assert np.allclose(first, third, rtol=1e-12, atol=1e-12)
    assert first[:4].sum() > 0
