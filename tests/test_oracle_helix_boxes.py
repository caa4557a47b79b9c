"""Pins of the oracle's charged transport in a box geometry with a field
(section 2.3: the boundary found along the curved path).  The helix's first
exit from a box and first entry into one are checked against a brute-force
march along the helix written out here (the position after path s from
the rotation of the direction about z) with bisection of the first
sample outside or inside; against closed forms of the Lorentz circle (a
quarter turn to the plane at one radius, no exit from a box that holds the
whole circle); and the slab stack written as boxes, wide enough that no
track reaches its sides, reproduces the slab geometry's histories step by
step in the same field.  Energy closes exactly.
"""
import math

import numpy as np
import pytest

import ems_inputs as I
from parity_util import compare_logs, ledger_residual, tiny_mixed_primaries


def helix_point(p, u, kappa, s):
    """Position after path s on the helix about z of signed curvature kappa:
    the transverse direction turns by -kappa s (a positive charge in +Bz
    turns clockwise), the transverse position is the integral of it."""
    ux, uy, uz = u
    phi = kappa * s
    # the direction at path t is (ux cos(kappa t) + uy sin(kappa t),
    # -ux sin(kappa t) + uy cos(kappa t), uz); integrated from 0 to s
    x = p[0] + (ux * math.sin(phi) + uy * (1.0 - math.cos(phi))) / kappa
    y = p[1] + (uy * math.sin(phi) - ux * (1.0 - math.cos(phi))) / kappa
    return np.array([x, y, p[2] + uz * s])


def first_change(p, u, kappa, pred, smax, n=20000):
    """Smallest s in (0, smax] where pred(point) turns true, by sampling and
    bisection; inf if it never does on the samples."""
    ss = np.linspace(0.0, smax, n + 1)[1:]
    prev = 0.0
    for s in ss:
        if pred(helix_point(p, u, kappa, s)):
            lo, hi = prev, s
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                if pred(helix_point(p, u, kappa, mid)):
                    hi = mid
                else:
                    lo = mid
                if hi - lo < 1e-13 * max(1.0, hi):
                    break
            return hi
        prev = s
    return math.inf


def one_box_oracle(oracle_mod, lo, hi, world_lo, world_hi):
    geo = I.BoxGeometry(lo=np.array([lo], dtype=np.float64), hi=np.array([hi], dtype=np.float64),
                        material=np.zeros(1, np.uint32), materials=[I.LEAD, I.LIQUID_ARGON],
                        world_lo=tuple(world_lo), world_hi=tuple(world_hi), world_material=1)
    return oracle_mod.Oracle(geo, I.RunConfig(bz_tesla=3.8))


def unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def test_exit_from_a_box_matches_a_march_along_the_helix(oracle_mod):
    rng = np.random.default_rng(3)
    lo, hi = np.array([-4.0, -3.0, -2.0]), np.array([5.0, 2.5, 6.0])
    o = one_box_oracle(oracle_mod, lo, hi, lo - 10.0, hi + 10.0)
    n_checked = 0
    for _ in range(150):
        p = lo + (hi - lo) * rng.uniform(0.05, 0.95, 3)
        u = unit(rng.normal(size=3))
        kappa = rng.choice([-1.0, 1.0]) * 10 ** rng.uniform(-1.5, 0.7)
        d, ax, f = o.geo_helix_distance(0, p, u, kappa)
        outside = lambda q: bool(np.any(q < lo) or np.any(q > hi))
        smax = 4.0 * (2.0 * math.pi / abs(kappa)) + 30.0
        ref = first_change(p, u, kappa, outside, smax)
        if not math.isfinite(ref):
            assert not math.isfinite(d) or d > smax * 0.999
            continue
        n_checked += 1
        assert d == pytest.approx(ref, rel=1e-7, abs=1e-9), (p, u, kappa)
        q = helix_point(p, u, kappa, d)
        assert q[ax] == pytest.approx(f, abs=1e-7) and f in (lo[ax], hi[ax])
    assert n_checked > 100


def test_entry_into_boxes_matches_a_march_along_the_helix(oracle_mod):
    rng = np.random.default_rng(4)
    geo = I.towers(cells=3, n_layers=3, pitch_mm=10.0, crack_mm=2.0, margin_mm=5.0)
    o = oracle_mod.Oracle(geo, I.RunConfig(bz_tesla=3.8))
    lo, hi = np.asarray(geo.lo), np.asarray(geo.hi)
    wlo, whi = np.asarray(geo.world_lo), np.asarray(geo.world_hi)
    world = len(lo)
    n_checked = 0
    for _ in range(400):
        p = wlo + (whi - wlo) * rng.uniform(0.02, 0.98, 3)
        u = unit(rng.normal(size=3))
        if o.geo_locate(p, u) != world:
            continue
        kappa = rng.choice([-1.0, 1.0]) * 10 ** rng.uniform(-1.0, 0.5)
        d, ax, f = o.geo_helix_distance(world, p, u, kappa)

        def left(q):
            if np.any(q < wlo) or np.any(q > whi):
                return True
            return bool(np.any(np.all((q >= lo) & (q <= hi), axis=1)))

        ref = first_change(p, u, kappa, left, 60.0, n=6000)
        if not math.isfinite(ref):
            continue
        n_checked += 1
        assert d == pytest.approx(ref, rel=1e-7, abs=1e-8), (p, u, kappa)
    assert n_checked > 100


def test_lorentz_circle_closed_forms(oracle_mod):
    lo, hi = np.array([-50.0, -50.0, -50.0]), np.array([50.0, 50.0, 50.0])
    o = one_box_oracle(oracle_mod, lo, hi, lo - 1.0, hi + 1.0)
    # from the origin along +y with kappa > 0 the circle has its centre at
    # (1/kappa, 0): the plane x = X (0 < X < 2/kappa) is met after
    # acos(1 - kappa X) / kappa
    for kappa, X in ((0.1, 3.0), (0.1, 19.0), (0.05, 40.0)):
        box = one_box_oracle(oracle_mod, [-50.0, -50.0, -50.0], [X, 50.0, 50.0], [-51.0, -51.0, -51.0],
                             [51.0, 51.0, 51.0])
        d, ax, f = box.geo_helix_distance(0, [0.0, 0.0, 0.0], [0.0, 1.0, 0.0], kappa)
        assert ax == 0 and f == X
        assert d == pytest.approx(math.acos(1.0 - kappa * X) / kappa, rel=1e-12)
    # a circle that fits in the box (u_z = 0) never leaves it
    d, _, _ = o.geo_helix_distance(0, [0.0, 0.0, 0.0], [1.0, 0.0, 0.0], 0.5)
    assert math.isinf(d)
    # with u_z != 0 it leaves through a z face after (50 - z0) / u_z
    u = unit([1.0, 0.0, 0.25])
    d, ax, f = o.geo_helix_distance(0, [0.0, 0.0, 0.0], u, 0.5)
    assert ax == 2 and f == 50.0 and d == pytest.approx(50.0 / u[2], rel=1e-15)
    # the search stops at smax
    d, _, _ = o.geo_helix_distance(0, [0.0, 0.0, 0.0], u, 0.5, smax=10.0)
    assert math.isinf(d)


def test_wide_slab_stack_as_boxes_has_the_same_histories_in_a_field(oracle_mod):
    # no track reaches the sides of a stack 20 m wide: the transverse safety
    # of the slab geometry never limits a step, and the box geometry's exit
    # along the helix is the same z plane
    geo = I.calorimeter(half_xy_mm=10000.0)
    cfg = I.RunConfig(seed=23, bz_tesla=3.8)
    prim = tiny_mixed_primaries()
    prim["ekin"] *= 20.0
    a = oracle_mod.Oracle(geo, cfg).run(prim, n_events=48, log_cap=400000)
    b = oracle_mod.Oracle(I.boxes_from_slabs(geo), cfg).run(prim, n_events=48, log_cap=400000)
    assert a["n_log"] == b["n_log"] and a["n_log"] > 1000
    compare_logs(b["log"][: b["n_log"]], a["log"][: a["n_log"]], e_rtol=1e-12, pos_atol=1e-9)
    assert np.allclose(a["edep"], b["edep"][:, :-1], rtol=1e-12, atol=1e-12)
    for f in ("n_steps", "n_created", "n_null", "n_pair", "n_annih"):
        assert np.array_equal(a["ledger"][f], b["ledger"][f]), f


def test_towers_in_a_field_close_energy(oracle_mod):
    geo = I.towers(cells=3, n_layers=10)
    cfg = I.RunConfig(seed=29, bz_tesla=3.8)
    prim = I.beam(6, I.ELECTRON, 500.0, smear_rad=0.3, seed=5)
    prim["pos"][:, 0] = np.linspace(-25.0, 25.0, 6)   # some start in the cracks
    r = oracle_mod.Oracle(geo, cfg).run(prim, n_events=6, log_cap=400000)
    assert ledger_residual(r["edep"], r["ledger"], prim).max() < 1e-12
    log = r["log"][: r["n_log"]]
    world = len(geo.lo)
    # charged steps in the world volume happen, and tracks cross between
    # towers and cracks along curved paths
    charged = log["species"] != 0
    assert np.any(charged & (log["slab_after"] == world))
    assert r["edep"][:, world].sum() > 0.0
