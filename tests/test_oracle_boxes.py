"""Pins of the oracle's box geometry (non-overlapping boxes in a world box,
brute-force navigation).

The slab stack written as boxes reproduces the slab geometry's histories
step by step; located volumes and boundary distances are checked against the
definitions on random and on-face points (the volume just before and just
after the boundary, the face on the ray); uncollided photons through boxes
and world gaps follow exp(-sum Sigma x); transversely segmented showers agree
in distribution with the unsegmented stack; energy closes exactly.
"""
import math

import numpy as np
import pytest

import ems_inputs as I
from parity_util import compare_logs, ledger_residual, tiny_mixed_primaries

NA = 6.02214076e23


def slab_equivalent_logs(oracle_mod, cfg, prim, n_events):
    geo = I.calorimeter()
    a = oracle_mod.Oracle(geo, cfg).run(prim, n_events=n_events, log_cap=400000, exit_cap=100000)
    b = oracle_mod.Oracle(I.boxes_from_slabs(geo), cfg).run(prim, n_events=n_events, log_cap=400000,
                                                              exit_cap=100000)
    return a, b


@pytest.mark.parametrize("mask", [I.P_ALL, I.P_ALL | I.P_MSC | I.P_FLUCT])
def test_slab_stack_as_boxes_has_the_same_histories(oracle_mod, mask):
    cfg = I.RunConfig(seed=21, process_mask=mask)
    prim = tiny_mixed_primaries()
    prim["ekin"] *= 20.0
    a, b = slab_equivalent_logs(oracle_mod, cfg, prim, 48)
    la, lb = a["log"][: a["n_log"]].copy(), b["log"][: b["n_log"]].copy()
    # the box geometry reports every boundary (walls included) as limiter 0
    la["limiter"][la["limiter"] == oracle_mod.LIMITERS["WALL"]] = oracle_mod.LIMITERS["ZPLANE"]
    assert a["n_log"] == b["n_log"]
    compare_logs(lb, la, e_rtol=1e-12, pos_atol=1e-9)
    assert np.allclose(a["edep"], b["edep"][:, :-1], rtol=1e-12, atol=1e-12)
    assert np.all(b["edep"][:, -1] == 0.0)
    for f in ("n_steps", "n_created", "n_null", "n_pair", "n_annih"):
        assert np.array_equal(a["ledger"][f], b["ledger"][f]), f
    assert a["n_exits"] == b["n_exits"]


def inside_by_definition(lo, hi, p, u):
    ok = (p > lo) & (p < hi) | (p == lo) & (u >= 0) | (p == hi) & (u < 0)
    return ok.all(axis=-1)


@pytest.fixture(scope="module")
def towers_oracle(oracle_mod):
    geo = I.towers(cells=5, n_layers=6)
    return geo, oracle_mod.Oracle(geo, I.RunConfig(seed=1))


def test_locate_matches_the_definition(towers_oracle):
    geo, o = towers_oracle
    rng = np.random.default_rng(3)
    wl, wh = np.array(geo.world_lo), np.array(geo.world_hi)
    pts = rng.uniform(wl, wh, size=(3000, 3))
    # put a third of the points exactly on box faces
    k = rng.integers(0, geo.n_boxes, 1000)
    ax = rng.integers(0, 3, 1000)
    side = rng.integers(0, 2, 1000)
    pts[:1000][np.arange(1000), ax] = np.where(side == 1, geo.hi[k, ax], geo.lo[k, ax])
    dirs = rng.normal(size=(3000, 3))
    dirs[::7, 0] = 0.0
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    for p, u in zip(pts, dirs):
        inside = np.nonzero(inside_by_definition(geo.lo, geo.hi, p[None, :], u[None, :]))[0]
        assert len(inside) <= 1
        want = int(inside[0]) if len(inside) else (geo.n_boxes if inside_by_definition(
            wl[None, :], wh[None, :], p[None, :], u[None, :])[0] else -1)
        assert o.geo_locate(p, u) == want


def test_boundary_distance_by_its_definition(towers_oracle):
    """just before the boundary the track is still in its volume, just after
    it is not, and the face coordinate is on the ray"""
    geo, o = towers_oracle
    rng = np.random.default_rng(4)
    wl, wh = np.array(geo.world_lo), np.array(geo.world_hi)
    n_checked = 0
    for _ in range(1500):
        p = rng.uniform(wl, wh)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        v = o.geo_locate(p, u)
        if v < 0:
            continue
        d, ax, face = o.geo_distance(v, p, u)
        assert 0.0 < d < np.inf
        assert p[ax] + d * u[ax] == pytest.approx(face, abs=1e-9)
        eps = 1e-7 * max(1.0, d)
        if d > 2 * eps:
            assert o.geo_locate(p + (d - eps) * u, u) == v
        after = o.geo_locate(p + (d + eps) * u, u)
        assert after != v
        n_checked += 1
    assert n_checked > 1000


def test_uncollided_photons_through_boxes_and_gaps(oracle_mod):
    """1 MeV photons along +z through three 1 mm lead boxes separated by 2 mm
    of world liquid argon (8 mm in all): unscattered fraction exp(-3 S_Pb - 8 S_lAr)"""
    lo = np.array([[-50, -50, 2.0], [-50, -50, 5.0], [-50, -50, 8.0]], dtype=float)
    hi = lo + np.array([100.0, 100.0, 1.0])
    geo = I.BoxGeometry(lo=lo, hi=hi, material=np.zeros(3, dtype=np.uint32), materials=[I.LEAD, I.LIQUID_ARGON],
                        world_lo=(-60.0, -60.0, 0.0), world_hi=(60.0, 60.0, 11.0), world_material=1)
    cfg = I.RunConfig(seed=5)
    o = oracle_mod.Oracle(geo, cfg)
    n = 4000
    prim = I.beam(n, I.GAMMA, 1.0)
    r = o.run(prim, exit_cap=10 * n)
    x = r["exits"][: r["n_exits"]]
    un = np.sum((x["ekin"] == 1.0) & (x["dir"][:, 2] == 1.0) & (x["pos"][:, 2] == 11.0))

    def sigma(m):
        nat = m[2] * NA / m[1] * 1e-3
        return (m[0] * nat * oracle_mod.formula("SIGMA_KN", m, 0, 1.0) +
                nat * oracle_mod.formula("SIGMA_PE", m, 0, 1.0) + nat * oracle_mod.formula("SIGMA_PAIR", m, 0, 1.0))
    p = math.exp(-3 * sigma(I.LEAD) - 8 * sigma(I.LIQUID_ARGON))
    assert abs(un / n - p) < 4 * math.sqrt(p * (1 - p) / n) + 2e-3


def test_segmented_showers_match_the_slab_stack(oracle_mod):
    """towers without cracks are the slab stack cut transversely: the same
    per-layer deposits in distribution, exact energy closure"""
    geo = I.towers(cells=5, crack_mm=0.0, n_layers=50, margin_mm=0.0)
    cfg = I.RunConfig(seed=6)
    n = 64
    prim = I.beam(n, I.ELECTRON, 1000.0, smear_rad=1e-3, seed=6)
    prim["pos"][:, 0] = np.linspace(-15.0, 15.0, n)  # across tower faces at +-20 mm ... and inside
    r = oracle_mod.Oracle(geo, cfg).run(prim)
    assert ledger_residual(r["edep"], r["ledger"], prim).max() < 1e-12
    layers_b = r["edep"][:, :-1].reshape(n, 25, 100).sum(axis=1).reshape(n, 50, 2).sum(axis=2)
    s = oracle_mod.Oracle(I.calorimeter(half_xy_mm=100.0), cfg).run(prim)
    layers_s = s["edep"].reshape(n, 50, 2).sum(axis=2)
    mb, ms = layers_b.mean(axis=0), layers_s.mean(axis=0)
    sig = np.sqrt(layers_b.var(axis=0) / n + layers_s.var(axis=0) / n)
    assert np.all(np.abs(mb - ms) <= 3.5 * sig + 0.01 * ms + 1e-9)
    assert r["ledger"]["n_steps"].sum() > s["ledger"]["n_steps"].sum()  # more boundaries


def test_box_geometry_validation(oracle_mod):
    cfg = I.RunConfig()
    base = I.towers(cells=3, n_layers=2)
    bad = []
    g = I.towers(cells=3, n_layers=2)
    g.hi = g.hi.copy()
    g.hi[0, 0] = g.hi[0, 0] + 50.0  # overlaps its neighbour
    bad.append(g)
    g = I.towers(cells=3, n_layers=2)
    g.lo = g.lo.copy()
    g.lo[0, 2] = -1.0  # outside the world
    bad.append(g)
    for g in bad:
        with pytest.raises(ValueError):
            oracle_mod.Oracle(g, cfg)
    o = oracle_mod.Oracle(base, cfg)
    p = I.beam(2, I.ELECTRON, 10.0)
    p["pos"][1] = (1e4, 0.0, 0.0)
    with pytest.raises(Exception):
        o.run(p)
