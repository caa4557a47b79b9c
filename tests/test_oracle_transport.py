"""Pins of the oracle's transport loop: exact energy ledger, thin-slab photon
attenuation against exp(-Sigma x), CSDA range against the integrated stopping
power, order independence of the stack, slab bookkeeping against a
brute-force locate, the helix against the circular orbit of the Lorentz
force, the iteration profile and the watchdog."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import ems_inputs as I

ME = 0.51099895


def ledger_residual(res, prim):
    L = res["ledger"]
    ein = np.bincount(prim["event"], weights=prim["ekin"], minlength=len(L))
    out = res["edep"].sum(axis=1) + L["escaped"].sum(axis=1) + L["killed"] + \
        2 * ME * (L["n_pair"].astype(np.int64) - L["n_annih"].astype(np.int64))
    return np.abs(out - ein) / ein


@pytest.fixture(scope="module")
def cal32(oracle_mod):
    geo, cfg, prim = I.workload("cal_1GeV_e-_x32")
    o = oracle_mod.Oracle(geo, cfg)
    return o, prim, o.run(prim, log_cap=400000, profile_cap=4000)


def test_ledger_identity_1gev(cal32):
    o, prim, res = cal32
    assert ledger_residual(res, prim).max() < 1e-12
    assert np.all(res["ledger"]["killed"] == 0)
    # edep per event equals the ledger's deposit sum
    assert np.allclose(res["edep"].sum(axis=1), res["ledger"]["edep"], rtol=1e-13)


def test_ledger_identity_field_mixed_species(oracle_mod):
    geo = I.calorimeter()
    cfg = I.RunConfig(seed=3, bz_tesla=3.8)
    prim = I.mixed_species(12, e_lo_MeV=100.0, e_hi_MeV=3000.0, seed=3)
    res = oracle_mod.Oracle(geo, cfg).run(prim)
    assert ledger_residual(res, prim).max() < 1e-12
    rnd = I.random_tracks(200, 10, geo, 1e-3, 50.0, seed=5)
    res = oracle_mod.Oracle(geo, cfg).run(rnd, n_events=10)
    assert ledger_residual(res, rnd).max() < 1e-12


def test_shower_sanity_1gev(cal32):
    """Parity unpinned against Geant4 (not available): only coarse sanity of a
    1 GeV shower -- containment and the position of the shower maximum."""
    o, prim, res = cal32
    edep = res["edep"].mean(axis=0)
    assert edep.sum() / 1000.0 > 0.95
    layer = edep.reshape(50, 2).sum(axis=1)
    assert 3 <= int(np.argmax(layer)) <= 12


def test_step_log_consistent_with_ledger(cal32):
    o, prim, res = cal32
    log = res["log"]
    assert res["n_log"] == len(log) == int(res["ledger"]["n_steps"].sum())
    dep = np.bincount(log["event"], weights=log["edep"], minlength=32)
    assert np.allclose(dep, res["ledger"]["edep"], rtol=1e-12)
    # each (event, id, step) appears once
    keys = set(zip(log["event"].tolist(), log["id"].tolist(), log["step"].tolist()))
    assert len(keys) == len(log)


def test_slab_index_matches_brute_force_locate(cal32):
    o, prim, res = cal32
    z = o.geo.z_mm
    log = res["log"]
    alive = log[log["slab_after"] >= 0]
    k = alive["slab_after"]
    zz = alive["pos_after"][:, 2]
    assert np.all(zz >= z[k] - 1e-9) and np.all(zz <= z[k + 1] + 1e-9)


def test_iteration_profile(cal32):
    o, prim, res = cal32
    prof = res["profile"]
    assert prof.sum() == res["ledger"]["n_steps"].sum()
    assert prof[0].tolist() == [0, 32, 0]
    assert res["n_iter"] == len(prof)


def test_order_independence(oracle_mod):
    geo, cfg, prim = I.workload("cal_1GeV_e-_x32")
    o = oracle_mod.Oracle(geo, cfg)
    a = o.run(prim[:6], stack_order=0)
    b = o.run(prim[:6], stack_order=1)
    assert np.allclose(a["edep"], b["edep"], rtol=1e-12, atol=1e-12)
    for f in ("n_steps", "n_created", "n_null", "n_pair", "n_annih"):
        assert np.array_equal(a["ledger"][f], b["ledger"][f])


@pytest.mark.parametrize("E", [0.1, 1.0, 10.0])
def test_thin_slab_photon_attenuation(oracle_mod, E):
    """Fraction of photons crossing 2.3 mm of lead without interacting is
    exp(-Sigma_tot x), Sigma_tot from the interpolated tables."""
    geo = I.single_slab(2.3, I.LEAD)
    cfg = I.RunConfig(seed=7)
    o = oracle_mod.Oracle(geo, cfg)
    n = 20000
    prim = I.beam(n, I.GAMMA, E)
    res = o.run(prim)
    direct = np.sum(res["ledger"]["n_steps"] == 1)
    assert np.all(res["edep"][res["ledger"]["n_steps"] == 1] == 0)
    sig = sum(o.lookup(0, t, E) for t in ("sigma_compton", "sigma_phot")) + \
        (o.lookup(0, "sigma_conv", E) if E > 2 * ME else 0.0)
    p = math.exp(-sig * 2.3)
    assert abs(direct - n * p) < 4 * math.sqrt(n * p * (1 - p)) + 1


@pytest.mark.parametrize("T0", [5.0, 50.0])
def test_csda_range(oracle_mod, T0):
    """Continuous loss only: the path length of an electron in a 100 mm lead
    block equals R(T0) from the table (0.1%) and the direct integral of
    dE/S(E) from the stopping-power formulas (0.5%)."""
    geo = I.single_slab(100.0, I.LEAD)
    cfg = I.RunConfig(seed=5, process_mask=I.P_CONT)
    o = oracle_mod.Oracle(geo, cfg)
    prim = I.beam(3, I.ELECTRON, T0)
    prim["pos"][:, 2] = 1.0
    res = o.run(prim)
    L = res["ledger"]["charged_len"]
    R = o.lookup(0, "R_e-", T0)
    assert np.allclose(L, R, rtol=1e-3)
    mat = I.LEAD

    def S(E):
        return oracle_mod.formula("SION_E", mat, 0.2, E) + oracle_mod.formula("SBREM", mat, 0.1, E)

    Es = np.geomspace(1e-3, T0, 200)
    direct = sum(integrate.quad(lambda e: 1 / S(e), a, b, epsrel=1e-10)[0] for a, b in zip(Es[:-1], Es[1:]))
    assert L[0] == pytest.approx(direct, rel=5e-3)
    assert np.all(res["ledger"]["escaped"] == 0)


@pytest.mark.parametrize("species,q", [(I.ELECTRON, -1.0), (I.POSITRON, +1.0)])
def test_helix_follows_lorentz_circle(oracle_mod, species, q):
    """No material interactions (empty process mask): a track moving
    perpendicular to Bz circles with radius p/(k_B B); positive charges turn
    clockwise seen from +z.  Every logged position lies on the circle at the
    phase the path length predicts."""
    geo = I.single_slab(400.0, I.LIQUID_ARGON)
    B, T = 3.8, 10.0
    cfg = I.RunConfig(seed=9, bz_tesla=B, process_mask=0, max_steps_per_track=40)
    o = oracle_mod.Oracle(geo, cfg)
    prim = I.beam(1, species, T)
    prim["pos"] = [[5.0, -3.0, 200.0]]
    prim["dir"] = [[1.0, 0.0, 0.0]]
    res = o.run(prim, log_cap=100)
    log = res["log"]
    p = math.sqrt(T * (T + 2 * ME))
    R = p / (0.299792458 * B)
    # centre: to the right of the velocity for positive charge (clockwise)
    cx, cy = 5.0, -3.0 - q * R
    s = np.cumsum(log["step_len"])
    phase0 = math.atan2(-3.0 - cy, 5.0 - cx)
    ang = phase0 - q * s / R
    xp = cx + R * np.cos(ang)
    yp = cy + R * np.sin(ang)
    assert np.allclose(log["pos_after"][:, 0], xp, rtol=0, atol=1e-9)
    assert np.allclose(log["pos_after"][:, 1], yp, rtol=0, atol=1e-9)
    assert np.all(log["pos_after"][:, 2] == 200.0)
    assert res["ledger"]["killed"][0] == T  # watchdog after 40 steps
    assert ledger_residual(res, prim).max() < 1e-15


def test_watchdog_accounts_killed_energy(oracle_mod):
    geo, cfg, prim = I.workload("cal_1GeV_e-_x32")
    cfg.max_steps_per_track = 5
    res = oracle_mod.Oracle(geo, cfg).run(prim[:4])
    assert np.all(res["ledger"]["killed"] > 0)
    assert ledger_residual(res, prim[:4]).max() < 1e-12


def test_invalid_primaries_rejected(oracle_mod):
    geo, cfg, prim = I.workload("cal_1GeV_e-_x32")
    o = oracle_mod.Oracle(geo, cfg)
    for field, val in (("ekin", -1.0), ("ekin", np.nan), ("species", 3)):
        bad = prim[:2].copy()
        bad[field][1] = val
        with pytest.raises(ValueError):
            o.run(bad, n_events=2)
    bad = prim[:2].copy()
    bad["dir"][0] = 0.0
    with pytest.raises(ValueError):
        o.run(bad, n_events=2)
    bad = prim[:2].copy()
    bad["pos"][0, 2] = -1.0
    with pytest.raises(ValueError):
        o.run(bad, n_events=2)
    with pytest.raises(ValueError):
        o.run(prim[:2], n_events=1)


def test_empty_run(oracle_mod):
    geo, cfg, prim = I.workload("cal_1GeV_e-_x32")
    res = oracle_mod.Oracle(geo, cfg).run(prim[:0], n_events=3)
    assert np.all(res["edep"] == 0) and np.all(res["ledger"]["n_steps"] == 0)


def test_event_key_not_row_decides_history(oracle_mod):
    """A run of one event with key k equals row k of a larger run."""
    geo, cfg, prim = I.workload("cal_1GeV_e-_x32")
    o = oracle_mod.Oracle(geo, cfg)
    full = o.run(prim[:5])
    one = prim[3:4].copy()
    one["event"] = 0
    sub = o.run(one, n_events=1, event_keys=[3])
    assert np.array_equal(sub["edep"][0], full["edep"][3])
    assert np.array_equal(sub["ledger"][0], full["ledger"][3])


def test_exits_close_the_ledger_and_sit_on_the_boundary(oracle_mod):
    """Outgoing tracks: their energies add up to each event's escaped energy
    per species, every exit point lies on the stack's boundary and every
    exit direction points out of the stack (with and without field)."""
    geo = I.calorimeter()
    H, z0, zN = geo.half_xy_mm, geo.z_mm[0], geo.z_mm[-1]
    for bz in (0.0, 3.8):
        cfg = I.RunConfig(seed=9, bz_tesla=bz)
        prim = I.random_tracks(400, 8, geo, 1e-2, 200.0, seed=21)
        res = oracle_mod.Oracle(geo, cfg).run(prim, n_events=8, exit_cap=100000)
        x = res["exits"]
        assert res["n_exits"] == len(x) > 0
        esc = np.zeros((8, 3))
        np.add.at(esc, (x["event"], x["species"]), x["ekin"])
        assert np.allclose(esc, res["ledger"]["escaped"], rtol=1e-12, atol=1e-12)
        p, d = x["pos"], x["dir"]
        back = np.isclose(p[:, 2], zN, atol=1e-9) & (d[:, 2] > 0)
        front = np.isclose(p[:, 2], z0, atol=1e-9) & (d[:, 2] < 0)
        if bz == 0.0:
            side = (np.isclose(np.abs(p[:, 0]), H, atol=1e-9) & (p[:, 0] * d[:, 0] > 0)) | \
                   (np.isclose(np.abs(p[:, 1]), H, atol=1e-9) & (p[:, 1] * d[:, 1] > 0))
        else:
            # charged tracks leave through the field-safety margin, photons
            # through the walls
            side = (H - np.maximum(np.abs(p[:, 0]), np.abs(p[:, 1])) < 1e-6 + 1e-9)
        assert np.all(back | front | side)


@pytest.mark.parametrize("E", [0.3, 1.0])
def test_uncollided_exits_follow_attenuation(oracle_mod, E):
    """Photons leaving 2.3 mm of lead with their initial energy and
    direction are the uncollided ones: their number is binomial with
    p = exp(-Sigma x), Sigma from the cross-section formulas (not the
    tables); they leave through the back plane on the beam axis."""
    geo = I.single_slab(2.3, I.LEAD)
    o = oracle_mod.Oracle(geo, I.RunConfig(seed=13))
    n = 20000
    res = o.run(I.beam(n, I.GAMMA, E), exit_cap=4 * n)
    x = res["exits"]
    same = (x["species"] == I.GAMMA) & (x["ekin"] == E) & (x["dir"][:, 2] == 1.0)
    assert np.all(np.isclose(x["pos"][same][:, 2], 2.3, atol=1e-12))
    assert np.all(x["pos"][same][:, :2] == 0.0)
    mat = I.LEAD
    n_at = mat[2] / mat[1] * 6.02214076e23 * 1e-3  # atoms per mm^3
    sig = n_at * (mat[0] * oracle_mod.formula("SIGMA_KN", mat, 0.0, E) +
                  oracle_mod.formula("SIGMA_PE", mat, 0.0, E) +
                  (oracle_mod.formula("SIGMA_PAIR", mat, 0.0, E) if E > 2 * ME else 0.0))
    p = math.exp(-sig * 2.3)
    k = int(same.sum())
    # the tables interpolate the formulas to well below the statistical error
    assert abs(k - n * p) < 4 * math.sqrt(n * p * (1 - p)) + 1
