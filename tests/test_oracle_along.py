"""Pins of the oracle's optional along-step processes of e-/e+: multiple
Coulomb scattering (Gaussian, Highland width) and fluctuations of the
restricted energy loss (gamma distribution, Bethe second moment).

Radiation lengths are tied to PDG's tabulated values, the Highland width to
its closed-form special case, the sampled angles and losses to their
distributions and to the pinned Philox draws, the loss variance to the
second moment of the oracle's (pinned) Moller and Bhabha spectra, and the
transport to single-slab experiments whose outcome is fixed by one step.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import ems_inputs as I

ME = 0.51099895
NA = 6.02214076e23


def el(Z, A, rho=1.0):
    return (float(Z), float(A), rho, 100.0)


# PDG radiation lengths in g/cm^2 (atomic and nuclear properties tables)
X0_PDG = [
    (el(1, 1.008), 63.04), (el(2, 4.002602), 94.32), (el(4, 9.0121831), 65.19),
    (el(6, 12.0107), 42.70), (el(8, 15.999), 34.24), (el(18, 39.948), 19.55),
    (el(26, 55.845), 13.84), (el(74, 183.84), 6.76), (el(82, 207.2), 6.37),
]


@pytest.mark.parametrize("mat,x0", X0_PDG)
def test_radiation_length_matches_pdg(oracle_mod, mat, x0):
    got = oracle_mod.formula("X0", mat, 0, 0) * mat[2] / 10.0  # mm -> g/cm^2
    assert got == pytest.approx(x0, rel=2e-3)


def test_compound_radiation_length(oracle_mod):
    # PbWO4: 7.39 g/cm^2 (PDG); 1/X0 adds over the elements
    m = I.LEAD_TUNGSTATE
    assert oracle_mod.formula("X0", m, 0, 0) * m[2] / 10.0 == pytest.approx(7.39, rel=3e-3)


@pytest.mark.parametrize("T", [1.0, 30.0, 1e4])
def test_highland_special_case(oracle_mod, T):
    """at x = beta^2 X0 the logarithm vanishes: theta_0 = 13.6 MeV / p"""
    p = math.sqrt(T * (T + 2 * ME))
    beta = p / (T + ME)
    x0 = oracle_mod.formula("X0", I.LEAD, 0, 0)
    assert oracle_mod.formula("HIGHLAND", I.LEAD, 0, T, beta ** 2 * x0) == pytest.approx(13.6 / p, rel=1e-12)
    # sqrt(x) growth with the log correction: ratio between x and 100 x
    a = oracle_mod.formula("HIGHLAND", I.LEAD, 0, T, 0.01 * x0)
    b = oracle_mod.formula("HIGHLAND", I.LEAD, 0, T, 1.0 * x0)
    L = math.log(1.0 / beta ** 2)
    assert b / a == pytest.approx(10 * (1 + 0.038 * L) / (1 + 0.038 * (math.log(0.01) + L)), rel=1e-12)
    # where the correction turns negative there is no deflection
    assert oracle_mod.formula("HIGHLAND", I.LEAD, 0, T, 1e-13 * x0) == 0.0


@pytest.fixture(scope="module")
def slab_oracle(oracle_mod):
    geo = I.single_slab(10.0, material=I.LEAD)
    return oracle_mod.Oracle(geo, I.RunConfig(seed=4))


def test_msc_deflection_uses_its_draws(oracle_mod, slab_oracle):
    """space angle = theta_0 sqrt(-2 ln u1), azimuth 2 pi u2, with u1, u2 the
    track's draws 65536 and 65537, about any incoming direction"""
    key = (3, 4)
    d = np.array([0.3, -0.4, math.sqrt(1 - 0.25)])
    for i in range(50):
        out = slab_oracle.sample_along("msc", 0, 50.0, 0.3, key, i, 7, direction=tuple(d))
        th0, u = out[0], out[1:]
        u1 = oracle_mod.uniform(key, i, 7, 65536)
        th = min(math.pi, th0 * math.sqrt(-2 * math.log(u1)))
        assert np.linalg.norm(u) == pytest.approx(1.0, abs=1e-14)
        assert math.acos(max(-1.0, min(1.0, float(np.dot(u, d))))) == pytest.approx(th, abs=1e-7)


def test_msc_projected_angles_are_gaussian(slab_oracle):
    n = 4000
    out = np.array([slab_oracle.sample_along("msc", 0, 1000.0, 0.5, (1, 2), i, 0) for i in range(n)])
    th0 = out[0, 0]
    assert 1e-3 < th0 < 0.1
    px = np.arctan2(out[:, 1], out[:, 3]) / th0
    py = np.arctan2(out[:, 2], out[:, 3]) / th0
    assert stats.kstest(px, "norm").pvalue > 1e-3
    assert stats.kstest(py, "norm").pvalue > 1e-3
    # theta^2 / theta_0^2 is chi^2 with two degrees of freedom
    th2 = np.arccos(np.clip(out[:, 3], -1, 1)) ** 2 / th0 ** 2
    assert stats.kstest(th2, stats.chi2(2).cdf).pvalue > 1e-3


@pytest.mark.parametrize("positron", [False, True])
def test_fluct_variance_is_second_moment_of_delta_spectrum(oracle_mod, positron):
    """for T >> cut the sub-cut second moment of the (pinned) Moller / Bhabha
    spectrum and the spin-0 Bethe form agree to O(cut / T)"""
    T, cut, s = 1000.0, 0.2, 1.0
    mat = I.LEAD
    nel = mat[0] * mat[2] * NA / mat[1] * 1e-3
    which = "DSDE_BHABHA" if positron else "DSDE_MOLLER"
    f = lambda w: w * w * oracle_mod.formula(which, mat, 0, T, w / T) / T
    lo = 1e-9
    m2 = nel * s * integrate.quad(f, lo, cut, epsrel=1e-10, limit=200)[0]
    v = oracle_mod.formula("FLUCT_VAR_P" if positron else "FLUCT_VAR_E", mat, cut, T, s)
    assert v == pytest.approx(m2, rel=1e-3)
    # at low energy the cut is the kinematic limit for e- (T/2)
    T2 = 0.3
    v2 = oracle_mod.formula("FLUCT_VAR_E", mat, cut, T2, s)
    g = T2 / ME + 1
    b2 = 1 - 1 / g ** 2
    assert v2 == pytest.approx(nel * s * 2 * math.pi * 2.8179403262e-12 ** 2 * ME / b2 * (T2 / 2) * (1 - b2 / 2),
                               rel=1e-12)


@pytest.mark.parametrize("k", [0.3, 2.5, 300.0])
def test_fluct_loss_is_gamma_distributed(slab_oracle, k):
    T, s = 20.0, 0.5
    var = slab_oracle.sample_along("fluct_e-", 0, T, s, (5, 6), 0, 0, mean=1.0)[1]
    mean = math.sqrt(k * var)
    n = 6000
    x = np.array([slab_oracle.sample_along("fluct_e-", 0, T, s, (5, 6), i, 3, mean=mean)[0] for i in range(n)])
    assert abs(x.mean() - mean) < 5 * math.sqrt(var / n)
    assert stats.kstest(x, stats.gamma(k, scale=var / mean).cdf).pvalue > 1e-3


def test_msc_single_slab_exit_angles(oracle_mod):
    """1 GeV e- through 1 mm of lead with only multiple scattering: one step
    through the slab, exit angles Gaussian with the Highland width of 1 mm"""
    geo = I.single_slab(1.0, material=I.LEAD)
    cfg = I.RunConfig(seed=9, process_mask=I.P_MSC)
    o = oracle_mod.Oracle(geo, cfg)
    n = 3000
    prim = I.beam(n, I.ELECTRON, 1000.0)
    r = o.run(prim, exit_cap=2 * n)
    assert r["n_exits"] == n
    x = r["exits"]
    assert np.all(x["ekin"] == 1000.0)
    assert np.allclose(x["pos"][:, 2], 1.0)
    th0 = oracle_mod.formula("HIGHLAND", I.LEAD, 0, 1000.0, 1.0)
    px = np.arctan2(x["dir"][:, 0], x["dir"][:, 2]) / th0
    assert stats.kstest(px, "norm").pvalue > 1e-3
    assert np.array_equal(r["ledger"]["n_steps"], np.ones(n, dtype=np.uint64))


def test_fluct_single_slab_loss(oracle_mod):
    """50 MeV e- through 1 mm of liquid argon, continuous loss only: one step;
    with fluctuations the deposit has the same mean and the Bethe variance"""
    geo = I.single_slab(1.0, material=I.LIQUID_ARGON)
    n = 4000
    prim = I.beam(n, I.ELECTRON, 50.0)
    base = oracle_mod.Oracle(geo, I.RunConfig(seed=2, process_mask=I.P_CONT)).run(prim[:1])
    mu = base["edep"][0, 0]
    r = oracle_mod.Oracle(geo, I.RunConfig(seed=2, process_mask=I.P_CONT | I.P_FLUCT)).run(prim)
    assert np.array_equal(r["ledger"]["n_steps"], np.ones(n, dtype=np.uint64))
    d = r["edep"][:, 0]
    var = oracle_mod.formula("FLUCT_VAR_E", I.LIQUID_ARGON, 0.2, 50.0, 1.0)
    assert abs(d.mean() - mu) < 5 * math.sqrt(var / n)
    assert d.var() == pytest.approx(var, rel=0.1)
    assert stats.kstest(d, stats.gamma(mu * mu / var, scale=var / mu).cdf).pvalue > 1e-3


def test_showers_with_msc_and_fluct_close_energy_and_backscatter(oracle_mod):
    """full physics with both along-step processes on the calorimeter: exact
    energy closure; multiple scattering sends electrons back out of the front
    face, which the other processes do not (the Gaussian core over steps of
    up to the range underestimates backscattering; no magnitude is claimed)"""
    geo = I.calorimeter(n_layers=10)
    prim = I.beam(64, I.ELECTRON, 2.0, seed=1)
    out = {}
    for tag, mask in (("off", I.P_ALL), ("on", I.P_ALL | I.P_MSC | I.P_FLUCT)):
        o = oracle_mod.Oracle(geo, I.RunConfig(seed=8, process_mask=mask))
        r = o.run(prim, exit_cap=100000)
        L = r["ledger"]
        tot = r["edep"].sum(axis=1) + L["escaped"].sum(axis=1) + L["killed"] + \
            2 * ME * (L["n_pair"].astype(np.int64) - L["n_annih"].astype(np.int64))
        np.testing.assert_allclose(tot, 2.0, rtol=1e-12)
        x = r["exits"][: r["n_exits"]]
        out[tag] = int(np.sum((x["species"] == I.ELECTRON) & (x["pos"][:, 2] == 0.0)))
    assert out["off"] <= 1 and out["on"] >= 4, out


def test_deflection_back_at_an_inner_plane_keeps_the_slab(oracle_mod):
    """a track scattered back on reaching an inner plane stays in its slab
    (its next step runs inside it); no step has zero length"""
    geo = I.calorimeter(n_layers=10)
    prim = I.beam(32, I.ELECTRON, 5.0, seed=2)
    o = oracle_mod.Oracle(geo, I.RunConfig(seed=3, process_mask=I.P_ALL | I.P_MSC))
    r = o.run(prim, log_cap=400000)
    log = r["log"][: r["n_log"]]
    zpl = oracle_mod.LIMITERS["ZPLANE"]
    assert np.all(log["step_len"][log["limiter"] == zpl] > 0.0)
    order = np.lexsort((log["step"], log["id"], log["event"]))
    L = log[order]
    same = (L["event"][1:] == L["event"][:-1]) & (L["id"][1:] == L["id"][:-1])
    prev_slab = L["slab_after"][:-1][same]
    cur = L[1:][same]
    zp = cur["limiter"] == zpl
    stayed = zp & (cur["slab_after"] == prev_slab)
    assert stayed.sum() > 0
    z = geo.z_mm
    for rec, s0 in zip(cur[stayed], prev_slab[stayed]):
        assert rec["pos_after"][2] in (z[s0], z[s0 + 1])
