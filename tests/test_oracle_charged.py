"""Pins of the oracle's charged-particle stepping (e-/e+).

The paper takes its electron and positron physics from G4HepEm (section 2.2)
and does not spell out how a charged step is limited or how discrete
interactions are sampled along a step that loses energy.  The oracle's
reading is a null-collision (thinning) scheme over the energy range a step
can reach, with a step function of the range and linear or range-table
energy loss.  These tests tie that reading to results fixed independently of
its code:

* the probability that a track crosses a thin slab without a discrete
  interaction is exp(-integral of Sigma(E(s)) ds) along its continuous-slowing
  -down path, and which process acts first follows the same integral;
* the restricted collision stopping power reduces, at T_cut = T_max, to the
  closed unrestricted formulas of ICRU Report 37 (Moller for e-, Bhabha for
  e+), and tends at high energy to the Fermi plateau fixed by the density
  effect;
* logged steps obey the properties of the step function and of the
  continuous loss: a step never exceeds the range, short ranges are taken in
  one step, long ones approach the fraction alpha of the range, and the range
  decreases by the path length.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import ems_inputs as I

ME = 0.51099895
RE = 2.8179403262e-12
NA = 6.02214076e23
PB, LAR = I.LEAD, I.LIQUID_ARGON
TCUT, KCUT = 0.2, 0.1

E_TABS = (("sigma_moller", 2 * TCUT), ("sigma_brem", KCUT))
P_TABS = (("sigma_bhabha", TCUT), ("sigma_brem", KCUT), ("sigma_annih", 0.0))


def csda_path(o, sp, T0, L, tabs, n=20001):
    """Energy along the continuous-slowing-down path of the oracle's own
    tables, E(s) = R^-1(R(T0) - s), and the interpolated discrete cross
    sections there (zero at and below each threshold)."""
    R0 = o.lookup(0, "R_e-" if sp == I.ELECTRON else "R_e+", T0)
    assert R0 > L, "the track must cross the slab without stopping"
    s = np.linspace(0.0, L, n)
    E = np.array([o.inverse_range(0, sp, R0 - x) for x in s])
    sig = np.array([[o.lookup(0, t, e) if e > th else 0.0 for e in E] for t, th in tabs])
    return s, E, sig


def survival_expected(o, sp, T0, L, tabs):
    def total(x):
        R0 = o.lookup(0, "R_e-" if sp == I.ELECTRON else "R_e+", T0)
        e = o.inverse_range(0, sp, R0 - x)
        return sum(o.lookup(0, t, e) if e > th else 0.0 for t, th in tabs)
    pts = np.linspace(0.0, L, 41)
    lam = sum(integrate.quad(total, a, b, epsabs=0, epsrel=1e-11, limit=200)[0] for a, b in zip(pts[:-1], pts[1:]))
    no_loss = L * sum(o.lookup(0, t, T0) if T0 > th else 0.0 for t, th in tabs)
    return math.exp(-lam), math.exp(-no_loss)


# ------------------------------------------------------------------ survival
# (species, T0 MeV, slab mm, material, seed): low energies in lead, where the
# cross sections change fastest along the path (0.45 MeV e- crosses the Moller
# threshold 2 T_cut = 0.4 MeV inside the slab), and one case in argon
SURVIVAL = [
    (I.ELECTRON, 0.45, 0.05, PB, 41),
    (I.ELECTRON, 0.6, 0.05, PB, 42),
    (I.ELECTRON, 0.6, 1.0, LAR, 43),
    (I.POSITRON, 0.5, 0.1, PB, 44),
    (I.POSITRON, 0.4, 1.0, LAR, 45),
]


@pytest.mark.parametrize("sp,T0,L,mat,seed", SURVIVAL)
def test_survival_without_discrete_interaction(oracle_mod, sp, T0, L, mat, seed):
    """2x10^6 tracks along the normal of one slab with continuous loss and
    the discrete processes of the species on: the fraction that leaves it
    without any discrete interaction (no secondary, no annihilation) is
    binomial with p = exp(-integral of Sigma_tot(E(s)) ds) along the CSDA
    path.  Taking Sigma at the entry energy instead (no energy loss inside
    the thinning) is excluded by the same data."""
    N = 2_000_000
    mask = I.P_CONT | I.P_EIONI | I.P_EBREM | (I.P_ANNIH if sp == I.POSITRON else 0)
    geo = I.single_slab(L, material=mat)
    o = oracle_mod.Oracle(geo, I.RunConfig(seed=seed, process_mask=mask))
    led = o.run(I.beam(N, sp, T0), n_events=N)["ledger"]
    assert led["killed"].sum() == 0.0
    survived = (led["n_created"].sum(axis=1) == 0) & (led["n_annih"] == 0)
    p_obs = survived.mean()
    p_exp, p_noloss = survival_expected(o, sp, T0, L, P_TABS if sp == I.POSITRON else E_TABS)
    sd = math.sqrt(p_exp * (1 - p_exp) / N)
    print(f"survival {p_obs:.6f}, expected {p_exp:.6f} ({(p_obs - p_exp) / sd:+.2f} sd), "
          f"without loss {p_noloss:.6f} ({(p_obs - p_noloss) / sd:+.1f} sd)")
    assert abs(p_obs - p_exp) < 4 * sd
    assert abs(p_obs - p_noloss) > 6 * sd


@pytest.mark.parametrize("sp,T0,L,seed", [(I.ELECTRON, 2.0, 0.4, 51), (I.POSITRON, 2.0, 0.4, 52)])
def test_first_interaction_process_mix(oracle_mod, sp, T0, L, seed):
    """Which process acts first: the fraction of tracks whose first discrete
    interaction is process i is the integral of
    Sigma_i(E(s)) exp(-integral_0^s Sigma_tot) ds over the slab."""
    N = 300_000
    mask = I.P_CONT | I.P_EIONI | I.P_EBREM | (I.P_ANNIH if sp == I.POSITRON else 0)
    tabs = P_TABS if sp == I.POSITRON else E_TABS
    codes = [5, 6, 7] if sp == I.POSITRON else [4, 6]  # Bhabha, brems, annihilation / Moller, brems
    geo = I.single_slab(L, material=PB)
    o = oracle_mod.Oracle(geo, I.RunConfig(seed=seed, process_mask=mask))
    out = o.run(I.beam(N, sp, T0), n_events=N, log_cap=12 * N)
    assert out["n_log"] <= 12 * N
    log = out["log"]
    prim = log[(log["id"] == 0) & np.isin(log["process"], codes)]
    # first such step of each event's primary
    order = np.lexsort((prim["step"], prim["event"]))
    prim = prim[order]
    first = prim[np.r_[True, prim["event"][1:] != prim["event"][:-1]]]
    counts = np.array([(first["process"] == c).sum() for c in codes], dtype=np.float64)
    s, E, sig = csda_path(o, sp, T0, L, tabs)
    lam = integrate.cumulative_trapezoid(sig.sum(axis=0), s, initial=0.0)
    frac = np.array([integrate.trapezoid(sig[i] * np.exp(-lam), s) for i in range(len(tabs))])
    # the selection must also be distinguishable from picking by the
    # cross sections at the entry energy
    entry = np.array([o.lookup(0, t, T0) if T0 > th else 0.0 for t, th in tabs])
    frac_entry = (1 - math.exp(-L * entry.sum())) * entry / entry.sum()
    sd = np.sqrt(N * frac * (1 - frac))
    print("first interactions", counts, "expected", N * frac, "entry-energy", N * frac_entry)
    assert np.all(np.abs(counts - N * frac) < 4 * sd + 1)


# -------------------------------------------------------- collision loss
def n_electrons(m):
    return m[0] * m[2] * NA / m[1] * 1e-3  # per mm^3


def density_term(m, T):
    """asymptotic density-effect correction with the plasma energy
    28.816 eV sqrt(rho Z / A), clamped at zero (the reading of the restricted
    loss)"""
    g = T / ME + 1
    bg = math.sqrt(g * g - 1)
    hw = 28.816e-6 * math.sqrt(m[2] * m[0] / m[1])
    return max(0.0, 2 * math.log(hw / (m[3] * 1e-6)) + 2 * math.log(bg) - 1)


def unrestricted_icru37(m, T, positron):
    """ICRU Report 37 unrestricted collision stopping power of electrons
    (Moller) and positrons (Bhabha), MeV/mm"""
    tau = T / ME
    g = tau + 1
    b2 = 1 - 1 / (g * g)
    im = m[3] * 1e-6 / ME
    if positron:
        t2 = tau + 2
        F = 2 * math.log(2) - b2 / 12 * (23 + 14 / t2 + 10 / t2 ** 2 + 4 / t2 ** 3)
    else:
        F = 1 - b2 + (tau * tau / 8 - (2 * tau + 1) * math.log(2)) / (g * g)
    pref = 2 * math.pi * RE ** 2 * ME * n_electrons(m) / b2
    return pref * (math.log(tau * tau * (tau + 2) / (2 * im * im)) + F - density_term(m, T))


@pytest.mark.parametrize("mat", [PB, LAR])
@pytest.mark.parametrize("T", [0.01, 0.3, 2.0, 30.0, 1e3, 1e5])
def test_unrestricted_collision_loss_closed_forms(oracle_mod, mat, T):
    """The restricted Berger-Seltzer forms with the cut at the largest energy
    transfer (T/2 for identical electrons, T for positrons) equal the closed
    unrestricted ICRU 37 formulas, above and below the onset of the density
    effect (lead: T > 11 MeV, argon: T > 6.5 MeV)."""
    se = oracle_mod.formula("SION_E", mat, T / 2, T)
    sp = oracle_mod.formula("SION_P", mat, T, T)
    assert se == pytest.approx(unrestricted_icru37(mat, T, False), rel=1e-10)
    assert sp == pytest.approx(unrestricted_icru37(mat, T, True), rel=1e-10)
    if T >= 30.0:
        assert density_term(mat, T) > 0.0


def test_electron_positron_collision_loss_difference(oracle_mod):
    """Unrestricted e- minus e+ loss depends only on the Moller and Bhabha
    functions F-(tau) - F+(tau): the logarithm, the mean excitation energy
    and the density effect cancel.  The difference changes sign near
    tau = 1 (positrons lose more at low energy, electrons at high)."""
    for mat in (PB, LAR):
        for T in np.geomspace(0.005, 1e6, 25):
            tau = T / ME
            g = tau + 1
            b2 = 1 - 1 / (g * g)
            t2 = tau + 2
            fm = 1 - b2 + (tau * tau / 8 - (2 * tau + 1) * math.log(2)) / (g * g)
            fp = 2 * math.log(2) - b2 / 12 * (23 + 14 / t2 + 10 / t2 ** 2 + 4 / t2 ** 3)
            pref = 2 * math.pi * RE ** 2 * ME * n_electrons(mat) / b2
            d = oracle_mod.formula("SION_E", mat, T / 2, T) - oracle_mod.formula("SION_P", mat, T, T)
            assert d == pytest.approx(pref * (fm - fp), rel=1e-8, abs=1e-14)
    # limits of F- - F+: -2 ln 2 + ... at tau -> 0 is negative; 1/8 - 2 ln 2
    # + 23/12 + 2 ln 2 - ... -> positive at tau -> infinity
    assert oracle_mod.formula("SION_E", PB, 0.005, 0.01) < oracle_mod.formula("SION_P", PB, 0.01, 0.01)
    assert oracle_mod.formula("SION_E", PB, 5e3, 1e4) > oracle_mod.formula("SION_P", PB, 1e4, 1e4)


@pytest.mark.parametrize("mat,hw_eV", [(PB, 61.07), (LAR, 22.85)])
def test_restricted_loss_fermi_plateau(oracle_mod, mat, hw_eV):
    """With the asymptotic density effect the restricted loss saturates: as
    T -> infinity at fixed T_cut the logarithmic rise cancels and the loss
    tends to 2 pi r_e^2 m n_el ln(2 m T_cut / (hbar omega_p)^2), independent
    of the mean excitation energy (derived from the restricted Moller and
    Bhabha forms; plasma energies 61.07 eV for lead and 22.85 eV for liquid
    argon from 28.816 eV sqrt(rho Z/A)).  A wrong sign or coefficient of the
    density term, or a wrong plasma energy, fails this."""
    pref = 2 * math.pi * RE ** 2 * ME * n_electrons(mat)
    plateau = pref * math.log(2 * ME * TCUT / (hw_eV * 1e-6) ** 2)
    for which in ("SION_E", "SION_P"):
        for T in (1e6, 1e8):
            assert oracle_mod.formula(which, mat, TCUT, T) == pytest.approx(plateau, rel=2e-4)
        # and the approach is a saturation, not a rise: 100 TeV vs 1 TeV
        a, b = oracle_mod.formula(which, mat, TCUT, 1e6), oracle_mod.formula(which, mat, TCUT, 1e8)
        assert abs(b - a) < 1e-5 * a
    # changing I moves the loss at low energy but not the plateau
    heavy_I = (mat[0], mat[1], mat[2], mat[3] * 1.5)
    assert oracle_mod.formula("SION_E", heavy_I, TCUT, 1e8) == pytest.approx(plateau, rel=2e-4)
    assert oracle_mod.formula("SION_E", heavy_I, TCUT, 1.0) < 0.97 * oracle_mod.formula("SION_E", mat, TCUT, 1.0)


# -------------------------------------------------- step function and loss
@pytest.fixture(scope="module")
def cont_only_log(oracle_mod):
    """Tracks anywhere in the calorimeter with continuous loss only (no
    discrete process): every step is limited by the step function, a plane,
    a wall, or ends the track."""
    geo = I.calorimeter()
    cfg = I.RunConfig(seed=61, process_mask=I.P_CONT)
    o = oracle_mod.Oracle(geo, cfg)
    rng = np.random.default_rng(7)
    p = I.random_tracks(4000, 40, geo, 1e-3, 1.0, seed=62, species=I.ELECTRON)
    hi = rng.random(len(p)) < 0.5
    p["ekin"][hi] = np.exp(rng.uniform(math.log(1.0), math.log(1e4), hi.sum()))
    p["species"][rng.random(len(p)) < 0.5] = I.POSITRON
    out = o.run(p, n_events=40, log_cap=2_000_000)
    assert out["n_log"] <= 2_000_000
    return o, geo, out["log"]


def with_material(geo, log):
    """Material of the slab each step was taken in: the slab after the
    previous step of the same track (the step log is in stack order, each
    track's steps consecutive)."""
    log = log[log["species"] != I.GAMMA]
    log = np.sort(log, order=["event", "id", "species", "step"])
    prev_slab = np.empty(len(log), dtype=np.int64)
    prev_slab[1:] = log["slab_after"][:-1]
    first = np.r_[True, (log["event"][1:] != log["event"][:-1]) | (log["id"][1:] != log["id"][:-1]) |
                  (log["species"][1:] != log["species"][:-1])]
    keep = ~first & (prev_slab >= 0)
    log = log[keep]
    mat = geo.material[prev_slab[keep]]
    return log, mat


def test_step_function_properties(cont_only_log):
    """Steps limited by the step function (alpha = 0.2, rho = 1 mm):
    never longer than the range; a range at or below rho is taken in one step
    that stops the track; above rho the step lies between
    alpha R + rho (1 - alpha) and alpha R + 2 rho (1 - alpha), grows with R,
    tends to the fraction alpha of R for R >> rho, and to rho as R -> rho
    (continuity of the two branches)."""
    o, geo, log = cont_only_log
    alpha, rho = 0.2, 1.0
    log, mat = with_material(geo, log)
    cont = log["limiter"] == 3
    stop = log["limiter"] == 5
    sp = log["species"]
    R = np.array([o.lookup(int(m), "R_e-" if s == I.ELECTRON else "R_e+", e)
                  for m, s, e in zip(mat, sp, log["e_before"])])
    s = log["step_len"]
    assert cont.sum() > 1000 and stop.sum() > 1000
    # never beyond the range
    assert np.all(s <= R * (1 + 1e-12))
    # stopping steps of short ranges are exactly the range
    short = stop & (R <= rho)
    assert short.sum() > 100
    assert np.allclose(s[short], R[short], rtol=1e-12, atol=0)
    # no step-function-limited step where the range is at most rho
    assert not np.any(cont & (R <= rho * (1 - 1e-12)))
    rc, sc = R[cont], s[cont]
    assert np.all(sc >= alpha * rc + rho * (1 - alpha) * (1 - 1e-12))
    assert np.all(sc <= alpha * rc + 2 * rho * (1 - alpha) * (1 + 1e-12))
    # monotone in R
    k = np.argsort(rc)
    assert np.all(np.diff(sc[k]) >= -1e-12 * sc[k][1:])
    # s / R -> alpha for R >> rho, s -> rho for R -> rho
    big = rc > 200 * rho
    assert big.sum() > 10 and np.all(np.abs(sc[big] / rc[big] - alpha) < 2 * rho / rc[big])
    # continuity at R = rho: the step function is 1-Lipschitz there,
    # |s(R) - rho| <= R - rho
    near = (rc > rho) & (rc < 2 * rho)
    assert near.sum() > 20 and np.all(np.abs(sc[near] - rho) <= (rc[near] - rho) * (1 + 1e-9))


def test_continuous_loss_follows_the_range(cont_only_log):
    """Along any step the range decreases by the path length,
    R(E_after) = R(E_before) - s (the loss is the exact inverse of the range
    table for steps of at least 1% of the range); shorter steps lose s S(E)
    (linear loss), which differs from the range rule only at second order in
    s / R.  A step that reaches the range or leaves less than the tracking
    cut stops the track."""
    o, geo, log = cont_only_log
    log, mat = with_material(geo, log)
    sp = log["species"]
    rn = np.where(sp == I.ELECTRON, "R_e-", "R_e+")
    sn = np.where(sp == I.ELECTRON, "S_e-", "S_e+")
    alive = log["e_after"] > 0.0
    Rb = np.array([o.lookup(int(m), r, e) for m, r, e in zip(mat, rn, log["e_before"])])
    Sb = np.array([o.lookup(int(m), r, e) for m, r, e in zip(mat, sn, log["e_before"])])
    Ra = np.array([o.lookup(int(m), r, e) if e > 0 else 0.0 for m, r, e in zip(mat, rn, log["e_after"])])
    s = log["step_len"]
    longs = alive & (s >= 0.01 * Rb)
    shorts = alive & (s < 0.01 * Rb)
    assert longs.sum() > 1000 and shorts.sum() > 1000
    assert np.allclose(Ra[longs], Rb[longs] - s[longs], rtol=0, atol=1e-10 * Rb[longs].max())
    assert np.allclose(log["edep"][shorts], s[shorts] * Sb[shorts], rtol=1e-12, atol=0)
    # the deposit is the energy lost (tracks that leave the stack excepted)
    kept = (log["slab_after"] >= 0) | np.isin(log["limiter"], (5, 6))
    lost = (log["e_before"] - log["e_after"])[kept]
    assert np.all(np.abs(log["edep"][kept] - lost) <= 1e-14 * log["e_before"][kept])
    # stopped tracks: no kinetic energy left
    assert np.all(log["e_after"][log["limiter"] == 5] == 0.0)


# ------------------------------------------------------- null-collision bound
def bound_intervals(rng):
    """energy intervals [a, b] of a step: narrow and wide ones around every
    process threshold (brems 0.1, Bhabha 0.2, Moller 0.4 MeV) and random ones
    from 1 keV to 1 GeV"""
    ivs = []
    for th in (0.1, 0.2, 0.4):
        for w in (1e-4, 1e-3, 1e-2, 0.05, 0.3):
            for f in (0.1, 0.5, 0.9):
                ivs.append((th * (1 - w * f), th * (1 + w * (1 - f))))
    for _ in range(200):
        a = math.exp(rng.uniform(math.log(1e-3), math.log(1e3)))
        ivs.append((a, a * math.exp(rng.uniform(0.0, 1.5))))
    return ivs


@pytest.mark.parametrize("sp", [I.ELECTRON, I.POSITRON])
def test_null_collision_bound_is_the_maximum_over_the_step(cal_oracle, sp):
    """The thinning bound of a step whose energy spans [a, b] is the maximum
    of the interpolated discrete total over [a, b] (processes counted from
    their thresholds on): never below the largest value found by dense
    brute-force sampling of the interval (a lower bound would under-sample
    interactions), and not above it by more than the sampling resolution (a
    loose bound only costs null collisions, but the maximum is what the
    reading takes)."""
    rng = np.random.default_rng(71 + sp)
    for m in (0, 1):
        for a, b in bound_intervals(rng):
            xs = np.unique(np.r_[np.geomspace(a, b, 3001), a, b])
            dense = max(cal_oracle.sigma_total(m, sp, x) for x in xs)
            bound = cal_oracle.sigma_bound(m, sp, a, b)
            assert bound >= dense * (1 - 1e-12), (m, a, b, bound, dense)
            assert bound <= dense * (1 + 1e-3), (m, a, b, bound, dense)
