"""Pins of the oracle's compound materials (lead tungstate, and compounds
that reduce to a single element).

A compound's per-atom cross sections are the sums of its elements' at their
partial atom densities (Bragg additivity), its per-electron ones scale with
its electron density, and pair production and bremsstrahlung pick their
target element in proportion to the partial cross sections.  The tests tie
each of these to something outside the compound code: separate
single-element contexts at the partial densities, the PDG electron density
and radiation length of PbWO4, exact reduction to the element, and the
sampled target frequencies.
"""
import math

import numpy as np
import pytest

import ems_inputs as I

NA = 6.02214076e23
PBWO4 = I.LEAD_TUNGSTATE
ELEMENTS = PBWO4[4]
M_FORMULA = sum(a * n for _, a, n in ELEMENTS)
ALPHA = 1 / 137.035999084
RE = 2.8179403262e-12


def partial(el, I_eV=PBWO4[3]):
    """element el of PbWO4 alone, at the density it has inside the compound"""
    z, a, n = el
    return (z, a, PBWO4[2] * n * a / M_FORMULA, I_eV)


def single_slab(mat, cfg):
    import oracle
    geo = I.single_slab(10.0, material=mat)
    return oracle.Oracle(geo, cfg)


CFG = I.RunConfig(seed=3)


@pytest.fixture(scope="module")
def compound_tables(oracle_mod):
    o = single_slab(PBWO4, CFG)
    t = o.tables()[0]
    o.close()
    return t


@pytest.fixture(scope="module")
def element_tables(oracle_mod):
    out = []
    for el in ELEMENTS:
        o = single_slab(partial(el), CFG)
        out.append(o.tables()[0])
        o.close()
    return out


def test_per_atom_and_per_electron_tables_add_over_elements(compound_tables, element_tables):
    import oracle
    for name in ("sigma_compton", "sigma_phot", "sigma_conv", "sigma_moller", "sigma_brem",
                 "sigma_bhabha", "sigma_annih"):
        k = oracle.TABLE_NAMES.index(name)
        ref = sum(t[k] for t in element_tables)
        np.testing.assert_allclose(compound_tables[k], ref, rtol=1e-13, atol=0, err_msg=name)


def test_stopping_power_is_compound_ionisation_plus_element_radiative_loss(oracle_mod, compound_tables):
    """S = collision loss with the compound's I and electron density + sum of
    the elements' sub-cut radiative losses, at every node"""
    import oracle
    nb = CFG.n_bins
    E = CFG.emin_MeV * (CFG.emax_MeV / CFG.emin_MeV) ** (np.arange(nb + 1) / nb)
    for name, which in (("S_e-", "SION_E"), ("S_e+", "SION_P")):
        k = oracle.TABLE_NAMES.index(name)
        for j in range(0, nb + 1, 7):
            ref = oracle_mod.formula(which, PBWO4, CFG.electron_cut_MeV, E[j]) + sum(
                oracle_mod.formula("SBREM", partial(el), CFG.gamma_cut_MeV, E[j]) for el in ELEMENTS)
            assert compound_tables[k][j] == pytest.approx(ref, rel=1e-12), (name, j)
    # collision loss depends on the material only through its electron
    # density, I and plasma energy: a single pseudo-element with the
    # atom-averaged Z and A (same <Z/A>) has the same
    pseudo = PBWO4[:4]
    for E in (0.3, 3.0, 300.0, 3e5):
        for which in ("SION_E", "SION_P"):
            assert oracle_mod.formula(which, PBWO4, CFG.electron_cut_MeV, E) == pytest.approx(
                oracle_mod.formula(which, pseudo, CFG.electron_cut_MeV, E), rel=1e-13)


def test_electron_density_matches_pdg(compound_tables):
    """Compton table / Klein-Nishina = electron density, PDG <Z/A> = 0.41315
    for PbWO4"""
    import oracle
    k = oracle.TABLE_NAMES.index("sigma_compton")
    E = 1.0
    nb = CFG.n_bins
    j = round(math.log(E / CFG.emin_MeV) / math.log(CFG.emax_MeV / CFG.emin_MeV) * nb)
    Ej = CFG.emin_MeV * (CFG.emax_MeV / CFG.emin_MeV) ** (j / nb)
    n_el = compound_tables[k][j] / oracle.formula("SIGMA_KN", PBWO4, 0, Ej)
    assert n_el == pytest.approx(PBWO4[2] * NA * 0.41315 * 1e-3, rel=1e-4)


def test_radiation_length_matches_pdg(compound_tables):
    """At 100 TeV the pair cross section is 7/9 of 1/X0 (complete screening,
    up to the small 1/54 term); PDG X0(PbWO4) = 0.8903 cm"""
    import oracle
    k = oracle.TABLE_NAMES.index("sigma_conv")
    sig = compound_tables[k][-1]  # top node, E = 1e8 MeV
    # the -1/54 term: sum_i n_i 4 a r_e^2 Z_i (Z_i + 1) / 54
    n_formula = PBWO4[2] * NA / M_FORMULA * 1e-3
    small = sum(n * n_formula * 4 * ALPHA * RE ** 2 * z * (z + 1) / 54 for z, _, n in ELEMENTS)
    x0 = 7 / 9 / (sig + small)
    assert x0 == pytest.approx(8.903, rel=0.03)


def test_one_element_compound_is_the_element(oracle_mod):
    """Lead written as a one-element compound: identical tables and
    identical histories (no extra draw)"""
    pb1 = I.compound(I.LEAD[2], I.LEAD[3], ((82, 207.2, 1),))
    geo_a = I.calorimeter(n_layers=4)
    geo_b = I.calorimeter(n_layers=4, absorber=pb1)
    a = oracle_mod.Oracle(geo_a, CFG)
    b = oracle_mod.Oracle(geo_b, CFG)
    assert np.array_equal(a.tables(), b.tables())
    prim = I.beam(6, I.ELECTRON, 2000.0, seed=5)
    ra, rb = a.run(prim), b.run(prim)
    assert np.array_equal(ra["edep"], rb["edep"])
    assert np.array_equal(ra["ledger"], rb["ledger"])
    a.close()
    b.close()


def test_split_element_selection_frequencies(oracle_mod):
    """Lead split into two 'elements' of 1 and 3 atoms: tables equal lead's
    (to rounding) and the target is element 1 three times in four, at any
    energy"""
    split = I.compound(I.LEAD[2], I.LEAD[3], ((82, 207.2, 1), (82, 207.2, 3)))
    a = single_slab(I.LEAD, CFG)
    b = single_slab(split, CFG)
    np.testing.assert_allclose(b.tables(), a.tables(), rtol=1e-13, atol=0)
    n = 4000
    for which, E in (("pair", 20.0), ("pair", 5e4), ("brem", 3.0), ("brem", 1e4)):
        idx = np.array([b.sample(which, 0, E, (11, 12), i, 0)[15] for i in range(n)])
        assert set(np.unique(idx)) <= {0.0, 1.0}
        f = idx.mean()
        assert abs(f - 0.75) < 5 * math.sqrt(0.75 * 0.25 / n), (which, E, f)
    a.close()
    b.close()


@pytest.mark.parametrize("which", ["pair", "brem"])
def test_pbwo4_selection_follows_partial_cross_sections(oracle_mod, which):
    o = single_slab(PBWO4, CFG)
    E = 1000.0
    fn = "SIGMA_PAIR" if which == "pair" else "SIGMA_BREM"
    w = []
    for el in ELEMENTS:
        m = partial(el)
        nat = m[2] * NA / m[1] * 1e-3
        w.append(nat * oracle_mod.formula(fn, m, CFG.gamma_cut_MeV, E))
    p = np.array(w) / sum(w)
    n = 6000
    idx = np.array([o.sample(which, 0, E, (21, 22), i, 0)[15] for i in range(n)]).astype(int)
    cnt = np.bincount(idx, minlength=3)
    # interpolation between log nodes moves the fractions by far less than
    # the statistical band
    for k in range(3):
        assert abs(cnt[k] / n - p[k]) < 5 * math.sqrt(p[k] * (1 - p[k]) / n) + 1e-3, (k, cnt, p)
    o.close()


def test_pbwo4_calorimeter_energy_closure(oracle_mod):
    """energy in = deposited + escaped + killed on the PbWO4 / lAr stack"""
    geo = I.calorimeter(n_layers=10, absorber=PBWO4)
    o = oracle_mod.Oracle(geo, CFG)
    prim = I.beam(8, I.ELECTRON, 1000.0, seed=9)
    r = o.run(prim)
    led = r["ledger"]
    # rest energy: +2 m_e per pair created, -2 m_e per annihilation
    tot = led["edep"] + led["escaped"].sum(axis=1) + led["killed"] + \
        2 * 0.51099895 * (led["n_pair"].astype(np.int64) - led["n_annih"].astype(np.int64))
    np.testing.assert_allclose(tot, 1000.0, rtol=1e-9)
    np.testing.assert_allclose(r["edep"].sum(axis=1), led["edep"], rtol=1e-12)
    o.close()
