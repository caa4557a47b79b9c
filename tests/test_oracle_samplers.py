"""Pins of the oracle's interaction samplers.

Each sampler's histogram is compared (chi-square) with the differential cross
section it must follow -- those differentials are themselves pinned against
the closed-form totals in test_oracle_physics.py -- and every sample must
conserve energy and momentum exactly (to rounding).
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

ME = 0.51099895
N = 40000


def _samples(o, which, mat, E, n=N, key=(11, 5), direction=(0.3, -0.2, 0.9)):
    return np.array([o.sample(which, mat, E, key, t, 3, direction) for t in range(n)])


def _chi2(x, pdf, edges):
    counts, _ = np.histogram(x, edges)
    expect = np.array([integrate.quad(pdf, a, b, epsabs=0, epsrel=1e-10, limit=200)[0] for a, b in zip(edges[:-1], edges[1:])])
    expect *= counts.sum() / expect.sum()
    keep = expect > 5
    chi2 = ((counts[keep] - expect[keep]) ** 2 / expect[keep]).sum()
    return stats.chi2.sf(chi2, keep.sum() - 1)


def _unit(v):
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("E", [0.1, 2.0, 50.0])
def test_compton_sampler(cal_oracle, oracle_mod, E):
    s = _samples(cal_oracle, "compton", 0, E)
    eps0 = 1 / (1 + 2 * E / ME)
    pdf = lambda e: oracle_mod.formula("DSDE_COMPTON", (82.0, 207.2, 11.35, 823.0), 0, E, e)
    assert _chi2(s[:, 0], pdf, np.geomspace(eps0, 1, 41)) > 1e-3
    u = _unit(np.array([0.3, -0.2, 0.9]))
    for r in s[:200]:
        Eg, Te = r[2], r[6]
        assert Eg + Te == pytest.approx(E, rel=1e-14)
        pe = math.sqrt(Te * (Te + 2 * ME))
        assert np.allclose(E * u, Eg * r[3:6] + pe * r[7:10], rtol=0, atol=1e-12 * E)
        # photon scattering angle obeys the Compton relation
        cost = np.dot(u, r[3:6])
        assert Eg == pytest.approx(E / (1 + E / ME * (1 - cost)), rel=1e-9)


@pytest.mark.parametrize("E", [0.1, 2.0, 50.0])
def test_compton_angles_follow_klein_nishina(cal_oracle, E):
    """The scattering angle against the Klein-Nishina cross section per unit
    cos(theta), written here in its angular form (independent of the
    energy-fraction form the sampler uses): with P = E'/E = 1 / (1 +
    kappa (1 - cos)), dsigma/dcos is proportional to P^2 (P + 1/P - sin^2)."""
    s = _samples(cal_oracle, "compton", 0, E)
    u = _unit(np.array([0.3, -0.2, 0.9]))
    cost = np.clip(s[:, 3:6] @ u, -1.0, 1.0)
    kap = E / ME

    def kn(c):
        P = 1.0 / (1.0 + kap * (1.0 - c))
        return P * P * (P + 1.0 / P - (1.0 - c * c))
    assert _chi2(cost, kn, np.linspace(-1.0, 1.0, 41)) > 1e-3
    # the azimuth about the incoming direction is uniform
    ref = _unit(np.cross(u, [0.0, 0.0, 1.0]))
    ref2 = np.cross(u, ref)
    phi = np.arctan2(s[:, 3:6] @ ref2, s[:, 3:6] @ ref)
    counts, _ = np.histogram(phi, np.linspace(-math.pi, math.pi, 17))
    assert stats.chisquare(counts).pvalue > 1e-3


@pytest.mark.parametrize("E", [3.0, 40.0, 5000.0])
def test_pair_sampler(cal_oracle, oracle_mod, E):
    s = _samples(cal_oracle, "pair", 0, E)
    eps0 = ME / E
    pdf = lambda e: oracle_mod.formula("DSDE_PAIR", (82.0, 207.2, 11.35, 823.0), 0, E, e)
    assert _chi2(s[:, 0], pdf, np.linspace(eps0, 0.5, 31)) > 1e-3
    for r in s[:200]:
        assert r[2] == -1.0  # photon absorbed
        assert r[6] + r[10] + 2 * ME == pytest.approx(E, rel=1e-14)
    # which lepton takes eps is an unbiased coin
    fr = np.mean(s[:, 10] + ME > s[:, 6] + ME)
    frac_eps_to_positron = np.mean(np.isclose(s[:, 10] + ME, s[:, 0] * E, rtol=1e-12))
    assert abs(frac_eps_to_positron - 0.5) < 5 * 0.5 / math.sqrt(N)
    assert 0.4 < fr < 0.6


@pytest.mark.parametrize("T", [0.5, 30.0, 1e4])
def test_brems_sampler(cal_oracle, oracle_mod, T):
    s = _samples(cal_oracle, "brem", 1, T)
    pdf = lambda k: oracle_mod.formula("DSDK_BREM", (18.0, 39.948, 1.396, 188.0), 0.1, T, k)
    assert _chi2(s[:, 0], pdf, np.geomspace(0.1, T, 31)) > 1e-3
    for r in s[:200]:
        assert r[2] + r[6] == pytest.approx(T, rel=1e-14)


@pytest.mark.parametrize("T", [0.45, 5.0, 500.0])
def test_moller_sampler(cal_oracle, oracle_mod, T):
    s = _samples(cal_oracle, "moller", 0, T)
    pdf = lambda e: oracle_mod.formula("DSDE_MOLLER", (82.0, 207.2, 11.35, 823.0), 0, T, e)
    assert _chi2(s[:, 0], pdf, np.geomspace(0.2 / T, 0.5, 31)) > 1e-3
    u = _unit(np.array([0.3, -0.2, 0.9]))
    p = math.sqrt(T * (T + 2 * ME))
    for r in s[:200]:
        T1, Td = r[2], r[6]
        assert T1 + Td == pytest.approx(T, rel=1e-14)
        p1, pd = math.sqrt(T1 * (T1 + 2 * ME)), math.sqrt(Td * (Td + 2 * ME))
        assert np.allclose(p * u, p1 * r[3:6] + pd * r[7:10], rtol=0, atol=1e-10 * p)


@pytest.mark.parametrize("T", [0.25, 5.0, 500.0])
def test_bhabha_sampler(cal_oracle, oracle_mod, T):
    s = _samples(cal_oracle, "bhabha", 0, T)
    pdf = lambda e: oracle_mod.formula("DSDE_BHABHA", (82.0, 207.2, 11.35, 823.0), 0, T, e)
    assert _chi2(s[:, 0], pdf, np.geomspace(0.2 / T, 1.0, 31)) > 1e-3
    u = _unit(np.array([0.3, -0.2, 0.9]))
    p = math.sqrt(T * (T + 2 * ME))
    for r in s[:200]:
        T1, Td = r[2], r[6]
        assert T1 + Td == pytest.approx(T, rel=1e-14)
        p1, pd = math.sqrt(T1 * (T1 + 2 * ME)), math.sqrt(Td * (Td + 2 * ME))
        assert np.allclose(p * u, p1 * r[3:6] + pd * r[7:10], rtol=0, atol=1e-9 * p)


@pytest.mark.parametrize("T", [0.05, 3.0, 300.0])
def test_annihilation_sampler(cal_oracle, T):
    s = _samples(cal_oracle, "annih", 0, T)
    g = T / ME + 1
    sq = math.sqrt(g * g - 1)
    emin = 1 / (g + 1 + sq)

    def S(e):
        return -(g + 1) ** 2 + (g * g + 4 * g + 1) / e - 1 / e ** 2

    # Heitler's photon spectrum S(eps) + S(1 - eps) counts both photons; the
    # first photon alone follows S(eps), the second takes 1 - eps
    edges = np.geomspace(emin, 1 - emin, 31)
    assert _chi2(s[:, 0], S, edges) > 1e-3
    both = np.concatenate([s[:, 6], s[:, 10]]) / (T + 2 * ME)
    assert _chi2(both, lambda e: S(e) + S(1 - e), edges) > 1e-3
    u = _unit(np.array([0.3, -0.2, 0.9]))
    p = math.sqrt(T * (T + 2 * ME))
    for r in s[:200]:
        assert r[2] == -1.0
        assert r[6] + r[10] == pytest.approx(T + 2 * ME, rel=1e-14)
        assert np.allclose(p * u, r[6] * r[7:10] + r[10] * r[11:14], rtol=0, atol=1e-9 * (T + 2 * ME))


def test_samplers_use_consecutive_draws_from_index_two(cal_oracle, oracle_mod):
    # a Moller trial takes (a, b) = (U2, U3); the first accepted eps is
    # reproducible from those draws
    key = (3, 9)
    T, cut = 10.0, 0.2
    for t in range(50):
        r = cal_oracle.sample("moller", 0, T, key, t, 0)
        if r[1] == 1:
            a = oracle_mod.uniform(key, t, 0, 2)
            x = cut / T
            assert r[0] == pytest.approx(x / (1 - a * (1 - 2 * x)), rel=1e-15)
