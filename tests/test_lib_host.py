"""CPU checks of the GPU library: the shared object loads and exports every
entry point of include/ems.h, its independently built tables agree with the
oracle's, its argument validation rejects bad input, and its per-track step
code (run on the host through the test hook, never by ems_run) reproduces the
oracle's histories step by step."""
import os
import re

import numpy as np
import pytest

import ems_inputs as I
from parity_util import compare_logs, ledger_residual, tiny_mixed_primaries

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def E():
    import paper_2209_15445_amd as E
    E.lib()
    return E


def header_functions():
    txt = open(os.path.join(ROOT, "include", "ems.h")).read()
    return sorted(set(re.findall(r"^\s*(?:ems_status|const char\*|uint32_t)\s+(ems_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_entry_point(E):
    names = header_functions()
    assert len(names) >= 26
    for n in names:
        assert hasattr(E.lib(), n), n
    assert E.lib().ems_abi_version() == E.ABI_VERSION


@pytest.mark.parametrize("mask", [I.P_ALL, I.P_CONT | I.P_COMPTON, 0])
def test_tables_agree_with_oracle(E, oracle_mod, mask):
    geo = I.calorimeter()
    cfg = I.RunConfig(process_mask=mask)
    lt = E.host_tables(E.make_config(cfg, 1), geo)
    ot = oracle_mod.Oracle(geo, cfg).tables()
    assert np.array_equal(lt == 0, ot == 0)
    nz = ot != 0
    assert np.max(np.abs(lt[nz] - ot[nz]) / np.abs(ot[nz])) < 1e-12


def _bad(E, cfg, geo):
    import ctypes as C
    gh = E._GeoHolder(geo)
    n = C.c_uint64()
    return E.lib().ems_workspace_bytes(C.byref(cfg), C.byref(gh.g), C.byref(n))


def test_config_and_geometry_validation(E):
    geo = I.calorimeter()
    good = E.make_config(I.RunConfig(), 4)
    assert _bad(E, good, geo) == E.OK
    c = E.make_config(I.RunConfig(), 4)
    c.abi_version = 99
    assert _bad(E, c, geo) == E.E_VERSION
    for field, val in (("n_bins", 1), ("emin_MeV", -1.0), ("max_events", 0), ("track_capacity", 3),
                       ("max_steps_per_track", 0), ("lin_loss_limit", 1.5), ("precision", 7),
                       ("refill_below", 64), ("interact_min", 65), ("photon_steps_per_visit", 0),
                       ("photon_refill_below", 64), ("short_electron_MeV", -1.0),
                       ("short_electron_MeV", float("nan"))):
        c = E.make_config(I.RunConfig(), 4)
        setattr(c, field, val)
        assert _bad(E, c, geo) == E.E_INVALID, field
    g2 = I.calorimeter()
    g2.z_mm = g2.z_mm.copy()
    g2.z_mm[5] = g2.z_mm[4]
    assert _bad(E, good, g2) == E.E_INVALID
    g3 = I.calorimeter()
    g3.material = g3.material.copy()
    g3.material[0] = 7
    assert _bad(E, good, g3) == E.E_INVALID


def test_workspace_grows_with_capacity_and_events(E):
    geo = I.calorimeter()

    def ws(n, cap, short):
        return E.workspace_bytes(E.make_config(I.RunConfig(), n, track_capacity=cap, short_electron_MeV=short), geo)
    a, b, c = ws(10, 1024, 0.0), ws(10, 2048, 0.0), ws(1000, 1024, 0.0)
    assert b - a == 6 * 1024 * 76
    assert c > a and a % 256 == 0
    # short electrons: two buffers of half the capacity and a spill buffer of
    # 5/8 of it
    assert ws(10, 1024, 1.0) - a == (2 * 512 + 640) * 76
    assert ws(10, 2048, 1.0) - ws(10, 1024, 1.0) == (6 * 1024 + 2 * 512 + 640) * 76


def test_invalid_primaries_rejected_by_host_path(E):
    geo, cfg, prim = I.workload("cal_1GeV_e-_x32")
    c = E.make_config(cfg, 4)
    for field, val in (("ekin", 0.0), ("ekin", np.inf), ("species", 5), ("event", 9)):
        bad = prim[:3].copy()
        bad[field][2] = val
        with pytest.raises(E.EmsError) as ei:
            E.debug_host_transport(c, geo, bad, 4)
        assert ei.value.code == E.E_INVALID


@pytest.mark.parametrize("bz", [0.0, 3.8])
def test_host_step_code_history_parity(E, oracle_mod, bz):
    """Every step of 48 tracks (16 each gamma/e-/e+ at 10 MeV) equal to the
    oracle's, with and without field."""
    geo = I.calorimeter()
    cfg = I.RunConfig(seed=11, bz_tesla=bz)
    prim = tiny_mixed_primaries()
    h = E.debug_host_transport(E.make_config(cfg, 48), geo, prim, 48, log_cap=200000)
    r = oracle_mod.Oracle(geo, cfg).run(prim, log_cap=200000)
    st = compare_logs(h["log"], r["log"], e_rtol=1e-10, pos_atol=1e-8)
    assert st["n"] == r["n_log"]
    assert np.allclose(h["edep"], r["edep"], rtol=1e-10, atol=1e-10)
    for f in ("n_steps", "n_created", "n_null", "n_pair", "n_annih"):
        assert np.array_equal(h["ledger"][f], r["ledger"][f]), f
    assert ledger_residual(h["edep"], h["ledger"], prim).max() < 1e-12


def test_host_step_code_random_tracks(E, oracle_mod):
    """Isotropic tracks anywhere in the stack (backward and grazing
    directions, all species, 1 keV-50 MeV) with field."""
    geo = I.calorimeter()
    cfg = I.RunConfig(seed=5, bz_tesla=3.8)
    prim = I.random_tracks(300, 20, geo, 1e-3, 50.0, seed=8)
    h = E.debug_host_transport(E.make_config(cfg, 20), geo, prim, 20, log_cap=200000)
    r = oracle_mod.Oracle(geo, cfg).run(prim, n_events=20, log_cap=200000)
    compare_logs(h["log"], r["log"], e_rtol=1e-10, pos_atol=1e-8)


def test_host_step_code_1gev_showers(E, oracle_mod):
    geo, cfg, prim = I.workload("cal_1GeV_e-_x32")
    h = E.debug_host_transport(E.make_config(cfg, 6), geo, prim[:6], 6)
    r = oracle_mod.Oracle(geo, cfg).run(prim[:6])
    assert np.array_equal(h["ledger"]["n_steps"], r["ledger"]["n_steps"])
    assert np.allclose(h["edep"], r["edep"], rtol=1e-9, atol=1e-9)


def test_host_step_code_event_keys(E, oracle_mod):
    geo, cfg, prim = I.workload("cal_1GeV_e-_x32")
    p = prim[:2].copy()
    keys = np.array([17, 4242], dtype=np.uint32)
    h = E.debug_host_transport(E.make_config(cfg, 2), geo, p, 2, keys=keys)
    r = oracle_mod.Oracle(geo, cfg).run(p, n_events=2, event_keys=keys)
    assert np.allclose(h["edep"], r["edep"], rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("case", ["1GeV_e-", "mixed_species_bz3.8"])
def test_host_mixed_precision_against_fp64_oracle(E, oracle_mod, case):
    """The mixed form (FP32 tables, step lengths and sampling; FP64 positions,
    boundaries and energies) on the host: conservation 1e-5, secondary counts
    per-mil, per-layer means within 3 sigma + 0.5% of the FP64 oracle."""
    from parity_util import mixed_precision_check
    if case == "1GeV_e-":
        geo, cfg, prim = I.workload("cal_1GeV_e-_x32")
    else:
        geo = I.calorimeter()
        cfg = I.RunConfig(seed=3, bz_tesla=3.8)
        prim = I.mixed_species(24, 1e3, 5e3, seed=3)
    n = len(prim)
    h = E.debug_host_transport(E.make_config(cfg, n, precision=E.MIXED), geo, prim, n)
    r = oracle_mod.Oracle(geo, cfg).run(prim, n_events=n)
    rep = mixed_precision_check(h["edep"], h["ledger"], r["edep"], r["ledger"], prim)
    assert rep["rms"] < 0.01


# ---------------------------------------------------------------- compounds
def test_compound_tables_agree_with_oracle(E, oracle_mod):
    geo = I.calorimeter(absorber=I.LEAD_TUNGSTATE)
    for mask in (I.P_ALL, I.P_CONV | I.P_EBREM | I.P_CONT):
        cfg = I.RunConfig(process_mask=mask)
        lt = E.host_tables(E.make_config(cfg, 1), geo)
        ot = oracle_mod.Oracle(geo, cfg).tables()
        assert np.array_equal(lt == 0, ot == 0)
        nz = ot != 0
        assert np.max(np.abs(lt[nz] - ot[nz]) / np.abs(ot[nz])) < 1e-12


def test_compound_validation(E):
    good = E.make_config(I.RunConfig(), 4)
    assert _bad(E, good, I.calorimeter(absorber=I.LEAD_TUNGSTATE)) == E.OK
    bad_mats = [
        I.compound(8.3, 600.7, ((82, 207.2, 1), (74, 183.84, 1), (8, 16.0, 4), (1, 1.0, 1), (2, 4.0, 1))),
        (82.0, 207.2, 8.3, 600.7, ((82.0, 207.2, 0.0),)),
        I.compound(8.3, 600.7, ((0.5, 207.2, 1),)),
        I.compound(8.3, 600.7, ((82, -1.0, 1),)),
        I.compound(0.0, 600.7, ((82, 207.2, 1),)),
    ]
    for m in bad_mats:
        assert _bad(E, good, I.calorimeter(absorber=m)) == E.E_INVALID, m


@pytest.mark.parametrize("bz", [0.0, 3.8])
def test_host_step_code_history_parity_pbwo4(E, oracle_mod, bz):
    """Every step of 48 tracks in the lead tungstate stack (element selection
    on pair production and bremsstrahlung) equal to the oracle's"""
    geo = I.calorimeter(absorber=I.LEAD_TUNGSTATE)
    cfg = I.RunConfig(seed=13, bz_tesla=bz)
    prim = tiny_mixed_primaries()
    prim["ekin"] *= 30.0
    h = E.debug_host_transport(E.make_config(cfg, 48), geo, prim, 48, log_cap=400000)
    r = oracle_mod.Oracle(geo, cfg).run(prim, log_cap=400000)
    st = compare_logs(h["log"], r["log"], e_rtol=1e-10, pos_atol=1e-8)
    assert st["n"] == r["n_log"]
    assert r["ledger"]["n_pair"].sum() > 5
    assert np.allclose(h["edep"], r["edep"], rtol=1e-10, atol=1e-10)
    for f in ("n_steps", "n_created", "n_null", "n_pair", "n_annih"):
        assert np.array_equal(h["ledger"][f], r["ledger"][f]), f
    assert ledger_residual(h["edep"], h["ledger"], prim).max() < 1e-12


def test_host_step_code_1gev_showers_pbwo4(E, oracle_mod):
    geo, cfg, prim = I.workload("calPbWO4_1GeV_e-_x32")
    h = E.debug_host_transport(E.make_config(cfg, 6), geo, prim[:6], 6)
    r = oracle_mod.Oracle(geo, cfg).run(prim[:6])
    assert np.array_equal(h["ledger"]["n_steps"], r["ledger"]["n_steps"])
    assert np.allclose(h["edep"], r["edep"], rtol=1e-9, atol=1e-9)


# ---------------------------------------------------------------- along-step processes
@pytest.mark.parametrize("bz", [0.0, 3.8])
def test_host_step_code_history_parity_msc_fluct(E, oracle_mod, bz):
    """multiple scattering and loss fluctuations on: every step of 48
    tracks (and the PbWO4 stack for the compound radiation length) equal to
    the oracle's"""
    for absorber in (I.LEAD, I.LEAD_TUNGSTATE):
        geo = I.calorimeter(absorber=absorber)
        cfg = I.RunConfig(seed=17, bz_tesla=bz, process_mask=I.P_ALL | I.P_MSC | I.P_FLUCT)
        prim = tiny_mixed_primaries()
        prim["ekin"] *= 10.0
        h = E.debug_host_transport(E.make_config(cfg, 48), geo, prim, 48, log_cap=400000)
        r = oracle_mod.Oracle(geo, cfg).run(prim, log_cap=400000)
        # a gamma draw of small shape k scales by u^(1/k), which multiplies
        # the rounding difference of k by up to ~1/k: energies to 1e-9
        st = compare_logs(h["log"], r["log"], e_rtol=1e-9, pos_atol=1e-8)
        assert st["n"] == r["n_log"]
        assert np.allclose(h["edep"], r["edep"], rtol=1e-9, atol=1e-9)
        for f in ("n_steps", "n_created", "n_null", "n_pair", "n_annih"):
            assert np.array_equal(h["ledger"][f], r["ledger"][f]), f
        assert ledger_residual(h["edep"], h["ledger"], prim).max() < 1e-12


def test_unknown_process_bits_rejected(E):
    c = E.make_config(I.RunConfig(process_mask=I.P_ALL | I.P_MSC | I.P_FLUCT), 4)
    assert _bad(E, c, I.calorimeter()) == E.OK
    c = E.make_config(I.RunConfig(process_mask=I.P_ALL | (1 << 9)), 4)
    assert _bad(E, c, I.calorimeter()) == E.E_INVALID


# ---------------------------------------------------------------- box geometry
def _box_parity(E, oracle_mod, geo, cfg, prim, n_events, e_rtol=1e-10):
    h = E.debug_host_transport(E.make_config(cfg, n_events), geo, prim, n_events, log_cap=1_000_000)
    r = oracle_mod.Oracle(geo, cfg).run(prim, n_events=n_events, log_cap=1_000_000)
    st = compare_logs(h["log"], r["log"], e_rtol=e_rtol, pos_atol=1e-8)
    assert st["n"] == r["n_log"]
    assert np.allclose(h["edep"], r["edep"], rtol=e_rtol, atol=e_rtol)
    for f in ("n_steps", "n_created", "n_null", "n_pair", "n_annih"):
        assert np.array_equal(h["ledger"][f], r["ledger"][f]), f
    assert ledger_residual(h["edep"], h["ledger"], prim).max() < 1e-12
    return h, r


@pytest.mark.parametrize("mask", [I.P_ALL, I.P_ALL | I.P_MSC | I.P_FLUCT])
def test_host_box_navigation_matches_brute_force_oracle(E, oracle_mod, mask):
    """the step code walking the hierarchy (towers with cracks of world
    material) against the oracle's walk over all boxes, step by step"""
    geo = I.towers(cells=5, n_layers=10)
    cfg = I.RunConfig(seed=23, process_mask=mask)
    prim = tiny_mixed_primaries()
    prim["ekin"] *= 20.0
    rng = np.random.default_rng(2)
    prim["pos"][:, 0] = rng.uniform(-70, 70, len(prim))
    prim["pos"][:, 1] = rng.uniform(-70, 70, len(prim))
    h, r = _box_parity(E, oracle_mod, geo, cfg, prim, 48, e_rtol=1e-9 if mask & I.P_FLUCT else 1e-10)
    assert h["edep"][:, -1].sum() > 0.0  # the cracks were crossed


def test_host_box_random_tracks(E, oracle_mod):
    geo = I.towers(cells=5, n_layers=10)
    cfg = I.RunConfig(seed=24)
    rng = np.random.default_rng(5)
    n = 300
    prim = I.primaries(n)
    prim["event"] = rng.integers(0, 20, n)
    prim["species"] = rng.integers(0, 3, n)
    prim["ekin"] = np.exp(rng.uniform(np.log(1e-3), np.log(50.0), n))
    prim["pos"] = rng.uniform(np.array(geo.world_lo) * 0.999, np.array(geo.world_hi) * 0.999 + [0, 0, 0.0], (n, 3))
    prim["pos"][:, 2] = rng.uniform(0.0, geo.world_hi[2], n)
    d = rng.normal(size=(n, 3))
    prim["dir"] = d / np.linalg.norm(d, axis=1)[:, None]
    _box_parity(E, oracle_mod, geo, cfg, prim, 20)


def test_host_box_9x9_towers_showers(E, oracle_mod):
    """8100 boxes (13-bit volume indices): 1 GeV showers equal to the oracle's"""
    geo = I.towers()
    assert geo.n_boxes == 8100
    cfg = I.RunConfig(seed=25)
    prim = I.beam(4, I.ELECTRON, 1000.0, smear_rad=1e-3, seed=3)
    prim["pos"][:, 0] = [0.0, 19.7, -19.9, 5.0]
    _box_parity(E, oracle_mod, geo, cfg, prim, 4)


@pytest.mark.parametrize("mask", [I.P_ALL, I.P_ALL | I.P_MSC | I.P_FLUCT])
def test_host_box_navigation_in_a_field_matches_the_oracle(E, oracle_mod, mask):
    """charged tracks on the helix through towers and cracks (the step code's
    crossings found through the hierarchy) against the oracle's crossings
    over all boxes, step by step, at 3.8 T"""
    geo = I.towers(cells=5, n_layers=10)
    cfg = I.RunConfig(seed=33, bz_tesla=3.8, process_mask=mask)
    prim = tiny_mixed_primaries()
    prim["ekin"] *= 20.0
    rng = np.random.default_rng(12)
    prim["pos"][:, 0] = rng.uniform(-70, 70, len(prim))
    prim["pos"][:, 1] = rng.uniform(-70, 70, len(prim))
    d = rng.normal(size=(len(prim), 3))
    d[:, 2] = np.abs(d[:, 2]) + 0.3
    prim["dir"] = d / np.linalg.norm(d, axis=1)[:, None]
    h, r = _box_parity(E, oracle_mod, geo, cfg, prim, 48, e_rtol=1e-9)
    log = r["log"][: r["n_log"]]
    assert np.any((log["species"] != 0) & (log["slab_after"] == geo.n_boxes))  # charged steps in the cracks


def test_host_box_random_tracks_in_a_field(E, oracle_mod):
    geo = I.towers(cells=5, n_layers=10)
    cfg = I.RunConfig(seed=34, bz_tesla=3.8)
    rng = np.random.default_rng(6)
    n = 300
    prim = I.primaries(n)
    prim["event"] = rng.integers(0, 20, n)
    prim["species"] = rng.integers(0, 3, n)
    prim["ekin"] = np.exp(rng.uniform(np.log(1e-2), np.log(50.0), n))
    prim["pos"] = rng.uniform(np.array(geo.world_lo) * 0.999, np.array(geo.world_hi) * 0.999, (n, 3))
    prim["pos"][:, 2] = rng.uniform(0.0, geo.world_hi[2], n)
    d = rng.normal(size=(n, 3))
    prim["dir"] = d / np.linalg.norm(d, axis=1)[:, None]
    _box_parity(E, oracle_mod, geo, cfg, prim, 20, e_rtol=1e-9)


def test_box_validation(E):
    good = E.make_config(I.RunConfig(), 4)
    geo = I.towers(cells=3, n_layers=2)
    assert _bad(E, good, geo) == E.OK
    g = I.towers(cells=3, n_layers=2)
    g.hi = g.hi.copy()
    g.hi[0, 0] += 50.0
    assert _bad(E, good, g) == E.E_INVALID
    g = I.towers(cells=3, n_layers=2)
    g.material = g.material.copy()
    g.material[1] = 5
    assert _bad(E, good, g) == E.E_INVALID
    assert _bad(E, E.make_config(I.RunConfig(bz_tesla=1.0), 4), geo) == E.OK  # a field is taken
    big = I.towers(cells=9, n_layers=50)
    assert _bad(E, E.make_config(I.RunConfig(max_steps_per_track=(1 << 19) - 1), 4), big) == E.OK
    assert _bad(E, E.make_config(I.RunConfig(max_steps_per_track=1 << 19), 4), big) == E.E_INVALID
    p = I.beam(2, I.ELECTRON, 10.0)
    p["pos"][1] = (1e4, 0.0, 0.0)
    with pytest.raises(E.EmsError):
        E.debug_host_transport(good, geo, p, 2)


def test_ctypes_structs_match_the_header(E, tmp_path):
    """Every field of the binding's structs sits at the offset the C header
    gives it (a C program built against include/ems.h prints them)."""
    import ctypes as C
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    structs = {"ems_material": E.Material, "ems_geometry": E.Geometry, "ems_config": E.Config,
               "ems_run_stats": E.RunStats, "ems_server_info": E.ServerInfo}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "ems.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    # the numpy record types of the read-back calls: C struct, dtype, C field
    # name of each dtype field in order
    records = {"ems_ledger": (E.LEDGER_DTYPE, [n for n in E.LEDGER_DTYPE.names]),
               "ems_primary": (E.PRIMARY_DTYPE, ["event", "species", "ekin_MeV", "pos_mm", "dir"]),
               "ems_step_record": (E.STEP_DTYPE, [n for n in E.STEP_DTYPE.names])}
    for cname, (dt, cfields) in records.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for cf in cfields:
            lines.append(f'  printf("{cname} {cf} %zu\\n", offsetof({cname}, {cf}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == C.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])
    for cname, (dt, cfields) in records.items():
        assert got[(cname, "sizeof")] == dt.itemsize, cname
        for name, cf in zip(dt.names, cfields):
            assert got[(cname, cf)] == dt.fields[name][1], (cname, cf)


def test_static_workspace_refuses_a_configuration_beyond_its_size(E):
    # checked before any HIP call: runs without a GPU
    import ctypes as C
    geo, cfg, _ = I.workload("cal_1GeV_e-_x32")
    big = E.make_config(cfg, 32, track_capacity=1 << 20)
    gh = E._GeoHolder(geo)
    h = C.c_void_p()
    rc = E.lib().ems_create_static(C.byref(big), C.byref(gh.g), None, C.byref(h))
    assert rc == E.E_CAPACITY and h.value is None
    msg = E.lib().ems_last_error().decode()
    assert "static workspace holds" in msg and str(64 << 20) in msg
    bad = E.make_config(cfg, 32, track_capacity=1 << 14)
    bad.abi_version = 1
    assert E.lib().ems_create_static(C.byref(bad), C.byref(gh.g), None, C.byref(h)) == E.E_VERSION


def test_range_table_inverse_finds_the_node_of_a_one_by_one_walk(tmp_path):
    """The strided walk of the range-table inverse (the step code's
    inverse_range, compiled for the host) against a plain walk down the
    table, node by node, for walks of every length up to the whole table."""
    import shutil
    import subprocess
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = tmp_path / "step_scans_check"
    subprocess.run([hipcc, "-O1", "-std=c++17", "-I", os.path.join(root, "paper_2209_15445_amd", "csrc"),
                    os.path.join(root, "tests", "step_scans_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    lines = r.stdout.strip().split("\n")
    assert r.returncode == 0, r.stdout
    assert lines[-2].startswith("double:") and lines[-1].startswith("float:")
    for line in lines[-2:]:
        assert line.endswith(" 0 mismatches") and int(line.split()[1]) > 4_000_000
