"""Helpers for comparing step logs and tallies between two transport runs."""
import numpy as np

ME = 0.51099895


def sort_log(log):
    order = np.lexsort((log["step"], log["id"], log["event"]))
    return log[order]


def compare_logs(a, b, e_rtol=1e-9, pos_atol=1e-7, dep_rtol=None):
    """Step-by-step comparison of two step logs (any order).  Energies after
    the step to e_rtol and deposits to dep_rtol (default e_rtol), both
    relative to the energy before the step; positions to pos_atol.  Returns a
    dict with the number of steps and the largest energy, deposit and
    position differences; raises AssertionError with the first divergence."""
    dep_rtol = e_rtol if dep_rtol is None else dep_rtol
    a, b = sort_log(a), sort_log(b)
    assert len(a) == len(b), f"step counts differ: {len(a)} vs {len(b)}"
    for f in ("event", "species", "id", "step", "slab_after", "limiter", "process"):
        bad = np.nonzero(a[f] != b[f])[0]
        assert len(bad) == 0, f"field {f} differs first at sorted step {bad[0]}: {a[bad[0]]} vs {b[bad[0]]}"
    scale = np.maximum(np.abs(a["e_before"]), 1e-3)
    de = np.max(np.abs(a["e_after"] - b["e_after"]) / scale) if len(a) else 0.0
    dd = np.max(np.abs(a["edep"] - b["edep"]) / scale) if len(a) else 0.0
    dp = np.max(np.abs(a["pos_after"] - b["pos_after"])) if len(a) else 0.0
    assert de <= e_rtol and dd <= dep_rtol, f"energy differs: {de}, deposit differs: {dd}"
    assert dp <= pos_atol, f"position differs: {dp}"
    return dict(n=len(a), de=de, dd=dd, dp=dp)


def ledger_residual(edep, ledger, prim):
    ein = np.bincount(prim["event"], weights=prim["ekin"], minlength=len(ledger))
    out = edep.sum(axis=1) + ledger["escaped"].sum(axis=1) + ledger["killed"] + \
        2 * ME * (ledger["n_pair"].astype(np.int64) - ledger["n_annih"].astype(np.int64))
    return np.abs(out - ein) / np.maximum(ein, 1e-300)


def tiny_mixed_primaries(n_each=16, E=10.0):
    """16 events of each species at 10 MeV along +z from the front face."""
    import ems_inputs as I
    p = I.primaries(3 * n_each)
    p["event"] = np.arange(3 * n_each)
    p["species"] = np.repeat([I.GAMMA, I.ELECTRON, I.POSITRON], n_each)
    p["ekin"] = E
    p["dir"] = [0.0, 0.0, 1.0]
    return p


def mixed_precision_check(edep_m, ledger_m, edep_o, ledger_o, prim, n_layers=50):
    """The mixed form against the FP64 oracle on the same events: energy
    conservation per event to 1e-5, per-species secondary counts to the
    per-mil level, per-layer mean deposits within 3 sigma + 0.5%.  Returns the
    per-layer relative error of the mean (and its statistical error)."""
    n = edep_m.shape[0]
    assert ledger_residual(edep_m, ledger_m, prim).max() < 1e-5
    cm = np.asarray(ledger_m["n_created"], dtype=np.float64).sum(axis=0)
    co = np.asarray(ledger_o["n_created"], dtype=np.float64).sum(axis=0)
    assert np.all(np.abs(cm - co) <= 1e-3 * co + 2), (cm, co)
    lm = edep_m.reshape(n, n_layers, -1).sum(axis=2)
    lo = edep_o.reshape(n, n_layers, -1).sum(axis=2)
    mm, mo = lm.mean(axis=0), lo.mean(axis=0)
    sig = np.sqrt(lm.var(axis=0) / n + lo.var(axis=0) / n)
    assert np.all(np.abs(mm - mo) <= 3 * sig + 0.005 * np.abs(mo) + 1e-9)
    live = mo > 1e-3 * mo.max()
    rel = (mm - mo)[live] / mo[live]
    return dict(rel=rel, stat=(sig[live] / mo[live]), rms=float(np.sqrt(np.mean(rel ** 2))),
                max=float(np.abs(rel).max()))


def compare_exits(a, b, e_rtol=1e-9, pos_atol=1e-7, dir_atol=1e-9):
    """Two lists of outgoing tracks (primary records) as multisets: same
    count per (event, species) and, sorted by energy, the same energies,
    exit points and directions within the tolerances."""
    assert len(a) == len(b), (len(a), len(b))
    def order(x):
        # equal energies occur (both photons of an annihilation at rest):
        # ties are broken by the exit point, all coarsened far above the
        # tolerances so that rounding differences cannot reorder
        e = np.round(np.log(x["ekin"]) * 1e6)
        p = np.round(x["pos"] * 1e4)
        return np.lexsort((p[:, 2], p[:, 1], p[:, 0], e, x["species"], x["event"]))
    ka, kb = order(a), order(b)
    a, b = a[ka], b[kb]
    assert np.array_equal(a["event"], b["event"]) and np.array_equal(a["species"], b["species"])
    assert np.allclose(a["ekin"], b["ekin"], rtol=e_rtol, atol=0.0)
    assert np.allclose(a["pos"], b["pos"], rtol=0.0, atol=pos_atol)
    assert np.allclose(a["dir"], b["dir"], rtol=0.0, atol=dir_atol)
