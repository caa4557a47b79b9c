"""Helpers for comparing step logs and tallies between two transport runs."""
import numpy as np

ME = 0.51099895


def sort_log(log):
    order = np.lexsort((log["step"], log["id"], log["event"]))
    return log[order]


def compare_logs(a, b, e_rtol=1e-9, pos_atol=1e-7):
    """Step-by-step comparison of two step logs (any order).  Returns a dict
    with the number of steps, integer mismatches and the largest energy and
    position differences; raises AssertionError with the first divergence."""
    a, b = sort_log(a), sort_log(b)
    assert len(a) == len(b), f"step counts differ: {len(a)} vs {len(b)}"
    for f in ("event", "species", "id", "step", "slab_after", "limiter", "process"):
        bad = np.nonzero(a[f] != b[f])[0]
        assert len(bad) == 0, f"field {f} differs first at sorted step {bad[0]}: {a[bad[0]]} vs {b[bad[0]]}"
    scale = np.maximum(np.abs(a["e_before"]), 1e-3)
    de = np.max(np.abs(a["e_after"] - b["e_after"]) / scale) if len(a) else 0.0
    dd = np.max(np.abs(a["edep"] - b["edep"]) / scale) if len(a) else 0.0
    dp = np.max(np.abs(a["pos_after"] - b["pos_after"])) if len(a) else 0.0
    assert de <= e_rtol and dd <= e_rtol, f"energy differs: {de}, {dd}"
    assert dp <= pos_atol, f"position differs: {dp}"
    return dict(n=len(a), de=de, dp=dp)


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
