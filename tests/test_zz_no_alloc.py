"""The entry point that allocates nothing (ems_create_static) against
ems_create on the same inputs, through the C ABI: two contexts in a row in
the static workspace, the second with a smaller input, each giving the
deposits, ledgers and (second call) step log of a context in a caller
workspace.  FP64 bar: integer counts equal, per-slab deposits and energies
to 1e-9 relative, positions to 1e-7 mm, energy conservation to 1e-9."""
import numpy as np
import pytest

import ems_inputs as I
from parity_util import compare_logs, ledger_residual

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_15445_amd as E
    E.lib()
    return E


def transport(E, cfg, geo, prim, n_events, static, log_cap=0):
    flags = E.F_FULL_LEDGER | (E.F_STEPLOG if log_cap else 0)
    c = E.make_config(cfg, n_events, track_capacity=1 << 16, flags=flags, steplog_capacity=log_cap)
    t = E.Transport(c, geo, static_workspace=static)
    try:
        assert (t.workspace is None) == static
        t.enqueue(prim)
        t.run()
        out = dict(edep=t.edep(), ledger=t.ledger(), stats=t.stats())
        if log_cap:
            out["log"], out["n_log"] = t.steplog()
    finally:
        t.close()
    return out


def check_same(a, b, prim):
    for f in ("n_steps", "n_created", "n_null", "n_pair", "n_annih"):
        assert np.array_equal(a["ledger"][f], b["ledger"][f]), f
    assert a["stats"]["steps"] == b["stats"]["steps"] and a["stats"]["created"] == b["stats"]["created"]
    assert np.allclose(a["edep"], b["edep"], rtol=1e-9, atol=1e-9)
    assert np.allclose(a["ledger"]["escaped"], b["ledger"]["escaped"], rtol=1e-9, atol=1e-9)
    assert ledger_residual(a["edep"], a["ledger"], prim).max() < 1e-9


def test_static_workspace_twice_second_smaller(E):
    geo, cfg, prim = I.workload("cal_1GeV_e-_x32")
    first, second = prim[:8], prim[:3]
    print("static workspace: 8 x 1 GeV e-", flush=True)
    s1 = transport(E, cfg, geo, first, 8, static=True)
    r1 = transport(E, cfg, geo, first, 8, static=False)
    check_same(s1, r1, first)
    assert s1["ledger"]["n_steps"].sum() > 10000
    print("static workspace: 3 x 1 GeV e- with step log", flush=True)
    s2 = transport(E, cfg, geo, second, 3, static=True, log_cap=200000)
    r2 = transport(E, cfg, geo, second, 3, static=False, log_cap=200000)
    check_same(s2, r2, second)
    assert s2["n_log"] == r2["n_log"] and s2["n_log"] <= 200000
    dev = compare_logs(s2["log"], r2["log"], e_rtol=1e-11, pos_atol=1e-9, dep_rtol=3e-11)
    print(f"steps {dev['n']}: largest relative energy difference {dev['de']:.3g}, position {dev['dp']:.3g} mm",
          flush=True)
    # the first context's tallies did not leak into the second
    assert np.allclose(s2["edep"], r2["edep"], rtol=1e-9, atol=1e-9)


def test_static_workspace_refusals(E):
    geo, cfg, prim = I.workload("cal_1GeV_e-_x32")
    big = E.make_config(cfg, 32, track_capacity=1 << 20)
    with pytest.raises(E.EmsError) as ex:
        E.Transport(big, geo, static_workspace=True)
    assert ex.value.code == E.E_CAPACITY and "static workspace" in str(ex.value)
    timed = E.make_config(cfg, 4, track_capacity=1 << 14, flags=E.F_KERNEL_TIMING)
    with pytest.raises(E.EmsError) as ex:
        E.Transport(timed, geo, static_workspace=True)
    assert ex.value.code == E.E_INVALID
    c = E.make_config(cfg, 4, track_capacity=1 << 14)
    held = E.Transport(c, geo, static_workspace=True)
    try:
        with pytest.raises(E.EmsError) as ex:
            E.Transport(c, geo, static_workspace=True)
        assert ex.value.code == E.E_BUSY
    finally:
        held.close()
    # released by ems_destroy: the next context gets it
    again = E.Transport(c, geo, static_workspace=True)
    again.enqueue(prim[:1])
    again.run()
    edep, led = again.edep(0, 1), again.ledger(0, 1)
    again.close()
    assert edep.sum() > 0.5 * prim["ekin"][0]
    assert ledger_residual(edep, led, prim[:1]).max() < 1e-9
