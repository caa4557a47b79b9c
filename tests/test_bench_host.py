"""Host-side checks of the benchmark's bookkeeping: the counter tables under
profiles/ hold rows for the benchmark's default launch configuration of
both forms, measured on the kernel sources as they are now (the benchmark
reports counter-measured traffic and atomics only while the digests match),
and a refused multi-GPU request exits with a message."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def default_keys():
    src = open(os.path.join(ROOT, "bench.py")).read()
    # the defaults the keys are built from, as bench.py declares them
    assert '"--steps-per-visit", type=int, default=16' in src
    assert '"--steps-per-visit-mixed", type=int, default=32' in src
    assert '"--refill-below", type=int, default=32' in src
    assert '"--interact-min", type=int, default=24' in src
    assert '"--photon-steps-per-visit", type=int, default=None' in src
    assert '"--photon-refill-below", type=int, default=None' in src
    assert bench.PHOTON_LAUNCH["slab"] == (32, 24)
    assert '"--workload", default="cal_10GeV_e-_x10k"' in src
    assert '"--mixed-workload", default="cal_10GeV_e-_x100k"' in src
    import paper_2209_15445_amd as E
    return [bench.counter_key("cal_10GeV_e-_x10k", True, 16, 32, 24, 32, 24,
                              bench.SHORT_MEV.get(("cal_10GeV_e-_x10k", E.FP64), 0.0)),
            bench.counter_key("cal_10GeV_e-_x100k", False, 32, 32, 24, 32, 24,
                              bench.SHORT_MEV.get(("cal_10GeV_e-_x100k", E.MIXED), 0.0))]


@pytest.mark.parametrize("table", ["traffic.txt", "atomics.txt"])
def test_counter_tables_match_the_kernel_sources(table):
    for key in default_keys():
        for kernel in ("k_visit<e-/e+>", "k_visit<photons>"):
            v = bench.counted_for(kernel, key, table)
            assert v is not None and v > 0, (table, kernel, key)


def test_counter_key_names_form_and_launch():
    assert bench.counter_key("w", True, 16, 32, 24, 32, 24) == "w/fp64/v16r32i24pv32pr24"
    assert bench.counter_key("w", False, 32, 8, 0, 1, 0) == "w/mixed/v32r8i0pv1pr0"
    assert bench.counter_key("w", False, 32, 8, 0, 1, 0, 0.5) == "w/mixed/v32r8i0pv1pr0s0.5"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in (r.stdout + r.stderr)
