"""Pins of the oracle's counter-based RNG (Philox4x32-10 and the draw layout).

The generator is pinned to the published known-answer vectors and to an
independent installed implementation (PyTorch's header-only philox engine,
compiled here with g++).  The draw layout (which block and which half of it
gives U_i, and the child-id block) is checked against direct Philox calls.
"""
import os
import random
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers(oracle_mod):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, expect in rows:
        assert oracle_mod.philox(ctr, key) == expect


@pytest.fixture(scope="module")
def torch_philox(tmp_path_factory):
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if not shutil.which("g++") or not os.path.exists(os.path.join(inc, "ATen/core/PhiloxRNGEngine.h")):
        pytest.skip("g++ or torch headers unavailable")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", inc, "-o", exe,
                           os.path.join(HERE, "philox_torch_ref.cpp")])
    return exe


def test_philox_matches_torch_engine(oracle_mod, torch_philox):
    rng = random.Random(1234)
    for _ in range(40):
        ctr = [rng.getrandbits(32) for _ in range(4)]
        key = [rng.getrandbits(32) for _ in range(2)]
        out = subprocess.check_output([torch_philox] + ["%08x" % x for x in ctr + key], text=True)
        assert [int(x, 16) for x in out.split()] == oracle_mod.philox(ctr, key)


def _u(lo, hi):
    return (((hi << 32) | lo) >> 12) * 2.0 ** -52 + 2.0 ** -53


def test_draw_layout(oracle_mod):
    key = [7, 123456]
    tid = 0x1234_5678_9ABC_DEF0
    for step in (0, 1, 99):
        for i in range(6):
            w = oracle_mod.philox([tid & 0xFFFFFFFF, tid >> 32, step, i // 2], key)
            lo, hi = (w[0], w[1]) if i % 2 == 0 else (w[2], w[3])
            assert oracle_mod.uniform(key, tid, step, i) == _u(lo, hi)
        for k in range(3):
            w = oracle_mod.philox([tid & 0xFFFFFFFF, tid >> 32, step, 0x80000000 | k], key)
            assert oracle_mod.child_id(key, tid, step, k) == w[0] | (w[1] << 32)


def test_uniforms_open_interval_and_uniform(oracle_mod):
    key = [1, 2]
    u = np.array([oracle_mod.uniform(key, t, s, i) for t in range(200) for s in range(25) for i in range(4)])
    assert np.all(u > 0.0) and np.all(u < 1.0)
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    # extreme words map strictly inside (0, 1)
    assert 0.0 < _u(0, 0) < 1e-15 and 0.0 < 1.0 - _u(0xFFFFFFFF, 0xFFFFFFFF) < 1e-15
