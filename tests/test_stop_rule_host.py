"""The stop rule of lp_solve and the serving layer (host C++, stop_rule.h),
compiled on its own and driven with change sequences: it must take the p of
every round and stop where the rule stated in include/lp.h says."""

import os
import shutil
import subprocess

import numpy as np
import pytest

from tests._util import rule_schedule

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("stop_rule") / "stop_rule")
    subprocess.run([cxx, "-std=c++17", "-O2", "-o", exe,
                    os.path.join(ROOT, "tests", "host", "stop_rule_main.cpp")], check=True)
    return exe


def _run(exe, p0, target, changes):
    inp = f"{p0} {target!r} {len(changes)} " + " ".join(repr(float(c)) for c in changes)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    ps, done = [], None
    for line in out:
        if line.startswith("done"):
            done = int(line.split()[1])
        elif line and line != "open":
            ps.append(int(line))
    return ps, done


def test_geometric_changes_stop_by_hand(harness):
    """c_r = 0.1 * 0.3^(r-1) at p = 1, target 1e-6: the estimate c Q / (1 - Q) with
    Q = 0.3 first reaches target / 2 when c <= 5e-7 * 0.7 / 0.3 = 1.17e-6, i.e. at
    round 11 (0.1 * 0.3^10 = 5.9e-7; 0.1 * 0.3^9 = 2.0e-6 is too large)."""
    ch = [0.1 * 0.3 ** r for r in range(20)]
    ps, done = _run(harness, 1, 1e-6, ch)
    assert done == 11 and ps == [1] * 11


def test_stall_halves_p(harness):
    """Changes that shrink by less than half per round are a stall at p > 1: p
    halves after the second round of each p, down to 1."""
    ch = [0.5, 0.4, 0.35, 0.3, 0.26, 0.22] + [0.1 * 0.2 ** r for r in range(12)]
    ps, done = _run(harness, 8, 1e-4, ch)
    assert ps[:6] == [8, 8, 4, 4, 2, 2] and ps[6] == 1
    ps_py, done_py = rule_schedule(ch, 8, 1e-4)
    assert ps == ps_py and (done is not None) == done_py


def test_zero_change_settles(harness):
    ps, done = _run(harness, 4, 1e-8, [0.3, 0.0, 0.0, 0.0])
    assert ps == [4, 4, 2, 1] and done == 4


@pytest.mark.parametrize("seed", range(6))
def test_random_sequences_match_the_stated_rule(harness, seed):
    rng = np.random.default_rng(seed)
    for _ in range(20):
        n = int(rng.integers(5, 60))
        ratios = rng.uniform(0.05, 1.1, n)
        ch = list(np.cumprod(ratios) * rng.uniform(1e-3, 1.0))
        if rng.random() < 0.2:
            ch[int(rng.integers(0, n))] = 0.0
        p0 = int(rng.choice([1, 2, 4, 8, 16]))
        target = float(10.0 ** rng.uniform(-8, -2))
        ps, done = _run(harness, p0, target, ch)
        ps_py, done_py = rule_schedule(ch, p0, target)
        assert ps == ps_py and (done is not None) == done_py
        if done is not None:
            assert done == len(ps_py)
