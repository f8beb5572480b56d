"""The serving layer's arena allocator (host C++, arena.h), compiled on its own
and driven with random take/give sequences against a brute-force model of the
arena: every range it hands out is the lowest free run that fits, ranges never
overlap, and the free list is whole again once everything is given back."""

import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("arena") / "arena")
    subprocess.run([cxx, "-std=c++17", "-O2", "-o", exe,
                    os.path.join(ROOT, "tests", "host", "arena_main.cpp")], check=True)
    return exe


def _lowest_fit(used, size, b):
    """Brute force: lowest offset o with [o, o + b) inside [0, size) and clear of
    every used range (free runs start at 0 or at the end of a used range)."""
    starts = sorted({0} | {o + n for o, n in used})
    for o in starts:
        if o + b <= size and all(o + b <= uo or uo + un <= o for uo, un in used):
            return o
    return -1


@pytest.mark.parametrize("seed", range(6))
def test_random_take_give_against_brute_force(harness, seed):
    rng = np.random.default_rng(seed)
    size = int(rng.integers(1000, 5000))
    ops, model, used = [f"{size}"], [], []
    # the model replays the same decisions; the harness output is checked after
    for _ in range(400):
        if used and rng.random() < 0.45:
            o, n = used.pop(int(rng.integers(len(used))))
            ops.append(f"g {o} {n}")
            model.append(("g", o, n))
        else:
            b = int(rng.integers(1, size // 3))
            o = _lowest_fit(used, size, b)
            ops.append(f"t {b}")
            model.append(("t", b, o))
            if o >= 0:
                used.append((o, b))
    for o, n in used:
        ops.append(f"g {o} {n}")
    ops.append("f")
    out = subprocess.run([harness], input="\n".join(ops) + "\n", capture_output=True, text=True,
                         check=True).stdout.split("\n")
    takes = [int(x) for x in out[:-2]]
    want = [o for kind, _, o in model if kind == "t"]
    assert takes == want
    assert out[-2].split() == ["0", str(size)]


def test_exact_fit_and_refusal(harness):
    ops = "100\nt 40\nt 60\nt 1\ng 0 40\nt 41\nt 40\nf\n"
    out = subprocess.run([harness], input=ops, capture_output=True, text=True, check=True).stdout.split()
    # 0, 40, no room, then 41 does not fit the freed 40 bytes, 40 does (at 0)
    assert out[:5] == ["0", "40", "-1", "-1", "0"]
    assert out[5:] == []
