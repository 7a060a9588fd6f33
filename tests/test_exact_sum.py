"""The device's per-step dipole accumulator (sfhk_exact_sum.hpp), compiled for the host: every total
must be the correctly rounded exact sum of the values added (Python's Fraction arithmetic, rounded
by float()), whatever their order, signs and magnitudes; non-finite values follow IEEE addition."""
import math
import os
import struct
import subprocess
from fractions import Fraction

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "native", "exact_sum_driver.cpp")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("exact") / "exact_sum")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror", "-o", exe, DRIVER], check=True)
    return exe


def _bits(x: float) -> str:
    return "%016x" % struct.unpack("<Q", struct.pack("<d", x))[0]


def _from_bits(h: str) -> float:
    return struct.unpack("<d", struct.pack("<Q", int(h, 16)))[0]


def _run(exe, groups):
    inp = "\n".join(" ".join(_bits(v) for v in g) for g in groups) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return [_from_bits(h) for h in out.split()]


def _exact(g):
    tot = sum((Fraction(v) for v in g), Fraction(0))
    try:
        return float(tot)  # correctly rounded (ties to even)
    except OverflowError:
        return math.inf if tot > 0 else -math.inf


def _same(a, b):
    return (math.isnan(a) and math.isnan(b)) or struct.pack("<d", a) == struct.pack("<d", b)


def test_random_groups_are_correctly_rounded_exact_sums(driver):
    rng = np.random.default_rng(123)
    groups = []
    for k in range(400):
        n = int(rng.integers(1, 200))
        kind = k % 5
        if kind == 0:    # similar magnitudes, both signs (cancellation)
            g = rng.standard_normal(n) * 10.0 ** rng.uniform(-20, 20)
        elif kind == 1:  # wide dynamic range
            g = rng.standard_normal(n) * 2.0 ** rng.integers(-1070, 1000, n)
        elif kind == 2:  # near-total cancellation: pairs x, -x plus a tiny remainder
            x = rng.standard_normal(n) * 1e10
            g = np.concatenate([x, -x[::-1], rng.standard_normal(3) * 1e-300])
        elif kind == 3:  # subnormals and the smallest normals
            g = rng.integers(-2 ** 52, 2 ** 52, n).astype(np.float64) * 2.0 ** -1074
        else:            # huge values whose sum stays finite or overflows
            g = rng.uniform(0.5, 1.0, n) * 1.7e308 * rng.choice([-1, 1], n)
        groups.append([float(v) for v in g])
    got = _run(driver, groups)
    for g, r in zip(groups, got):
        assert _same(r, _exact(g)), (g[:5], r, _exact(g))


def test_order_does_not_matter(driver):
    rng = np.random.default_rng(7)
    g = list(rng.standard_normal(500) * 2.0 ** rng.integers(-60, 60, 500))
    perms = [list(np.array(g)[rng.permutation(len(g))]) for _ in range(20)]
    got = _run(driver, [g] + perms)
    assert all(_same(x, got[0]) for x in got)
    assert _same(got[0], _exact(g))


def test_ties_round_to_even_and_edge_values(driver):
    one = 1.0
    ulp = 2.0 ** -52
    groups = [
        [one, ulp / 2],                  # tie: stays at 1 (even)
        [one + ulp, ulp / 2],            # tie: rounds up to the even neighbour
        [one, ulp / 2, 2.0 ** -200],     # above the tie: rounds up
        [0.0, -0.0],                     # zeros
        [5e-324, -5e-324, 5e-324],       # smallest subnormal
        [2.0 ** -1022, -(2.0 ** -1074)], # normal minus a subnormal
        [1.7976931348623157e308, 1.7976931348623157e308],  # overflow
        [math.inf, 1.0], [-math.inf, 1.0], [math.inf, -math.inf], [math.nan, 1.0],
    ]
    want = [1.0, 1.0 + 2 * ulp, 1.0 + ulp, 0.0, 5e-324, 2.0 ** -1022 - 2.0 ** -1074, math.inf,
            math.inf, -math.inf, math.nan, math.nan]
    got = _run(driver, groups)
    for g, r, w in zip(groups, got, want):
        assert _same(r, w), (g, r, w)
