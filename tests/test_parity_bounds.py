"""The conserved-totals bound against a float64 model of the library's
reduction (CPU): per-thread strided sums over 1024 x 256 threads, a tree of 8
levels per block of 256, then the 1024 block partials added in order. The
error of that model against the exactly rounded sum stays inside
sum_rounding_depth(n) eps64 sum|x|."""
import math

import numpy as np
import pytest

from parity_bounds import EPS, conserved_totals_bound, sum_rounding_depth


def model_sum(x):
    T = 1024 * 256
    m = -(-x.size // T)
    rows = np.zeros(m * T)
    rows[: x.size] = x
    rows = rows.reshape(m, T)
    acc = np.zeros(T)
    for r in rows:                       # each thread: its cells in stride order
        acc = acc + r
    blk = acc.reshape(1024, 256)
    o = 128
    while o > 0:                         # the block tree
        blk = blk.copy()
        blk[:, :o] = blk[:, :o] + blk[:, o:2 * o]
        o //= 2
    tot = 0.0
    for v in blk[:, 0]:                  # the partials in block order
        tot = tot + float(v)
    return tot


@pytest.mark.parametrize("n,kind", [(1000, "mixed"), (300_000, "mixed"), (3_000_000, "positive"),
                                    (3_000_000, "cancel")])
def test_reduction_error_inside_its_depth_bound(n, kind):
    rng = np.random.default_rng(n)
    if kind == "positive":
        x = 1.0 + 0.3 * rng.random(n)
    elif kind == "mixed":
        x = rng.standard_normal(n) * 10.0 ** rng.integers(-3, 4, n)
    else:                                # large terms that cancel
        x = np.concatenate([1e8 + rng.random(n // 2), -(1e8 + rng.random(n // 2))])
        rng.shuffle(x)
    exact = math.fsum(x)
    err = abs(model_sum(x) - exact)
    assert err <= sum_rounding_depth(n) * EPS["fp64"] * float(np.abs(x).sum())


def test_depth_counts_each_stage():
    assert sum_rounding_depth(1) == 0 + 8 + 1023
    assert sum_rounding_depth(262144) == 0 + 8 + 1023
    assert sum_rounding_depth(262145) == 1 + 8 + 1023
    assert sum_rounding_depth(24576**2) == 2303 + 8 + 1023


def test_zero_field_has_zero_bound():
    b = conserved_totals_bound(512 * 512, 10, [3.0, 0.0])
    assert b[0] > 0 and b[1] == 0.0
