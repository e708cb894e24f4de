"""The table statistics against hand-computed values of their definitions."""

import math

import pytest

from paper_2506_17650_amd.metrics import (best_over_grid, compare, geometric_mean,
                                          shifted_geometric_mean)


def test_shifted_geometric_mean_hand_values():
    # (0 + 10)(90 + 10) = 1000, square root 31.6227..., minus the shift
    assert math.isclose(shifted_geometric_mean([0, 90]), math.sqrt(1000) - 10, rel_tol=1e-13)
    assert math.isclose(shifted_geometric_mean([7, 7, 7]), 7.0, rel_tol=1e-13)
    # the shift damps small counts: SGM10 of {1, 100} is far above GM = 10
    assert shifted_geometric_mean([1, 100]) > 23.0
    assert math.isclose(shifted_geometric_mean([2, 8], shift=0.0), 4.0, rel_tol=1e-13)
    assert math.isnan(shifted_geometric_mean([]))


def test_geometric_mean_hand_values():
    assert math.isclose(geometric_mean([1.0, 100.0]), 10.0, rel_tol=1e-13)
    assert math.isclose(geometric_mean([0.5, 2.0, 1.0]), 1.0, rel_tol=1e-13)


def _run(opt, it, s=None):
    return {"optimal": opt, "iterations": it, "seconds": s}


def test_best_over_grid_picks_fewest_optimal():
    grid = {1e-1: [_run(True, 50), _run(False, 900), _run(False, 10)],
            1e-2: [_run(True, 40), _run(True, 800), _run(False, 5)],
            1e-3: [_run(True, 40), _run(True, 700), _run(False, 1)]}
    runs, rates = best_over_grid(grid)
    assert rates == [1e-2, 1e-3, None]  # ties keep the first rate in grid order
    assert [r["iterations"] for r in runs] == [40, 700, 10]


def test_compare_counts_and_means():
    base = [_run(True, 100, 1.0), _run(True, 200, 2.0), _run(False, 999), _run(True, 50, 0.5)]
    var = [_run(True, 80, 0.8), _run(True, 300, 3.0), _run(True, 120), _run(True, 50, 0.4)]
    out = compare({"base": base, "var": var}, "base")
    assert out["common_optimal"] == 3
    b, v = out["rows"]["base"], out["rows"]["var"]
    assert b["optimal"] == 3 and v["optimal"] == 4
    assert v["improved"] == 1 and v["worsened"] == 1  # instance 3 ties
    assert b["improved"] == 0 and b["worsened"] == 0
    assert math.isclose(v["iter_mean"], (80 + 300 + 50) / 3)
    want = math.exp((math.log(90) + math.log(310) + math.log(60)) / 3) - 10
    assert math.isclose(v["iter_sgm10"], want, rel_tol=1e-14)
    assert math.isclose(v["time_gm"], (0.8 * 3.0 * 0.4) ** (1 / 3), rel_tol=1e-14)


def test_compare_rejects_ragged_inputs():
    with pytest.raises(ValueError):
        compare({"a": [_run(True, 1)], "b": [_run(True, 1), _run(True, 2)]}, "a")
