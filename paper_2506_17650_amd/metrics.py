"""Summary statistics of the paper's benchmark tables (Section 4.1).

Per method, over a set of LP instances:
  #Opt             instances that end OPTIMAL within the limits;
  #Iter SGM10/Mean shifted geometric mean (shift 10) and arithmetic mean of
                   iteration counts over the instances that every compared
                   method solves;
  Time GM/Mean     geometric and arithmetic mean of solve times over the
                   same instances;
  #Imp / #Wors     instances with fewer / more iterations than the baseline
                   (reading: counted over the instances both solve).
The online learning rate is chosen per instance from a grid (Section 4.1):
the rate with the fewest iterations among the OPTIMAL runs, the first one in
grid order on ties.
"""

from __future__ import annotations

import math
from typing import Mapping, Sequence


def shifted_geometric_mean(values: Sequence[float], shift: float = 10.0) -> float:
    """exp(mean(log(v + shift))) - shift; nan for an empty sequence."""
    if len(values) == 0:
        return math.nan
    return math.exp(sum(math.log(v + shift) for v in values) / len(values)) - shift


def geometric_mean(values: Sequence[float]) -> float:
    """exp(mean(log(v))) for positive values; nan for an empty sequence."""
    if len(values) == 0:
        return math.nan
    return math.exp(sum(math.log(v) for v in values) / len(values))


def best_over_grid(runs_by_rate: Mapping[float, Sequence[Mapping]]) -> tuple[list, list]:
    """Per-instance choice of the learning rate.

    runs_by_rate[rate][i] is instance i's run ({"optimal", "iterations", ...})
    under that rate. Returns (chosen runs, chosen rates); an instance that
    no rate solves keeps the first rate's run and gets rate None.
    """
    rates = list(runs_by_rate)
    count = len(runs_by_rate[rates[0]])
    runs, chosen = [], []
    for i in range(count):
        best, best_rate = None, None
        for r in rates:
            run = runs_by_rate[r][i]
            if run["optimal"] and (best is None or run["iterations"] < best["iterations"]):
                best, best_rate = run, r
        runs.append(best if best is not None else runs_by_rate[rates[0]][i])
        chosen.append(best_rate)
    return runs, chosen


def compare(methods: Mapping[str, Sequence[Mapping]], baseline: str) -> dict:
    """One row per method, as in the paper's tables.

    methods[name][i] is instance i's run: {"optimal": bool, "iterations":
    int, "seconds": float (may be None)}. Every method lists the same
    instances in the same order.
    """
    names = list(methods)
    count = len(methods[baseline])
    for nm in names:
        if len(methods[nm]) != count:
            raise ValueError(f"{nm}: {len(methods[nm])} runs, baseline has {count}")
    common = [i for i in range(count) if all(methods[nm][i]["optimal"] for nm in names)]
    base = methods[baseline]
    rows = {}
    for nm in names:
        runs = methods[nm]
        its = [runs[i]["iterations"] for i in common]
        secs = [runs[i]["seconds"] for i in common if runs[i].get("seconds") is not None]
        both = [i for i in range(count) if runs[i]["optimal"] and base[i]["optimal"]]
        rows[nm] = {
            "optimal": sum(1 for r in runs if r["optimal"]),
            "iter_sgm10": shifted_geometric_mean(its),
            "iter_mean": sum(its) / len(its) if its else math.nan,
            "time_gm": geometric_mean(secs) if len(secs) == len(common) else None,
            "time_mean": sum(secs) / len(secs) if secs and len(secs) == len(common) else None,
            "improved": sum(1 for i in both if runs[i]["iterations"] < base[i]["iterations"]),
            "worsened": sum(1 for i in both if runs[i]["iterations"] > base[i]["iterations"]),
        }
    return {"instances": count, "common_optimal": len(common), "rows": rows}
