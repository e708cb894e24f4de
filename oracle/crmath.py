"""Correctly rounded FP64 log, exp and power (oracle; test infrastructure).

The method evaluates elementary functions in two places: the primal-weight
update at a restart, w <- exp(theta ln(dy / dx) + (1 - theta) ln w) (PDLP's
rule, adopted in Section 3.2), and the adaptive step's factors (j + 1)^-e.
A function value is taken here as its plain definition: the FP64 number
nearest the exact value (reading R33), the same order-free principle the
oracle applies to sums. Each is evaluated with Python's decimal module at 60
significant digits (decimal's ln and exp are correctly rounded at that
precision) and converted to the nearest double, so the only double rounding
is of a value already exact to ~1e-60, far below FP64's resolution.
"""

from __future__ import annotations

from decimal import Decimal, localcontext

_PREC = 60


def cr_log(x: float) -> float:
    """ln x rounded to the nearest double, x > 0 finite."""
    if not x > 0.0:
        raise ValueError("cr_log needs x > 0")
    with localcontext() as ctx:
        ctx.prec = _PREC
        return float(Decimal(x).ln())


def cr_exp(a: float) -> float:
    """e^a rounded to the nearest double."""
    with localcontext() as ctx:
        ctx.prec = _PREC
        return float(Decimal(a).exp())


def cr_pow(x: float, y: float) -> float:
    """x^y = e^(y ln x) rounded to the nearest double, x > 0."""
    if not x > 0.0:
        raise ValueError("cr_pow needs x > 0")
    with localcontext() as ctx:
        ctx.prec = _PREC
        return float((Decimal(y) * Decimal(x).ln()).exp())
