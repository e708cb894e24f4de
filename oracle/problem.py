"""Input validation and diagonal rescaling.

The LP is the paper's standard form (Section 2, eq. (1)) widened to
two-sided bounds and >= rows:

    min c^T x + c0   s.t.  A_E x = b_E,  A_I x >= b_I,  l <= x <= u.

Rescaling (Section 2, "Pock-Chambolle" and "Ruiz" preconditioning; the
paper applies it as preprocessing, Section 3.2) produces
A~ = D_r A D_c, b~ = D_r b, c~ = D_c c, l~ = l / D_c, u~ = u / D_c, so that
x = D_c x~ and y = D_r y~ map scaled solutions back. The paper's Ruiz
formula is garbled; the reading is standard infinity-norm equilibration with
the square root split between rows and columns, recomputed from the
original A and the accumulated diagonals at every pass.
"""

from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

from .exact import exact_norm, exact_row_sums


class InvalidLP(ValueError):
    pass


def validate(lp) -> None:
    """Raise InvalidLP unless the LP is well formed.

    Rules: n >= 1, m >= 0; row_ptr starts at 0, never decreases and ends at
    nnz < 2**31; every column index in [0, n) and no (row, column) pair
    twice; A, b, c finite; l < +inf, u > -inf, l <= u (no NaN); every row
    sense 0 ('=') or 1 ('>=').
    """
    m, n = int(lp.m), int(lp.n)
    if n < 1:
        raise InvalidLP("n must be at least 1")
    if m < 0:
        raise InvalidLP("m must be nonnegative")
    rp = np.asarray(lp.row_ptr, dtype=np.int64)
    if rp.shape != (m + 1,):
        raise InvalidLP("row_ptr must have m + 1 entries")
    if rp[0] != 0:
        raise InvalidLP("row_ptr[0] must be 0")
    if np.any(np.diff(rp) < 0):
        raise InvalidLP("row_ptr must be nondecreasing")
    nnz = int(rp[-1])
    if nnz >= 2**31:
        raise InvalidLP("nnz must be below 2**31")
    col = np.asarray(lp.col_idx)
    val = np.asarray(lp.val, dtype=np.float64)
    if col.shape != (nnz,) or val.shape != (nnz,):
        raise InvalidLP("col_idx and val must have nnz entries")
    if nnz and (col.min() < 0 or col.max() >= n):
        raise InvalidLP("column index out of range")
    rows = np.repeat(np.arange(m, dtype=np.int64), np.diff(rp))
    key = rows * n + col.astype(np.int64)
    if np.unique(key).size != nnz:
        raise InvalidLP("duplicate (row, column) entry")
    if not np.all(np.isfinite(val)):
        raise InvalidLP("A has a non-finite entry")
    b = np.asarray(lp.b, dtype=np.float64)
    c = np.asarray(lp.c, dtype=np.float64)
    if b.shape != (m,) or not np.all(np.isfinite(b)):
        raise InvalidLP("b must hold m finite values")
    if c.shape != (n,) or not np.all(np.isfinite(c)):
        raise InvalidLP("c must hold n finite values")
    l = np.asarray(lp.l, dtype=np.float64)
    u = np.asarray(lp.u, dtype=np.float64)
    if l.shape != (n,) or u.shape != (n,):
        raise InvalidLP("l and u must hold n values")
    if np.any(np.isnan(l)) or np.any(np.isnan(u)):
        raise InvalidLP("bounds must not be NaN")
    if np.any(l == np.inf) or np.any(u == -np.inf):
        raise InvalidLP("l must be below +inf and u above -inf")
    if np.any(l > u):
        raise InvalidLP("l must not exceed u")
    s = np.asarray(lp.sense)
    if s.shape != (m,) or np.any((s != 0) & (s != 1)):
        raise InvalidLP("row sense must be 0 or 1")
    if not np.isfinite(float(getattr(lp, "obj_offset", 0.0))):
        raise InvalidLP("objective offset must be finite")


@dataclasses.dataclass
class ScaledLP:
    """The rescaled LP the iteration runs on, plus what unscaling needs."""

    m: int
    n: int
    A: sp.csr_matrix  # A~
    AT: sp.csr_matrix  # transpose of A~, stored explicitly
    b: np.ndarray  # b~
    c: np.ndarray  # c~
    l: np.ndarray  # l~
    u: np.ndarray  # u~
    ineq: np.ndarray  # bool, m: True on >= rows
    Dr: np.ndarray
    Dc: np.ndarray
    c0: float
    b_norm: float  # ||b|| of the unscaled LP
    c_norm: float  # ||c|| of the unscaled LP


def _row_max(vals: np.ndarray, row_ptr: np.ndarray, m: int) -> np.ndarray:
    out = np.zeros(m)
    nonempty = np.diff(row_ptr) > 0
    if nonempty.any():
        out[nonempty] = np.maximum.reduceat(vals, row_ptr[:-1][nonempty])
    return out


def _col_sums(vals: np.ndarray, col: np.ndarray, row_ptr: np.ndarray, m: int, n: int):
    """Correctly rounded sum of each column's entries."""
    csc = sp.csr_matrix((vals, col, row_ptr), shape=(m, n)).tocsc()
    return exact_row_sums(csc.indptr, csc.data)


def rescale(lp, ruiz_iters: int = 10, pc_beta: float = 1.0, l2: bool = False) -> ScaledLP:
    """Ruiz infinity-norm passes, an optional L2-norm pass, then one
    Pock-Chambolle pass.

    Ruiz pass: r_i = max_j |A~_ij|, s_j = max_i |A~_ij| (0 read as 1), then
    D_r /= sqrt(r), D_c /= sqrt(s), with A~_ij = A_ij D_r,i D_c,j.
    L2 pass (l2=True; the preprocessing of the vanilla PDHG runs, Section
    4.2): r_i = |A~_i,:|_2, s_j = |A~_:,j|_2, applied the same way.
    Pock-Chambolle pass (exponent beta; skipped when beta < 0):
    r_i = sum_j |A~_ij|^beta, s_j = sum_i |A~_ij|^(2 - beta), applied the
    same way, so that with beta = 1 the scaled matrix has spectral norm at
    most 1. Sums are correctly rounded (module exact).
    """
    m, n = int(lp.m), int(lp.n)
    rp = np.asarray(lp.row_ptr, dtype=np.int64)
    col = np.asarray(lp.col_idx, dtype=np.int64)
    val = np.asarray(lp.val, dtype=np.float64)
    rows = np.repeat(np.arange(m, dtype=np.int64), np.diff(rp))
    absv = np.abs(val)
    Dr = np.ones(m)
    Dc = np.ones(n)
    for _ in range(ruiz_iters):
        a = absv * Dr[rows] * Dc[col]
        r = _row_max(a, rp, m)
        s = np.zeros(n)
        np.maximum.at(s, col, a)
        r[r == 0] = 1.0
        s[s == 0] = 1.0
        Dr = Dr / np.sqrt(r)
        Dc = Dc / np.sqrt(s)
    if l2:
        a = absv * Dr[rows] * Dc[col]
        a2 = a * a
        r = np.sqrt(exact_row_sums(rp, a2))
        s = np.sqrt(_col_sums(a2, col, rp, m, n))
        r[r == 0] = 1.0
        s[s == 0] = 1.0
        Dr = Dr / np.sqrt(r)
        Dc = Dc / np.sqrt(s)
    if pc_beta >= 0:
        a = absv * Dr[rows] * Dc[col]
        ar = a if pc_beta == 1.0 else a ** pc_beta
        ac = a if pc_beta == 1.0 else a ** (2.0 - pc_beta)
        r = exact_row_sums(rp, ar)
        s = _col_sums(ac, col, rp, m, n)
        r[r == 0] = 1.0
        s[s == 0] = 1.0
        Dr = Dr / np.sqrt(r)
        Dc = Dc / np.sqrt(s)
    sval = val * Dr[rows] * Dc[col]
    A = sp.csr_matrix((sval, col, rp), shape=(m, n))
    AT = A.T.tocsr()
    b = np.asarray(lp.b, dtype=np.float64)
    c = np.asarray(lp.c, dtype=np.float64)
    l = np.asarray(lp.l, dtype=np.float64)
    u = np.asarray(lp.u, dtype=np.float64)
    return ScaledLP(
        m=m, n=n, A=A, AT=AT, b=Dr * b, c=Dc * c, l=l / Dc, u=u / Dc,
        ineq=np.asarray(lp.sense) == 1, Dr=Dr, Dc=Dc,
        c0=float(getattr(lp, "obj_offset", 0.0)),
        b_norm=exact_norm(b), c_norm=exact_norm(c),
    )
