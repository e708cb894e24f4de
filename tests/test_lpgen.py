"""The seeded generators: shapes, fractions, determinism, planted KKT."""

import numpy as np
import pytest

from lpgen import config_lp, tiny_lp, random_lp
from lpgen.generators import summary


def _planted_kkt(lp):
    """KKT conditions of the planted point, checked directly on (A, b, c)."""
    A = lp.csr()
    x, y, z = lp.x_star, lp.y_star, lp.z_star
    Ax = A @ x
    E = lp.sense == 0
    I = ~E
    scale = 1.0 + np.abs(lp.b).max()
    out = {}
    out["eq"] = np.abs(Ax[E] - lp.b[E]).max(initial=0.0) / scale
    out["ineq"] = max(0.0, -(Ax[I] - lp.b[I]).min(initial=0.0)) / scale
    out["bounds"] = max(np.max(lp.l - x, initial=-np.inf), np.max(x - lp.u, initial=-np.inf), 0.0)
    out["dual_sign"] = max(0.0, -y[I].min(initial=0.0))
    # complementary slackness on rows: y_i (A_i x - b_i) = 0
    out["row_compl"] = np.abs(y[I] * (Ax[I] - lp.b[I])).max(initial=0.0) / scale
    # reduced cost equals z and is complementary to the bounds
    rc = lp.c - A.T @ y
    out["rc"] = np.abs(rc - z).max() / (1.0 + np.abs(lp.c).max())
    at_l = np.isfinite(lp.l) & (x == lp.l)
    at_u = np.isfinite(lp.u) & (x == lp.u)
    inside = ~(at_l | at_u)
    out["z_sign"] = max(0.0, -z[at_l].min(initial=0.0), z[at_u].max(initial=0.0))
    out["z_inside"] = np.abs(z[inside]).max(initial=0.0)
    # zero duality gap: c^T x = b^T y + l^T z+ - u^T z-
    zp = np.maximum(z, 0.0)
    zm = np.maximum(-z, 0.0)
    dual = lp.b @ y + np.sum(np.where(zp > 0, lp.l, 0.0) * zp) - np.sum(
        np.where(zm > 0, lp.u, 0.0) * zm)
    out["gap"] = abs(lp.c @ x - dual) / (1.0 + abs(lp.c @ x))
    return out


@pytest.mark.parametrize("name,scale", [("cfg0", 1.0), ("cfg1", 0.02), ("cfg2", 0.01),
                                        ("cfg3", 0.2), ("cfg4", 0.05)])
def test_planted_optimum_satisfies_kkt(name, scale):
    lp = config_lp(name, scale=scale)
    k = _planted_kkt(lp)
    for key, v in k.items():
        assert v <= 1e-12, (key, v)


def test_cfg0_shape_and_fractions():
    lp = config_lp("cfg0", seed=3)
    s = summary(lp)
    assert (s["m"], s["n"], s["nnz"]) == (200, 500, 2500)
    assert s["col_len_max"] == 5 and s["col_len_mean"] == 5.0
    assert s["eq_rows"] == 100
    assert np.all(lp.l == 0) and np.all(lp.u == 10)
    at_bound = (lp.x_star == 0) | (lp.x_star == 10)
    assert at_bound.sum() == 150  # exactly 30%
    I = lp.sense == 1
    assert (lp.y_star[I] == 0).sum() == 20  # exactly 20% of the >= rows slack


def test_cfg1_recipe_fractions():
    lp = config_lp("cfg1", scale=0.05)
    m, n = lp.m, lp.n
    assert (m, n) == (2500, 5000)
    assert (lp.sense == 0).sum() == 1000  # 40% equality
    free = ~np.isfinite(lp.l)
    nonneg = np.isfinite(lp.l) & ~np.isfinite(lp.u)
    box = np.isfinite(lp.l) & np.isfinite(lp.u)
    assert (free.sum(), nonneg.sum(), box.sum()) == (1000, 2500, 1500)
    assert np.all(lp.u[box] >= 1) and np.all(lp.u[box] <= 100)
    deg = np.bincount(lp.col_idx, minlength=n)
    assert deg.min() >= 2
    # power law: most columns have small degree, a heavy tail exists
    assert np.median(deg) <= 4 and deg.max() >= 50
    # row scales spread values over ~6 decades
    rmax = np.maximum.reduceat(np.abs(lp.val), lp.row_ptr[:-1])
    assert rmax.max() / rmax.min() > 1e4


def test_cfg3_cfg4_sizes():
    for i in range(5):
        lp = config_lp("cfg3", index=i)
        assert 1000 <= lp.m <= 50000 and lp.n == 2 * lp.m
        deg = np.bincount(lp.col_idx, minlength=lp.n)
        assert deg.min() >= 3 and deg.max() <= 8
    lp = config_lp("cfg4", index=0, scale=0.01)
    assert lp.n == int(2.5 * lp.m)


def test_cfg2_small_block_structure():
    lp = config_lp("cfg2", scale=0.01)
    s = summary(lp)
    # block rows are equalities; linking rows are >= rows at the end
    nlink = (lp.sense == 1).sum()
    assert nlink >= 1 and np.all(lp.sense[-nlink:] == 1)
    blk = lp.val[: lp.row_ptr[lp.m - nlink]]
    assert set(np.unique(blk)) <= {-1.0, 1.0}
    assert s["col_len_mean"] > 6.0


def test_seeded_determinism():
    a = config_lp("cfg1", scale=0.02)
    b = config_lp("cfg1", scale=0.02)
    for f in ("row_ptr", "col_idx", "val", "b", "c", "l", "u", "sense"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    c = config_lp("cfg1", seed=7, scale=0.02)
    assert not np.array_equal(a.val[:10], c.val[:10])


def test_csr_well_formed():
    lp = random_lp(5, 50, 80, degree=("uniform", 2, 6))
    rp = lp.row_ptr
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == lp.nnz
    for i in range(lp.m):
        cols = lp.col_idx[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cols) > 0)


def test_tiny_is_feasible():
    for s in range(10):
        lp = tiny_lp(s, 3, 5)
        assert lp.m == 3 and lp.n == 5 and np.all(np.isfinite(lp.u))


def test_study_set_families_and_determinism():
    from lpgen import study_lps
    a = study_lps(8)
    b = study_lps(8)
    assert [lp.m for lp in a] == [lp.m for lp in b]
    assert all(np.array_equal(x.val, y.val) for x, y in zip(a, b))
    # families cycle: cfg0 shape first (200 x 500), then the badly scaled one
    assert (a[0].m, a[0].n) == (200, 500) and (a[4].m, a[4].n) == (200, 500)
    assert a[1].n == 2 * a[1].m and np.isinf(a[1].u).any() and np.isinf(a[1].l).any()
    assert a[2].n == 2 * a[2].m and a[3].n == int(2.5 * a[3].m)
