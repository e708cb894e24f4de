"""Synthetic LP families and the planted-optimum construction.

Every generator takes a seed (an int or a tuple of ints handed to
``numpy.random.default_rng``) and draws its random numbers in a fixed,
documented order, so a seed names one problem exactly.

Planted optimum (shared by all families)
----------------------------------------
Given A, the row senses and the bounds, a primal-dual pair (x*, y*, z*) is
drawn first and b, c are built around it so that it satisfies the KKT
conditions of the LP exactly (up to the rounding of one sparse product):

* x*: in every bound class an exact 30% of the variables that have a finite
  bound sit on one (box variables pick l or u with probability 1/2); the rest
  are interior: U(l, u) for boxes, l + U(0, 10) / u - U(0, 10) for one-sided
  bounds, U(-10, 10) for free variables.
* y*: N(0, 1) on equality rows. Of the >= rows an exact 20% are slack with
  y* = 0 and b_i = A_i x* - U(0, 1); the others are tight with
  y* = |N(0, 1)| and b_i = A_i x*.
* z*: +|N(0, 1)| at a lower bound, -|N(0, 1)| at an upper bound, 0 otherwise.
* c = A^T y* + z*, so the reduced cost at y* is z*.

Then x* is primal feasible, y* is dual feasible, z* is complementary to x*,
and the duality gap is zero.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Iterator, Optional, Sequence

import numpy as np
import scipy.sparse as sp

__all__ = [
    "LP",
    "PlantedLP",
    "config_lp",
    "config_names",
    "random_lp",
    "plant_optimum",
    "tiny_lp",
    "block_angular_lp",
    "batch_lps",
    "serving_requests",
]


@dataclasses.dataclass
class LP:
    """An LP in CSR form: min c^T x + obj_offset, A x (= or >=) b, l <= x <= u."""

    m: int
    n: int
    row_ptr: np.ndarray  # int64, m + 1
    col_idx: np.ndarray  # int32, nnz, ascending within a row, no duplicates
    val: np.ndarray  # float64, nnz
    b: np.ndarray  # float64, m
    sense: np.ndarray  # int8, m: 0 is '=', 1 is '>='
    c: np.ndarray  # float64, n
    l: np.ndarray  # float64, n, may hold -inf
    u: np.ndarray  # float64, n, may hold +inf
    obj_offset: float = 0.0
    name: str = ""
    # planted optimum, when the generator built one
    x_star: Optional[np.ndarray] = None
    y_star: Optional[np.ndarray] = None
    z_star: Optional[np.ndarray] = None

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def csr(self) -> sp.csr_matrix:
        return sp.csr_matrix(
            (self.val, self.col_idx.astype(np.int64), self.row_ptr), shape=(self.m, self.n)
        )

    @property
    def planted_obj(self) -> Optional[float]:
        if self.x_star is None:
            return None
        return float(self.c @ self.x_star) + self.obj_offset


# A planted LP is an LP whose x_star / y_star / z_star are filled in.
PlantedLP = LP


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.Generator):
        return seed
    if isinstance(seed, (tuple, list)):
        return np.random.default_rng([int(s) for s in seed])
    return np.random.default_rng(int(seed))


def _degrees(rng: np.random.Generator, n: int, spec) -> np.ndarray:
    """Number of nonzeros per column.

    spec is ('fixed', k), ('uniform', lo, hi) (inclusive) or
    ('powerlaw', exponent, lo, hi): P(d) proportional to d**-exponent on
    the integers lo..hi.
    """
    kind = spec[0]
    if kind == "fixed":
        return np.full(n, int(spec[1]), dtype=np.int64)
    if kind == "uniform":
        return rng.integers(int(spec[1]), int(spec[2]) + 1, size=n).astype(np.int64)
    if kind == "powerlaw":
        expo, lo, hi = float(spec[1]), int(spec[2]), int(spec[3])
        d = np.arange(lo, hi + 1, dtype=np.float64)
        p = d ** (-expo)
        p /= p.sum()
        return rng.choice(np.arange(lo, hi + 1, dtype=np.int64), size=n, p=p)
    raise ValueError(f"unknown degree spec {spec!r}")


def _distinct_draws(rng: np.random.Generator, n_groups: int, counts: np.ndarray,
                    universe: int) -> tuple[np.ndarray, np.ndarray]:
    """For group g draw counts[g] distinct uniform members of range(universe).

    Returns (group, member) pairs. Draws with replacement, then redraws the
    duplicates inside a group until none are left.
    """
    if np.any(counts > universe):
        raise ValueError("a group asks for more distinct members than exist")
    group = np.repeat(np.arange(n_groups, dtype=np.int64), counts)
    member = rng.integers(0, universe, size=group.size, dtype=np.int64)
    while True:
        key = group * universe + member
        order = np.argsort(key, kind="stable")
        sk = key[order]
        dup = np.zeros(sk.size, dtype=bool)
        dup[1:] = sk[1:] == sk[:-1]
        if not dup.any():
            return group, member
        idx = order[dup]
        member[idx] = rng.integers(0, universe, size=idx.size, dtype=np.int64)


def _to_csr(m: int, n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray):
    key = rows.astype(np.int64) * n + cols.astype(np.int64)
    order = np.argsort(key, kind="stable")
    rows_s = rows[order]
    col_idx = cols[order].astype(np.int32)
    val = vals[order].astype(np.float64)
    counts = np.bincount(rows_s, minlength=m).astype(np.int64)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, col_idx, val


def _row_senses(rng: np.random.Generator, m: int, eq_frac: float) -> np.ndarray:
    m_eq = int(round(eq_frac * m))
    sense = np.ones(m, dtype=np.int8)
    sense[rng.permutation(m)[:m_eq]] = 0
    return sense


def _bounds(rng: np.random.Generator, n: int, spec) -> tuple[np.ndarray, np.ndarray]:
    """Variable bounds.

    spec is ('box', lo, hi) for every variable in [lo, hi];
    ('box_uniform', ulo, uhi) for [0, U(ulo, uhi)];
    ('mix', f_nonneg, f_box, f_free, ulo, uhi): exact fractions of [0, inf),
    [0, U(ulo, uhi)] and free variables, in a random permutation.
    """
    kind = spec[0]
    if kind == "box":
        return np.full(n, float(spec[1])), np.full(n, float(spec[2]))
    if kind == "box_uniform":
        u = rng.uniform(float(spec[1]), float(spec[2]), size=n)
        return np.zeros(n), u
    if kind == "mix":
        f_nonneg, f_box, f_free, ulo, uhi = spec[1:]
        assert abs(f_nonneg + f_box + f_free - 1.0) < 1e-12
        n_nonneg = int(round(f_nonneg * n))
        n_box = int(round(f_box * n))
        perm = rng.permutation(n)
        ubox = rng.uniform(float(ulo), float(uhi), size=n)
        l = np.zeros(n)
        u = np.full(n, np.inf)
        box = perm[n_nonneg:n_nonneg + n_box]
        free = perm[n_nonneg + n_box:]
        u[box] = ubox[box]
        l[free] = -np.inf
        return l, u
    raise ValueError(f"unknown bound spec {spec!r}")


def plant_optimum(rng: np.random.Generator, m: int, n: int, row_ptr, col_idx, val,
                  sense, l, u, *, at_bound_frac: float = 0.3, slack_frac: float = 0.2,
                  name: str = "") -> LP:
    """Draw (x*, y*, z*) and build b, c around them (module docstring)."""
    A = sp.csr_matrix((val, col_idx.astype(np.int64), row_ptr), shape=(m, n))
    fl = np.isfinite(l)
    fu = np.isfinite(u)
    # draws, in this order: interior fractions, sides, |N(0,1)| for z, then
    # one permutation per bound class
    frac = rng.random(n)
    side_upper = rng.random(n) < 0.5
    zmag = np.abs(rng.standard_normal(n))
    x = np.empty(n)
    at_l = np.zeros(n, dtype=bool)
    at_u = np.zeros(n, dtype=bool)
    classes = [(fl & fu), (fl & ~fu), (~fl & fu), (~fl & ~fu)]
    for ci, mask in enumerate(classes):
        idx = np.flatnonzero(mask)
        if ci == 3:  # free: never at a bound
            continue
        k = int(round(at_bound_frac * idx.size))
        chosen = idx[rng.permutation(idx.size)[:k]]
        if ci == 0:
            up = side_upper[chosen]
            at_u[chosen[up]] = True
            at_l[chosen[~up]] = True
        elif ci == 1:
            at_l[chosen] = True
        else:
            at_u[chosen] = True
    box = classes[0]
    x[box] = l[box] + frac[box] * (u[box] - l[box])
    lo_only = classes[1]
    x[lo_only] = l[lo_only] + 10.0 * frac[lo_only]
    up_only = classes[2]
    x[up_only] = u[up_only] - 10.0 * frac[up_only]
    free = classes[3]
    x[free] = -10.0 + 20.0 * frac[free]
    x[at_l] = l[at_l]
    x[at_u] = u[at_u]
    z = np.zeros(n)
    z[at_l] = zmag[at_l]
    z[at_u] = -zmag[at_u]

    # duals: draws in this order: N(0,1) for every row, slack permutation of
    # the >= rows, U(0,1) slack amounts for every row
    g = rng.standard_normal(m)
    ineq = np.flatnonzero(sense == 1)
    n_slack = int(round(slack_frac * ineq.size))
    slack_rows = ineq[rng.permutation(ineq.size)[:n_slack]]
    slack_amt = rng.random(m)
    y = g.copy()
    y[ineq] = np.abs(g[ineq])
    y[slack_rows] = 0.0
    b = A @ x
    b[slack_rows] -= slack_amt[slack_rows]
    c = A.T @ y + z
    return LP(m=m, n=n, row_ptr=row_ptr, col_idx=col_idx, val=val, b=b,
              sense=sense.astype(np.int8), c=c, l=l, u=u, obj_offset=0.0, name=name,
              x_star=x, y_star=y, z_star=z)


def random_lp(seed, m: int, n: int, *, degree=("fixed", 5), eq_frac: float = 0.5,
              row_scale: Optional[tuple[float, float]] = None, bounds=("box", 0.0, 10.0),
              name: str = "") -> LP:
    """Random sparse LP with a planted optimum.

    Column j gets degree[j] distinct uniformly random rows with N(0, 1)
    values, times a per-row scale log-uniform in row_scale when given.
    Draw order: degrees, (column, row) pairs, values, row scales, row senses,
    bounds, planted optimum.
    """
    rng = _rng(seed)
    deg = _degrees(rng, n, degree)
    deg = np.minimum(deg, m)
    cols, rows = _distinct_draws(rng, n, deg, m)
    vals = rng.standard_normal(cols.size)
    if row_scale is not None:
        lo, hi = row_scale
        s = np.exp(rng.uniform(math.log(lo), math.log(hi), size=m))
        vals = vals * s[rows]
    row_ptr, col_idx, val = _to_csr(m, n, rows, cols, vals)
    sense = _row_senses(rng, m, eq_frac)
    l, u = _bounds(rng, n, bounds)
    return plant_optimum(rng, m, n, row_ptr, col_idx, val, sense, l, u, name=name)


def block_angular_lp(seed, *, blocks: int = 64, block_rows: int = 30000,
                     block_cols: int = 80000, col_degree: int = 6, link_rows: int = 2000,
                     link_nnz_per_row: int = 2140, bounds=("box_uniform", 1.0, 100.0),
                     name: str = "", log=None) -> LP:
    """Block-angular, flow-like LP.

    Each diagonal block is block_rows x block_cols with col_degree distinct
    random rows per column holding +-1 (random sign); block rows are
    equalities. link_rows dense-ish linking >= rows follow, each with
    link_nnz_per_row distinct random columns holding N(0, 1).
    Draw order: block (column, row) pairs, signs, linking (row, column)
    pairs, linking values, bounds, planted optimum. ``log`` (optional)
    receives a line after each stage.
    """
    say = log if log is not None else (lambda msg: None)
    rng = _rng(seed)
    m = blocks * block_rows + link_rows
    n = blocks * block_cols
    nb = blocks * block_cols
    cols_b, rows_local = _distinct_draws(rng, nb, np.full(nb, col_degree, dtype=np.int64),
                                         block_rows)
    blk = cols_b // block_cols
    rows_b = rows_local + blk * block_rows
    signs = np.where(rng.random(cols_b.size) < 0.5, -1.0, 1.0)
    say(f"block entries drawn ({cols_b.size})")
    k = min(link_nnz_per_row, n)
    lrows, lcols = _distinct_draws(rng, link_rows, np.full(link_rows, k, dtype=np.int64), n)
    lvals = rng.standard_normal(lrows.size)
    say(f"linking entries drawn ({lrows.size})")
    rows = np.concatenate([rows_b, lrows + blocks * block_rows])
    cols = np.concatenate([cols_b, lcols])
    vals = np.concatenate([signs, lvals])
    del rows_b, cols_b, lrows, lcols, signs, lvals, blk, rows_local
    row_ptr, col_idx, val = _to_csr(m, n, rows, cols, vals)
    del rows, cols, vals
    say("CSR built")
    sense = np.zeros(m, dtype=np.int8)
    sense[blocks * block_rows:] = 1
    l, u = _bounds(rng, n, bounds)
    return plant_optimum(rng, m, n, row_ptr, col_idx, val, sense, l, u, name=name)


def tiny_lp(seed, m: int = 3, n: int = 4, *, m_eq: int = 1, density: float = 0.8,
            planted: bool = False) -> LP:
    """A tiny LP with finite boxes, small enough for vertex enumeration.

    Unplanted form: A has N(0,1) entries (each kept with probability
    density, at least one per row), x0 ~ U(l, u) with l = 0, u ~ U(1, 5),
    b = A x0 on equality rows and A x0 - U(0, 1) on >= rows, c ~ N(0, 1).
    The box makes it bounded and x0 makes it feasible.
    """
    rng = _rng(seed)
    dense = rng.standard_normal((m, n))
    keep = rng.random((m, n)) < density
    for i in range(m):
        if not keep[i].any():
            keep[i, rng.integers(0, n)] = True
    dense = np.where(keep, dense, 0.0)
    rows, cols = np.nonzero(dense)
    row_ptr, col_idx, val = _to_csr(m, n, rows.astype(np.int64), cols.astype(np.int64),
                                    dense[rows, cols])
    sense = np.ones(m, dtype=np.int8)
    sense[:m_eq] = 0
    l = np.zeros(n)
    u = rng.uniform(1.0, 5.0, size=n)
    if planted:
        return plant_optimum(rng, m, n, row_ptr, col_idx, val, sense, l, u,
                             name=f"tiny-planted-{seed}")
    x0 = l + rng.random(n) * (u - l)
    b = dense @ x0
    b[m_eq:] -= rng.random(m - m_eq)
    c = rng.standard_normal(n)
    return LP(m=m, n=n, row_ptr=row_ptr, col_idx=col_idx, val=val, b=b, sense=sense,
              c=c, l=l, u=u, obj_offset=0.0, name=f"tiny-{seed}")


# ---------------------------------------------------------------------------
# the five workload families
# ---------------------------------------------------------------------------

_CONFIGS = ("cfg0", "cfg1", "cfg2", "cfg2lit", "cfg3", "cfg4")


def config_names() -> tuple[str, ...]:
    return _CONFIGS


def _scaled(v: int, scale: float, lo: int = 1) -> int:
    return max(lo, int(round(v * scale)))


def config_lp(name: str, seed=None, scale: float = 1.0, index: int = 0, log=None) -> LP:
    """One LP of a workload family, optionally shrunk by ``scale``.

    cfg0  random sparse LP, m=200 (100 '=', 100 '>='), n=500, 5 nonzeros
          per column, N(0,1) values, bounds [0, 10].
    cfg1  badly scaled LP, m=50k (40% '='), n=100k, power-law column degree
          (exponent 2.2 on 2..2000), N(0,1) times row scales log-uniform in
          [1e-3, 1e3]; bounds 50% [0, inf), 30% [0, U(1,100)], 20% free.
    cfg2  block-angular LP: 64 blocks of 30k x 80k, 6 nonzeros per column,
          +-1 entries, plus 2k linking rows of ~2140 N(0,1) entries.
    cfg2lit  cfg2 with linking rows of the literal 2% density: 102,400
          entries each (nnz ~235M; the same blocks as cfg2).
    cfg3  one LP of the 256-LP batch (``index`` picks it): m log-uniform in
          [1k, 50k], n=2m, 3..8 nonzeros per column, 50% '=', bounds
          [0, U(1,100)].
    cfg4  one serving request (``index`` picks it): m log-uniform in
          [500, 500k], n=floor(2.5m), power-law degree (2.2 on 4..10), row
          scales log-uniform in [1e-2, 1e2], 50% '=', bounds as cfg1.
    """
    if name == "cfg0":
        seed = 0 if seed is None else seed
        m, n = _scaled(200, scale, 4), _scaled(500, scale, 8)
        return random_lp(seed, m, n, degree=("fixed", min(5, m)), eq_frac=0.5,
                         bounds=("box", 0.0, 10.0), name=f"cfg0-s{seed}")
    if name == "cfg1":
        seed = 1 if seed is None else seed
        m, n = _scaled(50000, scale, 8), _scaled(100000, scale, 16)
        hi = min(2000, max(2, m // 2))
        return random_lp(seed, m, n, degree=("powerlaw", 2.2, 2, hi), eq_frac=0.4,
                         row_scale=(1e-3, 1e3), bounds=("mix", 0.5, 0.3, 0.2, 1.0, 100.0),
                         name=f"cfg1-s{seed}-x{scale:g}")
    if name == "cfg2":
        seed = 2 if seed is None else seed
        blocks = max(1, int(round(64 * min(1.0, scale)))) if scale < 1.0 else 64
        br = _scaled(30000, scale if scale < 1.0 else 1.0, 8)
        bc = _scaled(80000, scale if scale < 1.0 else 1.0, 16)
        # keep the linking rows' share of nonzeros as in the full size
        nnz_blocks = blocks * bc * 6
        link_rows = _scaled(2000, scale, 1)
        link_nnz = max(1, min(blocks * bc, int(round(4.28e6 * nnz_blocks / 30.72e6 / link_rows))))
        return block_angular_lp(seed, blocks=blocks, block_rows=br, block_cols=bc,
                                col_degree=6, link_rows=link_rows, link_nnz_per_row=link_nnz,
                                name=f"cfg2-s{seed}-x{scale:g}")
    if name == "cfg2lit":
        seed = 2 if seed is None else seed
        return block_angular_lp(seed, link_nnz_per_row=102400, name=f"cfg2lit-s{seed}", log=log)
    if name == "cfg3":
        rng = _rng((3, index) if seed is None else seed)
        m = int(round(math.exp(rng.uniform(math.log(1000), math.log(50000)))))
        m = _scaled(m, scale, 8)
        return random_lp(rng, m, 2 * m, degree=("uniform", 3, 8), eq_frac=0.5,
                         bounds=("box_uniform", 1.0, 100.0), name=f"cfg3-{index}")
    if name == "cfg4":
        rng = _rng((4, index + 1) if seed is None else seed)
        m = int(round(math.exp(rng.uniform(math.log(500), math.log(500000)))))
        m = _scaled(m, scale, 8)
        n = int(math.floor(2.5 * m))
        return random_lp(rng, m, n, degree=("powerlaw", 2.2, 4, 10), eq_frac=0.5,
                         row_scale=(1e-2, 1e2), bounds=("mix", 0.5, 0.3, 0.2, 1.0, 100.0),
                         name=f"cfg4-{index}")
    raise ValueError(f"unknown config {name!r}")


def batch_lps(count: int = 256, scale: float = 1.0) -> list[LP]:
    """The cfg3 batch: LP i drawn from seed (3, i)."""
    return [config_lp("cfg3", index=i, scale=scale) for i in range(count)]


def study_lps(count: int = 24) -> list[LP]:
    """A mixed instance set for the variant study (it stands in for the
    paper's benchmark collections, which are not used here).

    Instance i comes from family i mod 4, member j = i // 4:
      0  the random sparse box LP (cfg0 shape), seed 100 + j;
      1  the badly scaled LP with power-law columns and free variables
         (cfg1 shape) at 1%..2% of full size, seed 200 + j;
      2  the batch LP family (cfg3) at 10% size, index j;
      3  the serving family (cfg4) at 1% size, index j.
    """
    out = []
    for i in range(count):
        fam, j = i % 4, i // 4
        if fam == 0:
            out.append(config_lp("cfg0", seed=100 + j))
        elif fam == 1:
            out.append(config_lp("cfg1", seed=200 + j, scale=(0.01, 0.015, 0.02)[j % 3]))
        elif fam == 2:
            out.append(config_lp("cfg3", index=j, scale=0.1))
        else:
            out.append(config_lp("cfg4", index=j, scale=0.01))
    return out


def serving_requests(count: int, rate_per_s: float, scale: float = 1.0,
                     first_index: int = 0) -> tuple[np.ndarray, Iterator[LP]]:
    """Poisson arrivals (seed (4, 0)) and a lazy stream of cfg4 requests.

    Returns (arrival_times_s, iterator over the LPs); request i is drawn from
    seed (4, i + 1), independent of the others and of the arrival process.
    """
    rng = _rng((4, 0))
    gaps = rng.exponential(1.0 / rate_per_s, size=first_index + count)[first_index:]
    times = np.cumsum(gaps)

    def it():
        for i in range(first_index, first_index + count):
            yield config_lp("cfg4", index=i, scale=scale)

    return times, it()


def summary(lp: LP) -> dict:
    """Shape statistics used in logs and in the generator tests."""
    rl = np.diff(lp.row_ptr)
    cl = np.bincount(lp.col_idx, minlength=lp.n)
    return {
        "m": lp.m, "n": lp.n, "nnz": lp.nnz,
        "row_len_mean": float(rl.mean()) if lp.m else 0.0,
        "row_len_max": int(rl.max()) if lp.m else 0,
        "col_len_mean": float(cl.mean()), "col_len_max": int(cl.max()),
        "eq_rows": int((lp.sense == 0).sum()),
    }


def as_batch(lps: Sequence[LP]) -> list[LP]:
    return list(lps)
