"""Pins of the FP64 oracle against facts fixed outside it.

Each test checks the oracle against the paper's definitions or mathematics
the oracle does not itself compute: closed forms, invariants, hand-derived
examples, finite differences of the loss definitions (Section 3.1, eq. (5)),
brute-force vertex enumeration, SciPy's HiGHS and planted optima.
"""

import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

import oracle
from oracle import pdhg as P
from oracle.params import (default_params, variant, SCHEDULE_ADAGRAD_DIAG,
                           SCHEDULE_ADAGRAD_NORM, SCHEDULE_CONSTANT)
from oracle.problem import InvalidLP, rescale, validate
from lpgen import LP, config_lp, tiny_lp, random_lp

from brute_force import brute_force

HERE = os.path.dirname(os.path.abspath(__file__))


def _lp_from_dense(A, b, sense, c, l, u, c0=0.0):
    A = np.asarray(A, dtype=float)
    M = sp.csr_matrix(A)
    M.sort_indices()
    return LP(m=A.shape[0], n=A.shape[1], row_ptr=M.indptr.astype(np.int64),
              col_idx=M.indices.astype(np.int32), val=M.data.astype(float),
              b=np.asarray(b, float), sense=np.asarray(sense, np.int8),
              c=np.asarray(c, float), l=np.asarray(l, float), u=np.asarray(u, float),
              obj_offset=c0)


def _highs(lp):
    A = lp.csr()
    E = lp.sense == 0
    I = ~E
    bounds = list(zip(np.where(np.isfinite(lp.l), lp.l, None),
                      np.where(np.isfinite(lp.u), lp.u, None)))
    res = linprog(lp.c, A_ub=-A[I] if I.any() else None, b_ub=-lp.b[I] if I.any() else None,
                  A_eq=A[E] if E.any() else None, b_eq=lp.b[E] if E.any() else None,
                  bounds=bounds, method="highs")
    assert res.status == 0
    return res.fun + lp.obj_offset


# ---------------------------------------------------------------------------
# validation
# ---------------------------------------------------------------------------


def test_validate_rejects_each_rule():
    good = tiny_lp(0, 3, 4)
    validate(good)

    def bad(**kw):
        d = dict(good.__dict__)
        d.update(kw)
        return LP(**d)

    cases = [
        bad(n=0),
        bad(row_ptr=np.array([1, 2, 3, 4])),
        bad(row_ptr=good.row_ptr[::-1].copy()),
        bad(col_idx=np.where(np.arange(good.nnz) == 0, 99, good.col_idx).astype(np.int32)),
        bad(val=np.where(np.arange(good.nnz) == 0, np.nan, good.val)),
        bad(b=np.array([np.inf, 0, 0])),
        bad(c=np.array([0, np.nan, 0, 0])),
        bad(l=np.array([np.inf, 0, 0, 0])),
        bad(u=np.array([-np.inf, 1, 1, 1])),
        bad(l=np.array([2.0, 0, 0, 0]), u=np.array([1.0, 1, 1, 1])),
        bad(sense=np.array([0, 2, 1], np.int8)),
    ]
    dup = _lp_from_dense([[1.0, 2.0]], [1.0], [0], [1, 1], [0, 0], [1, 1])
    dup.col_idx = np.array([0, 0], np.int32)
    cases.append(dup)
    for lp in cases:
        with pytest.raises(InvalidLP):
            validate(lp)


# ---------------------------------------------------------------------------
# rescaling (Section 2: Ruiz and Pock-Chambolle)
# ---------------------------------------------------------------------------


def test_ruiz_exact_on_scaled_permutation():
    # D1 P D2 has one entry per row and column; one Ruiz pass equilibrates
    # it exactly: every |A~_ij| becomes 1.
    rng = np.random.default_rng(0)
    n = 7
    perm = rng.permutation(n)
    A = np.zeros((n, n))
    A[np.arange(n), perm] = rng.uniform(0.01, 100, n) * rng.choice([-1, 1], n)
    lp = _lp_from_dense(A, np.ones(n), np.zeros(n), np.ones(n), np.zeros(n), np.ones(n))
    s = rescale(lp, ruiz_iters=1, pc_beta=-1)
    assert np.allclose(np.abs(s.A.data), 1.0, rtol=4e-16 * 4, atol=0)


def test_ruiz_equilibrates_random_matrix():
    lp = random_lp(11, 300, 600, degree=("uniform", 2, 8))
    s = rescale(lp, ruiz_iters=10, pc_beta=-1)
    a = abs(s.A)
    rmax = a.max(axis=1).toarray().ravel()
    cmax = a.max(axis=0).toarray().ravel()
    # infinity-norm equilibration converges with rate 1/2 in log scale
    assert np.all(np.abs(np.log(rmax)) < 1e-2)
    assert np.all(np.abs(np.log(cmax)) < 1e-2)


def test_ruiz_contracts_badly_scaled_rows():
    lp = config_lp("cfg1", scale=0.02)
    a0 = abs(lp.csr())
    spread0 = np.ptp(np.log(a0.max(axis=1).toarray().ravel()))
    s = rescale(lp, ruiz_iters=10, pc_beta=-1)
    a = abs(s.A)
    spread = np.ptp(np.log(a.max(axis=1).toarray().ravel()))
    assert spread0 > 10 and spread < 0.1


@pytest.mark.parametrize("beta", [0.0, 0.5, 1.0, 1.5, 2.0])
def test_pock_chambolle_spectral_bound(beta):
    # Pock & Chambolle: with sigma_i = 1/sum_j |A_ij|^beta and
    # tau_j = 1/sum_i |A_ij|^(2-beta), ||Sigma^1/2 A T^1/2||_2 <= 1.
    lp = random_lp(3, 40, 70, degree=("uniform", 1, 6))
    s = rescale(lp, ruiz_iters=0, pc_beta=beta)
    assert np.linalg.norm(s.A.toarray(), 2) <= 1.0 + 1e-12
    # and the bound is not vacuous: the unscaled matrix exceeds it
    assert np.linalg.norm(lp.csr().toarray(), 2) > 1.5


def test_rescale_preserves_the_lp():
    # x feasible for the LP <=> x / D_c feasible for the scaled LP, with the
    # same objective; checked on the planted point.
    lp = config_lp("cfg0", seed=4)
    s = rescale(lp)
    xs = lp.x_star / s.Dc
    ys = lp.y_star / s.Dr
    assert np.allclose(s.A @ xs, s.Dr * (lp.csr() @ lp.x_star), rtol=1e-13, atol=1e-12)
    assert math.isclose(s.c @ xs, lp.c @ lp.x_star, rel_tol=1e-13)
    assert math.isclose(s.b @ ys, lp.b @ lp.y_star, rel_tol=1e-13)


# ---------------------------------------------------------------------------
# KKT quantities
# ---------------------------------------------------------------------------


def _scaled_planted(lp, **kw):
    s = rescale(lp, **kw)
    x = lp.x_star / s.Dc
    y = lp.y_star / s.Dr
    return s, x, y


@pytest.mark.parametrize("name,scale", [("cfg0", 1.0), ("cfg1", 0.02), ("cfg3", 0.1)])
def test_kkt_zero_at_planted_optimum(name, scale):
    lp = config_lp(name, scale=scale)
    s, x, y = _scaled_planted(lp)
    parts = oracle.kkt_parts(s, x, y, s.A @ x, s.AT @ y)
    rel = oracle.rel_kkt(s, parts)
    assert rel[3] <= 1e-12
    assert math.isclose(parts["pobj"], lp.planted_obj, rel_tol=1e-12)


def test_kkt_hand_example():
    # min x1 + 2 x2  s.t.  x1 + x2 >= 1 (row 0),  x1 - x2 = 0 (row 1),
    # 0 <= x1 <= 5, x2 >= 0.  At x = (0.2, 0.3), y = (0.5, 0.25):
    #   b - Ax = (1 - 0.5, 0 - (-0.1)) = (0.5, 0.1), row 0 is >= so r_p = (0.5, 0.1)
    #   q = c - A^T y = (1 - 0.5 - 0.25, 2 - 0.5 + 0.25) = (0.25, 1.75)
    #   x1 boxed: lambda1 = 0.25, r_d1 = 0;  x2 only l finite: lambda2 = 1.75, r_d2 = 0
    #   primal obj = 0.2 + 0.6 = 0.8
    #   dual obj = b.y + l1 lambda1+ + l2 lambda2+ - u1 lambda1- = 0.5 + 0 + 0 - 0 = 0.5
    # Rescaling disabled (ruiz 0, no Pock-Chambolle) so the scaled LP is the LP.
    lp = _lp_from_dense([[1, 1], [1, -1]], [1, 0], [1, 0], [1, 2], [0, 0], [5, np.inf])
    s = rescale(lp, ruiz_iters=0, pc_beta=-1)
    x = np.array([0.2, 0.3])
    y = np.array([0.5, 0.25])
    p = oracle.kkt_parts(s, x, y, s.A @ x, s.AT @ y)
    assert math.isclose(p["rp2"], 0.25 + 0.01, rel_tol=1e-14)
    assert p["rd2"] == 0.0
    assert math.isclose(p["pobj"], 0.8, rel_tol=1e-14)
    assert math.isclose(p["dobj"], 0.5, rel_tol=1e-14)
    # relative errors: |b| = 1, |c| = sqrt(5)
    rel = oracle.rel_kkt(s, p)
    assert math.isclose(rel[0], math.sqrt(0.26) / 2.0, rel_tol=1e-14)
    assert math.isclose(rel[2], 0.3 / 2.3, rel_tol=1e-14)
    # a >= row that is satisfied contributes nothing; a free variable's whole
    # reduced cost is dual residual; an upper-only variable keeps q <= 0
    lp2 = _lp_from_dense([[1, 1, 1]], [-3], [1], [1, 2, -1], [0, -np.inf, -np.inf],
                         [np.inf, np.inf, 4])
    s2 = rescale(lp2, ruiz_iters=0, pc_beta=-1)
    x2 = np.array([1.0, 1.0, 1.0])
    y2 = np.array([0.5])
    p2 = oracle.kkt_parts(s2, x2, y2, s2.A @ x2, s2.AT @ y2)
    # q = (0.5, 1.5, -1.5): x1 lower-only -> lambda 0.5; x2 free -> r_d 1.5;
    # x3 upper-only -> lambda -1.5; dual obj = -1.5 + 0*0.5 - 4*1.5 = -7.5
    assert p2["rp2"] == 0.0
    assert math.isclose(p2["rd2"], 2.25, rel_tol=1e-14)
    assert math.isclose(p2["dobj"], -7.5, rel_tol=1e-14)


def test_weighted_kkt_hand_example():
    """KKT error in the primal-weight norm of the restart test (Section 3.2
    adopts PDLP's restart scheme), on the two hand-worked points of
    test_kkt_hand_example; every expected value is worked out by hand.

    Point 1: |r_p|^2 = 0.26, |r_d|^2 = 0, gap = 0.8 - 0.5 = 0.3.
      w = 2:   4 * 0.26 + 0 / 4 + 0.09 = 1.13
      w = 1/2: 0.26 / 4 + 0 * 4 + 0.09 = 0.155
    Point 2: |r_p|^2 = 0, |r_d|^2 = 2.25, p = 1 + 2 - 1 = 2, d = -7.5, gap = 9.5.
      w = 2:   0 + 2.25 / 4 + 90.25 = 90.8125
      w = 1/2: 0 + 2.25 * 4 + 90.25 = 99.25
    Swapping w and 1/w exchanges the two rows of each point, dropping the
    square on w gives 0.52 + 0.09 at point 1, and dropping the gap removes
    the 0.09 / 90.25: each such slip fails one of the four values.
    """
    lp = _lp_from_dense([[1, 1], [1, -1]], [1, 0], [1, 0], [1, 2], [0, 0], [5, np.inf])
    s = rescale(lp, ruiz_iters=0, pc_beta=-1)
    x, y = np.array([0.2, 0.3]), np.array([0.5, 0.25])
    p1 = oracle.kkt_parts(s, x, y, s.A @ x, s.AT @ y)
    lp2 = _lp_from_dense([[1, 1, 1]], [-3], [1], [1, 2, -1], [0, -np.inf, -np.inf],
                         [np.inf, np.inf, 4])
    s2 = rescale(lp2, ruiz_iters=0, pc_beta=-1)
    x2, y2 = np.array([1.0, 1.0, 1.0]), np.array([0.5])
    p2 = oracle.kkt_parts(s2, x2, y2, s2.A @ x2, s2.AT @ y2)
    cases = [(p1, 2.0, 1.13), (p1, 0.5, 0.155), (p2, 2.0, 90.8125), (p2, 0.5, 99.25)]
    for parts, om, sq in cases:
        assert math.isclose(oracle.weighted_kkt(parts, om), math.sqrt(sq), rel_tol=1e-15), (om, sq)


def test_weak_duality_sign():
    # For primal-feasible x and y with zero dual residual, gap >= 0.
    lp = config_lp("cfg0", seed=2)
    s, xs, ys = _scaled_planted(lp)
    rng = np.random.default_rng(1)
    for _ in range(5):
        # feasible primal points: convex combinations with another feasible
        # point are not available, so perturb y instead (x stays x*);
        # all variables are boxed, so r_d = 0 for any y with y_I >= 0
        y = ys + 0.1 * rng.standard_normal(lp.m)
        y[lp.sense == 1] = np.maximum(y[lp.sense == 1], 0.0)
        p = oracle.kkt_parts(s, xs, y, s.A @ xs, s.AT @ y)
        assert p["rd2"] == 0.0
        assert p["pobj"] - p["dobj"] >= -1e-9


# ---------------------------------------------------------------------------
# the PDHG step, eq. (6)
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_planted_optimum_is_a_fixed_point(seed):
    lp = config_lp("cfg0", seed=seed)
    s, x, y = _scaled_planted(lp)
    rng = np.random.default_rng(seed)
    for _ in range(4):
        eta = rng.uniform(0.1, 3.0)
        omega = rng.uniform(0.2, 5.0)
        T = rng.uniform(0.5, 2.0, lp.n)
        S = rng.uniform(0.5, 2.0, lp.m)
        g = s.c - s.AT @ y
        a = P.pdhg_attempt(s, x, y, s.A @ x, g, T, S, eta, omega)
        assert np.abs(a["x_new"] - x).max() <= 1e-12 * (1 + np.abs(x).max())
        assert np.abs(a["y_new"] - y).max() <= 1e-12 * (1 + np.abs(y).max())


def test_projections_hold():
    lp = config_lp("cfg1", scale=0.02)
    s = rescale(lp)
    st = P.initial_state(s)
    rng = np.random.default_rng(0)
    y = rng.standard_normal(lp.m)
    g = s.c - s.AT @ y
    a = P.pdhg_attempt(s, st.x, y, st.Ax, g, st.T, st.S, 5.0, 1.0)
    assert np.all(a["x_new"] >= s.l) and np.all(a["x_new"] <= s.u)
    assert np.all(a["y_new"][lp.sense == 1] >= 0)
    eq = lp.sense == 0
    assert np.array_equal(a["y_new"][eq], a["y_half"][eq])


def test_step_rule_hand_example():
    with open(os.path.join(HERE, "golden", "step_rule_1var.json")) as f:
        g = json.load(f)
    d = g["lp"]
    lp = _lp_from_dense(d["A"], d["b"], d["sense"], d["c"], d["l"], d["u"])
    r = oracle.solve(lp, default_params(), trace=3, stop_k=3)
    tr = {e.k: e for e in r.trace}
    eta1 = 1 + 2 ** -0.6
    y2 = 1 + eta1
    eta2 = (1 + 3 ** -0.6) * eta1
    x3 = eta2 * eta1
    assert 0 < x3 < 10
    dy3 = eta2 * (1 - 2 * x3)
    bar3 = 0.5 * (x3 ** 2 + dy3 ** 2) / abs(dy3 * x3)
    assert eta2 > bar3  # attempt 3 rejected
    eta3 = min((1 - 4 ** -0.3) * bar3, (1 + 4 ** -0.6) * eta2)
    x4 = eta3 * eta1
    dy4 = eta3 * (1 - 2 * x4)
    bar4 = 0.5 * (x4 ** 2 + dy4 ** 2) / abs(dy4 * x4)
    assert eta3 <= bar4  # attempt 4 accepted
    eta4 = min((1 - 5 ** -0.3) * bar4, (1 + 5 ** -0.6) * eta3)
    assert tr[0].eta == 1.0 and tr[0].omega == 1.0
    assert (tr[1].x[0], tr[1].y[0], tr[1].attempts) == (0.0, 1.0, 1)
    assert math.isclose(tr[1].eta, eta1, rel_tol=1e-15)
    assert tr[2].x[0] == 0.0 and math.isclose(tr[2].y[0], y2, rel_tol=1e-15)
    assert math.isclose(tr[2].eta, eta2, rel_tol=1e-15)
    assert tr[3].attempts == 4
    assert math.isclose(tr[3].x[0], x4, rel_tol=1e-14)
    assert math.isclose(tr[3].y[0], y2 + dy4, rel_tol=1e-14)
    assert math.isclose(tr[3].eta, eta4, rel_tol=1e-14)


def test_max_step_retries_zero_fails_on_first_rejection():
    # the same LP rejects its third attempt (above); with no retries allowed
    # that rejection is a numerical failure
    with open(os.path.join(HERE, "golden", "step_rule_1var.json")) as f:
        d = json.load(f)["lp"]
    lp = _lp_from_dense(d["A"], d["b"], d["sense"], d["c"], d["l"], d["u"])
    r = oracle.solve(lp, default_params(max_step_retries=0))
    assert r.status == P.NUMERICAL_ERROR and r.iterations == 2


# ---------------------------------------------------------------------------
# online gradients, eq. (7), against finite differences of the losses, eq. (5)
# ---------------------------------------------------------------------------


def _lagrangian(s, x, y):
    # eq. (2): L(x, y) = c^T x - y^T A x + b^T y (scaled LP)
    return float(s.c @ x - y @ (s.A @ x) + s.b @ y)


@pytest.mark.parametrize("seed", [0, 1])
def test_online_gradients_match_finite_differences(seed):
    lp = config_lp("cfg0", seed=seed)
    s = rescale(lp)
    rng = np.random.default_rng(10 + seed)
    x = np.clip(lp.x_star / s.Dc + rng.standard_normal(lp.n), s.l, s.u)
    y = lp.y_star / s.Dr + rng.standard_normal(lp.m)
    y[lp.sense == 1] = np.maximum(y[lp.sense == 1], 0.0)
    Ax = s.A @ x
    eta, omega = 0.7, 1.3
    T = rng.uniform(0.5, 1.5, lp.n)
    S = rng.uniform(0.5, 1.5, lp.m)
    g = s.c - s.AT @ y
    a = P.pdhg_attempt(s, x, y, Ax, g, T, S, eta, omega)
    r = s.b - Ax
    Gp, Gd = P.online_gradients(s, g, a["x_half"], r, a["r_tilde"], a["y_half"], eta, omega)
    L0 = _lagrangian(s, x, y)

    def loss_p(Tv):  # eq. (5), primal
        xn = P.pdhg_attempt(s, x, y, Ax, g, Tv, S, eta, omega)["x_new"]
        return _lagrangian(s, xn, y) - L0

    def loss_d(Sv):  # eq. (5), dual, with x^{k+1} held at the T-step
        yn = P.pdhg_attempt(s, x, y, Ax, g, T, Sv, eta, omega)["y_new"]
        return L0 - _lagrangian(s, x, yn)

    checked_p = checked_d = 0
    for j in rng.choice(lp.n, 60, replace=False):
        h = 0.05 * T[j]
        xh_lo = x[j] - eta / omega * (T[j] - h) * g[j]
        xh_hi = x[j] - eta / omega * (T[j] + h) * g[j]
        inside = [(s.l[j] <= v <= s.u[j]) for v in (xh_lo, a["x_half"][j], xh_hi)]
        if len(set(inside)) != 1:
            continue  # a kink within the difference step
        Tp = T.copy(); Tp[j] += h
        Tm = T.copy(); Tm[j] -= h
        fd = (loss_p(Tp) - loss_p(Tm)) / (2 * h)
        assert math.isclose(fd, Gp[j], rel_tol=1e-8, abs_tol=1e-12), j
        checked_p += 1
    for i in rng.choice(lp.m, 60, replace=False):
        h = 0.05 * S[i]
        if lp.sense[i] == 1:
            ys = [y[i] + eta * omega * v * a["r_tilde"][i] for v in (S[i] - h, S[i] + h)]
            if (ys[0] >= 0) != (ys[1] >= 0):
                continue
        Sp = S.copy(); Sp[i] += h
        Sm = S.copy(); Sm[i] -= h
        fd = (loss_d(Sp) - loss_d(Sm)) / (2 * h)
        assert math.isclose(fd, Gd[i], rel_tol=1e-8, abs_tol=1e-12), i
        checked_d += 1
    assert checked_p > 30 and checked_d > 30
    # sign structure (Section 3.1): the primal gradient is never positive
    assert np.all(Gp <= 0)


# ---------------------------------------------------------------------------
# the learner: schedule, AdaGrad, projection, phi
# ---------------------------------------------------------------------------


def _mini_state(n, m):
    s = P.State(x=np.zeros(n), y=np.zeros(m), T=np.ones(n), S=np.ones(m), Hp=np.zeros(n),
                Hd=np.zeros(m), Hp_norm=0.0, Hd_norm=0.0, eta=1.0, omega=1.0, k=0, t=0,
                attempts=0, restarts=0, x_anchor=np.zeros(n), y_anchor=np.zeros(m),
                anchor_parts=None, x_sum=np.zeros(n), y_sum=np.zeros(m), w=0.0,
                Ax=np.zeros(m), prev_cand_kkt=math.inf)
    return s


def test_adagrad_diag_closed_form():
    # constant gradient G < 0: H_t = t G^2, so T_t = 1 + lr * sum_{s<=t} 1/sqrt(s)
    p = default_params(lr=0.01, normalize=False, schedule=SCHEDULE_ADAGRAD_DIAG)
    st = _mini_state(3, 2)
    G = np.array([-2.0, -0.5, 0.0])
    for t in range(1, 9):
        P.learner_update(G, np.zeros(2), 1.0, 1.0, st, p)
        expect = 1.0 + 0.01 * sum(1.0 / math.sqrt(q) for q in range(1, t + 1))
        assert math.isclose(st.T[0], expect, rel_tol=1e-14)
        assert math.isclose(st.T[1], expect, rel_tol=1e-14)
        assert st.T[2] == 1.0  # zero gradient, zero accumulator: no change
    assert np.all(st.S == 1.0)


def test_adagrad_norm_and_constant_closed_forms():
    G = np.array([-3.0, -4.0])  # |G| = 5
    p = default_params(lr=0.1, normalize=False, schedule=SCHEDULE_ADAGRAD_NORM)
    st = _mini_state(2, 1)
    for t in range(1, 4):
        P.learner_update(G, np.zeros(1), 1.0, 1.0, st, p)
    # P_t = 1 - lr * G/5 * sum 1/sqrt(s)
    h = sum(1.0 / math.sqrt(q) for q in range(1, 4))
    assert np.allclose(st.T, 1.0 + 0.1 * np.array([3.0, 4.0]) / 5.0 * h, rtol=1e-14)
    p = default_params(lr=0.1, normalize=False, schedule=SCHEDULE_CONSTANT)
    st = _mini_state(2, 1)
    P.learner_update(G, np.zeros(1), 1.0, 1.0, st, p)
    assert np.allclose(st.T, [1.3, 1.4], rtol=1e-14)


def test_normalized_equals_unnormalized_at_constant_norm():
    # Diagonal AdaGrad is invariant to a constant rescaling of the gradient,
    # so dividing by a normalizer that stays constant changes nothing.
    rng = np.random.default_rng(3)
    Gs = [-np.abs(rng.standard_normal(4)) for _ in range(5)]
    Gd = [rng.standard_normal(3) for _ in range(5)]
    a = _mini_state(4, 3)
    b = _mini_state(4, 3)
    pa = default_params(lr=0.05, normalize=True)
    pb = default_params(lr=0.05, normalize=False)
    for gp, gd in zip(Gs, Gd):
        P.learner_update(gp, gd, 7.0, 3.0, a, pa)
        P.learner_update(gp, gd, 7.0, 3.0, b, pb)
    assert np.allclose(a.T, b.T, rtol=1e-13) and np.allclose(a.S, b.S, rtol=1e-13)


def test_zero_normalizer_skips_that_side_and_floor_projects():
    p = default_params(lr=10.0, normalize=True, precond_floor=0.25)
    st = _mini_state(2, 2)
    P.learner_update(np.array([-1.0, 0.0]), np.array([1.0, -1.0]), 0.0, 2.0, st, p)
    assert np.all(st.T == 1.0)  # |g|^2 = 0: primal side skipped
    # dual: G/2 = (0.5, -0.5), AdaGrad step (1, -1) * lr -> (1-10, 1+10)
    assert st.S[0] == 0.25 and st.S[1] == 11.0


def test_phi_schedule_and_sign_structure():
    lp = config_lp("cfg0", seed=1)
    phi, K = 5, 23
    p = default_params(lr=0.05, phi=phi, max_iter=K)
    r = oracle.solve(lp, p, trace=K)
    tr = r.trace
    changes = [k for k in range(K) if not np.array_equal(tr[k].T, tr[k + 1].T)
               or not np.array_equal(tr[k].S, tr[k + 1].S)]
    assert all(k % phi == 0 for k in changes)
    assert len(changes) == (K - 1) // phi + 1
    for k in range(K):
        assert np.all(tr[k + 1].T >= tr[k].T)  # G^p <= 0: T never decreases


def test_lr_zero_keeps_identity_preconditioners():
    lp = config_lp("cfg0", seed=0)
    r = oracle.solve(lp, default_params(lr=0.0, max_iter=300), trace=300)
    for e in r.trace:
        assert np.all(e.T == 1.0) and np.all(e.S == 1.0)


def test_restart_keeps_preconditioners():
    lp = config_lp("cfg0", seed=0)
    p = default_params(lr=0.05, phi=1, max_iter=130)
    r = oracle.solve(lp, p, trace=130)
    tr = {e.k: e for e in r.trace}
    # an artificial restart fires at k = 64 (t = 64 >= 0.36 k); T carries over
    assert tr[64].restarts == 0 and tr[65].restarts == 1
    assert np.all(tr[65].T >= tr[64].T) and not np.all(tr[64].T == 1.0)


# ---------------------------------------------------------------------------
# restart decision (reading of PDLP's scheme)
# ---------------------------------------------------------------------------


def test_restart_decision_table():
    p = default_params()
    rd = P.restart_decision
    # (i) sufficient decay, candidate = average (strictly lower)
    assert rd(0.5, 0.15, 1.0, math.inf, 10, 100, p) == (True, True, 0.15)
    # (ii) necessary decay and no progress since the last evaluation
    assert rd(0.7, 0.75, 1.0, 0.6, 10, 100, p) == (True, False, 0.7)
    # (ii) necessary decay but still improving: no restart
    assert rd(0.7, 0.75, 1.0, 0.71, 10, 100, p) == (False, False, 0.7)
    # (iii) artificial: t >= 0.36 k
    assert rd(0.9, 0.95, 1.0, 0.5, 36, 100, p)[0] is True
    assert rd(0.9, 0.95, 1.0, 0.5, 35, 100, p)[0] is False
    # ties go to the current iterate
    assert rd(0.5, 0.5, 1.0, math.inf, 1, 100, p)[1] is False
    # boundary of (i) is inclusive
    assert rd(0.2, 0.3, 1.0, math.inf, 1, 100, p)[0] is True


# ---------------------------------------------------------------------------
# end to end: the LP optimum
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("seed,m,n,m_eq", [(s, m, n, me) for s, (m, n, me) in
                                            zip(range(8), itertools.cycle(
                                                [(3, 5, 1), (2, 4, 0), (4, 6, 2), (3, 3, 3)]))])
def test_tiny_lps_match_vertex_enumeration(seed, m, n, m_eq):
    lp = tiny_lp(seed, m, n, m_eq=m_eq)
    best, xv, nv = brute_force(lp)
    if xv is None:
        pytest.skip("generated LP has no vertex")  # not expected; tiny_lp is feasible
    r = oracle.solve(lp, default_params(tol=1e-9, max_iter=200000))
    assert r.status == P.OPTIMAL
    assert math.isclose(r.primal_obj, best, rel_tol=1e-7, abs_tol=1e-7)
    # when the optimal vertex is unique, x matches it
    assert abs(r.dual_obj - best) <= 1e-6 * (1 + abs(best))


def test_tiny_planted_vertex():
    lp = tiny_lp(21, 3, 5, m_eq=1, planted=True)
    best, _, _ = brute_force(lp)
    assert math.isclose(best, lp.planted_obj, rel_tol=1e-9, abs_tol=1e-9)
    r = oracle.solve(lp, default_params(tol=1e-9, max_iter=200000))
    assert math.isclose(r.primal_obj, best, rel_tol=1e-7, abs_tol=1e-7)


@pytest.mark.parametrize("seed", range(10))
def test_cfg0_reaches_planted_objective(seed):
    lp = config_lp("cfg0", seed=seed)
    r = oracle.solve(lp, default_params(max_iter=20000))
    assert r.status == P.OPTIMAL and r.rel_kkt <= 1e-4
    obj = lp.planted_obj
    assert abs(r.primal_obj - obj) <= 2e-4 * (1 + abs(obj))


@pytest.mark.parametrize("seed", [0, 2])
def test_cfg0_tight_tolerance_matches_planted_and_highs(seed):
    lp = config_lp("cfg0", seed=seed)
    r = oracle.solve(lp, default_params(tol=1e-9, max_iter=100000))
    assert r.status == P.OPTIMAL
    assert math.isclose(r.primal_obj, lp.planted_obj, rel_tol=1e-8)
    assert math.isclose(r.primal_obj, _highs(lp), rel_tol=1e-8)
    # y* is unique here (350 interior columns over 200 rows, full row rank)
    A = lp.csr().toarray()
    interior = (lp.x_star > lp.l) & (lp.x_star < lp.u)
    assert np.linalg.matrix_rank(A[:, interior]) == lp.m
    assert np.linalg.norm(r.y - lp.y_star) <= 1e-6 * np.linalg.norm(lp.y_star)


def test_cfg1_small_matches_highs():
    lp = config_lp("cfg1", scale=0.02)
    r = oracle.solve(lp, default_params(tol=1e-7, max_iter=100000))
    assert r.status == P.OPTIMAL
    assert math.isclose(r.primal_obj, _highs(lp), rel_tol=1e-5)


@pytest.mark.parametrize("name", ["NoNorm-Freq", "Norm-Freq", "NoNorm-Infreq", "Norm-Infreq"])
def test_variants_converge(name):
    lp = config_lp("cfg0", seed=5)
    r = oracle.solve(lp, variant(name, lr=1e-2))
    assert r.status == P.OPTIMAL
    assert abs(r.primal_obj - lp.planted_obj) <= 2e-4 * (1 + abs(lp.planted_obj))


def test_no_constraints_box_lp():
    # m = 0: minimize c^T x over a box; the optimum sits at l where c > 0
    lp = LP(m=0, n=3, row_ptr=np.zeros(1, np.int64), col_idx=np.zeros(0, np.int32),
            val=np.zeros(0), b=np.zeros(0), sense=np.zeros(0, np.int8),
            c=np.array([1.0, -2.0, 0.5]), l=np.array([0.0, -1.0, 2.0]),
            u=np.array([4.0, 3.0, 5.0]), obj_offset=1.5)
    r = oracle.solve(lp, default_params(tol=1e-9))
    assert r.status == P.OPTIMAL
    assert np.allclose(r.x, [0.0, 3.0, 2.0], atol=1e-8)
    assert math.isclose(r.primal_obj, 1.5 + 0 - 6 + 1, rel_tol=1e-9)


def test_objective_offset_and_free_variables():
    lp = config_lp("cfg1", scale=0.01)
    lp.obj_offset = 123.0
    r = oracle.solve(lp, default_params(tol=1e-6, max_iter=100000))
    assert r.status == P.OPTIMAL
    assert math.isclose(r.primal_obj, _highs(lp), rel_tol=1e-4)


def test_primal_weight_hand_example():
    # min -2x  s.t.  x = 4,  0 <= x <= 10.  Scales stay 1 (1x1 matrix [1]),
    # w0 = |c|/|b| = 2/4 = 0.5, eta0 = 1.  First attempt (eq. (6)):
    #   g = -2;  x_half = 0 - (eta/w) * g = 0 + 2 * 2 = 4  ->  x' = 4
    #   r~ = b - (2 A x' - A x) = 4 - 8 = -4;  y' = 0 + (eta w) * r~ = -2
    #   movement = 0.5*0.5*16 + 0.5*4/0.5 = 8, interaction = |-2 * 4| = 8,
    #   eta_bar = 1 >= eta: accepted (all numbers exact in binary).
    # Swapping eta/w and eta*w would give x' = 1, y' = -8.
    lp = _lp_from_dense([[1.0]], [4.0], [0], [-2.0], [0.0], [10.0])
    r = oracle.solve(lp, default_params(), trace=1, stop_k=1)
    e0, e1 = r.trace
    assert e0.omega == 0.5 and e0.eta == 1.0
    assert e1.x[0] == 4.0 and e1.y[0] == -2.0 and e1.attempts == 1
    assert e1.eta == min((1 - 2 ** -0.3) * 1.0, (1 + 2 ** -0.6) * 1.0)


def test_restart_primal_weight_update():
    # At a restart to the current iterate the primal weight moves to the
    # geometric mean (smoothing 0.5) of |dy|/|dx| and the old weight, where
    # dx, dy are the distances from the previous anchor (the start point).
    lp = config_lp("cfg0", seed=0)
    r = oracle.solve(lp, default_params(max_iter=70), trace=range(60, 70))
    tr = {e.k: e for e in r.trace}
    assert tr[64].restarts == 0 and tr[65].restarts == 1
    st0 = P.initial_state(rescale(lp))
    # the candidate is either the current iterate or the average; recover
    # which from the new anchor (== the restart point)
    xa, ya = r.state.x_anchor, r.state.y_anchor
    dx = np.linalg.norm(xa - st0.x)
    dy = np.linalg.norm(ya - st0.y)
    assert math.isclose(tr[65].omega, math.sqrt(dy / dx * tr[64].omega), rel_tol=1e-12)


# ---------------------------------------------------------------------------
# vanilla PDHG of Section 4.2: L2 pass, power iteration, constant steps,
# no restarts
# ---------------------------------------------------------------------------


def _rank_one_lp(seed, m=6, n=9):
    rng = np.random.default_rng(seed)
    uu = rng.uniform(0.1, 10.0, m) * rng.choice([-1, 1], m)
    vv = rng.uniform(0.1, 10.0, n) * rng.choice([-1, 1], n)
    A = np.outer(uu, vv)
    lp = _lp_from_dense(A, np.ones(m), np.zeros(m), np.ones(n), np.zeros(n), np.full(n, 5.0))
    return lp, uu, vv


@pytest.mark.parametrize("seed", [0, 1])
def test_l2_pass_rank_one_closed_form(seed):
    # A = u v^T: |A_i,:| = |u_i| |v|, |A_:,j| = |v_j| |u|, so one L2 pass gives
    # A~_ij = sign(u_i v_j) sqrt(|u_i v_j|) / sqrt(|u| |v|)
    lp, uu, vv = _rank_one_lp(seed)
    s = rescale(lp, ruiz_iters=0, pc_beta=-1, l2=True)
    want = np.sign(np.outer(uu, vv)) * np.sqrt(np.abs(np.outer(uu, vv))) / math.sqrt(
        np.linalg.norm(uu) * np.linalg.norm(vv))
    assert np.allclose(s.A.toarray(), want, rtol=1e-14, atol=0)
    assert np.allclose(s.Dr, 1.0 / np.sqrt(np.abs(uu) * np.linalg.norm(vv)), rtol=1e-14, atol=0)


def test_l2_pass_exact_on_scaled_permutation():
    rng = np.random.default_rng(4)
    n = 8
    A = np.zeros((n, n))
    A[np.arange(n), rng.permutation(n)] = rng.uniform(0.01, 100, n) * rng.choice([-1, 1], n)
    lp = _lp_from_dense(A, np.ones(n), np.zeros(n), np.ones(n), np.zeros(n), np.ones(n))
    s = rescale(lp, ruiz_iters=0, pc_beta=-1, l2=True)
    assert np.allclose(np.abs(s.A.data), 1.0, rtol=1e-15, atol=0)


def test_l2_pass_sits_between_ruiz_and_pock_chambolle():
    # with all three passes the Pock-Chambolle bound still holds, and the L2
    # pass changes the result (it runs, and before the last pass)
    lp = random_lp(5, 50, 90, degree=("uniform", 1, 6))
    s1 = rescale(lp, 10, 1.0, l2=True)
    s0 = rescale(lp, 10, 1.0, l2=False)
    assert np.linalg.norm(s1.A.toarray(), 2) <= 1.0 + 1e-12
    assert not np.array_equal(s1.Dr, s0.Dr)


@pytest.mark.parametrize("seed", [0, 3])
def test_power_iteration_rank_one_exact(seed):
    lp, uu, vv = _rank_one_lp(seed)
    s = rescale(lp, ruiz_iters=0, pc_beta=-1)
    nu = P.spectral_norm_estimate(s, 50, 1e-12)
    assert math.isclose(nu, np.linalg.norm(uu) * np.linalg.norm(vv), rel_tol=1e-14)


def test_power_iteration_known_spectrum():
    # A = Q1 diag(sv) Q2^T with a clear gap: the estimate converges to max(sv)
    rng = np.random.default_rng(7)
    q1, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    q2, _ = np.linalg.qr(rng.standard_normal((20, 20)))
    sv = np.array([3.0, 2.0, 1.5, 1.0, 0.9, 0.5, 0.4, 0.3, 0.2, 0.1, 0.05, 0.01])
    A = q1 @ np.hstack([np.diag(sv), np.zeros((12, 8))]) @ q2.T
    lp = _lp_from_dense(A, np.ones(12), np.zeros(12), np.ones(20), np.zeros(20), np.ones(20))
    s = rescale(lp, ruiz_iters=0, pc_beta=-1)
    assert math.isclose(P.spectral_norm_estimate(s, 500, 1e-15), 3.0, rel_tol=1e-10)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_power_iteration_never_overshoots(seed):
    lp = random_lp(seed, 40, 70, degree=("uniform", 1, 6))
    s = rescale(lp, 10, -1.0, l2=True)
    true = np.linalg.norm(s.A.toarray(), 2)
    for iters in (1, 3, 10, 200):
        nu = P.spectral_norm_estimate(s, iters, 1e-7)
        assert nu <= true * (1 + 1e-12)
    assert nu >= 0.99 * true


def test_vanilla_constant_step_no_restarts():
    lp = config_lp("cfg0", seed=1)
    p = oracle.vanilla_params(0.0, max_iter=3000)
    r = oracle.solve(lp, p, trace=range(0, 3000, 250))
    s = rescale(lp, 10, -1.0, l2=True)
    eta0 = 0.9 / P.spectral_norm_estimate(s, p.power_iters, p.power_tol)
    st0 = P.initial_state(s, p)
    assert r.eta == eta0 == st0.eta
    assert r.omega == st0.omega
    assert r.restarts == 0 and r.attempts == r.iterations
    for e in r.trace:
        assert e.eta == eta0 and e.omega == st0.omega and e.attempts == e.k
    # the step-weighted average runs over every iteration
    assert math.isclose(r.state.w, r.iterations * eta0, rel_tol=1e-12)
    # tau sigma |A~|^2 = eta^2 |A~|^2 < 1 (Section 2)
    assert eta0 * np.linalg.norm(s.A.toarray(), 2) < 1.0


@pytest.mark.parametrize("lr", [0.0, 1e-1])
def test_vanilla_reaches_planted_objective(lr):
    lp = config_lp("cfg0", seed=0)
    r = oracle.solve(lp, oracle.vanilla_params(lr, max_iter=20000))
    assert r.status == P.OPTIMAL and r.restarts == 0
    obj = lp.planted_obj
    assert abs(r.primal_obj - obj) <= 2e-4 * (1 + abs(obj))


def test_vanilla_tiny_matches_vertex_enumeration():
    lp = tiny_lp(2, 3, 5, m_eq=1)
    best, xv, _ = brute_force(lp)
    assert xv is not None
    r = oracle.solve(lp, oracle.vanilla_params(1e-2, tol=1e-8, max_iter=200000))
    assert r.status == P.OPTIMAL
    assert math.isclose(r.primal_obj, best, rel_tol=1e-6, abs_tol=1e-6)


# ---------------------------------------------------------------------------
# preconditioner-weighted step rule
# ---------------------------------------------------------------------------


def test_weighted_step_rule_hand_example():
    from oracle.params import STEP_NORM_PRECOND, STEP_NORM_PLAIN
    with open(os.path.join(HERE, "golden", "weighted_step_1var.json")) as f:
        g = json.load(f)
    d = g["lp"]
    lp = _lp_from_dense(d["A"], d["b"], d["sense"], d["c"], d["l"], d["u"])
    want = {STEP_NORM_PRECOND: (1 - 2 ** -0.3) * 65 / 56,
            STEP_NORM_PLAIN: (1 - 2 ** -0.3) * 305 / 224}
    for norm, eta1 in want.items():
        p = default_params(step_norm=norm)
        s = rescale(lp, p.ruiz_iters, p.pc_beta)
        st = P.initial_state(s, p)
        st.T = np.array(g["start"]["T"])
        st.S = np.array(g["start"]["S"])
        r = P.solve_from_state(s, st, p, trace=1, stop_k=1)
        e = r.trace[-1]
        assert e.k == 1 and e.attempts == 1
        assert e.x[0] == 4.0 and e.y[0] == -1.75
        assert math.isclose(e.eta, eta1, rel_tol=1e-15), (norm, e.eta, eta1)


def test_weighted_step_rule_reduces_to_plain_at_identity():
    # lr = 0 keeps T = S = 1, where dividing by them changes nothing
    lp = config_lp("cfg0", seed=3)
    a = oracle.solve(lp, default_params(step_norm=1, max_iter=2000), trace=range(0, 2001, 100))
    b = oracle.solve(lp, default_params(step_norm=0, max_iter=2000), trace=range(0, 2001, 100))
    assert a.iterations == b.iterations and a.attempts == b.attempts
    for ea, eb in zip(a.trace, b.trace):
        assert np.array_equal(ea.x, eb.x) and ea.eta == eb.eta


@pytest.mark.parametrize("lr,phi", [(1e-2, 1), (1e-1, 1)])
def test_weighted_step_rule_converges(lr, phi):
    lp = config_lp("cfg0", seed=7)
    r = oracle.solve(lp, default_params(step_norm=1, lr=lr, phi=phi, max_iter=20000))
    assert r.status == P.OPTIMAL
    assert abs(r.primal_obj - lp.planted_obj) <= 2e-4 * (1 + abs(lp.planted_obj))
