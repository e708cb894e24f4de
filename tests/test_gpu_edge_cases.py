"""Edge cases of the method on the GPU against the FP64 oracle (C-ABI).

Each case runs the library and the oracle on the same LP with the same
parameters and compares them coordinate by coordinate (FP64):

* a rejected step attempt on the hand-worked one-variable LP (the adaptive
  step of eq. (6); tests/golden/step_rule_1var.json);
* max_step_retries = 0, so the first rejection ends the solve with
  NUMERICAL_ERROR, reporting the current iterate and its KKT error;
* a positive precond_floor that the online-gradient step actually clamps
  Sigma at (the projection onto the diagonal set of Algorithm 1);
* a zero normalizer (|b - A x| = 0 or |c - A^T y| = 0 at an update
  iteration): that side's update is skipped (normalized loss, Section 3.2);
* fixed variables (l = u), empty rows and an empty column;
* time_limit_s = 0: one launch sequence, then the final evaluation returns
  TIME_LIMIT with the iterate the oracle returns at the same iteration
  count (where it stops at the iteration limit).
"""

import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle.params import default_params
from lpgen import LP, config_lp
from gpu_common import (TRACE_TOL, check_final_fp64, ew_rel, lib_params, say as _say,
                        scal_rel)

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_17650_amd as P
    P.load()
    return P


def _lp_from_dense(A, b, sense, c, l, u, c0=0.0):
    A = np.asarray(A, dtype=float)
    M = sp.csr_matrix(A)
    M.sort_indices()
    return LP(m=A.shape[0], n=A.shape[1], row_ptr=M.indptr.astype(np.int64),
              col_idx=M.indices.astype(np.int32), val=M.data.astype(float),
              b=np.asarray(b, float), sense=np.asarray(sense, np.int8),
              c=np.asarray(c, float), l=np.asarray(l, float), u=np.asarray(u, float),
              obj_offset=c0)


def _trace(P, lp, op, ks, **kw):
    """Session states at every k in ks against the oracle's trace."""
    ref = oracle.solve(lp, op, trace=set(ks), stop_k=max(ks))
    tr = {e.k: e for e in ref.trace}
    states = {}
    with P.Session(lp, lib_params(P, op, **kw)) as s:
        for k in sorted(ks):
            if k not in tr:
                break
            s.run(k)
            x, y, T, S, st = s.state()
            e = tr[k]
            assert st.k == k and st.attempts == e.attempts, (k, st.attempts, e.attempts)
            assert st.restarts == e.restarts, (k, st.restarts, e.restarts)
            for name, a, b in (("x", x, e.x), ("y", y, e.y), ("T", T, e.T), ("S", S, e.S)):
                assert ew_rel(a, b) <= TRACE_TOL, (k, name, ew_rel(a, b))
            assert scal_rel(st.eta, e.eta) <= TRACE_TOL and scal_rel(st.omega, e.omega) <= TRACE_TOL
            states[k] = (x, y, T, S, st)
    return states, tr


def _golden_lp():
    with open(os.path.join(HERE, "golden", "step_rule_1var.json")) as f:
        g = json.load(f)
    d = g["lp"]
    return _lp_from_dense(d["A"], d["b"], d["sense"], d["c"], d["l"], d["u"])


def test_rejected_attempt_on_golden_lp(P):
    """Attempts 1 and 2 are accepted and attempt 3 is rejected; the retry
    with the reduced step is accepted (hand-worked values)."""
    lp = _golden_lp()
    _say("[golden 1-var] rejection and retry")
    states, _ = _trace(P, lp, default_params(), [0, 1, 2, 3])
    eta1 = 1 + 2 ** -0.6
    eta2 = (1 + 3 ** -0.6) * eta1
    x3 = eta2 * eta1
    dy3 = eta2 * (1 - 2 * x3)
    bar3 = 0.5 * (x3 ** 2 + dy3 ** 2) / abs(dy3 * x3)
    assert eta2 > bar3
    eta3 = min((1 - 4 ** -0.3) * bar3, (1 + 4 ** -0.6) * eta2)
    x1, y1, _, _, st1 = states[1]
    assert (x1[0], y1[0], st1.attempts) == (0.0, 1.0, 1)
    assert math.isclose(st1.eta, eta1, rel_tol=1e-15)
    x3g, y3g, _, _, st3 = states[3]
    assert st3.attempts == 4  # one rejected attempt on the way to k = 3
    assert math.isclose(x3g[0], eta3 * eta1, rel_tol=1e-14)


@pytest.mark.parametrize("which", ["golden", "cfg1x0.02"])
def test_no_retries_gives_numerical_error(P, which):
    # the small badly scaled LP rejects its first attempt after a few hundred
    # accepted ones
    lp = _golden_lp() if which == "golden" else config_lp("cfg1", scale=0.02)
    op = default_params(max_step_retries=0, max_iter=20000)
    ref = oracle.solve(lp, op)
    _say(f"[max_step_retries=0] {which}: oracle {ref.status_name} at k={ref.iterations}, "
         f"attempts {ref.attempts}")
    assert ref.status == oracle.pdhg.NUMERICAL_ERROR
    res = P.opdhg_solve(lp, lib_params(P, op))
    check_final_fp64(res, ref, label=which)
    r = res[2]
    assert r.status == P.capi.OPDHG_STATUS_NUMERICAL_ERROR and r.which == 0
    assert math.isfinite(r.rel_kkt) and scal_rel(r.eta, ref.eta) <= TRACE_TOL


def test_precond_floor_clamps_sigma(P):
    """With lr 0.5 the first AdaGrad step moves every entry by 0.5, so each
    Sigma_i that decreases lands on the floor 0.8."""
    lp = config_lp("cfg0", seed=4)
    op = default_params(lr=0.5, phi=1, precond_floor=0.8, max_iter=20000)
    _say("[precond floor 0.8]")
    states, tr = _trace(P, lp, op, [0, 1, 2, 3, 10, 30, 60])
    clamped = int(np.sum(states[1][3] == 0.8))
    assert clamped > 0 and clamped == int(np.sum(tr[1].S == 0.8))
    assert np.all(states[60][3] >= 0.8) and np.any(states[60][3] == 0.8)


@pytest.mark.parametrize("side", ["dual", "primal"])
def test_zero_normalizer_skips_that_side(P, side):
    """b = 0 makes |b - A x^0| = 0 (x^0 = 0 with l = 0): the first update
    leaves Sigma alone and moves T. c = 0 makes |c - A^T y^0| = 0: the first
    update leaves T alone and moves Sigma."""
    lp = config_lp("cfg0", seed=5)
    if side == "dual":
        lp.b = np.zeros(lp.m)
    else:
        lp.c = np.zeros(lp.n)
    op = default_params(lr=0.1, phi=1, normalize=True, max_iter=20000)
    _say(f"[zero normalizer] {side}")
    states, _ = _trace(P, lp, op, [0, 1, 2, 5, 20, 60])
    _, _, T1, S1, _ = states[1]
    skipped, moved = (S1, T1) if side == "dual" else (T1, S1)
    assert np.all(skipped == 1.0) and np.any(moved != 1.0)


def _fixed_and_empty_lp():
    """cfg0 with 10% of the variables fixed at their planted values (l = u),
    one empty equality row (b = 0), one empty >= row (b = -1) and one empty
    column (cost 1 on [0, 5])."""
    base = config_lp("cfg0", seed=7)
    rng = np.random.default_rng(70)
    A = base.csr().toarray()
    n0 = base.n
    fixed = rng.choice(n0, size=n0 // 10, replace=False)
    l = base.l.copy()
    u = base.u.copy()
    l[fixed] = base.x_star[fixed]
    u[fixed] = base.x_star[fixed]
    A = np.vstack([A, np.zeros((2, n0))])
    A = np.hstack([A, np.zeros((A.shape[0], 1))])
    b = np.concatenate([base.b, [0.0, -1.0]])
    sense = np.concatenate([base.sense, [0, 1]]).astype(np.int8)
    c = np.concatenate([base.c, [1.0]])
    l = np.concatenate([l, [0.0]])
    u = np.concatenate([u, [5.0]])
    return _lp_from_dense(A, b, sense, c, l, u)


def test_fixed_variables_empty_rows_and_column(P):
    lp = _fixed_and_empty_lp()
    op = default_params(lr=1e-2, phi=20, max_iter=20000)
    _say(f"[fixed / empty] m={lp.m} n={lp.n} nnz={lp.nnz}")
    _trace(P, lp, op, [0, 1, 2, 10, 64, 65, 100])
    ref = oracle.solve(lp, op)
    res = P.opdhg_solve(lp, lib_params(P, op))
    check_final_fp64(res, ref)
    x = res[0]
    fixed = lp.l == lp.u
    # a fixed variable sits on its scaled bound l / d_c, which unscales to l
    # up to one rounding of each operation
    assert np.all(np.abs(x[fixed] - lp.l[fixed]) <= 4e-16 * np.abs(lp.l[fixed]))
    assert x[-1] == 0.0 and res[2].status == P.capi.OPDHG_STATUS_OPTIMAL


def test_time_limit_zero(P):
    """time_limit_s = 0: the host asks for a final evaluation after the
    first launch sequence; the result is the oracle's at the same iteration
    count, where the oracle stops at the iteration limit."""
    lp = config_lp("cfg0", seed=2)
    op = default_params(lr=1e-2, max_iter=20000)
    x, y, r = P.opdhg_solve(lp, lib_params(P, op, time_limit_s=0.0))
    _say(f"[time limit 0] {P.opdhg_status_name(r.status)} at k={r.iterations}")
    assert r.status == P.capi.OPDHG_STATUS_TIME_LIMIT
    assert 0 < r.iterations <= 64
    op_k = default_params(lr=1e-2, max_iter=r.iterations)
    ref = oracle.solve(lp, op_k)
    assert ref.status == oracle.pdhg.ITERATION_LIMIT
    assert r.iterations == ref.iterations and r.attempts == ref.attempts
    assert r.restarts == ref.restarts and r.which == (1 if ref.which == "average" else 0)
    assert scal_rel(r.primal_obj, ref.primal_obj) <= 1e-6
    assert ew_rel(x, ref.x) <= 1e-6 and ew_rel(y, ref.y) <= 1e-6
    assert abs(r.rel_kkt - ref.rel_kkt) <= 1e-6 * ref.rel_kkt
