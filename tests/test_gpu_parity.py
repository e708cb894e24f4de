"""GPU path vs the FP64 oracle, through the C-ABI.

Trace parity: in FP64 the GPU's iterates, preconditioners, step sizes and
primal weights after each of the first 200 accepted iterations match the
oracle's to 1e-10 relative (|a-b| / |b|, 0 when both are 0), with the same
attempt and restart counts at every k. Final parity: the returned
objective, x and y match to 1e-6 relative, with the same status and
iteration count.
"""

import math
import sys

import numpy as np
import pytest

import oracle
from oracle.params import default_params, vanilla_params
from lpgen import LP, config_lp, tiny_lp

pytestmark = pytest.mark.gpu

TRACE_TOL = 1e-10
FINAL_TOL = 1e-6


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_17650_amd as P
    P.load()
    return P


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    nb = np.linalg.norm(b)
    d = np.linalg.norm(a - b)
    if nb == 0.0:
        return 0.0 if d == 0.0 else math.inf
    return d / nb


def lib_params(P, op, **kw):
    """Library parameters equal to oracle parameters op."""
    return P.opdhg_default_params(
        tol=op.tol, max_iter=op.max_iter, lr=op.lr, phi=op.phi, normalize=int(op.normalize),
        schedule=op.schedule, precond_floor=op.precond_floor, ruiz_iters=op.ruiz_iters,
        pc_beta=op.pc_beta, eval_every=op.eval_every, beta_suff=op.beta_suff,
        beta_nec=op.beta_nec, beta_art=op.beta_art, pw_smoothing=op.pw_smoothing,
        step_growth=op.step_growth, step_reduction=op.step_reduction,
        max_step_retries=op.max_step_retries, step_rule=op.step_rule,
        restart_scheme=op.restart_scheme, l2_rescale=int(op.l2_rescale),
        step_scale=op.step_scale, power_iters=op.power_iters, power_tol=op.power_tol,
        step_norm=op.step_norm, **kw)


def check_trace(P, lp, op, K=200, **kw):
    ref = oracle.solve(lp, op, trace=K, stop_k=K)
    tr = {e.k: e for e in ref.trace}
    worst = 0.0
    with P.Session(lp, lib_params(P, op, **kw)) as s:
        for k in range(0, K + 1):
            if k not in tr:
                break  # the oracle finished earlier
            s.run(k)
            x, y, T, S, st = s.state()
            e = tr[k]
            assert st.k == k, (k, st.k)
            assert st.attempts == e.attempts, ("attempts", k, st.attempts, e.attempts)
            assert st.restarts == e.restarts, ("restarts", k, st.restarts, e.restarts)
            errs = {"x": rel(x, e.x), "y": rel(y, e.y), "T": rel(T, e.T), "S": rel(S, e.S),
                    "eta": abs(st.eta - e.eta) / abs(e.eta),
                    "omega": abs(st.omega - e.omega) / abs(e.omega)}
            for name, v in errs.items():
                assert v <= TRACE_TOL, (k, name, v)
            worst = max(worst, max(errs.values()))
    return worst


def check_final(P, lp, op, **kw):
    ref = oracle.solve(lp, op)
    x, y, r = P.opdhg_solve(lp, lib_params(P, op, **kw))
    assert r.status == ref.status, (r.status, ref.status)
    assert r.iterations == ref.iterations and r.attempts == ref.attempts
    assert r.restarts == ref.restarts
    assert abs(r.primal_obj - ref.primal_obj) <= FINAL_TOL * abs(ref.primal_obj)
    assert rel(x, ref.x) <= FINAL_TOL and rel(y, ref.y) <= FINAL_TOL
    assert abs(r.rel_kkt - ref.rel_kkt) <= 1e-6 * max(ref.rel_kkt, 1e-12) + 1e-14
    return ref, r


@pytest.mark.parametrize("seed", range(10))
def test_cfg0_final_parity_fp64(P, seed):
    lp = config_lp("cfg0", seed=seed)
    _say(f"[cfg0 final] seed={seed}")
    ref, r = check_final(P, lp, default_params(max_iter=20000))
    assert r.status == 0 and r.rel_kkt <= 1e-4


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cfg0_trace_parity_plain(P, seed):
    _say(f"[cfg0 trace lr=0] seed={seed}")
    check_trace(P, config_lp("cfg0", seed=seed), default_params(max_iter=20000))


@pytest.mark.parametrize("lr,phi,norm", [(1e-2, 1, True), (1e-2, 20, True), (5e-2, 1, False),
                                         (5e-2, 20, False)])
def test_cfg0_trace_parity_online(P, lr, phi, norm):
    _say(f"[cfg0 trace] lr={lr} phi={phi} normalize={norm}")
    check_trace(P, config_lp("cfg0", seed=4), default_params(lr=lr, phi=phi, normalize=norm))


@pytest.mark.parametrize("schedule", [1, 2])
def test_trace_parity_other_schedules(P, schedule):
    _say(f"[cfg0 trace] schedule={schedule}")
    check_trace(P, config_lp("cfg0", seed=6),
                default_params(lr=1e-3, phi=5, schedule=schedule), K=120)


def test_cfg1_small_trace_parity(P):
    # power-law columns (long rows in A^T), free and one-sided bounds, row scales
    lp = config_lp("cfg1", scale=0.05)
    _say(f"[cfg1x0.05 trace] m={lp.m} n={lp.n} nnz={lp.nnz}")
    check_trace(P, lp, default_params(lr=1e-2, phi=20), K=200)


def test_cfg1_small_final_parity(P):
    lp = config_lp("cfg1", scale=0.02)
    _say(f"[cfg1x0.02 final] m={lp.m} n={lp.n}")
    check_final(P, lp, default_params(max_iter=40000))


@pytest.mark.parametrize("seed", range(6))
def test_tiny_lps(P, seed):
    lp = tiny_lp(seed, 3, 5, m_eq=1)
    _say(f"[tiny] seed={seed}")
    check_final(P, lp, default_params(tol=1e-8, max_iter=50000))


def test_no_rows(P):
    lp = LP(m=0, n=3, row_ptr=np.zeros(1, np.int64), col_idx=np.zeros(0, np.int32),
            val=np.zeros(0), b=np.zeros(0), sense=np.zeros(0, np.int8),
            c=np.array([1.0, -2.0, 0.5]), l=np.array([0.0, -1.0, 2.0]),
            u=np.array([4.0, 3.0, 5.0]), obj_offset=1.5)
    _say("[m=0]")
    ref, r = check_final(P, lp, default_params(tol=1e-9))
    assert r.status == 0


def test_iteration_limit_and_retries(P):
    lp = config_lp("cfg0", seed=1)
    _say("[limits]")
    ref, r = check_final(P, lp, default_params(max_iter=100))
    assert r.status == 1 and r.iterations == 100


def test_long_rows_whole_workgroup(P):
    # tile_nnz small enough that the dense-ish columns go to whole-workgroup tiles
    lp = config_lp("cfg1", scale=0.05)
    _say("[long-row tiles]")
    op = default_params(lr=1e-2)
    check_trace(P, lp, op, K=80, tile_nnz=512)
    check_trace(P, lp, op, K=80, tile_nnz=64, lanes=4)


def test_run_twice_bit_identical(P):
    lp = config_lp("cfg1", scale=0.03)
    _say("[determinism]")
    p = P.opdhg_default_params(max_iter=3000, lr=1e-2)
    a = P.opdhg_solve(lp, p)
    b = P.opdhg_solve(lp, p)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2].iterations == b[2].iterations


def test_batch_equals_solo(P):
    lps = [config_lp("cfg0", seed=s) for s in range(4)] + [config_lp("cfg3", index=i, scale=0.3)
                                                          for i in range(4)]
    _say(f"[batch] {len(lps)} LPs")
    p = P.opdhg_default_params(max_iter=5000, lr=1e-2)
    out = P.opdhg_solve_batch(lps, p)
    for lp, (x, y, r) in zip(lps, out):
        xs, ys, rs = P.opdhg_solve(lp, p)
        assert r.status == rs.status and r.iterations == rs.iterations
        assert np.array_equal(x, xs) and np.array_equal(y, ys)


def test_long_run_past_the_factor_table(P):
    # 11000 attempts with evaluations every 100 iterations: a launch sequence
    # holds at most 64 attempts, so every attempt past the host table's 8192
    # finds its own step-rule factor in the ring (a longer sequence would
    # have read clamped entries and moved the steps by ~1e-4 relative)
    lp = config_lp("cfg0", seed=1)
    op = default_params(tol=1e-9, max_iter=12000, eval_every=100, lr=1e-2)
    _say("[long run] cfg0 seed 1, eval_every 100, tol 1e-9")
    ref = oracle.solve(lp, op)
    assert ref.attempts > 8192 + 1000
    x, y, r = P.opdhg_solve(lp, lib_params(P, op))
    assert r.status == ref.status
    assert r.iterations == ref.iterations and r.attempts == ref.attempts
    assert r.restarts == ref.restarts
    # past the table the device computes the powers (not bit for bit the
    # host's), so the iterates agree to rounding, not exactly
    assert rel(x, ref.x) <= 1e-9 and rel(y, ref.y) <= 1e-9


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_results_independent_of_workgroup_count(P, prec):
    # each tile stores its own partial sums, so packing several tiles of an
    # LP into one workgroup (16 workgroups) gives the same numbers as one
    # tile per workgroup; FP32 sums them in plain FP64 and relies on this
    lp = config_lp("cfg1", scale=0.05, seed=2)
    pr = P.OPDHG_FP32 if prec == "fp32" else P.OPDHG_FP64
    _say(f"[workgroups] {prec} m={lp.m} n={lp.n} nnz={lp.nnz}")
    a = P.opdhg_solve(lp, P.opdhg_default_params(precision=pr, max_iter=4000, lr=1e-2,
                                                 tile_nnz=256, windows=P.OPDHG_WINDOWS_OFF))
    b = P.opdhg_solve(lp, P.opdhg_default_params(precision=pr, max_iter=4000, lr=1e-2,
                                                 tile_nnz=256, workgroups=16,
                                                 windows=P.OPDHG_WINDOWS_OFF))
    assert a[2].iterations == b[2].iterations and a[2].attempts == b[2].attempts
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_batch_prepared_on_device_equals_solo(P):
    # together these LPs reach the device-preparation threshold (2^20
    # nonzeros), so the automatic choice prepares the set on the device;
    # each alone is prepared on the host; the results agree bit for bit
    lps = [config_lp("cfg3", index=i) for i in (4, 9, 14, 16)]
    assert sum(lp.nnz for lp in lps) >= 1 << 20 and all(lp.nnz < 1 << 20 for lp in lps)
    _say(f"[batch, device preparation] {[lp.nnz for lp in lps]}")
    p = P.opdhg_default_params(max_iter=3000, lr=1e-2)
    out = P.opdhg_solve_batch(lps, p)
    for lp, (x, y, r) in zip(lps, out):
        xs, ys, rs = P.opdhg_solve(lp, p)
        assert r.status == rs.status and r.iterations == rs.iterations
        assert np.array_equal(x, xs) and np.array_equal(y, ys)


def test_fp32_batch_packs_tiles_equal_solo(P):
    # a batch whose chunks hold several tiles of one LP, in FP32
    lps = [config_lp("cfg3", index=i, scale=0.2) for i in range(6)]
    _say(f"[batch fp32] {len(lps)} LPs")
    p = P.opdhg_default_params(precision=P.OPDHG_FP32, max_iter=4000, lr=1e-2, tile_nnz=256,
                               workgroups=32)
    out = P.opdhg_solve_batch(lps, p)
    for lp, (x, y, r) in zip(lps, out):
        xs, ys, rs = P.opdhg_solve(lp, p)
        assert r.status == rs.status and r.iterations == rs.iterations
        assert np.array_equal(x, xs) and np.array_equal(y, ys)


def test_fp32_mode_error_reported(P):
    lp = config_lp("cfg0", seed=3)
    _say("[fp32]")
    ref = oracle.solve(lp, default_params(max_iter=20000))
    x, y, r = P.opdhg_solve(lp, P.opdhg_default_params(precision=P.OPDHG_FP32, max_iter=20000))
    assert r.status == 0 and r.rel_kkt <= 1e-4
    err_obj = abs(r.primal_obj - ref.primal_obj) / abs(ref.primal_obj)
    _say(f"  fp32 objective rel err {err_obj:.3e}, y rel err {rel(y, ref.y):.3e}")
    assert err_obj <= 1e-3


# FP32 trace tolerance. One FP32 step perturbs the iterate by about
# (row length) x 2^-24 relative to the row sums; after rescaling the rows
# are O(1), so 30 steps stay below ~30 x 1e-6. 2e-4 leaves a 5x margin.
# The step size is a ratio of differences of iterates (|dx|^2 over
# dy . A dx), so the iterates' rounding reaches it amplified by
# |x| / |dx| (~10-100 here): it gets 2e-3.
FP32_TRACE_TOL = 2e-4
FP32_ETA_TOL = 2e-3


@pytest.mark.parametrize("name,scale,tile,wg", [
    ("cfg1", 0.02, 256, 8),    # many stream tiles per workgroup: tiles overlap
    ("cfg1", 0.1, 512, 16),    # plus rows longer than a tile
    ("cfg0", 1.0, 64, 4),      # four lanes per row, ragged tails
])
def test_fp32_trace_close_to_oracle(P, name, scale, tile, wg):
    """FP32 iterates stay within FP32 rounding of the FP64 oracle's."""
    lp = config_lp(name, scale=scale)
    op = default_params(max_iter=100000, lr=1e-3, phi=5)
    K = 30
    ref = oracle.solve(lp, op, trace=K, stop_k=K)
    tr = {e.k: e for e in ref.trace}
    _say(f"[fp32-trace] {name} x{scale} tile {tile} wg {wg}: m={lp.m} n={lp.n} nnz={lp.nnz}")
    worst = 0.0
    with P.Session(lp, lib_params(P, op, precision=P.OPDHG_FP32, tile_nnz=tile,
                                  workgroups=wg)) as s:
        for k in (1, 2, 5, 10, 20, 30):
            if k not in tr:
                break
            s.run(k)
            x, y, T, S, st = s.state()
            e = tr[k]
            assert st.k == k and st.attempts == e.attempts, (k, st.attempts, e.attempts)
            errs = {"x": rel(x, e.x), "y": rel(y, e.y), "T": rel(T, e.T), "S": rel(S, e.S),
                    "eta": abs(st.eta - e.eta) / abs(e.eta)}
            worst = max(worst, max(v for nm, v in errs.items() if nm != "eta"))
            for nm, v in errs.items():
                assert v <= (FP32_ETA_TOL if nm == "eta" else FP32_TRACE_TOL), (k, nm, v)
    _say(f"  worst FP32 relative deviation {worst:.2e}")


# ---- vanilla PDHG of Section 4.2: constant steps, no restarts, Ruiz + L2 ----


@pytest.mark.parametrize("seed,lr", [(0, 0.0), (1, 1e-1), (2, 1e-2)])
def test_vanilla_trace_parity(P, seed, lr):
    _say(f"[vanilla trace] cfg0 seed={seed} lr={lr}")
    check_trace(P, config_lp("cfg0", seed=seed), vanilla_params(lr))


def test_vanilla_cfg1_small_trace_parity(P):
    lp = config_lp("cfg1", scale=0.05)
    _say(f"[vanilla trace] cfg1x0.05 m={lp.m} n={lp.n}")
    check_trace(P, lp, vanilla_params(1e-2), K=150)


@pytest.mark.parametrize("lr", [0.0, 1e-1])
def test_vanilla_final_parity(P, lr):
    lp = config_lp("cfg0", seed=0)
    _say(f"[vanilla final] cfg0 lr={lr}")
    ref, r = check_final(P, lp, vanilla_params(lr, max_iter=20000))
    assert r.status == 0 and r.restarts == 0 and r.attempts == r.iterations


def test_vanilla_iteration_limit(P):
    lp = config_lp("cfg1", scale=0.02)
    _say("[vanilla limit]")
    ref, r = check_final(P, lp, vanilla_params(1e-1, max_iter=300))
    assert r.status == 1 and r.iterations == 300 and r.restarts == 0


def test_vanilla_batch_equals_solo(P):
    lps = [config_lp("cfg0", seed=s) for s in range(3)] + [config_lp("cfg3", index=i, scale=0.2)
                                                          for i in range(3)]
    _say(f"[vanilla batch] {len(lps)} LPs")
    p = P.opdhg_vanilla_params(1e-2, max_iter=4000)
    out = P.opdhg_solve_batch(lps, p)
    for lp, (x, y, r) in zip(lps, out):
        xs, ys, rs = P.opdhg_solve(lp, p)
        assert r.status == rs.status and r.iterations == rs.iterations and r.restarts == 0
        assert np.array_equal(x, xs) and np.array_equal(y, ys)


# ---- preconditioner-weighted step rule (movement in the T^-1, Sigma^-1 norms) ----


@pytest.mark.parametrize("lr,phi,norm", [(1e-2, 1, True), (1e-1, 20, False)])
def test_weighted_step_trace_parity(P, lr, phi, norm):
    _say(f"[weighted step trace] cfg0 lr={lr} phi={phi} normalize={norm}")
    check_trace(P, config_lp("cfg0", seed=4),
                default_params(step_norm=1, lr=lr, phi=phi, normalize=norm))


def test_weighted_step_cfg1_small_trace_and_final(P):
    lp = config_lp("cfg1", scale=0.05)
    _say(f"[weighted step] cfg1x0.05 m={lp.m} n={lp.n}")
    check_trace(P, lp, default_params(step_norm=1, lr=1e-2, phi=5), K=150)
    small = config_lp("cfg1", scale=0.02)
    check_final(P, small, default_params(step_norm=1, lr=1e-3, phi=1, max_iter=40000))


def test_weighted_step_vanilla_trace_parity(P):
    # the constant step ignores the movement: weighting must change nothing there
    _say("[weighted step + vanilla]")
    check_trace(P, config_lp("cfg0", seed=5), vanilla_params(1e-1, step_norm=1), K=120)
