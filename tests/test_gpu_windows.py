"""Windowed sparse products (FP32) against the oracle, through the C-ABI.

Rows whose gathered vector entries fall into a few column ranges (the
block rows of a block-angular LP) run in windowed chunks: the ranges are
staged in LDS and each row sum is formed in a fixed order of its own. The
results are FP32 results, so they are held to the FP32 bounds of the tile
path: traces within the FP32 trace tolerances of the FP64 oracle, final
objectives within 1e-3 at rel KKT 1e-4, bit-identical reruns, batch = solo.
At the full block-angular size one step from the GPU's own iterate is
checked against one oracle step from the same point.
"""

import numpy as np
import pytest

import oracle
from oracle import pdhg as OP
from oracle.params import default_params
from lpgen import config_lp
from gpu_common import (adagrad_flip_slack, check_final_fp32, ew_mixed, ew_mixed_slack,
                        say as _say, scal_rel)

pytestmark = pytest.mark.gpu

# as in test_gpu_parity: FP32 rounding of row sums over 30 steps, per
# coordinate against its size plus the vector's scale, 5x margin; T and
# Sigma after the learner's sign-flip allowance (adagrad_flip_slack)
FP32_TRACE_TOL = 2e-4
FP32_ETA_TOL = 2e-3


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_17650_amd as P
    P.load()
    return P


def _lib(P, op, **kw):
    # these LPs are too small for the automatic choice (fewer than 128
    # chunks): windows are asked for explicitly
    return P.opdhg_default_params(
        precision=P.OPDHG_FP32, tol=op.tol, max_iter=op.max_iter, lr=op.lr, phi=op.phi,
        normalize=int(op.normalize), ruiz_iters=op.ruiz_iters, pc_beta=op.pc_beta,
        windows=P.OPDHG_WINDOWS_ALWAYS, **kw)


# block-angular LPs small enough for the oracle (cfg2 at a tenth: 18.2k x
# 48k), plus linking rows; the A side (block rows) is windowed, the A^T side
# too where the chunkings allow. window_buckets / window_rows force more
# passes and other chunkings. A chunk of one pass keeps its row sums in
# registers, a chunk of several in LDS: both kinds run in these cases.
CASES = [
    dict(window_buckets=0, window_rows=0),     # A: one pass per chunk but one (two)
    dict(window_buckets=2, window_rows=0),     # A: 4 passes of 2048 entries
    dict(window_buckets=3, window_rows=2500),  # A^T 2 passes, A 3; chunks ending mid-block
    dict(window_buckets=8, window_rows=3000),  # A^T one pass; A one or two
]


def _block_long():
    """6 blocks of 3000 x 8000 and 40 linking rows of 600 nonzeros: the
    linking rows are long, so they run as segments of the block chunks."""
    from lpgen import block_angular_lp
    return block_angular_lp(7, blocks=6, block_rows=3000, block_cols=8000, col_degree=6,
                            link_rows=40, link_nnz_per_row=600)


CASES_LONG = [
    dict(window_buckets=0, window_rows=0),     # A rows in one pass, linking rows as segments
    dict(window_buckets=2, window_rows=1500),  # A^T rows in 2 passes, A rows in 4
]


@pytest.mark.parametrize("kw", CASES_LONG)
def test_segmented_rows_trace_close_to_oracle(P, kw):
    _trace_case(P, _block_long(), kw, "block LP with long linking rows")


@pytest.mark.parametrize("kw", CASES)
def test_windowed_trace_close_to_oracle(P, kw):
    _trace_case(P, config_lp("cfg2", scale=0.1), kw, "cfg2x0.1")


def _trace_case(P, lp, kw, label):
    op = default_params(max_iter=100000, lr=1e-3, phi=5)
    K = 30
    ref = oracle.solve(lp, op, trace=K, stop_k=K)
    tr = {e.k: e for e in ref.trace}
    _say(f"[windows trace] {label} m={lp.m} n={lp.n} nnz={lp.nnz} {kw}")
    worst = 0.0
    with P.Session(lp, _lib(P, op, **kw)) as s:
        for k in (1, 2, 5, 10, 20, 30):
            s.run(k)
            x, y, T, S, st = s.state()
            e = tr[k]
            assert st.k == k and st.attempts == e.attempts, (k, st.attempts, e.attempts)
            slack = adagrad_flip_slack(op.lr, op.phi, k)
            errs = {"x": ew_mixed(x, e.x), "y": ew_mixed(y, e.y),
                    "T": ew_mixed_slack(T, e.T, slack), "S": ew_mixed_slack(S, e.S, slack),
                    "eta": scal_rel(st.eta, e.eta)}
            worst = max(worst, max(v for nm, v in errs.items() if nm != "eta"))
            for nm, v in errs.items():
                assert v <= (FP32_ETA_TOL if nm == "eta" else FP32_TRACE_TOL), (k, nm, v)
    _say(f"  worst FP32 per-coordinate deviation {worst:.2e}")


def test_windowed_solve_matches_tiles_and_oracle(P):
    lp = config_lp("cfg2", scale=0.1)
    _say("[windows solve]")
    ref = oracle.solve(lp, default_params(max_iter=40000))
    p = P.opdhg_default_params(precision=P.OPDHG_FP32, max_iter=40000,
                               windows=P.OPDHG_WINDOWS_ALWAYS)
    xw, yw, rw = P.opdhg_solve(lp, p)
    xt, yt, rt = P.opdhg_solve(lp, P.opdhg_default_params(precision=P.OPDHG_FP32, max_iter=40000,
                                                         windows=P.OPDHG_WINDOWS_OFF))
    for r in (rw, rt):
        check_final_fp32(r, ref)
    _say(f"  iterations windows {rw.iterations}, tiles {rt.iterations}, oracle {ref.iterations}")


def test_windowed_rerun_bit_identical_and_batch_equals_solo(P):
    lps = [config_lp("cfg2", scale=0.1), config_lp("cfg1", scale=0.05),
           config_lp("cfg2", scale=0.1, seed=5), _block_long()]
    _say("[windows determinism]")
    p = P.opdhg_default_params(precision=P.OPDHG_FP32, max_iter=3000, lr=1e-3, window_buckets=3,
                               windows=P.OPDHG_WINDOWS_ALWAYS)
    a = P.opdhg_solve(lps[0], p)
    b = P.opdhg_solve(lps[0], p)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2].iterations == b[2].iterations
    out = P.opdhg_solve_batch(lps, p)
    for lp, (x, y, r) in zip(lps, out):
        xs, ys, rs = P.opdhg_solve(lp, p)
        assert r.status == rs.status and r.iterations == rs.iterations
        assert np.array_equal(x, xs) and np.array_equal(y, ys)


def test_server_ignores_windows(P):
    # one captured sequence serves every mix: requests run in tiles, and
    # equal the solo solve with windows off
    lp = config_lp("cfg2", scale=0.1)
    p = P.opdhg_default_params(precision=P.OPDHG_FP32, max_iter=20000,
                               windows=P.OPDHG_WINDOWS_ALWAYS)
    off = P.opdhg_default_params(precision=P.OPDHG_FP32, max_iter=20000,
                                 windows=P.OPDHG_WINDOWS_OFF)
    solo = P.opdhg_solve(lp, off)
    with P.Server(64 << 20, precision=P.OPDHG_FP32) as srv:
        x, y, r = srv.wait(srv.submit(lp, p), 120.0)
    assert np.array_equal(x, solo[0]) and r.iterations == solo[2].iterations


def _one_step_check(P, lp, params, k):
    """Run the GPU to the first k' >= k whose next attempt is accepted, then
    compare that accepted attempt with one oracle attempt (FP64) from the
    GPU's own iterate, preconditioners and step, coordinate by coordinate."""
    slp = oracle.rescale(lp, params.ruiz_iters, params.pc_beta)
    with P.Session(lp, params) as s:
        for kk in range(k, k + 16):
            s.run(kk)
            x, y, T, S, st = s.state()
            s.run(kk + 1)
            x1, y1, T1, S1, st1 = s.state()
            if st1.attempts == st.attempts + 1 and st1.k == kk + 1:
                break
        else:
            raise AssertionError("no accepted first attempt in 16 iterations")
    g = slp.c - OP.AT_mul(slp, y)
    Ax = OP.A_mul(slp, x)
    a = OP.pdhg_attempt(slp, x, y, Ax, g, T, S, st.eta, st.omega)
    ex, ey = ew_mixed(x1, a["x_new"]), ew_mixed(y1, a["y_new"])
    _say(f"  one step from k={kk}: x per-coordinate {ex:.2e}, y {ey:.2e}")
    assert ex <= FP32_TRACE_TOL and ey <= FP32_TRACE_TOL


def test_windowed_full_size_one_step(P):
    """The full block-angular LP (1.92M x 5.12M, 35M nonzeros): every A^T row
    and every block row of A is windowed."""
    lp = config_lp("cfg2")
    _say(f"[windows full size] m={lp.m} n={lp.n} nnz={lp.nnz}")
    _one_step_check(P, lp, P.opdhg_default_params(precision=P.OPDHG_FP32, lr=1e-5, tol=0.0,
                                                  max_iter=10**6), 12)
