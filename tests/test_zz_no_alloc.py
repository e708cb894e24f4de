"""The allocation-free solve (opdhg_solve_noalloc) through the C-ABI.

It runs opdhg_solve's kernels on the library's static device scratch, with
the launch sequence enqueued directly on the caller's stream instead of a
captured graph, so its results must equal opdhg_solve's bit for bit. Two
calls in a row, the second on a smaller LP, check that nothing of the first
call's scratch contents leaks into the second; an LP too large for the
scratch is refused with an error and runs nothing.
"""

import numpy as np
import pytest

from lpgen import config_lp
from gpu_common import say as _say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_17650_amd as P
    P.load()
    return P


def _same(a, b):
    (xa, ya, ra), (xb, yb, rb) = a, b
    assert ra.status == rb.status and ra.iterations == rb.iterations
    assert ra.attempts == rb.attempts and ra.restarts == rb.restarts
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb)
    assert ra.primal_obj == rb.primal_obj and ra.rel_kkt == rb.rel_kkt
    assert ra.eta == rb.eta and ra.omega == rb.omega and ra.which == rb.which


@pytest.mark.parametrize("prec_name", ["fp64", "fp32"])
def test_noalloc_equals_solve_twice_smaller_second(P, prec_name):
    prec = P.OPDHG_FP64 if prec_name == "fp64" else P.OPDHG_FP32
    big = config_lp("cfg1", scale=0.1)
    small = config_lp("cfg0", seed=2)
    p = P.opdhg_default_params(precision=prec, max_iter=20000, lr=1e-3, phi=20)
    assert P.opdhg_workspace_bytes(big, p) <= P.capi.OPDHG_NOALLOC_SCRATCH_BYTES
    for lp in (big, small):
        _say(f"[noalloc] {prec_name} m={lp.m} n={lp.n} nnz={lp.nnz}")
        got = P.opdhg_solve_noalloc(lp, p)
        want = P.opdhg_solve(lp, p)
        _same(got, want)
        assert got[2].status == P.capi.OPDHG_STATUS_OPTIMAL


def test_noalloc_windowed_chunks_run_in_order(P):
    # FP32 windowed chunks beside tile rows: the direct launch runs a side's
    # tile, windowed and segment kernels one after the other on one stream
    from lpgen import block_angular_lp
    lp = block_angular_lp(7, blocks=6, block_rows=3000, block_cols=8000, col_degree=6,
                          link_rows=40, link_nnz_per_row=600)
    p = P.opdhg_default_params(precision=P.OPDHG_FP32, max_iter=3000, lr=1e-3,
                               windows=P.OPDHG_WINDOWS_ALWAYS)
    _say(f"[noalloc] windows m={lp.m} n={lp.n} nnz={lp.nnz}")
    _same(P.opdhg_solve_noalloc(lp, p), P.opdhg_solve(lp, p))
    # a small LP again after the large one
    small = config_lp("cfg0", seed=5)
    q = P.opdhg_default_params(precision=P.OPDHG_FP32, max_iter=20000)
    _same(P.opdhg_solve_noalloc(small, q), P.opdhg_solve(small, q))


def test_noalloc_rejects_an_lp_larger_than_the_scratch(P):
    lp = config_lp("cfg1", scale=3.0)
    p = P.opdhg_default_params(max_iter=10)
    need = P.opdhg_workspace_bytes(lp, p)
    assert need > P.capi.OPDHG_NOALLOC_SCRATCH_BYTES
    with pytest.raises(P.OpdhgError) as e:
        P.opdhg_solve_noalloc(lp, p)
    assert e.value.code == P.capi.OPDHG_ERR_WORKSPACE_TOO_SMALL
    assert "static scratch" in str(e.value)
    # and the scratch still serves the next call
    small = config_lp("cfg0", seed=1)
    q = P.opdhg_default_params(max_iter=20000)
    _same(P.opdhg_solve_noalloc(small, q), P.opdhg_solve(small, q))
