"""Rows longer than the split threshold in tile mode, against the FP64 oracle.

A row of more than kSplitNnz (16384) nonzeros that the step kernels take in
tiles is cut into pieces of kPieceNnz nonzeros, each summed by its own
workgroup; a finishing kernel merges a row's pieces in order and runs the
row epilogue. The LP here is block-angular with three linking rows of 20000
nonzeros, so the A side of every attempt takes that path (FP64 has no
windowed chunks; FP32 runs with windows off).
"""

import numpy as np
import pytest

import oracle
from oracle.params import default_params
from lpgen.generators import block_angular_lp
from gpu_common import check_final_fp32, check_final_fp64, lib_params, say

from test_gpu_parity import check_trace

pytestmark = pytest.mark.gpu

LINK_NNZ = 20000  # above the split threshold of 16384: five pieces per row


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_17650_amd as P
    P.load()
    return P


@pytest.fixture(scope="module")
def lp():
    return block_angular_lp(11, blocks=2, block_rows=400, block_cols=20000, col_degree=3,
                            link_rows=3, link_nnz_per_row=LINK_NNZ)


def test_split_rows_trace_parity_fp64(P, lp):
    say(f"[split rows trace] m={lp.m} n={lp.n} nnz={lp.nnz}")
    rows = np.diff(lp.row_ptr)
    assert int(rows.max()) == LINK_NNZ
    check_trace(P, lp, default_params(lr=1e-3, phi=5), K=120)


def test_split_rows_final_parity(P, lp):
    op = default_params(max_iter=20000)
    ref = oracle.solve(lp, op)
    say(f"[split rows final] oracle status {ref.status} after {ref.iterations} iterations")
    check_final_fp64(P.opdhg_solve(lp, lib_params(P, op)), ref, label="FP64")
    r32 = P.opdhg_solve(lp, lib_params(P, op, precision=P.OPDHG_FP32,
                                       windows=P.OPDHG_WINDOWS_OFF))[2]
    check_final_fp32(r32, ref, label="FP32")


def test_split_rows_batch_equals_solo(P, lp):
    # the split LP packed with an LP without long rows: each equals its solo solve
    other = block_angular_lp(12, blocks=2, block_rows=300, block_cols=2000, col_degree=3,
                             link_rows=2, link_nnz_per_row=500)
    p = lib_params(P, default_params(max_iter=3000, lr=1e-3, phi=5))
    for (xb, yb, rb), one in zip(P.opdhg_solve_batch([lp, other], p), (lp, other)):
        xs, ys, rs = P.opdhg_solve(one, p)
        assert np.array_equal(xb, xs) and np.array_equal(yb, ys)
        assert rb.iterations == rs.iterations and rb.status == rs.status
