"""Device-side preparation against host preparation, through the C-ABI.

With OPDHG_PREP_DEVICE the Ruiz, L2 and Pock-Chambolle passes, the scaled
values and vectors, and the first step size and primal weight are computed
by device kernels in the device order of the rows. Without windowed chunks
the device also builds both CSR copies (A in device order and its
transpose) from the caller's arrays, unless a column is longer than the
device's per-column ordering takes. Each row statistic follows the host's
expression and order, and each CSR copy the host's entry order, so the
whole solve must equal the host-prepared solve bit for bit; the host's
rescaling is in turn bitwise equal to the oracle's (test_library_host.py),
and every solve here is also checked against the oracle's.
"""

import numpy as np
import pytest

import oracle
from oracle.params import default_params, vanilla_params
from oracle.pdhg import spectral_norm_estimate
from lpgen import block_angular_lp, config_lp
from gpu_common import check_final_fp32, check_final_fp64, lib_params, say as _say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_17650_amd as P
    P.load()
    return P


def _lps():
    return {
        "cfg0": config_lp("cfg0", seed=3),
        "cfg1x0.05": config_lp("cfg1", scale=0.05),  # row scales over 6 decades, free variables
        "cfg4-2x0.01": config_lp("cfg4", index=2, scale=0.01),
        "cfg3-1x0.2": config_lp("cfg3", index=1, scale=0.2),
    }


_ORACLE = {}


def _oracle(name, lp, op, key):
    """The oracle's solve of one test LP, computed once per parameter set
    (both precisions compare with it)."""
    if (name, key) not in _ORACLE:
        _ORACLE[(name, key)] = oracle.solve(lp, op)
    return _ORACLE[(name, key)]


def _same(a, b):
    (xa, ya, ra), (xb, yb, rb) = a, b
    assert ra.status == rb.status and ra.iterations == rb.iterations
    assert ra.attempts == rb.attempts and ra.restarts == rb.restarts
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb)
    assert ra.primal_obj == rb.primal_obj and ra.eta == rb.eta and ra.omega == rb.omega


@pytest.mark.parametrize("prec_name", ["fp64", "fp32"])
@pytest.mark.parametrize("extra", [{}, {"l2_rescale": 1, "pc_beta": -1.0}])
def test_device_prep_equals_host_prep(P, prec_name, extra):
    prec = P.OPDHG_FP64 if prec_name == "fp64" else P.OPDHG_FP32
    for name, lp in _lps().items():
        _say(f"[prep] {name} {prec_name} {extra}")
        op = default_params(max_iter=3000, lr=1e-3, tol=1e-4, **extra)
        host = P.opdhg_solve(lp, lib_params(P, op, precision=prec, prep=P.OPDHG_PREP_HOST))
        dev = P.opdhg_solve(lp, lib_params(P, op, precision=prec, prep=P.OPDHG_PREP_DEVICE))
        _same(dev, host)
        ref = _oracle(name, lp, op, tuple(sorted(extra.items())))
        if prec == P.OPDHG_FP64:
            check_final_fp64(dev, ref, label=name)
        elif ref.status == oracle.pdhg.OPTIMAL:
            check_final_fp32(dev[2], ref, label=name)
        else:  # both stop at the iteration limit
            assert dev[2].status == ref.status and dev[2].iterations == ref.iterations, name


def test_device_prep_other_exponent_to_rounding(P):
    """A Pock-Chambolle exponent other than 1 takes powers: the device's pow
    and the host's may differ in the last bit, so the two preparations agree
    to rounding. Over 20 iterations the iterates stay within 1e-12."""
    lp = config_lp("cfg1", scale=0.05)
    kw = dict(precision=P.OPDHG_FP64, lr=1e-3, ruiz_iters=3, pc_beta=0.5, tol=0.0,
              max_iter=10**6)
    with P.Session(lp, P.opdhg_default_params(prep=P.OPDHG_PREP_HOST, **kw)) as a, \
            P.Session(lp, P.opdhg_default_params(prep=P.OPDHG_PREP_DEVICE, **kw)) as b:
        for k in (1, 5, 20):
            a.run(k)
            b.run(k)
            xa, ya, Ta, Sa, sa = a.state()
            xb, yb, Tb, Sb, sb = b.state()
            assert sa.attempts == sb.attempts
            for u, v in ((xa, xb), (ya, yb), (Ta, Tb), (Sa, Sb)):
                assert np.linalg.norm(u - v) <= 1e-12 * max(np.linalg.norm(u), 1e-300)
            assert abs(sa.eta - sb.eta) <= 1e-12 * abs(sa.eta)


def test_device_prep_windows_and_segments(P):
    # FP32 block LPs with windowed chunks, and long linking rows as segments
    lps = [config_lp("cfg2", scale=0.1),
           block_angular_lp(7, blocks=6, block_rows=3000, block_cols=8000, col_degree=6,
                            link_rows=40, link_nnz_per_row=600)]
    for lp in lps:
        _say(f"[prep windows] m={lp.m} n={lp.n}")
        kw = dict(precision=P.OPDHG_FP32, max_iter=2000, lr=1e-3, windows=P.OPDHG_WINDOWS_ALWAYS)
        host = P.opdhg_solve(lp, P.opdhg_default_params(prep=P.OPDHG_PREP_HOST, **kw))
        dev = P.opdhg_solve(lp, P.opdhg_default_params(prep=P.OPDHG_PREP_DEVICE, **kw))
        _same(dev, host)


def test_device_prep_batch_and_server(P):
    lps = list(_lps().values())
    op = default_params(max_iter=3000, lr=1e-3)
    kw = dict(precision=P.OPDHG_FP32, windows=P.OPDHG_WINDOWS_OFF)
    dev = lib_params(P, op, prep=P.OPDHG_PREP_DEVICE, **kw)
    solo = [P.opdhg_solve(lp, lib_params(P, op, prep=P.OPDHG_PREP_HOST, **kw)) for lp in lps]
    for got, ref in zip(P.opdhg_solve_batch(lps, dev), solo):
        _same(got, ref)
    with P.Server(64 << 20, precision=P.OPDHG_FP32) as srv:
        got = [srv.wait(srv.submit(lp, dev), 120.0) for lp in lps]
    for (name, lp), g, ref in zip(_lps().items(), got, solo):
        _same(g, ref)
        want = _oracle(name, lp, op, ())
        if want.status == oracle.pdhg.OPTIMAL:
            check_final_fp32(g[2], want, label=f"device-prepared served {name}")
        else:
            assert g[2].status == want.status and g[2].iterations == want.iterations, name


@pytest.mark.parametrize("prec_name", ["fp64", "fp32"])
def test_device_structure_falls_back_for_very_long_columns(P, prec_name):
    """A column of more than 4096 entries: the host builds the structure and
    the device rescales; a column of 4096 exactly: the device builds it.
    Both equal the host-prepared solve bit for bit and the oracle's."""
    from lpgen import random_lp
    prec = P.OPDHG_FP64 if prec_name == "fp64" else P.OPDHG_FP32
    for longest in (4096, 4097):
        lp = random_lp(21, 5000, 300, degree=("uniform", 3, 6))
        # one dense column: rows 0..longest-1 of column 0, values 1
        A = lp.csr().tolil()
        A[:, 0] = 0.0
        A[:longest, 0] = 1.0
        A = A.tocsr()
        A.sort_indices()
        lp.row_ptr = A.indptr.astype(np.int64)
        lp.col_idx = A.indices.astype(np.int32)
        lp.val = A.data.astype(float)
        assert np.bincount(lp.col_idx, minlength=lp.n)[0] == longest
        _say(f"[prep] longest column {longest}, {prec_name}, nnz {lp.nnz}")
        op = default_params(max_iter=1500, lr=1e-3, tol=1e-4)
        host = P.opdhg_solve(lp, lib_params(P, op, precision=prec, prep=P.OPDHG_PREP_HOST))
        dev = P.opdhg_solve(lp, lib_params(P, op, precision=prec, prep=P.OPDHG_PREP_DEVICE))
        _same(dev, host)
        ref = oracle.solve(lp, op)
        if prec == P.OPDHG_FP64:
            check_final_fp64(dev, ref, label=f"longest column {longest}")
        else:
            assert dev[2].status == ref.status or ref.status != oracle.pdhg.OPTIMAL


@pytest.mark.parametrize("prec_name", ["fp64", "fp32"])
def test_device_prep_long_rows_and_columns(P, prec_name):
    """Rows and columns of more than 256 nonzeros take a wave each in the
    maximum passes and the value pass (lengths that are not multiples of 64
    included); maxima and values are exact, so the result stays bitwise the
    host's."""
    from lpgen import random_lp
    prec = P.OPDHG_FP64 if prec_name == "fp64" else P.OPDHG_FP32
    lps = {
        "long rows": random_lp(11, 200, 3000, degree=("uniform", 20, 40)),
        "long columns": random_lp(12, 2000, 600, degree=("powerlaw", 1.1, 3, 1500)),
    }
    for name, lp in lps.items():
        rl = np.diff(lp.csr().indptr)
        cl = np.bincount(lp.csr().indices, minlength=lp.n)
        _say(f"[prep long] {name} {prec_name}: rows > 256: {int((rl > 256).sum())}, "
             f"columns > 256: {int((cl > 256).sum())}")
        assert (rl > 256).any() or (cl > 256).any()
        kw = dict(precision=prec, max_iter=1500, lr=1e-3, tol=1e-4)
        host = P.opdhg_solve(lp, P.opdhg_default_params(prep=P.OPDHG_PREP_HOST, **kw))
        dev = P.opdhg_solve(lp, P.opdhg_default_params(prep=P.OPDHG_PREP_DEVICE, **kw))
        _same(dev, host)


@pytest.mark.parametrize("prec_name", ["fp64", "fp32"])
def test_device_power_iteration_equals_host(P, prec_name):
    """Vanilla PDHG (constant step): the power iteration for |A~|_2 runs on
    the device after the device's rescaling. The solve equals the
    host-prepared one bit for bit, and its step size is step_scale over the
    oracle's estimate of the norm."""
    prec = P.OPDHG_FP64 if prec_name == "fp64" else P.OPDHG_FP32
    for name, lp in _lps().items():
        _say(f"[prep power] {name} {prec_name}")
        op = vanilla_params(1e-2, max_iter=1500)
        host = P.opdhg_solve(lp, lib_params(P, op, precision=prec, prep=P.OPDHG_PREP_HOST))
        dev = P.opdhg_solve(lp, lib_params(P, op, precision=prec, prep=P.OPDHG_PREP_DEVICE))
        _same(dev, host)
        slp = oracle.problem.rescale(lp, op.ruiz_iters, op.pc_beta, op.l2_rescale)
        nu = spectral_norm_estimate(slp, op.power_iters, op.power_tol)
        assert dev[2].eta == op.step_scale / nu, (name, dev[2].eta, op.step_scale / nu)
        if prec == P.OPDHG_FP64:
            check_final_fp64(dev, oracle.solve(lp, op), label=name)
