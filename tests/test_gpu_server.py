"""Serving loop on the GPU (opdhg_server_* through the C-ABI).

An LP's arithmetic depends only on its own data (rows reduced inside one
tile, exact cross-tile sums), so each result from the server must equal the
solo opdhg_solve of the same LP with the same parameters bit for bit, in
whatever mix it ran (the server runs tiles only, so the solo solves turn
windows off): submitted together, under a budget that admits only a
few at a time, or arriving while others iterate. Every served result is
also checked against the FP64 oracle's solve of the same LP: in FP64 the
same counts and the same iterate to 1e-6 per coordinate, in FP32 the same
status and the objective at the FP32 bound.
"""

import time

import numpy as np
import pytest

import oracle
from oracle.params import default_params, vanilla_params
from lpgen import config_lp
from gpu_common import check_final_fp32, check_final_fp64, lib_params

pytestmark = pytest.mark.gpu


def _P():
    import paper_2506_17650_amd as P
    P.load()
    return P


def _mix():
    lps = [config_lp("cfg0", seed=s) for s in range(3)]
    lps += [config_lp("cfg3", index=i, scale=0.02) for i in range(4)]
    lps += [config_lp("cfg4", index=i, scale=0.002) for i in range(3)]
    return lps


def _oparams(**kw):
    base = dict(tol=1e-4, max_iter=20000, lr=1e-3, phi=20)
    base.update(kw)
    return default_params(**base)


def _params(P, prec, **kw):
    # the server runs every request in tiles (one captured sequence serves
    # every mix), so the solo solves it is compared with use tiles too
    lib_kw = {k: kw.pop(k) for k in list(kw) if k in ("time_limit_s",)}
    return lib_params(P, _oparams(**kw), precision=prec, windows=P.OPDHG_WINDOWS_OFF, **lib_kw)


def _vs_oracle(P, prec, lp, res, op, label):
    if prec == P.OPDHG_FP64:
        check_final_fp64(res, oracle.solve(lp, op), label=label)
    else:
        check_final_fp32(res[2], oracle.solve(lp, op), label=label)


def _same(a, b):
    xa, ya, ra = a
    xb, yb, rb = b
    assert ra.status == rb.status
    assert ra.iterations == rb.iterations and ra.attempts == rb.attempts
    assert ra.restarts == rb.restarts
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb)
    assert ra.primal_obj == rb.primal_obj and ra.rel_kkt == rb.rel_kkt


@pytest.mark.parametrize("prec_name", ["fp32", "fp64"])
def test_mix_equals_solo(prec_name):
    P = _P()
    prec = P.OPDHG_FP32 if prec_name == "fp32" else P.OPDHG_FP64
    lps = _mix()
    solo = [P.opdhg_solve(lp, _params(P, prec)) for lp in lps]
    with P.Server(512 << 20, precision=prec) as srv:
        tickets = [srv.submit(lp, _params(P, prec)) for lp in lps]
        got = [srv.wait(t, 120.0) for t in tickets]
        st = srv.stats()
        assert st.completed == len(lps) and st.failed == 0 and st.active == 0
        lat = [srv.latency(t) for t in tickets]
    for i, (lp, a, b) in enumerate(zip(lps, got, solo)):
        _same(a, b)
        _vs_oracle(P, prec, lp, a, _oparams(), f"served LP {i} ({prec_name})")
    assert all(r.status == P.capi.OPDHG_STATUS_OPTIMAL for _, _, r in got)
    assert all(v > 0 for v in lat)


def test_tight_budget_admits_in_turn():
    P = _P()
    prec = P.OPDHG_FP32
    lps = [config_lp("cfg3", index=i, scale=0.03) for i in range(6)]
    params = _params(P, prec)
    need = [P.opdhg_workspace_bytes(lp, params) for lp in lps]
    budget = int(2.2 * max(need))  # two at a time at most
    solo = [P.opdhg_solve(lp, params) for lp in lps]
    with P.Server(64 << 20, precision=prec, budget_bytes=budget) as srv:
        tickets = [srv.submit(lp, params) for lp in lps]
        got = [srv.wait(t, 120.0) for t in tickets]
        st = srv.stats()
    assert st.peak_bytes <= budget
    assert st.completed == len(lps)
    for i, (lp, a, b) in enumerate(zip(lps, got, solo)):
        _same(a, b)
        _vs_oracle(P, prec, lp, a, _oparams(), f"budgeted LP {i}")


def test_over_budget_request_fails_alone():
    P = _P()
    prec = P.OPDHG_FP32
    small = config_lp("cfg0", seed=1)
    big = config_lp("cfg4", index=0, scale=0.01)
    params = _params(P, prec)
    budget = P.opdhg_workspace_bytes(small, params) * 2
    with P.Server(64 << 20, precision=prec, budget_bytes=budget) as srv:
        tb = srv.submit(big, params)
        ts = srv.submit(small, params)
        with pytest.raises(P.OpdhgError) as e:
            srv.wait(tb, 60.0)
        assert e.value.code == P.capi.OPDHG_ERR_OVER_BUDGET
        x, y, r = srv.wait(ts, 60.0)
    assert r.status == P.capi.OPDHG_STATUS_OPTIMAL


def test_cancel_running_and_queued():
    P = _P()
    prec = P.OPDHG_FP32
    lp = config_lp("cfg3", index=1, scale=0.05)
    endless = _params(P, prec, tol=0.0, max_iter=10**9, time_limit_s=1e9)
    with P.Server(64 << 20, precision=prec, max_active=1) as srv:
        t_run = srv.submit(lp, endless)
        t_queued = srv.submit(lp, endless)
        time.sleep(0.5)
        srv.cancel(t_queued)
        srv.cancel(t_run)
        for t in (t_run, t_queued):
            with pytest.raises(P.OpdhgError) as e:
                srv.wait(t, 60.0)
            assert e.value.code == P.capi.OPDHG_ERR_CANCELLED
        st = srv.stats()
        assert st.cancelled == 2 and st.active == 0 and st.bytes_in_use == 0
        # the server keeps serving after cancellations
        x, y, r = srv.wait(srv.submit(config_lp("cfg0", seed=2), _params(P, prec)), 60.0)
    assert r.status == P.capi.OPDHG_STATUS_OPTIMAL


def test_arrivals_while_others_iterate():
    P = _P()
    prec = P.OPDHG_FP32
    lps = [config_lp("cfg4", index=i, scale=0.003) for i in range(6)]
    params = _params(P, prec)
    solo = [P.opdhg_solve(lp, params) for lp in lps]
    with P.Server(256 << 20, precision=prec) as srv:
        tickets = []
        for lp in lps:
            tickets.append(srv.submit(lp, params))
            time.sleep(0.02)
        got = [srv.wait(t, 120.0) for t in tickets]
        assert srv.stats().replays > 0
    for i, (lp, a, b) in enumerate(zip(lps, got, solo)):
        _same(a, b)
        _vs_oracle(P, prec, lp, a, _oparams(), f"arriving LP {i}")


def test_vanilla_and_adaptive_requests_mixed():
    # the step rule and restart scheme are per request: vanilla PDHG and
    # restarted PDHG LPs iterate side by side and each equals its solo solve
    P = _P()
    prec = P.OPDHG_FP32
    lps = [config_lp("cfg0", seed=s) for s in range(4)]
    olist = [vanilla_params(lr, max_iter=20000) for lr in (0.0, 1e-1)]
    olist += [_oparams(), _oparams(lr=0.0)]
    plist = [lib_params(P, op, precision=prec, windows=P.OPDHG_WINDOWS_OFF) for op in olist]
    solo = [P.opdhg_solve(lp, q) for lp, q in zip(lps, plist)]
    with P.Server(64 << 20, precision=prec) as srv:
        tickets = [srv.submit(lp, q) for lp, q in zip(lps, plist)]
        got = [srv.wait(t, 120.0) for t in tickets]
    for i, (lp, a, b, op) in enumerate(zip(lps, got, solo, olist)):
        _same(a, b)
        _vs_oracle(P, prec, lp, a, op, f"mixed-scheme LP {i}")
    assert got[0][2].restarts == 0 and got[1][2].restarts == 0


def test_fp64_fallback_of_requests_short_of_tolerance():
    # With OPDHG_FALLBACK_FP64 an FP32 request that ends at its iteration
    # limit is solved again in FP64 with the same parameters: its result is
    # the plain FP64 solve's (and the oracle's), the server reports FP64 for
    # its ticket, and a request that reaches its tolerance keeps its FP32
    # result. Without the fallback the FP32 result comes back.
    P = _P()
    lps = [config_lp("cfg0", seed=s) for s in range(2)]
    short = _params(P, P.OPDHG_FP32, max_iter=30)  # stops at the iteration limit
    full = _params(P, P.OPDHG_FP32)
    with P.Server(256 << 20, precision=P.OPDHG_FP32, fallback=P.OPDHG_FALLBACK_FP64) as srv:
        t_short = srv.submit(lps[0], short)
        t_full = srv.submit(lps[1], full)
        got_short = srv.wait(t_short, 120.0)
        got_full = srv.wait(t_full, 120.0)
        st = srv.stats()
        prec_short, prec_full = srv.precision(t_short), srv.precision(t_full)
    assert st.fallbacks == 1 and st.completed == 2 and st.failed == 0
    assert prec_short == P.OPDHG_FP64 and prec_full == P.OPDHG_FP32
    assert got_short[2].status == P.capi.OPDHG_STATUS_ITERATION_LIMIT
    _same(got_short, P.opdhg_solve(lps[0], _params(P, P.OPDHG_FP64, max_iter=30)))
    _vs_oracle(P, P.OPDHG_FP64, lps[0], got_short, _oparams(max_iter=30), "fallback")
    assert got_full[2].status == P.capi.OPDHG_STATUS_OPTIMAL
    _same(got_full, P.opdhg_solve(lps[1], full))
    with P.Server(256 << 20, precision=P.OPDHG_FP32) as srv:
        t = srv.submit(lps[0], short)
        got = srv.wait(t, 120.0)
        assert srv.precision(t) == P.OPDHG_FP32 and srv.stats().fallbacks == 0
    assert got[2].status == P.capi.OPDHG_STATUS_ITERATION_LIMIT
    _same(got, P.opdhg_solve(lps[0], short))
