"""Restarted PDHG with online diagonal preconditioning, in plain FP64.

One iteration (Algorithm 1 of the paper):

  1. PDHG step with step size eta and primal weight w, eq. (6):
        x^{k+1/2} = x^k - (eta / w) T_k (c - A^T y^k)
        x^{k+1}   = proj_X(x^{k+1/2})                 X = [l, u]
        y^{k+1/2} = y^k + eta w S_k (b - A(2 x^{k+1} - x^k))
        y^{k+1}   = proj_Y(y^{k+1/2})                 Y = {y : y_I >= 0}
     The paper writes the standard form (X = R^n_+, Y = R^m); the box and
     the sign constraint on >= rows are the general form this solver takes.
     A step is tried with eta, judged by the step-size rule and retried with
     a smaller eta when rejected (reading of PDLP's rule, params.py); with
     the constant step of vanilla PDHG every attempt is accepted.
  2. If k mod phi != 0 the preconditioners stay.
  3. Otherwise the online gradients of eq. (7) are formed,
        G^p = -(eta / w) (g o 1[l <= x^{k+1/2} <= u]) o g,   g = c - A^T y^k
        G^d = -(eta w) (b - A x^k) o (b - A(2x^{k+1} - x^k)) o 1_dual
     (the diagonal of the outer products, since T and S are restricted to
     nonnegative diagonal matrices, Section 3.1),
  4. optionally divided by |c - A^T y^k|^2 and |b - A x^k|^2 (normalized
     online loss, Section 3.2),
  5. and T, S take one projected online-gradient step with the AdaGrad
     schedule (Section 4.1).

Every sparse product and every reduction is correctly rounded (module
exact), so the oracle's FP64 results do not depend on summation order.

Around it: evaluation every eval_every accepted iterations, restarts that
keep T, S and the AdaGrad state (Section 3.2: the next period starts from
the most recent preconditioners), termination on the relative KKT error.
T_0 = I and S_0 = I on the rescaled LP (Section 3.2).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Iterable, Optional, Union

import numpy as np

from .crmath import cr_exp, cr_log, cr_pow
from .exact import exact_dot, exact_norm, exact_spmv
from .kkt import kkt_parts, rel_kkt, weighted_kkt
from .params import (Params, RESTART_NONE, SCHEDULE_ADAGRAD_DIAG, SCHEDULE_ADAGRAD_NORM,
                     SCHEDULE_CONSTANT, STEP_CONSTANT, STEP_NORM_PRECOND)
from .problem import ScaledLP, rescale, validate

OPTIMAL = 0
ITERATION_LIMIT = 1
TIME_LIMIT = 2
NUMERICAL_ERROR = 3
RUNNING = 4  # returned only by a run paused at stop_k

STATUS_NAMES = {OPTIMAL: "OPTIMAL", ITERATION_LIMIT: "ITERATION_LIMIT",
                TIME_LIMIT: "TIME_LIMIT", NUMERICAL_ERROR: "NUMERICAL_ERROR",
                RUNNING: "RUNNING"}


@dataclasses.dataclass
class State:
    """Everything the iteration carries, in the scaled space."""

    x: np.ndarray
    y: np.ndarray
    T: np.ndarray
    S: np.ndarray
    Hp: np.ndarray  # AdaGrad accumulators (diagonal schedule)
    Hd: np.ndarray
    Hp_norm: float  # AdaGrad accumulators (norm schedule)
    Hd_norm: float
    eta: float
    omega: float
    k: int  # accepted iterations since the start (never reset)
    t: int  # accepted iterations since the last restart
    attempts: int
    restarts: int
    x_anchor: np.ndarray
    y_anchor: np.ndarray
    anchor_parts: Optional[dict]
    x_sum: np.ndarray
    y_sum: np.ndarray
    w: float  # sum of accepted step sizes in this restart period
    Ax: np.ndarray  # A~ x for the current x
    prev_cand_kkt: float

    def copy(self) -> "State":
        kw = {}
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            kw[f.name] = v.copy() if isinstance(v, np.ndarray) else (
                dict(v) if isinstance(v, dict) else v)
        return State(**kw)


@dataclasses.dataclass
class TraceEntry:
    k: int
    x: np.ndarray
    y: np.ndarray
    T: np.ndarray
    S: np.ndarray
    eta: float
    omega: float
    attempts: int
    restarts: int


@dataclasses.dataclass
class SolveResult:
    status: int
    x: np.ndarray  # unscaled
    y: np.ndarray  # unscaled
    iterations: int
    attempts: int
    restarts: int
    primal_obj: float
    dual_obj: float
    rel_primal: float
    rel_dual: float
    rel_gap: float
    rel_kkt: float
    eta: float
    omega: float
    which: str  # "current" or "average"
    trace: list
    state: State
    slp: ScaledLP

    @property
    def status_name(self) -> str:
        return STATUS_NAMES[self.status]


# ---------------------------------------------------------------------------
# the pieces of one iteration
# ---------------------------------------------------------------------------


def A_mul(slp: ScaledLP, x: np.ndarray) -> np.ndarray:
    """A~ x with correctly rounded rows."""
    return exact_spmv(slp.A.indptr, slp.A.indices, slp.A.data, x)


def AT_mul(slp: ScaledLP, y: np.ndarray) -> np.ndarray:
    """A~^T y with correctly rounded rows."""
    return exact_spmv(slp.AT.indptr, slp.AT.indices, slp.AT.data, y)


def spectral_norm_estimate(slp: ScaledLP, iters: int, tol: float) -> float:
    """Power iteration on A~^T A~ for |A~|_2 (the constant step of vanilla
    PDHG needs tau sigma |A~|_2^2 < 1, Section 2).

    v_0 = 1 / |1|; each round forms w = A~^T (A~ v), takes lam = |w| (for a
    unit v, |A~ v|^2 <= |w| <= |A~|_2^2, so lam never overshoots) and
    v = w / lam. It stops after `iters` rounds, when lam stops changing by
    more than tol relative to itself, or when w = 0. Returns sqrt(lam).
    """
    ones = np.ones(slp.n)
    v = ones / exact_norm(ones)
    lam = 0.0
    for _ in range(iters):
        w = AT_mul(slp, A_mul(slp, v))
        lam_new = exact_norm(w)
        if lam_new == 0.0:
            return 0.0
        v = w / lam_new
        done = abs(lam_new - lam) <= tol * lam_new
        lam = lam_new
        if done:
            break
    return math.sqrt(lam)


def initial_state(slp: ScaledLP, p: Optional[Params] = None) -> State:
    """Start point (reading): x = proj_X(0), y = 0, T = 1, S = 1, zero AdaGrad
    state, w = |c~| / |b~| (1 when either is tiny), eta = 1 / max |A~_ij|
    for the adaptive rule, eta = step_scale / |A~|_2 (estimate) for the
    constant step."""
    x = np.minimum(np.maximum(np.zeros(slp.n), slp.l), slp.u)
    y = np.zeros(slp.m)
    cn = exact_norm(slp.c)
    bn = exact_norm(slp.b)
    omega = cn / bn if (cn > 1e-10 and bn > 1e-10) else 1.0
    if p is not None and p.step_rule == STEP_CONSTANT:
        nu = spectral_norm_estimate(slp, p.power_iters, p.power_tol)
        eta = p.step_scale / nu if nu > 0.0 else p.step_scale
    else:
        amax = float(np.max(np.abs(slp.A.data))) if slp.A.nnz else 0.0
        eta = 1.0 / amax if amax > 0 else 1.0
    return State(
        x=x, y=y, T=np.ones(slp.n), S=np.ones(slp.m), Hp=np.zeros(slp.n), Hd=np.zeros(slp.m),
        Hp_norm=0.0, Hd_norm=0.0, eta=eta, omega=omega, k=0, t=0, attempts=0, restarts=0,
        x_anchor=x.copy(), y_anchor=y.copy(), anchor_parts=None,
        x_sum=np.zeros(slp.n), y_sum=np.zeros(slp.m), w=0.0, Ax=A_mul(slp, x),
        prev_cand_kkt=math.inf,
    )


def pdhg_attempt(slp: ScaledLP, x, y, Ax, g, T, S, eta: float, omega: float) -> dict:
    """One PDHG step with fixed (eta, w, T, S), eq. (6), on the general form.

    g = c~ - A~^T y is passed in (it does not depend on eta). The
    extrapolated product A(2x' - x) is formed as 2 A x' - A x from a fresh
    product A x' (reading; exact in exact arithmetic).
    """
    tau = eta / omega
    x_half = x - tau * T * g
    x_new = np.minimum(np.maximum(x_half, slp.l), slp.u)
    Ax_new = A_mul(slp, x_new)
    Ax_bar = 2.0 * Ax_new - Ax
    r_tilde = slp.b - Ax_bar
    sig = eta * omega
    y_half = y + sig * S * r_tilde
    y_new = np.where(slp.ineq, np.maximum(y_half, 0.0), y_half)
    return {"x_half": x_half, "x_new": x_new, "Ax_new": Ax_new, "r_tilde": r_tilde,
            "y_half": y_half, "y_new": y_new}


def step_size_rule(eta: float, omega: float, dx2: float, dy2: float, interaction: float,
                   attempts: int, p: Params) -> tuple[float, float, bool]:
    """PDLP's adaptive step (reading): returns (eta_bar, eta_next, accepted).

    eta_bar = (0.5 w |dx|^2 + 0.5 |dy|^2 / w) / |dy . A dx|, +inf when the
    interaction is zero; eta_next = min((1 - (j+1)^-0.3) eta_bar,
    (1 + (j+1)^-0.6) eta) where j counts every attempt so far, this one
    included (j >= 1, so the first factor is never 0); accepted iff
    eta <= eta_bar. The powers are correctly rounded (module crmath).
    """
    movement = 0.5 * omega * dx2 + 0.5 * dy2 / omega
    eta_bar = movement / interaction if interaction > 0.0 else math.inf
    kk = float(attempts + 1)
    first = (1.0 - cr_pow(kk, -p.step_reduction)) * eta_bar
    second = (1.0 + cr_pow(kk, -p.step_growth)) * eta
    return eta_bar, min(first, second), eta <= eta_bar


def online_gradients(slp: ScaledLP, g, x_half, r, r_tilde, y_half, eta: float,
                     omega: float) -> tuple[np.ndarray, np.ndarray]:
    """Diagonals of the online gradients of eq. (7), general form.

    Primal indicator 1[l <= x^{k+1/2} <= u] (both ends inclusive) is the
    derivative of the box projection and reduces to the paper's
    1[x^{k+1/2} >= 0] for X = R^n_+. The dual indicator is 1 on equality
    rows (the paper's unconstrained dual) and 1[y^{k+1/2} >= 0] on >= rows,
    the derivative of the sign projection. r = b - A x^k and
    r_tilde = b - A(2x^{k+1} - x^k).
    """
    tau = eta / omega
    ind_p = (x_half >= slp.l) & (x_half <= slp.u)
    Gp = np.where(ind_p, -(tau * g * g), 0.0)
    sig = eta * omega
    ind_d = np.where(slp.ineq, y_half >= 0.0, True)
    Gd = np.where(ind_d, -(sig * r * r_tilde), 0.0)
    return Gp, Gd


def _ogd_side(G: Optional[np.ndarray], scale: float, P: np.ndarray, H: np.ndarray, Hn: float,
              p: Params) -> tuple[np.ndarray, np.ndarray, float]:
    """One projected OGD step on one diagonal preconditioner.

    The gradient is G / scale (scale = 1 without normalization). The norm
    schedule accumulates |G / scale|^2 as |G|^2 / scale^2.
    """
    if G is None:
        return P, H, Hn
    if p.schedule == SCHEDULE_ADAGRAD_NORM:
        Hn = Hn + exact_dot(G, G) / (scale * scale)
    G = G / scale
    if p.schedule == SCHEDULE_ADAGRAD_DIAG:
        H = H + G * G
        step = np.where(H > 0.0, G / np.sqrt(np.where(H > 0.0, H, 1.0)), 0.0)
    elif p.schedule == SCHEDULE_ADAGRAD_NORM:
        step = G / math.sqrt(Hn) if Hn > 0.0 else np.zeros_like(G)
    elif p.schedule == SCHEDULE_CONSTANT:
        step = G
    else:
        raise ValueError("unknown schedule")
    P = np.maximum(P - p.lr * step, p.precond_floor)
    return P, H, Hn


def learner_update(Gp, Gd, g2: float, r2: float, st: State, p: Params) -> None:
    """Normalization (optional) and the projected OGD step, Algorithm 1.

    A side whose normalizer |g|^2 or |r|^2 is zero skips the update.
    The projection onto nonnegative diagonal matrices is a clamp at
    precond_floor.
    """
    sp_, sd_ = 1.0, 1.0
    if p.normalize:
        if g2 > 0.0:
            sp_ = g2
        else:
            Gp = None
        if r2 > 0.0:
            sd_ = r2
        else:
            Gd = None
    st.T, st.Hp, st.Hp_norm = _ogd_side(Gp, sp_, st.T, st.Hp, st.Hp_norm, p)
    st.S, st.Hd, st.Hd_norm = _ogd_side(Gd, sd_, st.S, st.Hd, st.Hd_norm, p)


def restart_decision(kkt_cur: float, kkt_avg: float, kkt_anchor: float, prev_cand: float,
                     t: int, k: int, p: Params) -> tuple[bool, bool, float]:
    """PDLP's adaptive restart test (reading): (restart, use_average, cand).

    The candidate is the average when its weighted KKT is strictly lower,
    else the current iterate. Restart on sufficient decay, on necessary
    decay while the candidate got worse since the last evaluation, or when
    the period is long relative to the whole run (artificial restart).
    """
    use_avg = kkt_avg < kkt_cur
    cand = kkt_avg if use_avg else kkt_cur
    restart = (cand <= p.beta_suff * kkt_anchor
               or (cand <= p.beta_nec * kkt_anchor and cand > prev_cand)
               or t >= p.beta_art * k)
    return restart, use_avg, cand


# ---------------------------------------------------------------------------
# the loop
# ---------------------------------------------------------------------------


def _evaluate(slp: ScaledLP, st: State, p: Params):
    """Evaluation at the top of an iteration: termination, then restart.

    Returns (status or None, best (x, y), which, parts, rel tuple)."""
    ATy = AT_mul(slp, st.y)
    cur = kkt_parts(slp, st.x, st.y, st.Ax, ATy)
    avg = None
    if st.w > 0.0:
        xa = st.x_sum / st.w
        ya = st.y_sum / st.w
        Axa = A_mul(slp, xa)
        avg = kkt_parts(slp, xa, ya, Axa, AT_mul(slp, ya))
    if st.anchor_parts is None:
        st.anchor_parts = cur
    rc = rel_kkt(slp, cur)
    ra = rel_kkt(slp, avg) if avg is not None else None
    if ra is not None and ra[3] < rc[3]:
        best = ((xa, ya), "average", avg, ra)
    else:
        best = ((st.x, st.y), "current", cur, rc)
    if best[3][3] <= p.tol:
        return (OPTIMAL,) + best
    if st.k >= p.max_iter:
        return (ITERATION_LIMIT,) + best
    if st.t > 0 and p.restart_scheme != RESTART_NONE:
        kc = weighted_kkt(cur, st.omega)
        ka = weighted_kkt(avg, st.omega) if avg is not None else math.inf
        kanc = weighted_kkt(st.anchor_parts, st.omega)
        restart, use_avg, cand = restart_decision(kc, ka, kanc, st.prev_cand_kkt, st.t, st.k, p)
        if restart:
            if use_avg:
                xc, yc, Axc, pc = xa, ya, Axa, avg
            else:
                xc, yc, Axc, pc = st.x, st.y, st.Ax, cur
            dxn = exact_norm(xc - st.x_anchor)
            dyn = exact_norm(yc - st.y_anchor)
            if dxn > 1e-10 and dyn > 1e-10:
                # primal-weight smoothing; exp and log correctly rounded (crmath)
                th = p.pw_smoothing
                st.omega = cr_exp(th * cr_log(dyn / dxn) + (1.0 - th) * cr_log(st.omega))
            st.x, st.y, st.Ax = xc.copy(), yc.copy(), Axc.copy()
            st.x_anchor, st.y_anchor = xc.copy(), yc.copy()
            st.anchor_parts = pc
            st.x_sum = np.zeros(slp.n)
            st.y_sum = np.zeros(slp.m)
            st.w = 0.0
            st.t = 0
            st.prev_cand_kkt = math.inf
            st.restarts += 1
        else:
            st.prev_cand_kkt = cand
    return None


def _over(d: np.ndarray, P: np.ndarray) -> np.ndarray:
    """d / P per coordinate, 0 where P = 0 (a zero preconditioner entry
    makes that coordinate's step 0)."""
    pos = P > 0.0
    return np.where(pos, d / np.where(pos, P, 1.0), 0.0)


def _iterate(slp: ScaledLP, st: State, p: Params) -> bool:
    """Algorithm 1 for one iteration; False on a numerical failure."""
    g = slp.c - AT_mul(slp, st.y)
    retries = 0
    while True:
        a = pdhg_attempt(slp, st.x, st.y, st.Ax, g, st.T, st.S, st.eta, st.omega)
        st.attempts += 1
        dx = a["x_new"] - st.x
        dy = a["y_new"] - st.y
        if p.step_norm == STEP_NORM_PRECOND:
            dx2 = exact_dot(dx, _over(dx, st.T))
            dy2 = exact_dot(dy, _over(dy, st.S))
        else:
            dx2 = exact_dot(dx, dx)
            dy2 = exact_dot(dy, dy)
        inter = abs(exact_dot(dy, a["Ax_new"] - st.Ax))
        if not (math.isfinite(dx2) and math.isfinite(dy2) and math.isfinite(inter)):
            return False
        if p.step_rule == STEP_CONSTANT:
            eta_next, accepted = st.eta, True
        else:
            _, eta_next, accepted = step_size_rule(st.eta, st.omega, dx2, dy2, inter,
                                                   st.attempts, p)
        if accepted:
            break
        st.eta = eta_next
        retries += 1
        if retries > p.max_step_retries or not (st.eta > 0.0 and math.isfinite(st.eta)):
            return False
    if p.lr > 0.0 and st.k % p.phi == 0:
        r = slp.b - st.Ax
        Gp, Gd = online_gradients(slp, g, a["x_half"], r, a["r_tilde"], a["y_half"],
                                  st.eta, st.omega)
        learner_update(Gp, Gd, exact_dot(g, g), exact_dot(r, r), st, p)
    eta = st.eta
    st.x_sum = st.x_sum + eta * a["x_new"]
    st.y_sum = st.y_sum + eta * a["y_new"]
    st.w += eta
    st.x, st.y, st.Ax = a["x_new"], a["y_new"], a["Ax_new"]
    st.k += 1
    st.t += 1
    st.eta = eta_next
    return True


def _wants(trace, k: int) -> bool:
    if trace is None or trace is False:
        return False
    if isinstance(trace, bool):
        return trace
    if isinstance(trace, int):
        return k <= trace
    return k in trace


def _result(slp: ScaledLP, st: State, status: int, best, trace) -> SolveResult:
    (xs, ys), which, parts, rel = best
    return SolveResult(
        status=status, x=slp.Dc * xs, y=slp.Dr * ys, iterations=st.k, attempts=st.attempts,
        restarts=st.restarts, primal_obj=parts["pobj"], dual_obj=parts["dobj"],
        rel_primal=rel[0], rel_dual=rel[1], rel_gap=rel[2], rel_kkt=rel[3], eta=st.eta,
        omega=st.omega, which=which, trace=trace, state=st, slp=slp)


def solve_from_state(slp: ScaledLP, st: State, p: Params,
                     trace: Union[None, int, Iterable[int]] = None,
                     stop_k: Optional[int] = None) -> SolveResult:
    """Run the loop from a given state; pause (status RUNNING) at k == stop_k."""
    tr = []
    want = set(trace) if (trace is not None and not isinstance(trace, (int, bool))) else trace
    while True:
        if _wants(want, st.k) and (not tr or tr[-1].k != st.k):
            tr.append(TraceEntry(st.k, st.x.copy(), st.y.copy(), st.T.copy(), st.S.copy(),
                                 st.eta, st.omega, st.attempts, st.restarts))
        if stop_k is not None and st.k >= stop_k:
            nan = (math.nan,) * 4
            parts = {"pobj": math.nan, "dobj": math.nan}
            return _result(slp, st, RUNNING, ((st.x, st.y), "current", parts, nan), tr)
        if st.k % p.eval_every == 0 or st.k >= p.max_iter:
            out = _evaluate(slp, st, p)
            if out is not None:
                return _result(slp, st, out[0], out[1:], tr)
        if not _iterate(slp, st, p):
            ATy = AT_mul(slp, st.y)
            parts = kkt_parts(slp, st.x, st.y, st.Ax, ATy)
            return _result(slp, st, NUMERICAL_ERROR,
                           ((st.x, st.y), "current", parts, rel_kkt(slp, parts)), tr)


def solve(lp, params: Optional[Params] = None,
          trace: Union[None, int, Iterable[int]] = None,
          stop_k: Optional[int] = None) -> SolveResult:
    """Validate, rescale, initialize and run; x and y come back unscaled."""
    p = params or Params()
    validate(lp)
    slp = rescale(lp, p.ruiz_iters, p.pc_beta, p.l2_rescale)
    st = initial_state(slp, p)
    return solve_from_state(slp, st, p, trace=trace, stop_k=stop_k)
