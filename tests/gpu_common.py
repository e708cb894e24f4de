"""Helpers shared by the GPU parity tests (not a test module).

Comparisons are element by element, so one wrong coordinate cannot hide
under the norm of a long vector:

  ew_rel(a, b)    max_j |a_j - b_j| / max(|b_j|, floor): relative error of
                  every coordinate (floor 1e-300, so a zero of the reference
                  must be matched by a zero); used where the GPU follows the
                  oracle's FP64 arithmetic.
  ew_mixed(a, b)  max_j |a_j - b_j| / (|b_j| + max_i |b_i|): relative error of
                  every coordinate against its own size plus the vector's
                  scale. Rounding enters an iterate's coordinate through the
                  step (eta / omega) T_j g_j or (eta omega) Sigma_i r_i, whose
                  size is set by the vector's scale, not by |x_j|: a
                  coordinate that passes near zero keeps an absolute error of
                  the vector's rounding level. Used for FP32 iterates.
"""

import sys

import numpy as np

import oracle

TRACE_TOL = 1e-10  # FP64 iterates over the first 200 iterations, per coordinate
FINAL_TOL = 1e-6   # FP64 final x, y and objective at rel KKT <= tol, per coordinate


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ew_rel(a, b, floor=1e-300):
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    assert a.shape == b.shape, (a.shape, b.shape)
    if a.size == 0:
        return 0.0
    d = np.abs(a - b)
    if not np.all(np.isfinite(d)):
        return np.inf
    return float(np.max(d / np.maximum(np.abs(b), floor)))


def ew_mixed(a, b):
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    assert a.shape == b.shape, (a.shape, b.shape)
    if a.size == 0:
        return 0.0
    d = np.abs(a - b)
    if not np.all(np.isfinite(d)):
        return np.inf
    scale = np.abs(b) + np.max(np.abs(b))
    if not np.any(scale > 0.0):
        return 0.0 if not np.any(d > 0.0) else np.inf
    return float(np.max(np.where(scale > 0.0, d / np.where(scale > 0.0, scale, 1.0),
                                 np.where(d > 0.0, np.inf, 0.0))))


def ew_mixed_slack(a, b, slack):
    """ew_mixed after an absolute allowance `slack` per coordinate:
    max_j max(|a_j - b_j| - slack, 0) / (|b_j| + max_i |b_i|)."""
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    if a.size == 0:
        return 0.0
    d = np.maximum(np.abs(a - b) - slack, 0.0)
    if not np.all(np.isfinite(d)):
        return np.inf
    scale = np.abs(b) + np.max(np.abs(b))
    return float(np.max(d / np.where(scale > 0.0, scale, 1.0)))


def adagrad_flip_slack(lr, phi, k):
    """Largest FP32-vs-FP64 difference of a preconditioner entry that comes
    from the learner's normalization alone, after k accepted iterations.

    The diagonal AdaGrad step moves an entry by lr G / sqrt(H) with
    H >= G^2, so by at most lr, whatever the size of G. A gradient entry near
    zero whose sign or relative size FP32 rounding changes can therefore
    move the entry by up to lr in one direction in FP32 and up to lr in the
    other in FP64: at most 2 lr per update, and there are floor((k-1)/phi)+1
    updates in the first k iterations (k >= 1).
    """
    if lr <= 0.0 or k < 1:
        return 0.0
    return 2.0 * lr * ((k - 1) // phi + 1)


def scal_rel(a, b):
    if a == b:
        return 0.0
    return abs(a - b) / abs(b) if b != 0.0 else np.inf


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


def check_final_fp64(res, ref, label=""):
    """A library result (x, y, r) against the oracle's, FP64: same status,
    counts and returned iterate; objective, x and y per coordinate within
    FINAL_TOL; the reported KKT error within 1e-6 relative."""
    x, y, r = res
    assert r.status == ref.status, (label, r.status, ref.status)
    assert r.iterations == ref.iterations and r.attempts == ref.attempts, (
        label, r.iterations, ref.iterations, r.attempts, ref.attempts)
    assert r.restarts == ref.restarts, (label, r.restarts, ref.restarts)
    assert scal_rel(r.primal_obj, ref.primal_obj) <= FINAL_TOL, (label, r.primal_obj,
                                                                 ref.primal_obj)
    ex, ey = ew_rel(x, ref.x), ew_rel(y, ref.y)
    if not (np.array_equal(x, ref.x) and np.array_equal(y, ref.y)):
        say(f"  {label}: final x, y not bit-identical (per-coordinate {ex:.2e}, {ey:.2e})")
    assert ex <= FINAL_TOL and ey <= FINAL_TOL, (label, ex, ey)
    assert abs(r.rel_kkt - ref.rel_kkt) <= 1e-6 * max(ref.rel_kkt, 1e-12) + 1e-14, (
        label, r.rel_kkt, ref.rel_kkt)


# FP32 results against the FP64 oracle at rel KKT <= 1e-4: both points are
# 1e-4-optimal, so their objectives differ by about the gap plus the
# residuals, each <= 1e-4 (1 + |p| + |d|): 2e-4 plus the FP32 rounding of x
# (~1e-7 relative), with a 5x margin. x and y are not unique (several optima),
# so only the objective and the KKT error are compared.
FP32_OBJ_TOL = 1e-3


def check_final_fp32(r, ref, tol=1e-4, label=""):
    assert r.status == ref.status == oracle.pdhg.OPTIMAL, (label, r.status, ref.status)
    assert r.rel_kkt <= tol, (label, r.rel_kkt)
    err = abs(r.primal_obj - ref.primal_obj) / (1.0 + abs(ref.primal_obj))
    assert err <= FP32_OBJ_TOL, (label, r.primal_obj, ref.primal_obj, err)
    return err
