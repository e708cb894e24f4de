"""Residuals, objectives and KKT errors of an iterate.

Sign convention: the Lagrangian is L(x, y) = c^T x - y^T A x + b^T y
(Section 2, eq. (2)), so y_i >= 0 on >= rows. For the bounds l <= x <= u
the reduced cost q = c - A^T y splits into a part lambda that the bounds
can absorb and a dual residual q - lambda. Per variable, lambda is the
projection of q onto R (both bounds finite), R+ (only l finite), R- (only u
finite) or {0} (free). The dual objective is
b^T y + sum_{l finite} l_j lambda_j^+ - sum_{u finite} u_j lambda_j^-.

The primal residual is b - A x on equality rows and max(0, b - A x) on >=
rows. Iterates always satisfy l <= x <= u and y_I >= 0 by projection, so
those parts of the KKT system hold exactly and are not measured.

Readings (the paper delegates restarts and termination to PDLP):
  weighted KKT, used by restarts:  sqrt(w^2 |r_p|^2 + |r_d|^2 / w^2 + gap^2)
      on the scaled LP;
  relative KKT, used for termination: max(|r_p| / (1 + |b|),
      |r_d| / (1 + |c|), |p - d| / (1 + |p| + |d|)) on the unscaled LP.
"""

from __future__ import annotations

import math

import numpy as np

from .exact import exact_dot


def kkt_parts(slp, x: np.ndarray, y: np.ndarray, Ax: np.ndarray, ATy: np.ndarray) -> dict:
    """Squared residual norms (scaled and unscaled) and both objectives.

    x, y live in the scaled space; Ax = A~ x and ATy = A~^T y are passed in
    so callers decide how they were computed. Every sum is correctly
    rounded (module exact).
    """
    rp = slp.b - Ax
    rp = np.where(slp.ineq, np.maximum(rp, 0.0), rp)
    q = slp.c - ATy
    fl = np.isfinite(slp.l)
    fu = np.isfinite(slp.u)
    lam = np.where(fl & fu, q,
                   np.where(fl, np.maximum(q, 0.0),
                            np.where(fu, np.minimum(q, 0.0), 0.0)))
    rd = q - lam
    lam_pos = np.maximum(lam, 0.0)
    lam_neg = np.maximum(-lam, 0.0)
    bound_term = exact_dot(np.where(fl, slp.l, 0.0), lam_pos) - exact_dot(
        np.where(fu, slp.u, 0.0), lam_neg)
    pobj = exact_dot(slp.c, x) + slp.c0
    dobj = exact_dot(slp.b, y) + bound_term + slp.c0
    # unscaled residuals: b - A x = D_r^-1 (b~ - A~ x~), c - A^T y = D_c^-1 (...)
    rpu = rp / slp.Dr
    rdu = rd / slp.Dc
    return {
        "rp2": exact_dot(rp, rp),
        "rd2": exact_dot(rd, rd),
        "rp2u": exact_dot(rpu, rpu),
        "rd2u": exact_dot(rdu, rdu),
        "pobj": pobj,
        "dobj": dobj,
    }


def weighted_kkt(parts: dict, omega: float) -> float:
    """KKT error in the primal-weight norm (restart criterion; reading)."""
    gap = parts["pobj"] - parts["dobj"]
    return math.sqrt(omega * omega * parts["rp2"] + parts["rd2"] / (omega * omega) + gap * gap)


def rel_kkt(slp, parts: dict) -> tuple[float, float, float, float]:
    """(rel_primal, rel_dual, rel_gap, max of the three) on the unscaled LP."""
    rel_p = math.sqrt(parts["rp2u"]) / (1.0 + slp.b_norm)
    rel_d = math.sqrt(parts["rd2u"]) / (1.0 + slp.c_norm)
    p, d = parts["pobj"], parts["dobj"]
    rel_g = abs(p - d) / (1.0 + abs(p) + abs(d))
    return rel_p, rel_d, rel_g, max(rel_p, rel_d, rel_g)
