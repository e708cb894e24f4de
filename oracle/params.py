"""Solver parameters of the oracle.

Values fixed by the paper (Section 4.1): relative tolerance 1e-4, update
period phi = 20 for the infrequent variants, the AdaGrad schedule, and the
online learning-rate grids. Everything else is a reading of the parts the
paper delegates to PDLP ("default values", Section 4.1; restarts "same
approach as PDLP", Section 3.2):

  step rule   eta_bar = (0.5 w |dx|^2 + 0.5 |dy|^2 / w) / |dy . A dx|
              (+inf when the interaction is 0); the next step is
              min((1 - (j+1)^-0.3) eta_bar, (1 + (j+1)^-0.6) eta); an attempt
              is accepted when eta <= eta_bar. j counts all attempts so far,
              the current one included (PDLP's counter; counting accepted
              iterations from 0 would make the first factor 0 and freeze
              eta at 0).
  restarts    every 64 accepted iterations; candidate = lower weighted KKT of
              the current and the step-weighted average iterate; restart on
              sufficient decay (0.2), necessary decay (0.8) without progress,
              or an artificial restart when t >= 0.36 k; primal weight
              smoothed with 0.5 at restarts; preconditioners and AdaGrad
              accumulators carried over (Section 3.2).
  termination max of relative primal residual, dual residual and gap on the
              unscaled LP, L2 norms, at most tol.
  rescaling   10 Ruiz passes (infinity norms, square-root split) followed by
              one Pock-Chambolle pass with beta = 1 (Section 2).
  AdaGrad     diagonal: H += G^2, P -= lr * G / sqrt(H) where H > 0, no
              epsilon; projection onto the nonnegative diagonal matrices
              (Section 3.1) is a clamp at precond_floor (default 0).
  indicators  primal: l <= x^{k+1/2} <= u (both ends inclusive), the
              derivative of the box projection; dual: 1 on equality rows and
              y^{k+1/2}_i >= 0 on >= rows, the derivative of the sign
              projection.

The vanilla PDHG of Section 4.2 (constant step sizes with tau sigma
|A|_2^2 < 1, Section 2; Ruiz then L2-norm rescaling; no restarts) is the
second configuration (readings):

  constant step  eta = step_scale / nu, nu the power-iteration estimate of
              |A~|_2 (module pdhg), so tau sigma |A~|^2 = eta^2 |A~|^2 <
              1 whenever nu > step_scale |A~|; every attempt is accepted
              and eta never changes. nu = 0 (no nonzeros) gives
              eta = step_scale.
  no restarts the evaluation every eval_every iterations only tests
              termination; the primal weight keeps its initial value and the
              average runs over all iterations.
  L2 pass     after the Ruiz passes and before the Pock-Chambolle pass:
              rows and columns divided by the square roots of their L2
              norms (0 read as 1).

A preconditioner-weighted step rule is an option (step_norm =
STEP_NORM_PRECOND): the movement of the adaptive rule measures dx and dy in
the norms of the preconditioned step, |dx|^2_{T^-1} = sum_j dx_j (dx_j / T_j)
and |dy|^2_{S^-1} likewise (a coordinate with T_j = 0 or S_i = 0 adds 0: its
step is 0), with the T and S the attempt used. With T = S = I it is the plain
rule.
"""

from __future__ import annotations

import dataclasses

SCHEDULE_ADAGRAD_DIAG = 0
SCHEDULE_ADAGRAD_NORM = 1
SCHEDULE_CONSTANT = 2

STEP_ADAPTIVE = 0
STEP_CONSTANT = 1

RESTART_ADAPTIVE = 0
RESTART_NONE = 1

STEP_NORM_PLAIN = 0
STEP_NORM_PRECOND = 1


@dataclasses.dataclass
class Params:
    tol: float = 1e-4
    max_iter: int = 100000
    lr: float = 0.0  # online learning rate alpha; 0 is plain PDLP
    phi: int = 20  # preconditioner update period
    normalize: bool = True  # normalized online loss
    schedule: int = SCHEDULE_ADAGRAD_DIAG
    precond_floor: float = 0.0
    ruiz_iters: int = 10
    pc_beta: float = 1.0  # Pock-Chambolle exponent; negative disables the pass
    eval_every: int = 64
    beta_suff: float = 0.2
    beta_nec: float = 0.8
    beta_art: float = 0.36
    pw_smoothing: float = 0.5
    step_growth: float = 0.6
    step_reduction: float = 0.3
    max_step_retries: int = 60
    step_rule: int = STEP_ADAPTIVE
    restart_scheme: int = RESTART_ADAPTIVE
    l2_rescale: bool = False
    step_scale: float = 0.9  # constant step: eta = step_scale / |A~|_2 estimate
    power_iters: int = 200  # power-iteration limit
    power_tol: float = 1e-7  # stop when the estimate of |A~|_2^2 moves less than this, relatively
    step_norm: int = STEP_NORM_PLAIN  # movement in plain or preconditioner-weighted norms


def default_params(**overrides) -> Params:
    return dataclasses.replace(Params(), **overrides)


def variant(name: str, lr: float) -> Params:
    """The four variants of Section 4.3: {NoNorm, Norm} x {Freq, Infreq}."""
    table = {
        "NoNorm-Freq": (False, 1),
        "Norm-Freq": (True, 1),
        "NoNorm-Infreq": (False, 20),
        "Norm-Infreq": (True, 20),
    }
    norm, phi = table[name]
    return default_params(lr=lr, normalize=norm, phi=phi)


def vanilla_params(lr: float, **overrides) -> Params:
    """Section 4.2: vanilla PDHG (constant steps, no restarts) after 10 Ruiz
    passes and one L2-norm pass, with the normalized online loss updated every
    iteration; iteration limit 5e4 and tolerance 1e-4."""
    base = dict(lr=lr, normalize=True, phi=1, step_rule=STEP_CONSTANT,
                restart_scheme=RESTART_NONE, l2_rescale=True, pc_beta=-1.0,
                ruiz_iters=10, max_iter=50000, tol=1e-4)
    base.update(overrides)
    return default_params(**base)
