"""FP64 CPU oracle for restarted PDHG with online preconditioning.

TEST INFRASTRUCTURE ONLY. This package is the slow, plain reference that the
GPU library is checked against. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the solver library never does,
and it shares no code, headers, tables or helpers with the library.

It follows "Enhanced PDHG for Linear Programming with Online Preconditioning"
(Lu & Zhang): the PDHG step with adaptive step size and primal weight
(Section 3.2, eq. (6)), the online gradients (eq. (7)) and the one-step
iteration of Algorithm 1, with normalized losses and infrequent updates
(Section 3.2) and the AdaGrad schedule (Section 4.1). The paper defers the
step-size rule, the restart scheme, the rescaling defaults and the
termination test to PDLP; those parts implement the readings listed in
``oracle/params.py`` and are marked "reading" where they occur.

Modules:
  params    solver parameters and their defaults
  problem   input validation and diagonal rescaling (Ruiz, L2, Pock-Chambolle)
  kkt       residuals, objectives, duality gap, relative KKT error
  pdhg      the iteration, the learner, restarts, the solve loop and traces

Parity status: every function here is pinned by a CPU test against a fact
fixed outside the oracle (closed forms, invariants, brute-force vertex
enumeration, SciPy's HiGHS, planted optima, finite differences of the loss
definitions). The constants of the PDLP step-size rule and restart scheme
are pinned only by hand-worked examples of the readings, not by the paper.
"""

from .params import Params, default_params, vanilla_params, variant  # noqa: F401
from .problem import validate, rescale, ScaledLP  # noqa: F401
from .kkt import kkt_parts, rel_kkt, weighted_kkt  # noqa: F401
from .pdhg import (  # noqa: F401
    SolveResult,
    TraceEntry,
    pdhg_attempt,
    step_size_rule,
    online_gradients,
    learner_update,
    restart_decision,
    solve,
    solve_from_state,
    initial_state,
    spectral_norm_estimate,
)
