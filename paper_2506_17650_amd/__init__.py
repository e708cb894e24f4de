"""opdhg: restarted PDHG with online preconditioning for LP on MI355X.

The solver is libopdhg.so (HIP kernels for gfx950 behind the C-ABI of
include/opdhg.h); this package is its Python binding. See capi.py.
"""

from .capi import (  # noqa: F401
    OpdhgError,
    Server,
    Session,
    load,
    opdhg_autotune,
    opdhg_batch_workspace_bytes,
    opdhg_build_info,
    opdhg_default_params,
    opdhg_last_error,
    opdhg_rescale,
    opdhg_spectral_norm,
    opdhg_vanilla_params,
    opdhg_server_default_cfg,
    opdhg_session_create,
    opdhg_solve,
    opdhg_solve_batch,
    opdhg_solve_noalloc,
    opdhg_status_name,
    opdhg_validate,
    opdhg_workspace_bytes,
    OPDHG_FP32,
    OPDHG_FP64,
    OPDHG_RESTART_ADAPTIVE,
    OPDHG_RESTART_NONE,
    OPDHG_STEP_ADAPTIVE,
    OPDHG_STEP_CONSTANT,
    OPDHG_STEP_NORM_PLAIN,
    OPDHG_STEP_NORM_PRECOND,
    OPDHG_WINDOWS_AUTO,
    OPDHG_WINDOWS_OFF,
    OPDHG_WINDOWS_ALWAYS,
    OPDHG_PREP_AUTO,
    OPDHG_PREP_HOST,
    OPDHG_PREP_DEVICE,
    OPDHG_FALLBACK_NONE,
    OPDHG_FALLBACK_FP64,
)
