"""ctypes binding of libopdhg.so: the C-ABI of include/opdhg.h, same names.

Argument marshalling only: LP arrays become contiguous host arrays of the
declared types, device workspaces come from torch (``torch.empty(...,
device="cuda")``) and streams from ``torch.cuda`` stream handles. Every step
of the solve runs in the library's HIP kernels; if the library is missing
this module raises instead of computing anything itself.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libopdhg.so")

# ---- constants (include/opdhg.h) ----
OPDHG_OK = 0
OPDHG_ERR_INVALID_ARGUMENT = -1
OPDHG_ERR_WORKSPACE_TOO_SMALL = -2
OPDHG_ERR_OVER_BUDGET = -3
OPDHG_ERR_DEVICE = -4
OPDHG_ERR_NOT_READY = -5
OPDHG_ERR_CANCELLED = -6
OPDHG_ERR_UNKNOWN_TICKET = -7
OPDHG_NOALLOC_SCRATCH_BYTES = 64 << 20  # static device scratch of opdhg_solve_noalloc

OPDHG_STATUS_OPTIMAL = 0
OPDHG_STATUS_ITERATION_LIMIT = 1
OPDHG_STATUS_TIME_LIMIT = 2
OPDHG_STATUS_NUMERICAL_ERROR = 3
OPDHG_STATUS_RUNNING = 4

OPDHG_FP64 = 0
OPDHG_FP32 = 1

OPDHG_SCHEDULE_ADAGRAD_DIAG = 0
OPDHG_SCHEDULE_ADAGRAD_NORM = 1
OPDHG_SCHEDULE_CONSTANT = 2
OPDHG_STEP_ADAPTIVE = 0
OPDHG_STEP_CONSTANT = 1
OPDHG_RESTART_ADAPTIVE = 0
OPDHG_RESTART_NONE = 1
OPDHG_STEP_NORM_PLAIN = 0
OPDHG_STEP_NORM_PRECOND = 1
OPDHG_WINDOWS_AUTO = 0
OPDHG_WINDOWS_OFF = 1
OPDHG_WINDOWS_ALWAYS = 2
OPDHG_PREP_AUTO = 0
OPDHG_PREP_HOST = 1
OPDHG_PREP_DEVICE = 2
OPDHG_FALLBACK_NONE = 0
OPDHG_FALLBACK_FP64 = 1

_p = ctypes.POINTER
c_i64, c_i32, c_dbl, c_sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t


class opdhg_lp(ctypes.Structure):
    _fields_ = [
        ("m", c_i64), ("n", c_i64), ("nnz", c_i64),
        ("row_ptr", _p(c_i64)), ("col_idx", _p(c_i32)), ("val", _p(c_dbl)),
        ("b", _p(c_dbl)), ("row_sense", _p(ctypes.c_int8)), ("c", _p(c_dbl)),
        ("l", _p(c_dbl)), ("u", _p(c_dbl)), ("obj_offset", c_dbl),
    ]


class opdhg_params(ctypes.Structure):
    _fields_ = [
        ("tol", c_dbl), ("max_iter", c_i64), ("time_limit_s", c_dbl),
        ("precision", c_i32), ("schedule", c_i32), ("lr", c_dbl), ("phi", c_i32),
        ("normalize", c_i32), ("precond_floor", c_dbl), ("ruiz_iters", c_i32),
        ("pc_beta", c_dbl), ("eval_every", c_i32), ("max_step_retries", c_i32),
        ("beta_suff", c_dbl), ("beta_nec", c_dbl), ("beta_art", c_dbl),
        ("pw_smoothing", c_dbl), ("step_growth", c_dbl), ("step_reduction", c_dbl),
        ("tile_nnz", c_i32), ("lanes", c_i32), ("workgroups", c_i32),
        ("step_rule", c_i32), ("restart_scheme", c_i32), ("l2_rescale", c_i32),
        ("power_iters", c_i32), ("step_scale", c_dbl), ("power_tol", c_dbl),
        ("step_norm", c_i32), ("windows", c_i32), ("window_buckets", c_i32),
        ("window_rows", c_i32), ("prep", c_i32), ("eval_slots", c_i32),
    ]


class opdhg_result(ctypes.Structure):
    _fields_ = [
        ("status", c_i32), ("which", c_i32), ("iterations", c_i64), ("attempts", c_i64),
        ("restarts", c_i64), ("primal_obj", c_dbl), ("dual_obj", c_dbl),
        ("rel_primal", c_dbl), ("rel_dual", c_dbl), ("rel_gap", c_dbl), ("rel_kkt", c_dbl),
        ("solve_seconds", c_dbl), ("eta", c_dbl), ("omega", c_dbl),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class opdhg_state(ctypes.Structure):
    _fields_ = [
        ("k", c_i64), ("t", c_i64), ("attempts", c_i64), ("restarts", c_i64),
        ("status", c_i32), ("need_eval", c_i32), ("eta", c_dbl), ("omega", c_dbl),
        ("w", c_dbl),
    ]


class opdhg_server_cfg(ctypes.Structure):
    _fields_ = [
        ("budget_bytes", c_sz), ("max_active", c_i32), ("attempts_per_replay", c_i32),
        ("precision", c_i32), ("workgroups", c_i32), ("prep_threads", c_i32),
        ("fallback", c_i32), ("poll_interval_s", c_dbl),
    ]


class opdhg_server_stats(ctypes.Structure):
    _fields_ = [
        ("submitted", c_i64), ("completed", c_i64), ("cancelled", c_i64), ("failed", c_i64),
        ("active", c_i64), ("queued", c_i64), ("replays", c_i64), ("bytes_in_use", c_sz),
        ("peak_bytes", c_sz), ("fallbacks", c_i64),
    ]


class opdhg_tuning(ctypes.Structure):
    _fields_ = [
        ("tile_nnz", c_i32), ("lanes", c_i32), ("workgroups", c_i32), ("candidates", c_i32),
        ("attempts_per_s", c_dbl), ("default_attempts_per_s", c_dbl),
        ("executed_fraction", c_dbl), ("windows", c_i32), ("window_rows", c_i32),
    ]


# exported symbols and their signatures (restype, argtypes)
SIGNATURES = {
    "opdhg_default_params": (None, [_p(opdhg_params)]),
    "opdhg_validate": (c_i32, [_p(opdhg_lp)]),
    "opdhg_workspace_bytes": (c_i32, [_p(opdhg_lp), _p(opdhg_params), _p(c_sz)]),
    "opdhg_rescale": (c_i32, [_p(opdhg_lp), _p(opdhg_params), _p(c_dbl), _p(c_dbl), _p(c_dbl)]),
    "opdhg_spectral_norm": (c_i32, [_p(opdhg_lp), _p(opdhg_params), _p(c_dbl)]),
    "opdhg_solve": (c_i32, [_p(opdhg_lp), _p(opdhg_params), ctypes.c_void_p, c_sz,
                            ctypes.c_void_p, _p(c_dbl), _p(c_dbl), _p(opdhg_result)]),
    "opdhg_solve_noalloc": (c_i32, [_p(opdhg_lp), _p(opdhg_params), ctypes.c_void_p, _p(c_dbl),
                                    _p(c_dbl), _p(opdhg_result)]),
    "opdhg_batch_workspace_bytes": (c_i32, [c_i32, _p(opdhg_lp), _p(opdhg_params), _p(c_sz)]),
    "opdhg_solve_batch": (c_i32, [c_i32, _p(opdhg_lp), _p(opdhg_params), ctypes.c_void_p, c_sz,
                                  ctypes.c_void_p, _p(_p(c_dbl)), _p(_p(c_dbl)),
                                  _p(opdhg_result)]),
    "opdhg_batch_prepare": (c_i32, [c_i32, _p(opdhg_lp), _p(opdhg_params),
                                    _p(ctypes.c_void_p)]),
    "opdhg_batch_bytes": (c_i32, [ctypes.c_void_p, _p(c_sz)]),
    "opdhg_batch_solve": (c_i32, [ctypes.c_void_p, ctypes.c_void_p, c_sz, ctypes.c_void_p,
                                  _p(_p(c_dbl)), _p(_p(c_dbl)), _p(opdhg_result)]),
    "opdhg_batch_destroy": (None, [ctypes.c_void_p]),
    "opdhg_prepare": (c_i32, [_p(opdhg_lp), _p(opdhg_params), _p(ctypes.c_void_p)]),
    "opdhg_prepared_bytes": (c_i32, [ctypes.c_void_p, _p(c_sz)]),
    "opdhg_session_create_prepared": (c_i32, [ctypes.c_void_p, ctypes.c_void_p, c_sz,
                                              ctypes.c_void_p, _p(ctypes.c_void_p)]),
    "opdhg_prepared_destroy": (None, [ctypes.c_void_p]),
    "opdhg_autotune_workspace_bytes": (c_i32, [c_i32, _p(opdhg_lp), _p(opdhg_params), _p(c_sz)]),
    "opdhg_autotune": (c_i32, [c_i32, _p(opdhg_lp), _p(opdhg_params), ctypes.c_void_p, c_sz,
                               ctypes.c_void_p, c_i32, _p(opdhg_tuning)]),
    "opdhg_session_create": (c_i32, [_p(opdhg_lp), _p(opdhg_params), ctypes.c_void_p, c_sz,
                                     ctypes.c_void_p, _p(ctypes.c_void_p)]),
    "opdhg_session_run": (c_i32, [ctypes.c_void_p, c_i64]),
    "opdhg_session_replay": (c_i32, [ctypes.c_void_p, c_i32]),
    "opdhg_session_state": (c_i32, [ctypes.c_void_p, _p(c_dbl), _p(c_dbl), _p(c_dbl),
                                    _p(c_dbl), _p(opdhg_state)]),
    "opdhg_session_result": (c_i32, [ctypes.c_void_p, _p(c_dbl), _p(c_dbl),
                                     _p(opdhg_result)]),
    "opdhg_session_time_primal_kernel": (c_i32, [ctypes.c_void_p, c_i32, _p(c_dbl)]),
    "opdhg_session_time_kernels": (c_i32, [ctypes.c_void_p, c_i32, _p(c_dbl), _p(c_dbl)]),
    "opdhg_session_destroy": (None, [ctypes.c_void_p]),
    "opdhg_server_default_cfg": (None, [_p(opdhg_server_cfg)]),
    "opdhg_server_create": (ctypes.c_void_p, [_p(opdhg_server_cfg), ctypes.c_void_p, c_sz,
                                              ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p]),
    "opdhg_server_submit": (c_i32, [ctypes.c_void_p, _p(opdhg_lp), _p(opdhg_params),
                                    _p(ctypes.c_uint64)]),
    "opdhg_server_poll": (c_i32, [ctypes.c_void_p, ctypes.c_uint64, _p(c_dbl), _p(c_dbl),
                                  _p(opdhg_result)]),
    "opdhg_server_wait": (c_i32, [ctypes.c_void_p, ctypes.c_uint64, c_dbl, _p(c_dbl),
                                  _p(c_dbl), _p(opdhg_result)]),
    "opdhg_server_cancel": (c_i32, [ctypes.c_void_p, ctypes.c_uint64]),
    "opdhg_server_get_stats": (c_i32, [ctypes.c_void_p, _p(opdhg_server_stats)]),
    "opdhg_server_latency": (c_i32, [ctypes.c_void_p, ctypes.c_uint64, _p(c_dbl)]),
    "opdhg_server_precision": (c_i32, [ctypes.c_void_p, ctypes.c_uint64, _p(c_i32)]),
    "opdhg_server_destroy": (None, [ctypes.c_void_p]),
    "opdhg_last_error": (ctypes.c_char_p, []),
    "opdhg_status_name": (ctypes.c_char_p, [c_i32]),
    "opdhg_build_info": (ctypes.c_char_p, []),
}

_lib: Optional[ctypes.CDLL] = None


class OpdhgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"opdhg error {code}: {msg}")
        self.code = code


def load() -> ctypes.CDLL:
    """Load libopdhg.so (built in-tree); raise if it is missing.

    torch is imported first: it ships its own HIP runtime under the same
    soname, and the library must resolve to that copy so that torch's
    device pointers and stream handles are valid in the library's runtime
    (two HIP runtimes in one process do not share devices).
    """
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2506_17650_amd.build`")
    import torch  # noqa: F401  (binds the process to torch's HIP runtime)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int) -> None:
    if rc != OPDHG_OK:
        raise OpdhgError(rc, load().opdhg_last_error().decode())


def _dptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(_p(ctype))


class _LPArrays:
    """Holds contiguous copies of an LP's arrays and the opdhg_lp view."""

    def __init__(self, lp):
        self.row_ptr = np.ascontiguousarray(lp.row_ptr, dtype=np.int64)
        self.col_idx = np.ascontiguousarray(lp.col_idx, dtype=np.int32)
        self.val = np.ascontiguousarray(lp.val, dtype=np.float64)
        self.b = np.ascontiguousarray(lp.b, dtype=np.float64)
        self.sense = np.ascontiguousarray(lp.sense, dtype=np.int8)
        self.c = np.ascontiguousarray(lp.c, dtype=np.float64)
        self.l = np.ascontiguousarray(lp.l, dtype=np.float64)
        self.u = np.ascontiguousarray(lp.u, dtype=np.float64)
        self.m, self.n = int(lp.m), int(lp.n)
        nnz = self.col_idx.size
        # the C-ABI trusts these lengths; a mismatch would read past an array
        sizes = {"row_ptr": (self.row_ptr.size, self.m + 1), "val": (self.val.size, nnz),
                 "b": (self.b.size, self.m), "sense": (self.sense.size, self.m),
                 "c": (self.c.size, self.n), "l": (self.l.size, self.n),
                 "u": (self.u.size, self.n)}
        bad = {k: v for k, v in sizes.items() if v[0] != v[1]}
        if bad or self.m < 0 or self.n < 0:
            raise ValueError(f"LP array lengths do not match m={self.m}, n={self.n}, "
                             f"nnz={nnz}: {bad}")
        self.struct = opdhg_lp(
            m=self.m, n=self.n, nnz=nnz,
            row_ptr=_dptr(self.row_ptr, c_i64), col_idx=_dptr(self.col_idx, c_i32),
            val=_dptr(self.val, c_dbl), b=_dptr(self.b, c_dbl),
            row_sense=_dptr(self.sense, ctypes.c_int8), c=_dptr(self.c, c_dbl),
            l=_dptr(self.l, c_dbl), u=_dptr(self.u, c_dbl),
            obj_offset=float(getattr(lp, "obj_offset", 0.0)))


def opdhg_default_params(**overrides) -> opdhg_params:
    p = opdhg_params()
    load().opdhg_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def opdhg_vanilla_params(lr: float = 0.0, **overrides) -> opdhg_params:
    """Vanilla PDHG as run in Section 4.2: constant steps from a power
    iteration, no restarts, 10 Ruiz passes then one L2-norm pass, normalized
    online loss updated every iteration, 5e4 iterations at most."""
    base = dict(lr=lr, normalize=1, phi=1, step_rule=OPDHG_STEP_CONSTANT,
                restart_scheme=OPDHG_RESTART_NONE, l2_rescale=1, pc_beta=-1.0,
                ruiz_iters=10, max_iter=50000, tol=1e-4)
    base.update(overrides)
    return opdhg_default_params(**base)


def opdhg_validate(lp) -> int:
    a = _LPArrays(lp)
    return load().opdhg_validate(ctypes.byref(a.struct))


def opdhg_last_error() -> str:
    return load().opdhg_last_error().decode()


def opdhg_status_name(status: int) -> str:
    return load().opdhg_status_name(int(status)).decode()


def opdhg_build_info() -> str:
    return load().opdhg_build_info().decode()


def opdhg_workspace_bytes(lp, params: opdhg_params) -> int:
    a = _LPArrays(lp)
    out = c_sz(0)
    _check(load().opdhg_workspace_bytes(ctypes.byref(a.struct), ctypes.byref(params),
                                        ctypes.byref(out)))
    return int(out.value)


def opdhg_batch_workspace_bytes(lps: Sequence, params: opdhg_params) -> int:
    arrs = [_LPArrays(lp) for lp in lps]
    structs = (opdhg_lp * len(arrs))(*[a.struct for a in arrs])
    out = c_sz(0)
    _check(load().opdhg_batch_workspace_bytes(len(arrs), structs, ctypes.byref(params),
                                              ctypes.byref(out)))
    return int(out.value)


def opdhg_spectral_norm(lp, params: opdhg_params) -> float:
    """Host-only power-iteration estimate of |A~|_2 after rescaling."""
    a = _LPArrays(lp)
    out = c_dbl(0.0)
    _check(load().opdhg_spectral_norm(ctypes.byref(a.struct), ctypes.byref(params),
                                      ctypes.byref(out)))
    return out.value


def opdhg_rescale(lp, params: opdhg_params):
    """Host-only rescaling: (scaled values in CSR order, d_row, d_col)."""
    a = _LPArrays(lp)
    sval = np.empty(a.val.size)
    dr = np.empty(a.m)
    dc = np.empty(a.n)
    _check(load().opdhg_rescale(ctypes.byref(a.struct), ctypes.byref(params),
                                _dptr(sval, c_dbl), _dptr(dr, c_dbl), _dptr(dc, c_dbl)))
    return sval, dr, dc


# ---------------------------------------------------------------------------
# device memory and streams (torch)
# ---------------------------------------------------------------------------


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the opdhg solver runs only on the device")
    return torch


def device_workspace(nbytes: int):
    """A torch uint8 device tensor of at least nbytes (256-byte aligned)."""
    torch = _torch()
    return torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device="cuda")


def _ws_ptr(ws) -> tuple[int, int]:
    ptr = ws.data_ptr()
    aligned = (ptr + 255) & ~255
    return aligned, ws.numel() - (aligned - ptr)


def _stream_handle(stream) -> int:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _prepared_session(a, params, workspace, stream):
    """A session over the LP arrays a, prepared once (opdhg_prepare): its
    handle and workspace (a device tensor when none is given)."""
    lib = load()
    pr = ctypes.c_void_p()
    _check(lib.opdhg_prepare(ctypes.byref(a.struct), ctypes.byref(params), ctypes.byref(pr)))
    try:
        need = c_sz(0)
        _check(lib.opdhg_prepared_bytes(pr, ctypes.byref(need)))
        ws = workspace if workspace is not None else device_workspace(int(need.value))
        ptr, size = _ws_ptr(ws)
        h = ctypes.c_void_p()
        _check(lib.opdhg_session_create_prepared(pr, ctypes.c_void_p(ptr), size,
                                                 ctypes.c_void_p(_stream_handle(stream)),
                                                 ctypes.byref(h)))
    finally:
        lib.opdhg_prepared_destroy(pr)
    return h, ws


def opdhg_solve(lp, params: Optional[opdhg_params] = None, workspace=None, stream=None):
    """Solve one LP on the GPU: returns (x, y, opdhg_result).

    With a caller's workspace this is the C opdhg_solve. Without one the
    workspace has to be sized first; opdhg_workspace_bytes followed by
    opdhg_solve would prepare the LP twice, so the LP is prepared once
    (opdhg_prepare) and solved through the session calls, which give the
    same result bit for bit."""
    params = params or opdhg_default_params()
    a = _LPArrays(lp)
    lib = load()
    x = np.empty(a.n)
    y = np.empty(max(a.m, 1))
    res = opdhg_result()
    if workspace is not None:
        ptr, size = _ws_ptr(workspace)
        _check(lib.opdhg_solve(ctypes.byref(a.struct), ctypes.byref(params), ctypes.c_void_p(ptr),
                               size, ctypes.c_void_p(_stream_handle(stream)), _dptr(x, c_dbl),
                               _dptr(y, c_dbl), ctypes.byref(res)))
        return x, y[: a.m], res
    h, ws = _prepared_session(a, params, None, stream)
    try:
        _check(lib.opdhg_session_run(h, -1))
        _check(lib.opdhg_session_result(h, _dptr(x, c_dbl), _dptr(y, c_dbl), ctypes.byref(res)))
    finally:
        lib.opdhg_session_destroy(h)
    return x, y[: a.m], res


def opdhg_solve_noalloc(lp, params: Optional[opdhg_params] = None, stream=None):
    """opdhg_solve on the library's static device scratch (no workspace, no
    allocation): returns (x, y, opdhg_result)."""
    params = params or opdhg_default_params()
    a = _LPArrays(lp)
    x = np.empty(a.n)
    y = np.empty(a.m)
    res = opdhg_result()
    _check(load().opdhg_solve_noalloc(ctypes.byref(a.struct), ctypes.byref(params),
                                      ctypes.c_void_p(_stream_handle(stream)), _dptr(x, c_dbl),
                                      _dptr(y, c_dbl), ctypes.byref(res)))
    return x, y, res


def opdhg_solve_batch(lps: Sequence, params: Optional[opdhg_params] = None, workspace=None,
                      stream=None):
    """Solve LPs packed into one set of launches: list of (x, y, result).

    The set is prepared once (opdhg_batch_prepare), the workspace sized
    from it (a device tensor when none is given), then solved."""
    params = params or opdhg_default_params()
    arrs = [_LPArrays(lp) for lp in lps]  # borrowed by the handle until the solve
    count = len(arrs)
    structs = (opdhg_lp * count)(*[a.struct for a in arrs])
    lib = load()
    h = ctypes.c_void_p()
    _check(lib.opdhg_batch_prepare(count, structs, ctypes.byref(params), ctypes.byref(h)))
    try:
        need = c_sz(0)
        _check(lib.opdhg_batch_bytes(h, ctypes.byref(need)))
        ws = workspace if workspace is not None else device_workspace(int(need.value))
        ptr, size = _ws_ptr(ws)
        xs = [np.empty(a.n) for a in arrs]
        ys = [np.empty(max(a.m, 1)) for a in arrs]
        xp = (_p(c_dbl) * count)(*[_dptr(v, c_dbl) for v in xs])
        yp = (_p(c_dbl) * count)(*[_dptr(v, c_dbl) for v in ys])
        res = (opdhg_result * count)()
        _check(lib.opdhg_batch_solve(h, ctypes.c_void_p(ptr), size,
                                     ctypes.c_void_p(_stream_handle(stream)), xp, yp, res))
    finally:
        lib.opdhg_batch_destroy(h)
    return [(xs[i], ys[i][: arrs[i].m], res[i]) for i in range(count)]


def opdhg_autotune(lps: Sequence, params: Optional[opdhg_params] = None, replays: int = 3,
                   stream=None):
    """Time the candidate tilings on these LPs: (opdhg_tuning, tuned params)."""
    import copy
    params = params or opdhg_default_params()
    arrs = [_LPArrays(lp) for lp in lps]
    count = len(arrs)
    structs = (opdhg_lp * count)(*[a.struct for a in arrs])
    need = c_sz(0)
    _check(load().opdhg_autotune_workspace_bytes(count, structs, ctypes.byref(params),
                                                 ctypes.byref(need)))
    ws = device_workspace(int(need.value))
    ptr, size = _ws_ptr(ws)
    out = opdhg_tuning()
    _check(load().opdhg_autotune(count, structs, ctypes.byref(params), ctypes.c_void_p(ptr),
                                 size, ctypes.c_void_p(_stream_handle(stream)), int(replays),
                                 ctypes.byref(out)))
    tuned = copy.copy(params)
    tuned.tile_nnz, tuned.lanes, tuned.workgroups = out.tile_nnz, out.lanes, out.workgroups
    tuned.windows, tuned.window_rows = out.windows, out.window_rows
    return out, tuned


class Session:
    """opdhg_session_*: step an LP under host control and read its state."""

    def __init__(self, lp, params: Optional[opdhg_params] = None, stream=None):
        self.params = params or opdhg_default_params()
        self._a = _LPArrays(lp)
        self._h, self._ws = _prepared_session(self._a, self.params, None, stream)

    def run(self, k_target: int = -1) -> None:
        _check(load().opdhg_session_run(self._h, int(k_target)))

    def replay(self, replays: int) -> None:
        _check(load().opdhg_session_replay(self._h, int(replays)))

    def state(self):
        n, m = self._a.n, self._a.m
        x, y, T, S = np.empty(n), np.empty(max(m, 1)), np.empty(n), np.empty(max(m, 1))
        st = opdhg_state()
        _check(load().opdhg_session_state(self._h, _dptr(x, c_dbl), _dptr(y, c_dbl),
                                          _dptr(T, c_dbl), _dptr(S, c_dbl), ctypes.byref(st)))
        return x, y[:m], T, S[:m], st

    def result(self):
        x, y = np.empty(self._a.n), np.empty(max(self._a.m, 1))
        res = opdhg_result()
        _check(load().opdhg_session_result(self._h, _dptr(x, c_dbl), _dptr(y, c_dbl),
                                           ctypes.byref(res)))
        return x, y[: self._a.m], res

    def time_primal_kernel(self, reps: int) -> float:
        out = c_dbl(0.0)
        _check(load().opdhg_session_time_primal_kernel(self._h, int(reps), ctypes.byref(out)))
        return float(out.value)

    def time_kernels(self, reps: int) -> tuple[float, float]:
        """(primal_ms, dual_ms): average device time of one launch of each."""
        a, b = c_dbl(0.0), c_dbl(0.0)
        _check(load().opdhg_session_time_kernels(self._h, int(reps), ctypes.byref(a),
                                                 ctypes.byref(b)))
        return float(a.value), float(b.value)

    def close(self) -> None:
        if self._h:
            load().opdhg_session_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def opdhg_session_create(lp, params=None, stream=None) -> Session:
    return Session(lp, params, stream)


def opdhg_server_default_cfg(**overrides) -> opdhg_server_cfg:
    cfg = opdhg_server_cfg()
    load().opdhg_server_default_cfg(ctypes.byref(cfg))
    for k, v in overrides.items():
        setattr(cfg, k, v)
    return cfg


class Server:
    """opdhg_server_*: continuous batching of LP solves over a device arena.

    The arena is one torch uint8 device tensor of arena_bytes; the server's
    compute, upload and download streams are torch streams at default
    priority. submit() copies the LP; wait() / poll() return
    (x, y, opdhg_result) or raise OpdhgError (NOT_READY from poll while the
    solve runs).
    """

    NOT_READY = OPDHG_ERR_NOT_READY

    def __init__(self, arena_bytes: int, cfg: Optional[opdhg_server_cfg] = None, **overrides):
        torch = _torch()
        self.cfg = cfg or opdhg_server_default_cfg(**overrides)
        self._arena = device_workspace(int(arena_bytes))
        ptr, size = _ws_ptr(self._arena)
        self._streams = [torch.cuda.Stream() for _ in range(3)]
        h = load().opdhg_server_create(ctypes.byref(self.cfg), ctypes.c_void_p(ptr), size,
                                       *[ctypes.c_void_p(int(st.cuda_stream))
                                         for st in self._streams])
        if not h:
            raise OpdhgError(OPDHG_ERR_DEVICE, load().opdhg_last_error().decode())
        self._h = ctypes.c_void_p(h)
        self._shapes = {}

    def submit(self, lp, params: Optional[opdhg_params] = None) -> int:
        params = params or opdhg_default_params(precision=self.cfg.precision)
        a = _LPArrays(lp)
        t = ctypes.c_uint64(0)
        _check(load().opdhg_server_submit(self._h, ctypes.byref(a.struct), ctypes.byref(params),
                                          ctypes.byref(t)))
        self._shapes[t.value] = (a.n, a.m)
        return t.value

    def _outputs(self, ticket):
        n, m = self._shapes[ticket]
        return np.empty(n), np.empty(max(m, 1)), opdhg_result(), m

    def poll(self, ticket: int):
        x, y, res, m = self._outputs(ticket)
        rc = load().opdhg_server_poll(self._h, ctypes.c_uint64(ticket), _dptr(x, c_dbl),
                                      _dptr(y, c_dbl), ctypes.byref(res))
        if rc != OPDHG_ERR_NOT_READY:
            self._shapes.pop(ticket, None)
        _check(rc)
        return x, y[:m], res

    def wait(self, ticket: int, timeout_s: float = -1.0):
        x, y, res, m = self._outputs(ticket)
        rc = load().opdhg_server_wait(self._h, ctypes.c_uint64(ticket), float(timeout_s),
                                      _dptr(x, c_dbl), _dptr(y, c_dbl), ctypes.byref(res))
        if rc != OPDHG_ERR_NOT_READY:
            self._shapes.pop(ticket, None)
        _check(rc)
        return x, y[:m], res

    def cancel(self, ticket: int) -> None:
        _check(load().opdhg_server_cancel(self._h, ctypes.c_uint64(ticket)))

    def stats(self) -> opdhg_server_stats:
        st = opdhg_server_stats()
        _check(load().opdhg_server_get_stats(self._h, ctypes.byref(st)))
        return st

    def latency(self, ticket: int) -> float:
        out = c_dbl(0.0)
        _check(load().opdhg_server_latency(self._h, ctypes.c_uint64(ticket), ctypes.byref(out)))
        return float(out.value)

    def precision(self, ticket: int) -> int:
        """Precision of the solve that produced the ticket's result (the
        server's, or OPDHG_FP64 after a fallback)."""
        out = c_i32(0)
        _check(load().opdhg_server_precision(self._h, ctypes.c_uint64(ticket), ctypes.byref(out)))
        return int(out.value)

    def close(self) -> None:
        if self._h:
            load().opdhg_server_destroy(self._h)
            self._h = None
            torch = _torch()
            torch.cuda.synchronize()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
