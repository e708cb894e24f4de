"""Host-side checks of libopdhg.so that need no GPU.

- The library exports every function include/opdhg.h declares, and the
  Python binding names only exported functions.
- opdhg_validate applies the same rules as the oracle's validation.
- opdhg_rescale (host C++) gives the oracle's rescaling bit for bit: both
  compute correctly rounded sums, so no tolerance is needed.
- opdhg_workspace_bytes grows with the LP and is smaller in FP32.
No test here launches a kernel.
"""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2506_17650_amd as P
from paper_2506_17650_amd import capi
from lpgen import config_lp, tiny_lp
from oracle.problem import InvalidLP, rescale, validate

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "opdhg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(opdhg_[a-z_0-9]+)\s*\(", text)))


def exported_symbols():
    out = subprocess.run(["nm", "-D", "--defined-only", capi.LIB_PATH], check=True,
                         capture_output=True, text=True).stdout
    return {line.split()[-1] for line in out.splitlines() if line.strip()}


def test_library_exports_every_declared_function():
    assert os.path.exists(capi.LIB_PATH), "build the library first"
    decl = declared_functions()
    assert len(decl) >= 25, decl
    missing = [f for f in decl if f not in exported_symbols()]
    assert not missing, missing


def test_binding_names_only_declared_functions():
    decl = set(declared_functions())
    assert set(capi.SIGNATURES) <= decl, set(capi.SIGNATURES) - decl
    lib = P.load()
    for name in capi.SIGNATURES:
        assert getattr(lib, name) is not None


def _broken_lps():
    """One invalid LP per validation rule, from a valid tiny LP."""
    base = tiny_lp(seed=3)

    def mutate(**kw):
        import copy
        lp = copy.deepcopy(base)
        for k, v in kw.items():
            setattr(lp, k, v)
        return lp

    rp = base.row_ptr.copy()
    ci = base.col_idx.copy()
    cases = {
        "n zero": mutate(n=0, c=np.zeros(0), l=np.zeros(0), u=np.zeros(0),
                         col_idx=np.zeros(0, np.int32), val=np.zeros(0),
                         row_ptr=np.zeros(base.m + 1, np.int64)),
        "row_ptr start": mutate(row_ptr=np.r_[1, rp[1:]]),
        "row_ptr end": mutate(row_ptr=np.r_[rp[:-1], rp[-1] - 1]),
        "column range": mutate(col_idx=np.r_[ci[:-1], base.n]),
        "nan value": mutate(val=np.r_[np.nan, base.val[1:]]),
        "inf b": mutate(b=np.r_[np.inf, base.b[1:]]),
        "inf c": mutate(c=np.r_[base.c[:-1], -np.inf]),
        "l = +inf": mutate(l=np.r_[np.inf, base.l[1:]]),
        "u = -inf": mutate(u=np.r_[-np.inf, base.u[1:]]),
        "l > u": mutate(l=np.r_[base.u[0] + 1.0, base.l[1:]]),
        "sense": mutate(sense=np.r_[2, base.sense[1:]].astype(np.int8)),
    }
    # a duplicate (row, col): repeat the first column of row 0
    if rp[1] - rp[0] >= 2:
        ci2 = ci.copy()
        ci2[rp[0] + 1] = ci2[rp[0]]
        cases["duplicate"] = mutate(col_idx=ci2)
    return base, cases


def test_validate_agrees_with_oracle():
    base, cases = _broken_lps()
    assert P.opdhg_validate(base) == 0
    validate(base)
    for name, lp in cases.items():
        with pytest.raises(InvalidLP):
            validate(lp)
        assert P.opdhg_validate(lp) == capi.OPDHG_ERR_INVALID_ARGUMENT, name


@pytest.mark.parametrize("name,seed,scale", [("cfg0", 0, 1.0), ("cfg0", 5, 1.0), ("cfg1", 1, 0.05),
                                             ("cfg4", 0, 0.06)])
def test_rescale_bitwise_equal_to_oracle(name, seed, scale):
    # the last case has enough nonzeros (about 370k) that the library splits
    # its column index and its row and column passes over several host threads
    lp = config_lp(name, seed=seed, scale=scale) if name != "cfg4" else \
        config_lp(name, index=seed, scale=scale)
    sval, dr, dc = P.opdhg_rescale(lp, P.opdhg_default_params())
    ref = rescale(lp, 10, 1.0)
    assert np.array_equal(dr, ref.Dr)
    assert np.array_equal(dc, ref.Dc)
    assert np.array_equal(sval, ref.A.data)


def test_workspace_bytes_monotone_and_precision():
    small = config_lp("cfg0", seed=0)
    big = config_lp("cfg1", seed=1, scale=0.05)
    p64 = P.opdhg_default_params()
    p32 = P.opdhg_default_params(precision=P.OPDHG_FP32)
    b_small = P.opdhg_workspace_bytes(small, p64)
    b_big = P.opdhg_workspace_bytes(big, p64)
    assert 0 < b_small < b_big
    assert P.opdhg_workspace_bytes(big, p32) < b_big
    # a batch needs at least the sum of its members' slots
    assert P.opdhg_batch_workspace_bytes([small, small], p64) >= b_small


def test_binding_refuses_mismatched_lengths():
    base, _ = _broken_lps()
    import copy
    lp = copy.deepcopy(base)
    lp.c = lp.c[:-1]
    with pytest.raises(ValueError):
        P.opdhg_validate(lp)


@pytest.mark.parametrize("name,seed,scale", [("cfg0", 2, 1.0), ("cfg1", 1, 0.05),
                                             ("cfg4", 1, 0.06)])
def test_l2_rescale_and_spectral_norm_bitwise_equal_to_oracle(name, seed, scale):
    # the vanilla PDHG preprocessing (Ruiz, then the L2 pass) and the
    # power-iteration estimate behind its constant step
    from oracle.pdhg import spectral_norm_estimate
    lp = config_lp(name, seed=seed, scale=scale) if name != "cfg4" else \
        config_lp(name, index=seed, scale=scale)
    params = P.opdhg_vanilla_params(0.0)
    sval, dr, dc = P.opdhg_rescale(lp, params)
    ref = rescale(lp, 10, -1.0, l2=True)
    assert np.array_equal(dr, ref.Dr) and np.array_equal(dc, ref.Dc)
    assert np.array_equal(sval, ref.A.data)
    nu = P.opdhg_spectral_norm(lp, params)
    assert nu == spectral_norm_estimate(ref, params.power_iters, params.power_tol)
    # with the Pock-Chambolle pass too (order: Ruiz, L2, Pock-Chambolle)
    both = P.opdhg_default_params(l2_rescale=1)
    sval2, dr2, dc2 = P.opdhg_rescale(lp, both)
    ref2 = rescale(lp, 10, 1.0, l2=True)
    assert np.array_equal(dr2, ref2.Dr) and np.array_equal(sval2, ref2.A.data)


def test_new_parameters_validated():
    lp = tiny_lp(seed=3)
    for k, v in [("step_rule", 2), ("restart_scheme", -1), ("l2_rescale", 2),
                 ("power_iters", 0), ("step_scale", 0.0), ("step_scale", float("inf")),
                 ("power_tol", -1.0), ("windows", 3), ("window_buckets", 33),
                 ("window_rows", 10241), ("prep", 3)]:
        with pytest.raises(P.OpdhgError) as e:
            P.opdhg_spectral_norm(lp, P.opdhg_default_params(**{k: v}))
        assert e.value.code == capi.OPDHG_ERR_INVALID_ARGUMENT, k


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes mirror has the C compiler's size and field offsets, and
    every numeric constant of the binding the header's value."""
    import ctypes
    import shutil
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = [getattr(capi, n) for n in dir(capi)
               if isinstance(getattr(capi, n), type) and issubclass(getattr(capi, n), ctypes.Structure)
               and n.startswith("opdhg_")]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "opdhg.h"', "int main(void) {"]
    want = []
    for st in structs:
        lines.append(f'  printf("%zu\\n", sizeof({st.__name__}));')
        want.append(ctypes.sizeof(st))
        for f, _ in st._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({st.__name__}, {f}));')
            want.append(getattr(st, f).offset)
    # every numeric constant of the binding that the header defines
    import re
    with open(os.path.join(ROOT, "include", "opdhg.h")) as f:
        defined = set(re.findall(r"^#define (OPDHG_\w+) ", f.read(), re.M))
    consts = sorted(n for n in dir(capi) if n in defined and isinstance(getattr(capi, n), int))
    for n in consts:
        lines.append(f'  printf("%lld\\n", (long long)({n}));')
        want.append(getattr(capi, n))
    lines += ["  return 0;", "}"]
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "abi"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert len(structs) >= 6 and len(consts) >= 30
    assert got == want


def test_constant_step_takes_device_preparation():
    # the power iteration behind the constant step runs on the device too:
    # the parameters are accepted and the slot is sized for the device's
    # raw data, larger than a host-prepared slot
    lp = tiny_lp(seed=3)
    dev = P.opdhg_workspace_bytes(lp, P.opdhg_vanilla_params(0.0, prep=capi.OPDHG_PREP_DEVICE))
    host = P.opdhg_workspace_bytes(lp, P.opdhg_vanilla_params(0.0, prep=capi.OPDHG_PREP_HOST))
    assert dev > host


def test_server_sequences_hold_at_most_64_attempts():
    # the step-rule factor ring covers 64 attempts per launch sequence; the
    # configuration is checked before the arena or any stream is used
    lib = capi.load()
    for bad in (0, 65, 1000):
        cfg = P.opdhg_server_default_cfg(attempts_per_replay=bad)
        h = lib.opdhg_server_create(ctypes.byref(cfg), ctypes.c_void_p(256), 1 << 20,
                                    None, None, None)
        assert not h, bad
        assert "configuration" in capi.opdhg_last_error()


def test_window_plans_pass_their_checks():
    """Windowed chunks (FP32) are planned for every shape and window setting
    the GPU tests use: each plan passes the library's index checks (slice
    entries inside the entry arrays, lane rows below the chunk's rows,
    window columns inside the staged window), or workspace sizing reports
    an internal error. Windows take workspace: at the default window size
    the block-angular LPs need more than in tiles (small windows may plan
    no chunk at all)."""
    from lpgen.generators import block_angular_lp
    lps = [block_angular_lp(5, blocks=4, block_rows=3000, block_cols=8000, col_degree=6,
                            link_rows=40, link_nnz_per_row=300),
           block_angular_lp(6, blocks=3, block_rows=2500, block_cols=9000, col_degree=4,
                            link_rows=3, link_nnz_per_row=6000),
           config_lp("cfg3", index=7, scale=0.2), config_lp("cfg1", scale=0.1)]
    for i, lp in enumerate(lps):
        base = P.opdhg_default_params(precision=P.OPDHG_FP32, windows=P.OPDHG_WINDOWS_OFF)
        tiles = P.opdhg_workspace_bytes(lp, base)
        for wb, wr in [(0, 0), (1, 0), (2, 1500), (3, 2500), (8, 3000), (28, 10240)]:
            p = P.opdhg_default_params(precision=P.OPDHG_FP32, windows=P.OPDHG_WINDOWS_ALWAYS,
                                       window_buckets=wb, window_rows=wr)
            ws = P.opdhg_workspace_bytes(lp, p)
            assert ws >= tiles, (i, wb, wr)
            if i < 2 and wb == 0:
                assert ws > tiles, (i, wb, wr)


def test_prepared_handle_sizes_as_workspace_bytes():
    """opdhg_prepare runs on the host only (validation, structure, tiling,
    windows, and the scaled data when the host prepares): the handle's
    workspace size equals opdhg_workspace_bytes for every precision, window
    setting and preparation mode, and the handle's error paths report
    without touching a device."""
    lib = capi.load()
    lps = [config_lp("cfg0", seed=1), config_lp("cfg2", scale=0.05),
           config_lp("cfg3", index=7, scale=0.2)]
    settings = [dict(), dict(precision=P.OPDHG_FP32),
                dict(precision=P.OPDHG_FP32, windows=P.OPDHG_WINDOWS_ALWAYS),
                dict(precision=P.OPDHG_FP32, prep=P.OPDHG_PREP_DEVICE),
                dict(prep=P.OPDHG_PREP_HOST)]
    for i, lp in enumerate(lps):
        a = capi._LPArrays(lp)
        for kw in settings:
            p = P.opdhg_default_params(**kw)
            pr = ctypes.c_void_p()
            capi._check(lib.opdhg_prepare(ctypes.byref(a.struct), ctypes.byref(p),
                                          ctypes.byref(pr)))
            try:
                got = ctypes.c_size_t(0)
                capi._check(lib.opdhg_prepared_bytes(pr, ctypes.byref(got)))
                assert got.value == P.opdhg_workspace_bytes(lp, p), (i, kw)
                # no workspace: refused before any device work, handle still unused
                h = ctypes.c_void_p()
                rc = lib.opdhg_session_create_prepared(pr, None, got.value, None, ctypes.byref(h))
                assert rc == capi.OPDHG_ERR_INVALID_ARGUMENT and not h.value
            finally:
                lib.opdhg_prepared_destroy(pr)
    # invalid LP and parameters are refused by opdhg_prepare, with no handle
    bad = tiny_lp(1)
    a = capi._LPArrays(bad)
    a.struct.m = -1
    pr = ctypes.c_void_p()
    p = P.opdhg_default_params()
    assert lib.opdhg_prepare(ctypes.byref(a.struct), ctypes.byref(p), ctypes.byref(pr)) != 0
    assert not pr.value
    a = capi._LPArrays(tiny_lp(2))
    p = P.opdhg_default_params(tol=-1.0)
    assert lib.opdhg_prepare(ctypes.byref(a.struct), ctypes.byref(p), ctypes.byref(pr)) \
        == capi.OPDHG_ERR_INVALID_ARGUMENT
    assert not pr.value
    assert lib.opdhg_prepared_bytes(None, ctypes.byref(ctypes.c_size_t(0))) \
        == capi.OPDHG_ERR_INVALID_ARGUMENT
    assert lib.opdhg_session_create_prepared(None, None, 0, None, ctypes.byref(ctypes.c_void_p())) \
        == capi.OPDHG_ERR_INVALID_ARGUMENT
    lib.opdhg_prepared_destroy(None)
