"""The C ABI on the CPU: the library loads, exports what include/cm.h
declares, and rejects invalid arguments before touching any device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2110_15425_amd import cm, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "cm.h")).read()
    return sorted(set(re.findall(r"^(?:cm_status|const char \*)\s*(cm_\w+)\(", text, re.M)))


def test_header_and_binding_agree():
    assert _declared() == sorted(cm.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = cm.lib()
    for name in _declared():
        assert hasattr(L, name), name
    out = os.popen(f"nm -D --defined-only {cm.LIB_PATH}").read()
    for name in _declared():
        assert re.search(rf"\bT {name}$", out, re.M), name


def _status(w):
    return cm.validate(w)


def test_valid_workloads_pass_validation():
    assert _status(W.ddm()) == cm.OK
    assert _status(W.conflict()) == cm.OK
    assert _status(W.grid_search()) == cm.OK
    assert _status(W.ddm(precision=W.FP32_STEP)) == cm.OK


@pytest.mark.parametrize("change", [
    dict(trials=0), dict(max_steps=0), dict(n_bins=0), dict(n_bins=3001), dict(flag_eps=-1.0),
    dict(flag_eps=float("nan")), dict(n_settings=0), dict(trials=2 ** 31), dict(reward=float("inf")),
    dict(n_units=2), dict(n_stimuli=9), dict(kind=7), dict(precision=9),
])
def test_invalid_sweeps_are_rejected(change):
    w = W.with_(W.ddm(), **change)
    assert _status(w) == cm.E_INVALID
    assert cm.lib().cm_last_error().decode() != ""


@pytest.mark.parametrize("slot,value", [("dt", 0.0), ("dt", -1.0), ("noise", -0.1), ("thresh", 0.0),
                                        ("start", 1.0), ("start", -1.5), ("drift", float("inf"))])
def test_invalid_ddm_parameters(slot, value):
    w = W.ddm()
    p = w["params"].copy()
    p[W.DDM_P[slot]] = value
    assert _status(W.with_(w, params=p)) == cm.E_INVALID


def test_invalid_lca_shapes():
    w = W.conflict()
    assert _status(W.with_(w, weights=w["weights"][:30])) == cm.E_INVALID
    assert _status(W.with_(w, grid=np.ones((64, 3)))) == cm.E_INVALID
    p = w["params"].copy()
    p[W.LCA_P["noise"]] = -1
    assert _status(W.with_(w, params=p)) == cm.E_INVALID


def test_unsupported_combinations():
    assert _status(W.ddm(precision=W.BF16_PROJ)) == cm.E_UNSUPPORTED
    assert _status(W.conflict(precision=W.BF16_PROJ)) == cm.E_UNSUPPORTED
    assert _status(W.rnn(precision=W.FP32_STEP)) == cm.E_UNSUPPORTED


def test_rate_network_shapes():
    assert _status(W.rnn()) == cm.OK
    assert _status(W.rnn(precision=W.BF16_PROJ)) == cm.OK
    for n in (64, 128, 192):
        assert _status(W.rnn(n_units=n)) == cm.OK
    for n in (32, 100, 320):
        assert _status(W.rnn(n_units=n)) == cm.E_INVALID
    w = W.rnn()
    assert _status(W.with_(w, weights=w["weights"][:1000])) == cm.E_INVALID
    assert cm.workspace_bytes(W.rnn()) >= 256 * 256 * 8
    assert cm.workspace_bytes(W.rnn(precision=W.BF16_PROJ)) >= 256 * 256 * 2


def test_bins_times_steps_bound():
    w = W.ddm(max_steps=70_000, n_bins=70_000)
    assert _status(w) == cm.E_INVALID


def test_workspace_bytes():
    assert cm.workspace_bytes(W.ddm()) % 256 == 0
    small = cm.workspace_bytes(W.conflict())
    big = cm.workspace_bytes(W.grid_search())
    assert big >= 4096 * 9 * 2 * 8 and big > small
    with pytest.raises(cm.CmError):
        cm.workspace_bytes(W.with_(W.ddm(), trials=0))


def test_abi_version_mismatch():
    w = W.ddm()
    m, s, keep = cm.structs(w)
    m.abi_version = 99
    assert cm.lib().cm_validate(C.byref(m), C.byref(s)) == cm.E_INVALID
    assert "abi_version" in cm.lib().cm_last_error().decode()


def test_null_arguments():
    L = cm.lib()
    assert L.cm_validate(None, None) == cm.E_INVALID
    m, s, keep = cm.structs(W.ddm())
    assert L.cm_workspace_bytes(C.byref(m), C.byref(s), None) == cm.E_INVALID
    assert L.cm_launch(None, C.byref(m), C.byref(s), None, None, 0, None) == cm.E_INVALID
    assert L.cm_create(0, None) == cm.E_INVALID
    t = C.c_uint64(0)
    assert L.cm_submit(None, 1, C.byref(m), C.byref(s), None, None, None, None, None,
                       C.byref(t)) == cm.E_INVALID
    d = C.c_int(0)
    assert L.cm_poll(None, 1, C.byref(d)) == cm.E_INVALID
    assert L.cm_serve_config(None, 4) == cm.E_INVALID


def test_closed_loop_validation():
    assert cm.validate(W.control_loop()) == cm.OK
    assert cm.validate(W.control_loop(costs=[0.0, 0.1], precision=W.FP32_STEP)) == cm.OK
    for bad in (dict(levels=0), dict(levels=1.5), dict(samples=0), dict(samples=5000),
                dict(levels=4096, samples=64), dict(amax=-1.0), dict(noise=-0.1)):
        assert cm.validate(W.control_loop(**bad)) == cm.E_INVALID, bad
    assert cm.validate(W.control_loop(precision=W.BF16_PROJ)) == cm.E_UNSUPPORTED
    w = W.control_loop(levels=10)
    assert cm.workspace_bytes(w) >= 100 * 9 * 2 * 8
    m, s, keep = cm.structs(w, weights_ptr=8)
    n = C.c_uint64(0)
    assert cm.lib().cm_unfused_workspace_bytes(C.byref(m), C.byref(s), C.byref(n)) == cm.E_UNSUPPORTED



def test_unfused_rejects_sweeps_beyond_32bit_run_indices():
    """The node-by-node kernels index runs with 32 bits: sweeps of 2^32 runs
    or more are refused (CM_E_INVALID) before anything is enqueued, up to
    2^32 - 1 accepted."""
    n = C.c_uint64(0)
    big = W.ddm(trials=(1 << 31) - 1, drifts=[0.1, 0.2, 0.3])  # 3 (2^31 - 1) > 2^32
    m, s, keep = cm.structs(big, grid_ptr=256)
    assert cm.lib().cm_validate(C.byref(m), C.byref(s)) == cm.OK
    assert cm.lib().cm_unfused_workspace_bytes(C.byref(m), C.byref(s), C.byref(n)) == cm.E_INVALID
    assert "2^32" in cm.lib().cm_last_error().decode()
    assert cm.lib().cm_launch_unfused(None, C.byref(m), C.byref(s), None, None, 0, None) == cm.E_INVALID
    ok = W.ddm(trials=(1 << 31) - 1, drifts=[0.1, 0.2])  # 2^32 - 2 runs
    m, s, keep = cm.structs(ok, grid_ptr=256)
    assert cm.lib().cm_unfused_workspace_bytes(C.byref(m), C.byref(s), C.byref(n)) == cm.OK
    assert n.value > 0
