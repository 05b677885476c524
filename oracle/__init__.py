"""Python face of the FP64 CPU oracle (``cmo.c``).

TEST INFRASTRUCTURE ONLY.  Tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the product path never does.  It loads
``libcmoracle.so`` (built by ``oracle/build.py``) through ctypes and shares no
code with the HIP library.

A workload is a plain dict (see ``paper_2110_15425_amd.workloads``):
``kind, precision, n_units, n_stimuli, n_signals, params, weights, grid,
n_settings, trials, seed, max_steps, n_bins, reward, cost, flag_eps``.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

NSTAT = 9
ST = dict(dec0=0, dec1=1, undec=2, correct=3, sumn0=4, sumn1=5, sumsq0=6, sumsq1=7, flagged=8)


class _Model(C.Structure):
    _fields_ = [("kind", C.c_int32), ("precision", C.c_int32), ("n_units", C.c_int32),
                ("n_stimuli", C.c_int32), ("n_signals", C.c_int32),
                ("params", C.POINTER(C.c_double)), ("n_params", C.c_int32),
                ("weights", C.POINTER(C.c_double)), ("n_weights", C.c_int64)]


class _Sweep(C.Structure):
    _fields_ = [("grid", C.POINTER(C.c_double)), ("n_settings", C.c_int64),
                ("trials", C.c_uint64), ("seed", C.c_uint64),
                ("max_steps", C.c_uint32), ("n_bins", C.c_uint32),
                ("reward", C.c_double), ("cost", C.c_double), ("flag_eps", C.c_double)]


class _Result(C.Structure):
    _fields_ = [("hist", C.POINTER(C.c_uint64)), ("stats", C.POINTER(C.c_uint64)),
                ("score", C.POINTER(C.c_double)), ("best", C.POINTER(C.c_int64)),
                ("run_choice", C.POINTER(C.c_int8)), ("run_step", C.POINTER(C.c_uint32)),
                ("run_flag", C.POINTER(C.c_uint8)), ("run_state", C.POINTER(C.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        L.cmo_run.argtypes = [C.POINTER(_Model), C.POINTER(_Sweep), C.POINTER(_Result), C.c_int]
        L.cmo_run.restype = C.c_int
        L.cmo_trajectory.argtypes = [C.POINTER(_Model), C.POINTER(_Sweep), C.c_int64, C.c_uint64,
                                     C.POINTER(C.c_double), C.POINTER(C.c_int8),
                                     C.POINTER(C.c_uint8)]
        L.cmo_trajectory.restype = C.c_uint32
        L.cmo_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.cmo_normals64.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_double)]
        L.cmo_normals32.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_float)]
        L.cmo_ddm_update.argtypes = [C.c_double] * 4
        L.cmo_ddm_update.restype = C.c_double
        L.cmo_lca_update.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double,
                                     C.c_double, C.c_double, C.c_double, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]
        L.cmo_conflict_drive.argtypes = [C.POINTER(C.c_double), C.c_double, C.c_double,
                                         C.c_double, C.c_double, C.c_double,
                                         C.POINTER(C.c_double)]
        L.cmo_conflict_correct.argtypes = [C.POINTER(C.c_double), C.c_double, C.c_double,
                                           C.POINTER(C.c_int32)]
        L.cmo_bf16_bits.argtypes = [C.c_double]
        L.cmo_bf16_bits.restype = C.c_uint16
        L.cmo_ddm_density.argtypes = [C.c_double] * 4 + [C.c_int, C.c_int, C.c_double,
                                                          C.POINTER(C.c_double),
                                                          C.POINTER(C.c_double)]
        L.cmo_ddm_density.restype = C.c_int
        L.cmo_timecourse.argtypes = [C.POINTER(_Model), C.POINTER(_Sweep), C.c_uint32,
                                     C.POINTER(C.c_int64), C.c_int]
        L.cmo_timecourse.restype = C.c_int
        L.cmo_tc_quant.argtypes = [C.c_double]
        L.cmo_tc_quant.restype = C.c_int64
        L.cmo_state_width.argtypes = [C.POINTER(_Model)]
        L.cmo_state_width.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def _structs(w):
    """Marshal a workload dict; returns (model, sweep, keepalive)."""
    params = np.ascontiguousarray(w["params"], dtype=np.float64)
    weights = w.get("weights")
    weights = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    grid = w.get("grid")
    grid = None if grid is None or w["n_signals"] == 0 else np.ascontiguousarray(grid, np.float64)
    m = _Model(int(w["kind"]), int(w["precision"]), int(w["n_units"]), int(w["n_stimuli"]),
               int(w["n_signals"]), _ptr(params, C.c_double), len(params),
               _ptr(weights, C.c_double), 0 if weights is None else weights.size)
    s = _Sweep(_ptr(grid, C.c_double), int(w["n_settings"]), int(w["trials"]), int(w["seed"]),
               int(w["max_steps"]), int(w["n_bins"]), float(w.get("reward", 0.0)),
               float(w.get("cost", 0.0)), float(w.get("flag_eps", 1e-10)))
    return m, s, (params, weights, grid)


def state_width(w):
    m, _, keep = _structs(w)
    return lib().cmo_state_width(C.byref(m))


def run(w, dumps=False, n_threads=0):
    """Run a whole sweep on the CPU.  Returns a dict of numpy arrays:
    hist [S,2,B] u64, stats [S,9] u64, score [S] f64 or None, best [2] i64 or
    None and, with dumps=True, per-run choice/step/flag/state."""
    m, s, keep = _structs(w)
    S, T, B = int(w["n_settings"]), int(w["trials"]), int(w["n_bins"])
    runs = S * T
    hist = np.zeros((S, 2, B), np.uint64)
    stats = np.zeros((S, NSTAT), np.uint64)
    scored = float(w.get("reward", 0.0)) != 0.0 or float(w.get("cost", 0.0)) != 0.0
    score = np.zeros(S, np.float64) if scored else None
    best = np.full(2, -1, np.int64) if scored else None
    out = dict(hist=hist, stats=stats, score=score, best=best)
    r = _Result(_ptr(hist, C.c_uint64), _ptr(stats, C.c_uint64), _ptr(score, C.c_double),
                _ptr(best, C.c_int64), None, None, None, None)
    if dumps:
        width = lib().cmo_state_width(C.byref(m))
        out["run_choice"] = np.zeros(runs, np.int8)
        out["run_step"] = np.zeros(runs, np.uint32)
        out["run_flag"] = np.zeros(runs, np.uint8)
        out["run_state"] = np.zeros((runs, width), np.float64)
        r.run_choice = _ptr(out["run_choice"], C.c_int8)
        r.run_step = _ptr(out["run_step"], C.c_uint32)
        r.run_flag = _ptr(out["run_flag"], C.c_uint8)
        r.run_state = _ptr(out["run_state"], C.c_double)
    rc = lib().cmo_run(C.byref(m), C.byref(s), C.byref(r), int(n_threads))
    if rc != 0:
        raise ValueError(f"oracle rejected the workload (code {rc})")
    return out


def trajectory(w, setting, trial):
    """One run's state after every executed step: (states [n, width], choice, flag)."""
    m, s, keep = _structs(w)
    width = lib().cmo_state_width(C.byref(m))
    buf = np.zeros((int(w["max_steps"]), width), np.float64)
    ch = C.c_int8(0)
    fl = C.c_uint8(0)
    n = lib().cmo_trajectory(C.byref(m), C.byref(s), int(setting), int(trial),
                             _ptr(buf, C.c_double), C.byref(ch), C.byref(fl))
    if n == 0:
        raise ValueError("oracle rejected the trajectory request")
    return buf[:n].copy(), int(ch.value), int(fl.value)


TC_WORDS = 6
TC = dict(count=0, x0=1, x1=2, x0sq=3, x1sq=4, energy=5)
TC_SCALE = 2.0 ** 32


def timecourse(w, every, n_threads=0):
    """Ensemble time course [settings, K = max_steps // every, 6] int64 (see
    cmo_timecourse: count, then fixed-point sums of x0, x1, x0^2, x1^2 and the
    conflict energy comp*x0*x1 over the runs that executed each sample step)."""
    m, s, keep = _structs(w)
    S, K = int(w["n_settings"]), int(w["max_steps"]) // int(every)
    tc = np.zeros((S, K, TC_WORDS), np.int64)
    rc = lib().cmo_timecourse(C.byref(m), C.byref(s), int(every), _ptr(tc, C.c_int64),
                              int(n_threads))
    if rc:
        raise ValueError(f"oracle rejected the time-course request (code {rc})")
    return tc


def tc_quant(v):
    return int(lib().cmo_tc_quant(float(v)))


def tc_moments(tc, scale=TC_SCALE):
    """Per (setting, sample): count and the means of x0, x1, x0^2, x1^2 and
    the energy over contributing runs (NaN where no run contributes)."""
    cnt = tc[..., 0].astype(np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        means = tc[..., 1:].astype(np.float64) / scale / cnt[..., None]
    return cnt, means


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().cmo_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(o, C.c_uint32))
    return o


def normals64(words):
    w = np.ascontiguousarray(words, np.uint32)
    z = np.zeros(2, np.float64)
    lib().cmo_normals64(_ptr(w, C.c_uint32), _ptr(z, C.c_double))
    return z


def normals32(words):
    w = np.ascontiguousarray(words, np.uint32)
    z = np.zeros(2, np.float32)
    lib().cmo_normals32(_ptr(w, C.c_uint32), _ptr(z, C.c_float))
    return z


def ddm_update(x, a, b, z):
    return lib().cmo_ddm_update(x, a, b, z)


def lca_update(x, inp, leak, comp, dt, b, z):
    xa = np.ascontiguousarray(x, np.float64)
    ia = np.ascontiguousarray(inp, np.float64)
    za = np.ascontiguousarray(z, np.float64)
    o = np.zeros(2, np.float64)
    lib().cmo_lca_update(_ptr(xa, C.c_double), _ptr(ia, C.c_double), leak, comp, dt, b,
                         _ptr(za, C.c_double), _ptr(o, C.c_double))
    return o


def conflict_drive(weights, gain, bias, offset, cA, cB):
    wt = np.ascontiguousarray(weights, np.float64)
    d = np.zeros((9, 2), np.float64)
    lib().cmo_conflict_drive(_ptr(wt, C.c_double), gain, bias, offset, cA, cB,
                             _ptr(d, C.c_double))
    return d


def conflict_correct(weights, gain, bias):
    wt = np.ascontiguousarray(weights, np.float64)
    c = np.zeros(9, np.int32)
    lib().cmo_conflict_correct(_ptr(wt, C.c_double), gain, bias, _ptr(c, C.c_int32))
    return c


def ddm_density(a, b, theta, start=0.0, cells=1000, max_steps=3000, tol=1e-15):
    """First-passage probabilities per step, (lower[N], upper[N])."""
    lo = np.zeros(max_steps, np.float64)
    up = np.zeros(max_steps, np.float64)
    rc = lib().cmo_ddm_density(a, b, theta, start, cells, max_steps, tol,
                               _ptr(lo, C.c_double), _ptr(up, C.c_double))
    if rc:
        raise ValueError("oracle rejected the density request")
    return lo, up


def bf16_bits(v):
    return int(lib().cmo_bf16_bits(float(v)))


def run_steps(w, out):
    """Executed run-steps of a sweep, from its integer statistics."""
    st = out["stats"].astype(np.uint64)
    return int(st[:, ST["sumn0"]].sum() + st[:, ST["sumn1"]].sum()
               + st[:, ST["undec"]].sum() * np.uint64(w["max_steps"]))
