"""Python binding of libcm (``include/cm.h``): argument marshalling only.

Every step of a sweep runs in libcm's HIP kernels.  PyTorch provides device
memory and the stream: buffers are ``torch`` CUDA tensors whose data
pointers go through the C ABI, and launches are enqueued on
``torch.cuda.current_stream()``.  If ``libcm.so`` is missing the binding
raises; there is no fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcm.so")

ABI_VERSION = 2
OK, E_INVALID, E_BUDGET, E_DEVICE, E_UNSUPPORTED, E_BUSY = range(6)
STATUS_NAMES = {0: "CM_OK", 1: "CM_E_INVALID", 2: "CM_E_BUDGET", 3: "CM_E_DEVICE",
                4: "CM_E_UNSUPPORTED", 5: "CM_E_BUSY"}
NSTAT = 9
TC_WORDS = 6  # time course per sample: count, sums of x0, x1, x0^2, x1^2, energy
TC_SCALE = 2.0 ** 32
ST = dict(dec0=0, dec1=1, undec=2, correct=3, sumn0=4, sumn1=5, sumsq0=6, sumsq1=7, flagged=8)

# every symbol include/cm.h declares
EXPORTS = ["cm_validate", "cm_workspace_bytes", "cm_create", "cm_destroy", "cm_set_tuning",
           "cm_get_tuning", "cm_launch", "cm_launch_scratch", "cm_launch_batch", "cm_launch_graph",
           "cm_graph_clear", "cm_queue_create", "cm_queue_submit", "cm_queue_poll",
           "cm_queue_destroy", "cm_launch_timecourse",
           "cm_unfused_workspace_bytes",
           "cm_launch_unfused", "cm_ddm_density", "cm_serve_config", "cm_submit", "cm_poll",
           "cm_ceiling",
           "cm_profile", "cm_profile_read", "cm_last_error"]


class CmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Model(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("kind", C.c_uint32), ("precision", C.c_uint32),
                ("n_units", C.c_uint32), ("n_stimuli", C.c_uint32), ("n_signals", C.c_uint32),
                ("params", C.POINTER(C.c_double)), ("n_params", C.c_uint32),
                ("weights", C.c_void_p), ("n_weights", C.c_uint64)]


class Sweep(C.Structure):
    _fields_ = [("grid", C.c_void_p), ("n_settings", C.c_uint64), ("trials", C.c_uint64),
                ("seed", C.c_uint64), ("max_steps", C.c_uint32), ("n_bins", C.c_uint32),
                ("reward", C.c_double), ("cost", C.c_double), ("flag_eps", C.c_double)]


class Result(C.Structure):
    _fields_ = [("hist", C.c_void_p), ("stats", C.c_void_p), ("score", C.c_void_p),
                ("best", C.c_void_p), ("run_choice", C.c_void_p), ("run_step", C.c_void_p),
                ("run_flag", C.c_void_p), ("run_state", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("block", C.c_uint32), ("runs_per_lane", C.c_uint32),
                ("steps_per_sync", C.c_uint32), ("tile_rows", C.c_uint32),
                ("lanes_per_run", C.c_uint32), ("waves_per_simd", C.c_uint32),
                ("tail_sweeps", C.c_uint32)]


class HostResult(C.Structure):
    _fields_ = [("hist", C.c_void_p), ("stats", C.c_void_p), ("score", C.c_void_p),
                ("best", C.c_void_p)]


_lib = None


def lib():
    """Load libcm.so (PyTorch first, so that one HIP runtime serves both)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  -- loads PyTorch's HIP runtime before libcm's dependency
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2110_15425_amd/build.py")
        L = C.CDLL(LIB_PATH)
        L.cm_validate.argtypes = [C.POINTER(Model), C.POINTER(Sweep)]
        L.cm_workspace_bytes.argtypes = [C.POINTER(Model), C.POINTER(Sweep), C.POINTER(C.c_uint64)]
        L.cm_create.argtypes = [C.c_int, C.POINTER(C.c_void_p)]
        L.cm_destroy.argtypes = [C.c_void_p]
        L.cm_set_tuning.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.POINTER(Tuning)]
        L.cm_get_tuning.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.POINTER(Tuning)]
        L.cm_launch.argtypes = [C.c_void_p, C.POINTER(Model), C.POINTER(Sweep), C.POINTER(Result),
                                C.c_void_p, C.c_uint64, C.c_void_p]
        L.cm_launch_scratch.argtypes = [C.c_void_p, C.POINTER(Model), C.POINTER(Sweep),
                                        C.POINTER(Result), C.c_void_p]
        L.cm_launch_batch.argtypes = [C.c_void_p, C.c_uint32, C.POINTER(Model), C.POINTER(Sweep),
                                      C.POINTER(Result), C.POINTER(C.c_void_p),
                                      C.POINTER(C.c_uint64), C.c_void_p]
        L.cm_launch_graph.argtypes = [C.c_void_p, C.c_uint32, C.POINTER(Model), C.POINTER(Sweep),
                                      C.POINTER(Result), C.POINTER(C.c_void_p),
                                      C.POINTER(C.c_uint64), C.c_void_p]
        L.cm_graph_clear.argtypes = [C.c_void_p]
        L.cm_queue_create.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                      C.c_uint32, C.POINTER(C.c_void_p)]
        L.cm_queue_submit.argtypes = [C.c_void_p, C.POINTER(Model), C.POINTER(Sweep), C.POINTER(Result),
                                      C.c_void_p, C.c_uint64, C.POINTER(HostResult), C.c_void_p,
                                      C.POINTER(C.c_uint64)]
        L.cm_queue_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_int)]
        L.cm_queue_destroy.argtypes = [C.c_void_p]
        L.cm_launch_timecourse.argtypes = [C.c_void_p, C.POINTER(Model), C.POINTER(Sweep),
                                           C.POINTER(Result), C.c_uint32, C.c_void_p, C.c_void_p,
                                           C.c_uint64, C.c_void_p]
        L.cm_unfused_workspace_bytes.argtypes = L.cm_workspace_bytes.argtypes
        L.cm_launch_unfused.argtypes = L.cm_launch.argtypes
        L.cm_ddm_density.argtypes = [C.c_void_p, C.POINTER(Model), C.POINTER(Sweep), C.c_uint32,
                                     C.c_double, C.c_void_p, C.c_void_p]
        L.cm_serve_config.argtypes = [C.c_void_p, C.c_uint32]
        L.cm_submit.argtypes = [C.c_void_p, C.c_uint32, C.POINTER(Model), C.POINTER(Sweep),
                                C.POINTER(Result), C.POINTER(C.c_void_p), C.POINTER(C.c_uint64),
                                C.POINTER(HostResult), C.c_void_p, C.POINTER(C.c_uint64)]
        L.cm_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_int)]
        L.cm_ceiling.argtypes = [C.c_void_p, C.POINTER(Model), C.c_uint32, C.c_uint64, C.c_void_p,
                                 C.c_void_p]
        L.cm_profile.argtypes = [C.c_void_p, C.c_int]
        L.cm_profile_read.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]
        L.cm_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name != "cm_last_error":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(status):
    if status != OK:
        raise CmError(status, lib().cm_last_error().decode())


def structs(w, weights_ptr=None, grid_ptr=None):
    """cm_model / cm_sweep for a workload dict; device pointers passed in."""
    params = np.ascontiguousarray(w["params"], np.float64)
    nw = 0 if w.get("weights") is None else int(np.asarray(w["weights"]).size)
    m = Model(ABI_VERSION, int(w["kind"]), int(w["precision"]), int(w["n_units"]),
              int(w["n_stimuli"]), int(w["n_signals"]),
              params.ctypes.data_as(C.POINTER(C.c_double)), params.size,
              weights_ptr, nw)
    s = Sweep(grid_ptr, int(w["n_settings"]), int(w["trials"]), int(w["seed"]),
              int(w["max_steps"]), int(w["n_bins"]), float(w.get("reward", 0.0)),
              float(w.get("cost", 0.0)), float(w.get("flag_eps", 1e-10)))
    return m, s, params


def validate(w):
    """Host-only validation; returns the cm_status."""
    m, s, keep = structs(w, weights_ptr=None if w.get("weights") is None else 8,
                         grid_ptr=None if w["n_signals"] == 0 else 8)
    return lib().cm_validate(C.byref(m), C.byref(s))


def workspace_bytes(w):
    m, s, keep = structs(w, weights_ptr=None if w.get("weights") is None else 8,
                         grid_ptr=None if w["n_signals"] == 0 else 8)
    n = C.c_uint64(0)
    check(lib().cm_workspace_bytes(C.byref(m), C.byref(s), C.byref(n)))
    return int(n.value)


def state_width(w):
    return {0: 1, 1: 2, 3: 2}.get(int(w["kind"]), 2 + int(w["n_units"]))


class Handle:
    """A libcm handle on one device."""

    def __init__(self, device=0):
        h = C.c_void_p()
        check(lib().cm_create(int(device), C.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().cm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable=True):
        check(lib().cm_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        """(summed simulation-kernel milliseconds, number of timed launches)."""
        ms, n = C.c_double(0), C.c_uint64(0)
        check(lib().cm_profile_read(self.h, C.byref(ms), C.byref(n)))
        return float(ms.value), int(n.value)

    def set_tuning(self, kind, precision, block=0, runs_per_lane=0, steps_per_sync=0,
                   tile_rows=0, lanes_per_run=0, waves_per_simd=0, tail_sweeps=0):
        t = Tuning(block, runs_per_lane, steps_per_sync, tile_rows, lanes_per_run, waves_per_simd,
                   tail_sweeps)
        check(lib().cm_set_tuning(self.h, int(kind), int(precision), C.byref(t)))

    def get_tuning(self, kind, precision):
        t = Tuning()
        check(lib().cm_get_tuning(self.h, int(kind), int(precision), C.byref(t)))
        return dict(block=t.block, runs_per_lane=t.runs_per_lane,
                    steps_per_sync=t.steps_per_sync, tile_rows=t.tile_rows,
                    lanes_per_run=t.lanes_per_run, waves_per_simd=t.waves_per_simd,
                    tail_sweeps=t.tail_sweeps)


class DeviceSweep:
    """Device-resident inputs, outputs and workspace of one sweep.

    ``launch()`` enqueues the whole sweep on the current torch stream;
    ``results()`` synchronises and copies the outputs to numpy."""

    def __init__(self, handle, w, dumps=False):
        import torch
        self.torch = torch
        self.handle = handle
        self.w = w
        dev = torch.device("cuda", handle.device)
        S, T, B = int(w["n_settings"]), int(w["trials"]), int(w["n_bins"])
        f64 = dict(dtype=torch.float64, device=dev)
        self.weights = None
        if w.get("weights") is not None:
            self.weights = torch.as_tensor(np.asarray(w["weights"], np.float64)).to(dev)
        self.grid = None
        if int(w["n_signals"]) > 0:
            self.grid = torch.as_tensor(np.ascontiguousarray(w["grid"], np.float64)).to(dev)
        self.hist = torch.empty((S, 2, B), dtype=torch.int64, device=dev)
        self.stats = torch.empty((S, NSTAT), dtype=torch.int64, device=dev)
        scored = float(w.get("reward", 0.0)) != 0.0 or float(w.get("cost", 0.0)) != 0.0
        self.score = torch.empty(S, **f64) if scored else None
        self.best = torch.empty(2, dtype=torch.int64, device=dev) if scored else None
        self.dumps = dumps
        if dumps:
            runs = S * T
            self.run_choice = torch.empty(runs, dtype=torch.int8, device=dev)
            self.run_step = torch.empty(runs, dtype=torch.int32, device=dev)
            self.run_flag = torch.empty(runs, dtype=torch.uint8, device=dev)
            self.run_state = torch.empty((runs, state_width(w)), **f64)
        self.model, self.sweep, self._params = structs(
            w, None if self.weights is None else self.weights.data_ptr(),
            None if self.grid is None else self.grid.data_ptr())
        n = C.c_uint64(0)
        check(lib().cm_workspace_bytes(C.byref(self.model), C.byref(self.sweep), C.byref(n)))
        self.workspace = torch.empty(int(n.value), dtype=torch.uint8, device=dev)
        ptr = lambda t: None if t is None else t.data_ptr()  # noqa: E731
        self.result = Result(ptr(self.hist), ptr(self.stats), ptr(self.score), ptr(self.best),
                             ptr(self.run_choice) if dumps else None,
                             ptr(self.run_step) if dumps else None,
                             ptr(self.run_flag) if dumps else None,
                             ptr(self.run_state) if dumps else None)

    def launch_unfused(self, stream=None):
        """The same sweep node by node (ablation of the fused kernels)."""
        torch = self.torch
        st = stream if stream is not None else torch.cuda.current_stream(self.handle.device)
        n = C.c_uint64(0)
        check(lib().cm_unfused_workspace_bytes(C.byref(self.model), C.byref(self.sweep), C.byref(n)))
        if getattr(self, "uf_workspace", None) is None or self.uf_workspace.numel() < n.value:
            self.uf_workspace = torch.empty(int(n.value), dtype=torch.uint8,
                                            device=self.workspace.device)
        check(lib().cm_launch_unfused(self.handle.h, C.byref(self.model), C.byref(self.sweep),
                                      C.byref(self.result), C.c_void_p(self.uf_workspace.data_ptr()),
                                      self.uf_workspace.numel(), C.c_void_p(st.cuda_stream)))

    def launch_timecourse(self, every, stream=None):
        """cm_launch_timecourse: the sweep plus its ensemble time course, kept
        in ``self.timecourse`` ([settings, max_steps // every, 6] int64)."""
        torch = self.torch
        st = stream if stream is not None else torch.cuda.current_stream(self.handle.device)
        K = int(self.w["max_steps"]) // max(1, int(every))
        self.timecourse = torch.empty((int(self.w["n_settings"]), K, TC_WORDS), dtype=torch.int64,
                                      device=self.workspace.device)
        check(lib().cm_launch_timecourse(self.handle.h, C.byref(self.model), C.byref(self.sweep),
                                         C.byref(self.result), int(every),
                                         C.c_void_p(self.timecourse.data_ptr()),
                                         C.c_void_p(self.workspace.data_ptr()),
                                         self.workspace.numel(), C.c_void_p(st.cuda_stream)))

    def launch(self, stream=None):
        torch = self.torch
        st = stream if stream is not None else torch.cuda.current_stream(self.handle.device)
        check(lib().cm_launch(self.handle.h, C.byref(self.model), C.byref(self.sweep),
                              C.byref(self.result), C.c_void_p(self.workspace.data_ptr()),
                              self.workspace.numel(), C.c_void_p(st.cuda_stream)))

    def launch_scratch(self, stream=None):
        """cm_launch_scratch: the same sweep with the library's static scratch
        array as its workspace (this object's workspace is not used)."""
        torch = self.torch
        st = stream if stream is not None else torch.cuda.current_stream(self.handle.device)
        check(lib().cm_launch_scratch(self.handle.h, C.byref(self.model), C.byref(self.sweep),
                                      C.byref(self.result), C.c_void_p(st.cuda_stream)))

    def results(self):
        self.torch.cuda.synchronize(self.handle.device)
        out = dict(hist=self.hist.cpu().numpy().view(np.uint64),
                   stats=self.stats.cpu().numpy().view(np.uint64),
                   score=None if self.score is None else self.score.cpu().numpy(),
                   best=None if self.best is None else self.best.cpu().numpy())
        if self.dumps:
            out["run_choice"] = self.run_choice.cpu().numpy()
            out["run_step"] = self.run_step.cpu().numpy().view(np.uint32)
            out["run_flag"] = self.run_flag.cpu().numpy()
            out["run_state"] = self.run_state.cpu().numpy()
        return out


def launch_batch(handle, sweeps, stream=None):
    """Enqueue several DeviceSweeps with one cm_launch_batch call."""
    import torch
    n = len(sweeps)
    st = stream if stream is not None else torch.cuda.current_stream(handle.device)
    models = (Model * n)(*[d.model for d in sweeps])
    sws = (Sweep * n)(*[d.sweep for d in sweeps])
    res = (Result * n)(*[d.result for d in sweeps])
    wsp = (C.c_void_p * n)(*[d.workspace.data_ptr() for d in sweeps])
    wsb = (C.c_uint64 * n)(*[d.workspace.numel() for d in sweeps])
    check(lib().cm_launch_batch(handle.h, n, models, sws, res, wsp, wsb, C.c_void_p(st.cuda_stream)))


def launch_graph(handle, sweeps, stream=None):
    """Enqueue several DeviceSweeps as cm_launch_batch would, replayed from the
    handle's graph cache (cm_launch_graph): captured on the first call with
    these exact arguments, launched as one graph afterwards."""
    import torch
    n = len(sweeps)
    st = stream if stream is not None else torch.cuda.current_stream(handle.device)
    models = (Model * n)(*[d.model for d in sweeps])
    sws = (Sweep * n)(*[d.sweep for d in sweeps])
    res = (Result * n)(*[d.result for d in sweeps])
    wsp = (C.c_void_p * n)(*[d.workspace.data_ptr() for d in sweeps])
    wsb = (C.c_uint64 * n)(*[d.workspace.numel() for d in sweeps])
    check(lib().cm_launch_graph(handle.h, n, models, sws, res, wsp, wsb, C.c_void_p(st.cuda_stream)))


def graph_clear(handle):
    """Drop every graph the handle keeps (cm_graph_clear)."""
    check(lib().cm_graph_clear(handle.h))


class DeviceQueue:
    """The device work queue (cm_queue_*): one persistent kernel of one kind
    and precision fed with DeviceSweeps from the host."""

    def __init__(self, handle, kind, precision, slots=64, groups_per_cu=2, idle_us=20000):
        self.handle = handle
        q = C.c_void_p(0)
        check(lib().cm_queue_create(handle.h, int(kind), int(precision), int(slots),
                                    int(groups_per_cu), int(idle_us), C.byref(q)))
        self.q = q

    def submit(self, d, stream=None, host=None):
        """Queue a DeviceSweep after the work on ``stream`` (default: the
        current torch stream); returns its ticket.  ``host``: a dict of
        pinned tensors (see host_buffers) that the kernel fills with the
        results before it marks the request done."""
        import torch
        st = stream if stream is not None else torch.cuda.current_stream(self.handle.device)
        hr = None
        if host is not None:
            ptr = lambda k: host[k].data_ptr() if k in host else None  # noqa: E731
            hr = C.byref(HostResult(ptr("hist"), ptr("stats"), ptr("score"), ptr("best")))
        t = C.c_uint64(0)
        check(lib().cm_queue_submit(self.q, C.byref(d.model), C.byref(d.sweep), C.byref(d.result),
                                    C.c_void_p(d.workspace.data_ptr()), d.workspace.numel(), hr,
                                    C.c_void_p(st.cuda_stream), C.byref(t)))
        return t.value

    def poll(self, ticket):
        done = C.c_int(0)
        check(lib().cm_queue_poll(self.q, int(ticket), C.byref(done)))
        return bool(done.value)

    def close(self):
        if self.q:
            check(lib().cm_queue_destroy(self.q))
            self.q = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve_config(handle, n_slots):
    """Give the handle n_slots serving streams (cm_serve_config)."""
    check(lib().cm_serve_config(handle.h, int(n_slots)))


def host_buffers(d):
    """Pinned host tensors matching a DeviceSweep's hist, stats, score and best."""
    import torch
    return {k: torch.empty(v.shape, dtype=v.dtype, pin_memory=True)
            for k, v in (("hist", d.hist), ("stats", d.stats), ("score", d.score),
                         ("best", d.best)) if v is not None}


def submit(handle, sweeps, host=None, producer=None):
    """Enqueue DeviceSweeps on a free serving slot of the handle (cm_submit);
    ``host`` is a list of dicts of pinned tensors (see host_buffers) that
    receive the results.  ``producer`` is the torch stream that wrote the
    inputs (default: the current stream).  Returns the ticket, or None when
    every slot is busy."""
    import torch
    n = len(sweeps)
    prod = producer if producer is not None else torch.cuda.current_stream(handle.device)
    models = (Model * n)(*[d.model for d in sweeps])
    sws = (Sweep * n)(*[d.sweep for d in sweeps])
    res = (Result * n)(*[d.result for d in sweeps])
    wsp = (C.c_void_p * n)(*[d.workspace.data_ptr() for d in sweeps])
    wsb = (C.c_uint64 * n)(*[d.workspace.numel() for d in sweeps])
    hr = None
    if host is not None:
        ptr = lambda hh, k: hh[k].data_ptr() if k in hh else None  # noqa: E731
        hr = (HostResult * n)(*[HostResult(ptr(hh, "hist"), ptr(hh, "stats"), ptr(hh, "score"),
                                           ptr(hh, "best")) for hh in host])
    t = C.c_uint64(0)
    st = lib().cm_submit(handle.h, n, models, sws, res, wsp, wsb, hr,
                         C.c_void_p(prod.cuda_stream), C.byref(t))
    if st == E_BUSY:
        return None
    check(st)
    return int(t.value)


def poll(handle, ticket):
    """True once all work of the ticket (result copies included) has finished."""
    d = C.c_int(0)
    check(lib().cm_poll(handle.h, int(ticket), C.byref(d)))
    return bool(d.value)


def ceiling(w, steps=1000, lanes=None, reps=3, handle=None):
    """Measured step-rate ceiling of the model's random numbers and update
    (cm_ceiling): run-steps per second with every lane busy and no tests,
    refills or reductions.  lanes defaults to 8 workgroups of 256 per CU."""
    import torch
    h = handle or default_handle()
    dev = torch.device("cuda", h.device)
    if lanes is None:
        lanes = 8 * 256 * torch.cuda.get_device_properties(dev).multi_processor_count
    m, s, keep = structs(w)
    out = torch.empty(int(lanes), dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream(h.device)

    def launch():
        check(lib().cm_ceiling(h.h, C.byref(m), int(steps), int(lanes),
                               C.c_void_p(out.data_ptr()), C.c_void_p(st.cuda_stream)))

    launch()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        launch()
    e1.record(st)
    torch.cuda.synchronize(h.device)
    sec = e0.elapsed_time(e1) / 1e3 / reps
    if not torch.isfinite(out).all():
        raise RuntimeError("ceiling kernel produced a non-finite state")
    return float(steps) * float(lanes) / sec


def ddm_density(w, cells=1000, tol=1e-15, handle=None):
    """Exact first-passage probabilities of a DDM sweep's settings on the GPU:
    array [settings, 2 (lower, upper), max_steps]."""
    import torch
    h = handle or default_handle()
    dev = torch.device("cuda", h.device)
    grid = None
    if int(w["n_signals"]) > 0:
        grid = torch.as_tensor(np.ascontiguousarray(w["grid"], np.float64)).to(dev)
    m, s, keep = structs(w, None, None if grid is None else grid.data_ptr())
    out = torch.empty((int(w["n_settings"]), 2, int(w["max_steps"])), dtype=torch.float64,
                      device=dev)
    st = torch.cuda.current_stream(h.device)
    check(lib().cm_ddm_density(h.h, C.byref(m), C.byref(s), int(cells), float(tol),
                               C.c_void_p(out.data_ptr()), C.c_void_p(st.cuda_stream)))
    torch.cuda.synchronize(h.device)
    return out.cpu().numpy()


_default_handle = None


def default_handle():
    global _default_handle
    if _default_handle is None:
        _default_handle = Handle(0)
    return _default_handle


def run(w, dumps=False, handle=None):
    """Run one sweep on the GPU and return its outputs as numpy arrays
    (same keys as the oracle's)."""
    ds = DeviceSweep(handle or default_handle(), w, dumps=dumps)
    ds.launch()
    return ds.results()


def timecourse(w, every, handle=None):
    """Run one sweep with its time course on the GPU: (outputs as in run(),
    timecourse [settings, max_steps // every, 6] int64)."""
    ds = DeviceSweep(handle or default_handle(), w)
    ds.launch_timecourse(every)
    out = ds.results()
    return out, ds.timecourse.cpu().numpy()


def run_steps(w, out):
    """Executed run-steps of a sweep, from its integer statistics."""
    st = out["stats"].astype(np.uint64)
    return int(st[:, ST["sumn0"]].sum() + st[:, ST["sumn1"]].sum()
               + st[:, ST["undec"]].sum() * np.uint64(w["max_steps"]))
