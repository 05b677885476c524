"""Serving loop: continuous batching of simulation sweeps on one GPU.

Requests (workload dicts) arrive over time.  The server admits them while
the device-memory budget and a free stream allow, groups the admitted
requests of one tick into batched launches (``cm_launch_batch``: sweeps of
the same kind and precision share one simulation kernel), and puts each
group on its own stream, so work from different requests overlaps on the
device while earlier groups are still running.  The streams, their
completion events and the result copies belong to libcm's serving queue
(``cm_submit`` / ``cm_poll``).  Inputs stay resident on the device from
admission to completion; only the small integer results come back, through
pinned host buffers, and a request's latency is measured from its arrival to
the moment its results are on the host.

Results do not depend on what else is in flight: every random number is
keyed by the request's own (seed, setting, trial, step) and every reduction
is an integer sum, so a request computes the same outputs alone and in any
mix.

The scheduling core (``Scheduler``) is pure Python and device-free so it can
be tested on the CPU; ``GpuBackend`` does the device work through libcm.
"""
import collections
import time

import numpy as np

from . import cm, workloads as W


def request_bytes(w):
    """Device bytes a request holds while in flight: inputs, outputs and
    libcm workspace."""
    S, T, B = int(w["n_settings"]), int(w["trials"]), int(w["n_bins"])
    nw = 0 if w.get("weights") is None else int(np.asarray(w["weights"]).size)
    ng = 0 if int(w["n_signals"]) == 0 else S * int(w["n_signals"])
    out = S * 2 * B * 8 + S * cm.NSTAT * 8 + S * 8 + 16
    return 8 * (nw + ng) + out + cm.workspace_bytes(w)


class Request:
    __slots__ = ("rid", "w", "arrival", "admitted", "done", "result", "nbytes")

    def __init__(self, rid, w, arrival):
        self.rid, self.w, self.arrival = rid, w, arrival
        self.admitted = self.done = None
        self.result = None
        self.nbytes = request_bytes(w)


class Scheduler:
    """Admission by memory budget and free streams; FIFO among waiting
    requests, but a request that does not fit does not block smaller ones
    behind it (they may pass it while it waits for memory)."""

    def __init__(self, backend, budget_bytes, n_streams=4, max_group=12):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.n_streams = n_streams
        self.max_group = max_group
        self.waiting = collections.deque()
        self.inflight = []  # (stream index, [requests], handle)
        self.free_streams = list(range(n_streams))
        self.used = 0
        self.finished = []

    def submit(self, req):
        if req.nbytes > self.budget:
            raise ValueError(f"request {req.rid} needs {req.nbytes} bytes, budget {self.budget}")
        self.waiting.append(req)

    def _admit(self, now):
        if not self.free_streams or not self.waiting:
            return
        group, keep = [], collections.deque()
        while self.waiting:
            r = self.waiting.popleft()
            if len(group) < self.max_group and self.used + r.nbytes <= self.budget:
                self.used += r.nbytes
                r.admitted = now
                group.append(r)
            else:
                keep.append(r)
        self.waiting = keep
        if group:
            si = self.free_streams.pop()
            token = self.backend.launch(si, [r.w for r in group])
            self.inflight.append((si, group, token))

    def _reap(self, now):
        still = []
        for si, group, token in self.inflight:
            results = self.backend.poll(token)
            if results is None:
                still.append((si, group, token))
                continue
            t = self.backend.clock()
            for r, res in zip(group, results):
                r.done = t
                r.result = res
                self.used -= r.nbytes
                self.finished.append(r)
            self.free_streams.append(si)
        self.inflight = still

    def tick(self):
        now = self.backend.clock()
        self._reap(now)
        self._admit(now)

    def idle(self):
        return not self.waiting and not self.inflight

    def drain(self, sleep=0.0002):
        while not self.idle():
            self.tick()
            if sleep:
                time.sleep(sleep)


class GpuBackend:
    """Device side of the server: libcm's serving queue (``cm_submit`` /
    ``cm_poll``) with one slot per scheduler stream.  Inputs are written on
    the current torch stream, which the slot waits for; results come back
    by asynchronous copies into pinned host memory enqueued by the library
    behind the batch."""

    def __init__(self, handle, n_streams=4, dumps=False):
        import torch
        self.torch = torch
        self.h = handle
        self.dumps = dumps
        cm.serve_config(handle, n_streams)

    @staticmethod
    def clock():
        return time.perf_counter()

    def launch(self, si, ws):
        ds = [cm.DeviceSweep(self.h, w, dumps=self.dumps) for w in ws]
        host = [cm.host_buffers(d) for d in ds]
        ticket = cm.submit(self.h, ds, host)
        if ticket is None:  # the scheduler frees a slot only after its ticket is done
            raise RuntimeError("libcm reports every serving slot busy")
        return (ticket, ds, host)

    def poll(self, token):
        ticket, ds, host = token
        if not cm.poll(self.h, ticket):
            return None
        out = []
        for d, hh in zip(ds, host):
            o = {k: (t.numpy().view(np.uint64) if k in ("hist", "stats") else t.numpy())
                 for k, t in hh.items()}
            if self.dumps:  # per-run dumps stay on the device; read them after the mix
                o["device_sweep"] = d
            out.append(o)
        return out


class QueueBackend(GpuBackend):
    """GpuBackend with the device work queue in front: requests of the
    queue's kind and precision (conflict-network sweeps in FP32 steps) join
    the work of one persistent kernel as they arrive (cm_queue_submit),
    without a launch of their own; the others go to the serving slots.
    A request the queue has no room for goes to its slot too."""

    def __init__(self, handle, n_streams=4, dumps=False, queue_slots=256,
                 groups_per_cu=2, idle_us=2000):
        super().__init__(handle, n_streams, dumps)
        self.queue = cm.DeviceQueue(handle, W.LCA, W.FP32_STEP, slots=queue_slots,
                                    groups_per_cu=groups_per_cu, idle_us=idle_us)

    def close(self):
        self.queue.close()

    @staticmethod
    def _queued(w):
        return int(w["kind"]) == W.LCA and int(w["precision"]) == W.FP32_STEP

    def launch(self, si, ws):
        queued, rest = [], []
        for i, w in enumerate(ws):
            if self._queued(w):
                d = cm.DeviceSweep(self.h, w, dumps=self.dumps)
                hh = cm.host_buffers(d)
                try:
                    queued.append((i, (d, hh), self.queue.submit(d, host=hh)))
                    continue
                except cm.CmError as e:
                    if e.status != cm.E_BUSY:
                        raise
            rest.append(i)
        slot = super().launch(si, [ws[i] for i in rest]) if rest else None
        return (queued, rest, slot, len(ws))

    def poll(self, token):
        queued, rest, slot, n = token
        for k, (i, d, t) in enumerate(queued):
            if t is not None and self.queue.poll(t):
                queued[k] = (i, d, None)  # retired: polled done once
        if any(t is not None for _, _, t in queued):
            return None
        slot_out = None
        if slot is not None:
            slot_out = super().poll(slot)
            if slot_out is None:
                return None
        out = [None] * n
        for i, (d, hh), _ in queued:  # views of the pinned buffers, as in GpuBackend
            o = {k: (t.numpy().view(np.uint64) if k in ("hist", "stats") else t.numpy()) for k, t in hh.items()}
            if self.dumps:
                o["device_sweep"] = d
            out[i] = o
        for i, o in zip(rest, slot_out or []):
            out[i] = o
        return out


def served_mix(n_requests, rate_hz=50.0, seed=11, max_runs=10 ** 6, fp32=True):
    """The served-mix workload: Poisson arrivals at rate_hz; each request picks
    one of the four model configurations uniformly, a log-uniform total run
    count in [10^3, max_runs] and a grid size uniform in [1, 4096]; trials per
    setting = max(1, round(runs / grid)).  Request i's noise seed is 1000 + i.
    Returns [(arrival offset in s, workload)]."""
    g = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    grid64 = W.control_grid(64)
    for i in range(n_requests):
        t += g.exponential(1.0 / rate_hz)
        cfg = int(g.integers(0, 4))
        runs = int(10 ** g.uniform(3.0, np.log10(max_runs)))
        G = int(g.integers(1, 4097))
        T = max(1, int(round(runs / G)))
        seed_i = 1000 + i
        if cfg == 0:
            w = W.ddm(trials=T, seed=seed_i, drifts=np.linspace(0.0, 0.6, G),
                      precision=W.FP32_STEP if fp32 else W.FP64)
        elif cfg in (1, 2):
            w = W.conflict(trials=T, seed=seed_i, grid=grid64[:G],
                           precision=W.FP32_STEP if fp32 else W.FP64,
                           reward=1.0 if cfg == 2 else 0.0, cost=0.1 if cfg == 2 else 0.0)
        else:
            w = W.rnn(trials=T, seed=seed_i, gains=np.linspace(0.5, 1.5, G),
                      precision=W.BF16_PROJ if fp32 else W.FP64)
        out.append((t, w))
    return out


def run_mix(handle, mix, budget_bytes=32 << 30, n_streams=4, dumps=False, queue=False, queue_opts=None,
            tick_s=0.0, on_done=None):
    """Replay a served mix in real time; returns the finished requests.  With
    ``dumps`` every request also writes its per-run outcomes, left on the
    device in ``result["device_sweep"]`` (its ``results()`` reads them).
    With ``queue`` the conflict-network FP32 requests go through the device
    work queue (QueueBackend, given ``queue_opts`` as keyword arguments).
    ``tick_s``: the loop's sleep between scheduler ticks; by default it
    spins (one host core busy), since a sleeping loop wakes late (measured
    on the C4 mix: p50 0.58 against 0.34 ms).  ``on_done(request)``, when
    given, is called as each request finishes, after which the request drops
    its results: their pinned host buffers go back to the allocator's cache
    for the requests still to come, instead of every request pinning fresh
    memory (which costs about 0.4 ms a request until the cache holds enough
    blocks)."""
    be = (QueueBackend(handle, n_streams, dumps=dumps, **(queue_opts or {})) if queue
          else GpuBackend(handle, n_streams, dumps=dumps))
    try:
        sch = Scheduler(be, budget_bytes, n_streams)
        t0 = be.clock()
        pending = collections.deque(Request(i, w, t0 + dt) for i, (dt, w) in enumerate(mix))
        seen = 0
        while pending or not sch.idle():
            now = be.clock()
            while pending and pending[0].arrival <= now:
                sch.submit(pending.popleft())
            sch.tick()
            if on_done is not None:
                for r in sch.finished[seen:]:
                    on_done(r)
                    r.result = None
                seen = len(sch.finished)
            if tick_s:
                time.sleep(tick_s)
        return sch.finished
    finally:
        if queue:
            be.close()


CONFIG_NAMES = {0: "ddm", 1: "conflict", 2: "grid_search", 3: "rate_network"}


def config_of(w):
    """Which of the mix's four model configurations a request is (0 DDM,
    1 conflict network, 2 its scored grid search, 3 rate network)."""
    kind = int(w["kind"])
    if kind == W.DDM:
        return 0
    if kind == W.RNN:
        return 3
    return 2 if float(w.get("reward", 0.0)) != 0.0 or float(w.get("cost", 0.0)) != 0.0 else 1


def latency_summary(finished):
    lat = np.array([r.done - r.arrival for r in finished]) * 1e3
    return dict(requests=len(lat), p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)), max_ms=float(lat.max()))


def latency_by_config(finished):
    """latency_summary per model configuration, keyed by its name."""
    out = {}
    for c, name in CONFIG_NAMES.items():
        sel = [r for r in finished if config_of(r.w) == c]
        if sel:
            out[name] = latency_summary(sel)
    return out
