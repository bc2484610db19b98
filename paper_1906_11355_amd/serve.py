"""Continuous-batching server for MCLAHE enhancement requests on one GPU.

Requests of mixed dimensionality, shape, dtype and parameters arrive as an
open-loop stream.  A request is admitted, first come first served, when its
device bytes (input, output and its own workspace, which holds its
histograms, clipped counts, LUTs and range) fit in the free part of a fixed
HBM arena and an in-flight slot is free.  Admitted requests are copied in on
a copy stream; whenever one of the compute streams is idle, every admitted
request not yet running is coalesced into one batched step
(``mclahe_run_batched_split``: one launch per pass and kernel class over all
of them).  With two or more compute streams, work admitted while a step runs
starts on the device beside it.  A step's completion event marks its
requests' outputs ready; their memory and slots are then returned and the
queue is admitted again.

Per-request state never leaves the device: the workspace sits in the arena
next to the request's output for the life of the request.  The histogram
arithmetic is the same integer arithmetic as the single-volume path, and the
outputs are bit-identical to it (a batched step runs the same kernels on the
same work units).

Admission (``admit``), the arena allocator (``Arena``) and the event loop
(``Server``) are plain host code with no GPU dependency; the loop drives a
backend object.  ``DeviceBackend`` is the HIP one; tests drive the loop with
a simulated backend and a fake clock.
"""
from __future__ import annotations

import bisect
import gc
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Iterable, List, Optional, Sequence

import numpy as np

ALIGN = 256

WAITING, STAGED, RUNNING, DONE, FAILED, REJECTED, TIMED_OUT = (
    "waiting", "staged", "running", "done", "failed", "rejected", "timed_out")


def align_up(n: int, a: int = ALIGN) -> int:
    return (int(n) + a - 1) // a * a


# ------------------------------------------------------------------ arena --
class Arena:
    """First-fit allocator over [0, capacity) with ALIGN-byte blocks.

    Free blocks are kept sorted by offset and merged with their neighbours
    on release, so a fully released arena is one block again.
    """

    def __init__(self, capacity: int):
        self.capacity = int(capacity) // ALIGN * ALIGN
        self._free_off: List[int] = [0] if self.capacity else []
        self._free_len: List[int] = [self.capacity] if self.capacity else []
        self._live = {}
        self.used = 0
        self.peak = 0

    def alloc(self, nbytes: int) -> Optional[int]:
        n = align_up(max(1, nbytes))
        for i, ln in enumerate(self._free_len):
            if ln >= n:
                off = self._free_off[i]
                if ln == n:
                    del self._free_off[i], self._free_len[i]
                else:
                    self._free_off[i] += n
                    self._free_len[i] -= n
                self._live[off] = n
                self.used += n
                self.peak = max(self.peak, self.used)
                return off
        return None

    def free(self, off: int) -> None:
        n = self._live.pop(off)            # KeyError on a double free
        self.used -= n
        i = bisect.bisect_left(self._free_off, off)
        self._free_off.insert(i, off)
        self._free_len.insert(i, n)
        if i + 1 < len(self._free_off) and off + n == self._free_off[i + 1]:       # merge right
            self._free_len[i] += self._free_len.pop(i + 1)
            self._free_off.pop(i + 1)
        if i > 0 and self._free_off[i - 1] + self._free_len[i - 1] == off:           # merge left
            self._free_len[i - 1] += self._free_len.pop(i)
            self._free_off.pop(i)

    @property
    def free_bytes(self) -> int:
        return self.capacity - self.used

    def largest_free(self) -> int:
        return max(self._free_len, default=0)

    def blocks(self):
        return sorted(self._live.items())


# ---------------------------------------------------------------- request --
@dataclass
class Request:
    """One enhancement request.  ``payload`` is the input array: a host
    (pinned) tensor when the server copies inputs in, a device tensor when
    inputs are already resident.  ``arrival`` is on the server's clock."""
    rid: int
    arrival: float
    shape: tuple
    kernel_size: tuple
    n_bins: int = 256
    clip_limit: float = 0.01
    adaptive: bool = False
    in_dtype: str = "float32"
    out_dtype: str = "float32"
    payload: object = None
    # filled in by the server
    status: str = WAITING
    need: int = 0
    off: int = -1
    t_admit: float = float("nan")
    t_launch: float = float("nan")     # host time its step was launched
    t_ready: float = float("nan")      # completion event, on the server clock
    t_seen: float = float("nan")       # host time the loop saw the completion
    step: int = -1
    error: str = ""
    result: dict = field(default_factory=dict)
    dev: dict = field(default_factory=dict)

    @property
    def voxels(self) -> int:
        return int(np.prod(self.shape))

    @property
    def latency(self) -> float:
        return self.t_ready - self.arrival


def admit(waiting: deque, arena: Arena, free_slots: int, need: Callable[[Request], int]):
    """Admit from the head of the FIFO while the head fits.

    Strict arrival order: a head that does not fit blocks the requests
    behind it (no starvation of large requests).  Returns [(request, offset)]
    and removes them from ``waiting``; the arena blocks are allocated.
    """
    out = []
    while waiting and free_slots > 0:
        r = waiting[0]
        off = arena.alloc(need(r))
        if off is None:
            break
        waiting.popleft()
        out.append((r, off))
        free_slots -= 1
    return out


@dataclass
class Step:
    sid: int
    stream: int
    reqs: list
    token: object
    t_launch: float


@dataclass
class Report:
    n_requests: int
    n_done: int
    n_failed: int
    n_rejected: int
    n_timed_out: int
    p50_ms: float
    p99_ms: float
    mean_ms: float
    max_ms: float
    seen_p50_ms: float
    seen_p99_ms: float
    voxels: int
    makespan_s: float
    gvox_s: float
    steps: int
    mean_batch: float
    max_batch: int
    max_concurrent_steps: int
    peak_arena_bytes: int

    def as_dict(self, digits=4):
        return {k: (round(v, digits) if isinstance(v, float) else v) for k, v in self.__dict__.items()}


def summarize(reqs: Sequence[Request], steps: int, batch_sizes, max_conc: int, peak: int) -> Report:
    done = [r for r in reqs if r.status == DONE]
    lat = np.array([r.latency for r in done], np.float64) * 1e3
    seen = np.array([r.t_seen - r.arrival for r in done], np.float64) * 1e3
    vox = int(sum(r.voxels for r in done))
    if done:
        t0 = min(r.arrival for r in reqs)
        t1 = max(r.t_ready for r in done)
        span = max(t1 - t0, 1e-12)
    else:
        span = 0.0
    pct = (lambda q: float(np.percentile(lat, q))) if lat.size else (lambda q: float("nan"))
    return Report(
        n_requests=len(reqs), n_done=len(done),
        n_failed=sum(r.status == FAILED for r in reqs),
        n_rejected=sum(r.status == REJECTED for r in reqs),
        n_timed_out=sum(r.status == TIMED_OUT for r in reqs),
        p50_ms=pct(50), p99_ms=pct(99),
        mean_ms=float(lat.mean()) if lat.size else float("nan"),
        max_ms=float(lat.max()) if lat.size else float("nan"),
        seen_p50_ms=float(np.percentile(seen, 50)) if seen.size else float("nan"),
        seen_p99_ms=float(np.percentile(seen, 99)) if seen.size else float("nan"),
        voxels=vox, makespan_s=span, gvox_s=(vox / span / 1e9) if span > 0 else 0.0,
        steps=steps, mean_batch=float(np.mean(batch_sizes)) if batch_sizes else 0.0,
        max_batch=int(max(batch_sizes, default=0)), max_concurrent_steps=max_conc,
        peak_arena_bytes=peak)


# ----------------------------------------------------------------- server --
class Server:
    """Event loop: arrivals -> completions -> admission -> steps.

    backend interface:
        clock() -> float                 seconds, the same clock as arrivals
        need(req) -> int                 arena bytes of one request
        stage(req, base_offset)          bind device views, issue the input copy
        launch(reqs, stream) -> token    one batched step on compute stream
        done(token) -> bool              non-blocking completion query
        ready_time(token) -> float       completion time on clock()
        finish(req)                      called once the outputs are ready
        wait(deadline, busy)             block briefly (until deadline at most)
        n_streams                        number of compute streams
    """

    def __init__(self, backend, budget_bytes: int, max_slots: int = 64, max_batch: int = 32,
                 max_queue: Optional[int] = None, queue_timeout: Optional[float] = None):
        if max_slots < 1 or max_batch < 1:
            raise ValueError("max_slots and max_batch must be >= 1")
        self.b = backend
        self.arena = Arena(budget_bytes)
        self.max_slots = max_slots
        self.max_batch = max_batch
        self.max_queue = max_queue
        self.queue_timeout = queue_timeout
        self.steps: List[Step] = []
        self.log: List[tuple] = []      # (time, event, ids) for tests

    def run(self, requests: Iterable[Request]) -> Report:
        # no cyclic garbage collection pauses inside the loop
        was = gc.isenabled()
        gc.disable()
        try:
            return self._run(requests)
        finally:
            if was:
                gc.enable()

    def _run(self, requests: Iterable[Request]) -> Report:
        b = self.b
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        pending, waiting, staged = deque(reqs), deque(), deque()
        active: List[Optional[Step]] = [None] * b.n_streams
        slots = 0
        batch_sizes, max_conc = [], 0
        next_stream = 0
        while pending or waiting or staged or any(active):
            progressed = False
            now = b.clock()
            # arrivals
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                r.need = b.need(r)
                if r.need > self.arena.capacity:
                    r.status, r.error = REJECTED, f"needs {r.need} bytes, arena holds {self.arena.capacity}"
                else:
                    waiting.append(r)
                progressed = True
            # requests that waited too long for admission
            if self.queue_timeout is not None and waiting:
                keep = deque()
                for r in waiting:
                    if now - r.arrival > self.queue_timeout:
                        r.status, r.error = TIMED_OUT, "not admitted in time"
                    else:
                        keep.append(r)
                if len(keep) != len(waiting):
                    waiting, progressed = keep, True
            # completions
            for s, st in enumerate(active):
                if st is not None and b.done(st.token):
                    t = b.ready_time(st.token)
                    for r in st.reqs:
                        r.t_ready, r.t_seen, r.status = t, now, DONE
                        b.finish(r)
                        self.arena.free(r.off)
                        slots -= 1
                    self.log.append((now, "done", [r.rid for r in st.reqs]))
                    active[s] = None
                    progressed = True
            # admission
            for r, off in admit(waiting, self.arena, self.max_slots - slots, lambda q: q.need):
                r.off, r.t_admit = off, now
                slots += 1
                try:
                    b.stage(r, off)
                except Exception as e:       # a failed copy fails this request only
                    r.status, r.error = FAILED, str(e)
                    self.arena.free(off)
                    slots -= 1
                    continue
                r.status = STAGED
                staged.append(r)
                progressed = True
            # bounded queue: the newest of the requests still not admitted are turned away
            while self.max_queue is not None and len(waiting) > self.max_queue:
                r = waiting.pop()
                r.status, r.error = REJECTED, "queue full"
            # one step per idle compute stream, with everything staged so far
            for k in range(b.n_streams):
                s = (next_stream + k) % b.n_streams
                if active[s] is not None or not staged:
                    continue
                batch = [staged.popleft() for _ in range(min(self.max_batch, len(staged)))]
                sid = len(self.steps)
                try:
                    token = b.launch(batch, s)
                except Exception as e:       # a HIP error fails this step's requests
                    # part of the step may already be queued: its blocks are
                    # released only after that work has left the stream
                    b.drain(s)
                    for r in batch:
                        r.status, r.error = FAILED, str(e)
                        self.arena.free(r.off)
                        slots -= 1
                    self.log.append((now, "failed", [r.rid for r in batch]))
                    progressed = True
                    continue
                for r in batch:
                    r.status, r.step, r.t_launch = RUNNING, sid, now
                st = Step(sid, s, batch, token, now)
                self.steps.append(st)
                active[s] = st
                batch_sizes.append(len(batch))
                self.log.append((now, "launch", [r.rid for r in batch]))
                next_stream = (s + 1) % b.n_streams
                progressed = True
            max_conc = max(max_conc, sum(a is not None for a in active))
            if not progressed:
                b.wait(pending[0].arrival if pending else None, any(a is not None for a in active))
        return summarize(reqs, len(self.steps), batch_sizes, max_conc, self.arena.peak)


# ---------------------------------------------------------- HIP backend --
class DeviceBackend:
    """The server's device side: one HBM arena, a copy stream, compute streams.

    Request i's arena block is [input | output | workspace]; the input part
    is absent when inputs are already resident (``h2d=False``, payloads are
    device tensors).  ``plain=True`` runs each step's requests with one
    ``mclahe_run`` per volume instead of one batched call (the serial
    baseline uses it with one stream, one slot and batches of one); a step
    of a single request always takes ``mclahe_run``.
    ``keep`` copies each finished request's output and state to the host
    (for tests; it synchronises).
    """

    def __init__(self, budget_bytes: int, n_streams: int = 2, h2d: bool = True, plain: bool = False,
                 keep: bool = False, table_bytes: int = 1 << 20, device: str = "cuda:0",
                 poll_s: float = 0.0):
        import torch
        from . import _lib
        self.torch, self._lib = torch, _lib
        self.dev = torch.device(device)
        self.h2d, self.plain, self.keep = h2d, plain, keep
        self.n_streams = n_streams
        self.poll_s = poll_s
        self.arena = torch.empty(align_up(budget_bytes), dtype=torch.uint8, device=self.dev)
        self.base = self.arena.data_ptr()
        if self.base % ALIGN:
            raise RuntimeError("arena base is not 256-byte aligned")
        self.copy_stream = torch.cuda.Stream(self.dev)
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(n_streams)]
        self.table_bytes = align_up(table_bytes)
        self.tables = [torch.empty(self.table_bytes, dtype=torch.uint8, device=self.dev)
                       for _ in range(n_streams)]
        self._plans = {}
        self.clock = time.perf_counter
        # GPU event times are mapped to clock() through one reference event:
        # of several records on an idle stream, each polled to completion,
        # keep the one seen in the narrowest host-time window
        torch.cuda.synchronize(self.dev)
        best = None
        for _ in range(32):
            ev = torch.cuda.Event(enable_timing=True)
            t0 = self.clock()
            ev.record(self.streams[0])
            while not ev.query():
                pass
            t1 = self.clock()
            if best is None or t1 - t0 < best[0]:
                best = (t1 - t0, ev, 0.5 * (t0 + t1))
        self.ref_window_s, self.ref, self.t_ref = best

    def plan(self, r: Request):
        key = (r.shape, r.kernel_size, r.n_bins, r.clip_limit, r.adaptive, r.in_dtype, r.out_dtype)
        p = self._plans.get(key)
        if p is None:
            p = self._lib.Plan(r.shape, r.kernel_size, r.n_bins, r.clip_limit,
                               "kernel" if r.adaptive else "global",
                               in_dtype=r.in_dtype, out_dtype=r.out_dtype)
            self._plans[key] = p
        return p

    def _sizes(self, r: Request):
        nin = r.voxels * np.dtype(r.in_dtype).itemsize if self.h2d else 0
        nout = r.voxels * np.dtype(r.out_dtype).itemsize
        return align_up(nin), align_up(nout), align_up(self.plan(r).workspace_size())

    def need(self, r: Request) -> int:
        return sum(self._sizes(r))

    def stage(self, r: Request, off: int) -> None:
        torch = self.torch
        nin, nout, nws = self._sizes(r)
        d = r.dev
        d["ws"], d["ws_bytes"] = self.base + off + nin + nout, nws
        d["out"] = self.base + off + nin
        d["out_off"] = off + nin
        d["ws_off"] = off + nin + nout
        d["ev"] = None
        if self.h2d:
            src = r.payload.view(torch.uint8).reshape(-1)
            with torch.cuda.stream(self.copy_stream):
                self.arena[off:off + src.numel()].copy_(src, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(self.copy_stream)
            d["in"], d["ev"] = self.base + off, ev
        else:
            d["in"] = r.payload.data_ptr()

    def launch(self, reqs: Sequence[Request], s: int):
        torch, _lib = self.torch, self._lib
        st = self.streams[s]
        for r in reqs:
            if r.dev["ev"] is not None:
                st.wait_event(r.dev["ev"])
        plans = [self.plan(r) for r in reqs]
        h = st.cuda_stream
        if self.plain or len(reqs) == 1:
            # a step of one request takes the single-volume entry (same kernels
            # and bits, no descriptor table to upload)
            for p, r in zip(plans, reqs):
                p.run_ptr(r.dev["in"], r.dev["out"], r.dev["ws"], r.dev["ws_bytes"], h)
        else:
            _lib.run_batched_split_ptr(plans, [r.dev["in"] for r in reqs], [r.dev["out"] for r in reqs],
                                       [r.dev["ws"] for r in reqs], [r.dev["ws_bytes"] for r in reqs],
                                       self.tables[s].data_ptr(), self.table_bytes, h)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(st)
        return ev

    def done(self, token) -> bool:
        return token.query()

    def ready_time(self, token) -> float:
        return self.t_ref + self.ref.elapsed_time(token) * 1e-3

    def finish(self, r: Request) -> None:
        if self.keep:
            nout = r.voxels * np.dtype(r.out_dtype).itemsize
            o = r.dev["out_off"]
            w = r.dev["ws_off"]
            r.result["out_bytes"] = self.arena[o:o + nout].cpu()
            r.result["ws_bytes"] = self.arena[w:w + self.plan(r).workspace_size()].cpu()
        r.dev.pop("ev", None)

    def drain(self, s: int) -> None:
        """Wait until everything queued on compute stream s has run."""
        self.streams[s].synchronize()

    def wait(self, deadline: Optional[float], busy: bool) -> None:
        # poll_s = 0: busy-poll (a serving loop owns a host core)
        dt = self.poll_s
        if deadline is not None:
            dt = min(dt, max(0.0, deadline - self.clock()))
        if dt > 0:
            time.sleep(dt)


# --------------------------------------------------------------- streams --
def make_requests(pool: Sequence[dict], rate_hz: float, n: int, seed: int = 5) -> List[Request]:
    """n requests drawn (seeded) from a pool of items, Poisson arrivals at
    rate_hz (rate_hz = inf: all arrive at time 0).  Pool entries are dicts
    with shape, kernel_size, n_bins, clip_limit, adaptive, in_dtype, payload."""
    rng = np.random.default_rng(seed)
    pick = rng.integers(0, len(pool), n)
    if np.isinf(rate_hz):
        arr = np.zeros(n)
    else:
        arr = np.cumsum(rng.exponential(1.0 / rate_hz, n))
    out = []
    for i, (k, t) in enumerate(zip(pick, arr)):
        it = pool[int(k)]
        out.append(Request(rid=i, arrival=float(t), shape=tuple(it["shape"]),
                           kernel_size=tuple(it["kernel_size"]), n_bins=int(it.get("n_bins", 256)),
                           clip_limit=float(it["clip_limit"]), adaptive=bool(it.get("adaptive", False)),
                           in_dtype=str(it["in_dtype"]), out_dtype=str(it.get("out_dtype", "float32")),
                           payload=it.get("payload")))
    return out


def shift_arrivals(reqs: Sequence[Request], t0: float) -> None:
    for r in reqs:
        r.arrival += t0
