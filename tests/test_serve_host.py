"""Serving loop host logic on the CPU: arena, FIFO admission by HBM budget and
slots, continuous batching, failure handling, overflow and time-outs.

The event loop is driven by a simulated backend with a fake clock: a step on
a compute stream takes a fixed time plus a time per voxel, steps on one
stream run one after another, input copies run one after another on a copy
stream.  No GPU is involved.
"""
import random
from collections import deque

import numpy as np
import pytest

from paper_1906_11355_amd.serve import (ALIGN, DONE, FAILED, REJECTED, TIMED_OUT, Arena, Request, Server,
                                        admit, align_up, make_requests)


class SimBackend:
    def __init__(self, n_streams=2, t_fixed=1e-4, t_vox=1e-9, t_copy_byte=0.0, fail_steps=(),
                 fail_stage=()):
        self.t = 0.0
        self.n_streams = n_streams
        self.t_fixed, self.t_vox, self.t_copy = t_fixed, t_vox, t_copy_byte
        self.stream_free = [0.0] * n_streams
        self.copy_free = 0.0
        self.inflight = []
        self.nlaunch = 0
        self.fail_steps, self.fail_stage = set(fail_steps), set(fail_stage)
        self.live = {}          # rid -> bytes between stage and finish
        self.max_live = 0
        self.launches = []      # (stream, start, end, rids)
        self.stages = []        # (time, arena offset, bytes)
        self.partial = []       # failed steps: (end of their queued part, [(offset, bytes)])

    def clock(self):
        return self.t

    def need(self, r):
        return align_up(r.voxels * 4) * 2 + 65536

    def stage(self, r, off):
        if r.rid in self.fail_stage:
            raise RuntimeError("injected copy failure")
        self.copy_free = max(self.t, self.copy_free) + r.voxels * 4 * self.t_copy
        r.dev["copy_done"] = self.copy_free
        r.dev["off"] = off
        self.stages.append((self.t, off, r.need))
        self.live[r.rid] = r.need
        self.max_live = max(self.max_live, sum(self.live.values()))

    def launch(self, reqs, s):
        k = self.nlaunch
        self.nlaunch += 1
        if k in self.fail_steps:
            # the first half of the step was queued before the error
            done_part = reqs[:len(reqs) // 2]
            if done_part:
                start = max([self.t, self.stream_free[s]] + [r.dev["copy_done"] for r in done_part])
                self.stream_free[s] = start + self.t_fixed + self.t_vox * sum(r.voxels for r in done_part)
            self.partial.append((len(self.stages), self.stream_free[s], [(r.dev["off"], r.need) for r in reqs]))
            for r in reqs:
                self.live.pop(r.rid, None)
            raise RuntimeError("injected HIP error")
        start = max([self.t, self.stream_free[s]] + [r.dev["copy_done"] for r in reqs])
        end = start + self.t_fixed + self.t_vox * sum(r.voxels for r in reqs)
        self.stream_free[s] = end
        tok = [end]
        self.inflight.append(tok)
        self.launches.append((s, start, end, [r.rid for r in reqs]))
        return tok

    def done(self, tok):
        if self.t >= tok[0]:
            if tok in self.inflight:
                self.inflight.remove(tok)
            return True
        return False

    def ready_time(self, tok):
        return tok[0]

    def finish(self, r):
        self.live.pop(r.rid, None)

    def drain(self, s):
        self.t = max(self.t, self.stream_free[s])

    def wait(self, deadline, busy):
        c = [tok[0] for tok in self.inflight if tok[0] > self.t]
        if deadline is not None:
            c.append(deadline)
        if not c:
            raise RuntimeError("the loop waits with nothing in flight and nothing pending")
        self.t = min(c)


def _reqs(n, rate, seed=0, sizes=(1000, 200000)):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n)) if np.isfinite(rate) else np.zeros(n)
    out = []
    for i in range(n):
        v = int(rng.integers(*sizes))
        out.append(Request(rid=i, arrival=float(t[i]), shape=(v,), kernel_size=(max(1, v // 4),)))
    return out


# ------------------------------------------------------------------ arena
def test_arena_alignment_merge_and_release():
    a = Arena(10 * ALIGN + 17)
    assert a.capacity == 10 * ALIGN
    x = a.alloc(1)
    y = a.alloc(ALIGN + 1)
    z = a.alloc(3 * ALIGN)
    assert (x, y, z) == (0, ALIGN, 3 * ALIGN)
    assert a.alloc(5 * ALIGN) is None and a.largest_free() == 4 * ALIGN
    a.free(y)
    assert a.alloc(2 * ALIGN) == ALIGN            # first fit reuses the hole
    a.free(ALIGN)
    a.free(x)
    a.free(z)
    assert a.used == 0 and a.largest_free() == a.capacity and len(a._free_off) == 1
    with pytest.raises(KeyError):
        a.free(z)


def test_arena_random_ops_never_overlap():
    rnd = random.Random(1)
    cap = 1 << 20
    a = Arena(cap)
    live = {}
    for _ in range(3000):
        if live and rnd.random() < 0.45:
            off = rnd.choice(list(live))
            a.free(off)
            del live[off]
        else:
            n = rnd.randint(1, 40000)
            off = a.alloc(n)
            if off is None:
                # first fit fails only when no free block is large enough
                assert a.largest_free() < align_up(n)
                continue
            assert off % ALIGN == 0 and off + align_up(n) <= cap
            live[off] = align_up(n)
        occ = np.zeros(cap // ALIGN, np.int32)
        for o, n in live.items():
            occ[o // ALIGN:(o + n) // ALIGN] += 1
        assert occ.max() <= 1
        assert a.used == sum(live.values())
    for off in list(live):
        a.free(off)
    assert a.used == 0 and a.largest_free() == cap


# -------------------------------------------------------------- admission
def test_admit_fifo_head_of_line_and_slots():
    a = Arena(100 * ALIGN)
    q = deque(_reqs(5, 1.0))
    sizes = {0: 30, 1: 60, 2: 20, 3: 5, 4: 1}
    need = lambda r: sizes[r.rid] * ALIGN
    got = admit(q, a, free_slots=10, need=need)
    assert [r.rid for r, _ in got] == [0, 1]                 # 2 does not fit: it blocks 3 and 4
    assert [r.rid for r in q] == [2, 3, 4]
    a.free(got[0][1])
    got2 = admit(q, a, free_slots=1, need=need)               # one slot left
    assert [r.rid for r, _ in got2] == [2]
    assert admit(q, a, free_slots=0, need=need) == []


# -------------------------------------------------------------- event loop
@pytest.mark.parametrize("rate", [50.0, 2000.0, float("inf")])
def test_all_complete_within_budget_and_slots(rate):
    b = SimBackend()
    budget = 4 << 20
    srv = Server(b, budget, max_slots=6, max_batch=4)
    reqs = _reqs(120, rate, seed=2)
    rep = srv.run(reqs)
    assert rep.n_done == 120 and all(r.status == DONE for r in reqs)
    assert b.max_live <= budget and srv.arena.peak <= srv.arena.capacity
    assert srv.arena.used == 0
    # never more than max_slots requests admitted at once
    ev = sorted([(r.t_admit, 1) for r in reqs] + [(r.t_ready, -1) for r in reqs], key=lambda e: (e[0], e[1]))
    live = np.cumsum([d for _, d in ev])
    assert live.max() <= 6
    # latency covers queueing: ready after arrival, admitted after arrival
    for r in reqs:
        assert r.t_admit >= r.arrival and r.t_ready > r.t_admit
    # admission is in arrival order
    adm = [r.t_admit for r in sorted(reqs, key=lambda r: (r.arrival, r.rid))]
    assert adm == sorted(adm)
    assert all(len(st.reqs) <= 4 for st in srv.steps)


def test_continuous_batching_overlaps_and_coalesces():
    b = SimBackend(n_streams=2, t_fixed=1e-3)
    srv = Server(b, 64 << 20, max_slots=64, max_batch=32)
    reqs = _reqs(60, 20000.0, seed=3)
    rep = srv.run(reqs)
    assert rep.n_done == 60
    assert rep.max_batch > 1 and rep.steps < 60                # requests were coalesced
    assert rep.max_concurrent_steps == 2                       # two steps in flight
    # some step started while the other stream's step was still running
    L = b.launches
    assert any(s1 != s2 and st2 < en1 and st1 < en2
               for i, (s1, st1, en1, _) in enumerate(L) for (s2, st2, en2, _) in L[i + 1:])
    # requests that arrived during a running step ran in a later step
    first = srv.steps[0]
    assert len(first.reqs) == 1 and all(r.step >= 1 for r in reqs if r.rid != first.reqs[0].rid)


def test_serial_configuration_is_serial():
    b = SimBackend(n_streams=1)
    srv = Server(b, 64 << 20, max_slots=1, max_batch=1)
    reqs = _reqs(30, 5000.0, seed=4)
    rep = srv.run(reqs)
    assert rep.n_done == 30 and rep.steps == 30 and rep.max_batch == 1 and rep.max_concurrent_steps == 1
    order = [r.rid for r in sorted(reqs, key=lambda r: r.t_ready)]
    assert order == list(range(30))


def test_latency_percentiles_exact_when_idle():
    # requests far apart: each waits for nothing, latency = its service time
    b = SimBackend(t_fixed=2e-3, t_vox=0.0)
    srv = Server(b, 64 << 20)
    reqs = [Request(rid=i, arrival=i * 1.0, shape=(100,), kernel_size=(10,)) for i in range(10)]
    rep = srv.run(reqs)
    assert rep.p50_ms == pytest.approx(2.0) and rep.p99_ms == pytest.approx(2.0)
    assert rep.makespan_s == pytest.approx(9.002)


def test_failed_step_frees_its_requests_only():
    b = SimBackend()
    srv = Server(b, 64 << 20, max_slots=8, max_batch=3)
    reqs = _reqs(40, 5000.0, seed=5)
    b.fail_steps = {2}
    rep = srv.run(reqs)
    failed = [r for r in reqs if r.status == FAILED]
    assert failed and rep.n_failed == len(failed) <= 3
    assert rep.n_done == 40 - len(failed)
    assert all("injected" in r.error for r in failed)
    assert srv.arena.used == 0


def test_failed_step_keeps_its_blocks_until_queued_work_ends():
    """A step that fails after queueing part of its work releases its arena
    blocks only once that work has run: no request staged after the failure
    lands in those blocks earlier."""
    b = SimBackend(t_vox=1e-8)
    srv = Server(b, 32 << 20, max_slots=8, max_batch=4)
    reqs = _reqs(60, 20000.0, seed=8, sizes=(100000, 400000))
    b.fail_steps = {1, 4}
    srv.run(reqs)
    assert len(b.partial) == 2
    reused = 0
    for first, end, blocks in b.partial:
        for t, off, size in b.stages[first:]:
            if any(off < o + n and o < off + size for o, n in blocks):
                reused += 1
                assert t >= end, (t, end)
    assert reused > 0                      # the case is exercised
    assert srv.arena.used == 0


def test_failed_copy_fails_that_request_only():
    b = SimBackend(fail_stage={7})
    srv = Server(b, 64 << 20)
    reqs = _reqs(20, 1000.0, seed=6)
    rep = srv.run(reqs)
    assert [r.rid for r in reqs if r.status == FAILED] == [7]
    assert rep.n_done == 19 and srv.arena.used == 0


def test_too_large_rejected_others_served():
    b = SimBackend()
    srv = Server(b, 2 << 20)
    reqs = _reqs(10, 1000.0, seed=7, sizes=(1000, 2000))
    reqs[4].shape = (10 ** 6,)            # 8 MB needed, 2 MB arena
    rep = srv.run(reqs)
    assert reqs[4].status == REJECTED and rep.n_rejected == 1 and rep.n_done == 9


def test_request_waits_for_memory_then_runs():
    # arena holds one request at a time: the next is queued, never dropped
    b = SimBackend(t_fixed=1e-3)
    one = align_up(50000 * 4) * 2 + 65536
    srv = Server(b, one + ALIGN, max_slots=8)
    reqs = [Request(rid=i, arrival=0.0, shape=(50000,), kernel_size=(100,)) for i in range(5)]
    rep = srv.run(reqs)
    assert rep.n_done == 5 and rep.max_concurrent_steps == 1 and rep.steps == 5
    readies = sorted(r.t_ready for r in reqs)
    assert np.all(np.diff(readies) > 0)


def test_queue_overflow_and_timeout():
    b = SimBackend(t_fixed=5e-3)
    srv = Server(b, 64 << 20, max_slots=1, max_batch=1, max_queue=3)
    reqs = _reqs(10, float("inf"), seed=8)
    rep = srv.run(reqs)
    assert rep.n_rejected == 6 and rep.n_done == 4          # 1 admitted + 3 queued
    b2 = SimBackend(t_fixed=5e-3)
    srv2 = Server(b2, 64 << 20, max_slots=1, max_batch=1, queue_timeout=0.012)
    reqs2 = _reqs(10, float("inf"), seed=8)
    rep2 = srv2.run(reqs2)
    # 5 ms per request, serial: those not admitted within 12 ms time out
    assert rep2.n_done + rep2.n_timed_out == 10 and rep2.n_done in (2, 3)
    for r in reqs2:
        if r.status == DONE:
            assert r.t_admit - r.arrival <= 0.012
        else:
            assert r.status == TIMED_OUT and np.isnan(r.t_admit)


def test_make_requests_seeded():
    pool = [dict(shape=(10, 12), kernel_size=(5, 6), clip_limit=0.02, in_dtype="uint16"),
            dict(shape=(8, 8, 8), kernel_size=(4, 4, 4), clip_limit=0.03, adaptive=True, in_dtype="float32")]
    a = make_requests(pool, 100.0, 50, seed=3)
    b = make_requests(pool, 100.0, 50, seed=3)
    assert [(r.arrival, r.shape) for r in a] == [(r.arrival, r.shape) for r in b]
    assert all(np.diff([r.arrival for r in a]) > 0)
    assert {r.shape for r in a} == {(10, 12), (8, 8, 8)}
    assert all(r.arrival == 0 for r in make_requests(pool, float("inf"), 5))
