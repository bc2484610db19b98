"""Host model of the persistent batched launch (no GPU).

tests/persist_model.cpp runs the ticket protocol of mc_persist.h (the very
functions the persistent kernel runs) with host threads standing in for
work-groups, on batch table images the library writes for real batches:
the 64-volume benchmark mix and small batches with zero-unit passes.  It
shows that every run ends, every unit runs exactly once and only after
every unit of its volume's previous pass, that every completion counter ends
at its pass's unit count, and that the abort word ends a run whose wait
gives up (a forced give-up at a chosen ticket, or a stalled producer with a
short poll budget) with every later unit skipped.  A planted protocol
mistake (counters read one unit ahead) is caught.
"""
import os
import subprocess
import tempfile

import pytest

from paper_1906_11355_amd import _lib
from paper_1906_11355_amd._lib import Plan

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1906_11355_amd", "csrc")
_EXE = None


def _model():
    global _EXE
    if _EXE is None:
        d = tempfile.mkdtemp(prefix="mclahe_persist_model_")
        exe = os.path.join(d, "persist_model")
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-pthread", "-I", CSRC,
                               os.path.join(ROOT, "tests", "persist_model.cpp"), "-o", exe])
        _EXE = exe
    return _EXE


def _image(plans):
    n = len(plans)
    ins = [(1 << 36) + i * (1 << 30) for i in range(n)]
    outs = [(1 << 37) + i * (1 << 30) for i in range(n)]
    img = _lib.batched_table(plans, ins, outs, 1 << 40)
    f = tempfile.NamedTemporaryFile(prefix="mclahe_table_", suffix=".bin", delete=False)
    f.write(img)
    f.close()
    return f.name


def _run(img, workers, delay_us=0, spins=-1, abort_ticket=-1, stall_ticket=-1, stall_ms=0, mutant=0,
         timeout=120):
    r = subprocess.run([_model(), img, str(workers), str(delay_us), str(spins), str(abort_ticket),
                        str(stall_ticket), str(stall_ms), str(mutant)],
                       capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, (r.returncode, r.stderr)
    a, head, ran, viol, dup, missing, ms = r.stdout.split()
    return dict(aborted=int(a), head=int(head), ran=int(ran), violations=int(viol), dup=int(dup),
                missing=int(missing), ms=float(ms))


def _mix_plans(n=64):
    from paper_1906_11355_amd import synth
    return [Plan(s["shape"], s["kernel_size"], 256, s["clip_limit"], "kernel" if s["adaptive"] else "global",
                 in_dtype="uint16" if s["kind"] == "2d" else "float32") for s in synth.mix_spec(n, 4)]


SMALL = [
    [Plan((40, 64), (8, 16), 64, 0.02)],                                              # one volume
    [Plan((40, 64), (8, 16), 64, 0.02, user_range=(0.0, 9.0)),                        # no range pass
     Plan((17, 33, 9), (5, 7, 3), 32, 0.1, "kernel"),
     Plan((30, 26, 25, 15), (8, 9, 7, 8), 128, 0.03, in_dtype="uint8")],
    [Plan((9, 8, 7, 6, 5), (3, 3, 3, 3, 3), 16, 0.05)] * 3,                           # generic map, repeated
]


@pytest.mark.parametrize("workers", [64, 512])
def test_mix_runs_every_unit_once_after_its_dependencies(workers):
    img = _image(_mix_plans())
    r = _run(img, workers, delay_us=20)
    assert r["aborted"] == 0
    assert r["violations"] == 0 and r["dup"] == 0 and r["missing"] == 0
    assert r["head"] >= r["ran"] + workers - 1       # every worker took one ticket past the end
    os.unlink(img)


@pytest.mark.parametrize("case", range(len(SMALL)))
def test_small_batches_and_zero_unit_passes(case):
    img = _image(SMALL[case])
    for workers in (1, 3, 256):
        r = _run(img, workers, delay_us=50)
        assert r["aborted"] == 0 and r["violations"] == 0 and r["dup"] == 0 and r["missing"] == 0, (workers, r)
    os.unlink(img)


def test_forced_give_up_ends_the_run():
    """A ticket told to give up sets the abort word; the run still ends, no
    unit runs before its dependencies, later units are skipped."""
    img = _image(_mix_plans(16))
    full = _run(img, 64)
    total = full["ran"]
    for t in (0, total // 3, total - 1):
        r = _run(img, 64, delay_us=10, abort_ticket=t)
        assert r["aborted"] == t + 1, (t, r)
        assert r["violations"] == 0 and r["dup"] == 0
        assert r["ran"] < total and r["missing"] > 0
    os.unlink(img)


def test_stalled_producer_with_short_poll_budget_aborts_and_drains():
    """A producer that stalls longer than the waits' poll budget: a waiter
    gives up, the abort word ends every later wait, the run drains."""
    img = _image(_mix_plans(16))
    r = _run(img, 64, spins=2000, stall_ticket=3, stall_ms=2000, timeout=60)
    assert r["aborted"] != 0 and r["violations"] == 0
    assert r["ms"] < 30000
    os.unlink(img)


def test_planted_protocol_mistake_is_caught():
    """Counters read one unit ahead: with more workers than units, waiters
    reach a pass boundary while its last units still run, and start early."""
    img = _image([Plan((64, 96), (8, 16), 64, 0.02), Plan((33, 40, 20), (7, 9, 5), 32, 0.05, "kernel")])
    seen = 0
    for _ in range(3):
        r = _run(img, 256, delay_us=500, mutant=1)
        seen += r["violations"]
    assert seen > 0
    r = _run(img, 256, delay_us=500)
    assert r["violations"] == 0 and r["missing"] == 0
    os.unlink(img)
