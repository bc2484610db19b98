"""Batched path: one launch per pass for all volumes (hipGraph) vs per-volume launches.

Every output and every intermediate array of every volume must be
bit-identical to mclahe_run of the same plan, on graph replays with eager work
and synchronisations between them, with new buffers between calls, and
against the oracle within the parity tolerance.
"""
import numpy as np
import pytest

from gpu_util import NP_CODE, assert_parity, collect, oracle_run, to_device_bytes

pytestmark = pytest.mark.gpu


def _volumes(seed=0):
    rng = np.random.default_rng(seed)
    vols = [
        (rng.integers(0, 60000, size=(300, 257)).astype(np.uint16), (64, 50), 256, 0.02, "global", np.float32),
        (rng.poisson(4.0, size=(40, 36, 28)).astype(np.float32), (10, 9, 7), 256, 0.03, "kernel", np.float32),
        (rng.poisson(2.0, size=(24, 20, 16, 8)).astype(np.float32), (6, 5, 4, 4), 512, 0.02, "global", np.float32),
        (rng.integers(0, 256, size=(1000,)).astype(np.uint8), (37,), 64, 0.1, "global", np.uint8),
        (rng.poisson(3.0, size=(6, 5, 4, 3, 7)).astype(np.float32), (3, 2, 2, 2, 3), 16, 0.1, "kernel", np.float32),
        (np.full((17, 19), 3.0, np.float32), (4, 5), 32, 0.02, "global", np.uint16),
        (rng.normal(0, 1, size=(50, 60)).astype(np.float32), (11, 12), 128, 0.05, "global", np.float32),
        (rng.poisson(1.0, size=(30, 30, 30)).astype(np.float32), (30, 30, 30), 64, 1.0, "kernel", np.float32),
    ]
    return vols


def _plans(vols):
    from paper_1906_11355_amd import _lib
    plans = []
    for x, ks, nb, clip, mode, od in vols:
        ur = (-1.0, 1.0) if x.ndim == 2 and x.dtype == np.float32 and mode == "global" and x.shape == (50, 60) else None
        plans.append(_lib.Plan(x.shape, ks, nb, clip, mode, ur, in_dtype=NP_CODE[x.dtype],
                               out_dtype=NP_CODE[np.dtype(od)]))
    return plans


def _run_plain(plans, vols, in_off=0):
    import torch
    res = []
    for p, (x, *_r, od) in zip(plans, vols):
        ib, ip = to_device_bytes(x, in_off)
        ob = torch.zeros(x.size * np.dtype(od).itemsize + 64, dtype=torch.uint8, device="cuda")
        ws = torch.full((p.workspace_size(),), 0xCD, dtype=torch.uint8, device="cuda")
        p.run_ptr(ip, ob.data_ptr(), ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        res.append(collect(p, ws, 0, ob, ob.data_ptr(), x.shape, od))
    return res


def _run_batched(plans, vols, ws=None, in_off=0):
    import torch
    from paper_1906_11355_amd import _lib
    ins, outs = [], []
    for x, *_r, od in vols:
        ins.append(to_device_bytes(x, in_off))
        outs.append(torch.zeros(x.size * np.dtype(od).itemsize + 64, dtype=torch.uint8, device="cuda"))
    need = _lib.batched_workspace_size(plans)
    if ws is None:
        ws = torch.full((need,), 0xEF, dtype=torch.uint8, device="cuda")
    _lib.run_batched_ptr(plans, [p for _, p in ins], [o.data_ptr() for o in outs], ws.data_ptr(),
                         ws.numel(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    offs = _lib.batched_workspace_offsets(plans)
    res = [collect(p, ws, off, o, o.data_ptr(), x.shape, od)
           for p, off, o, (x, *_r, od) in zip(plans, offs, outs, vols)]
    return res, ws


def _same(a, b, i):
    for k in ("out", "hist", "clipped", "lut", "range", "scale"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=f"volume {i}: {k} differs from the plain path")


def test_batched_bit_identical_to_plain():
    vols = _volumes()
    plans = _plans(vols)
    plain = _run_plain(plans, vols)
    batched, _ = _run_batched(plans, vols)
    for i, (a, b) in enumerate(zip(batched, plain)):
        _same(a, b, i)


def test_batched_matches_oracle():
    vols = _volumes(1)
    plans = _plans(vols)
    batched, _ = _run_batched(plans, vols)
    for p, g, (x, ks, nb, clip, mode, od) in zip(plans, batched, vols):
        r = oracle_run(x, ks, nb, clip, mode, p.user_range, od)
        assert_parity(g, r, od, what=f"batched {x.shape}")


def test_graph_replays_with_eager_work_between():
    import torch
    vols = _volumes(2)
    plans = _plans(vols)
    plain = _run_plain(plans, vols)
    ws = None
    for rep in range(4):
        # eager work of the program itself between replays
        a = torch.randn(1 << 20, device="cuda")
        (a * 2).sum().item()
        torch.cuda.synchronize()
        batched, ws = _run_batched(plans, vols, ws if rep % 2 else None)
        for i, (b, c) in enumerate(zip(batched, plain)):
            _same(b, c, i)


def test_batch_of_one_and_repeated_volume():
    vols = _volumes(3)
    plans = _plans(vols)
    plain = _run_plain(plans, vols)
    for i in (0, 2, 4):
        b, _ = _run_batched([plans[i]], [vols[i]])
        _same(b[0], plain[i], i)
    # the same plan twice in one batch
    b, _ = _run_batched([plans[1], plans[1]], [vols[1], vols[1]])
    _same(b[0], plain[1], 1)
    _same(b[1], plain[1], 1)


def test_unaligned_inputs_with_long_rows():
    """Inputs off a 16-byte boundary take the scalar-load decomposition in a
    batch as in a per-volume run: bit-identical to mclahe_run, and to the
    oracle within the parity bar."""
    rng = np.random.default_rng(9)
    vols = [
        (rng.integers(0, 256, size=(512, 512)).astype(np.uint8), (64, 64), 256, 0.01, "global", np.float32),
        (rng.integers(0, 60000, size=(64, 2048)).astype(np.uint16), (16, 256), 256, 0.02, "global", np.float32),
        (rng.poisson(6.0, size=(40, 1040)).astype(np.float32), (16, 260), 128, 0.03, "kernel", np.float32),
        (rng.poisson(3.0, size=(6, 10, 520)).astype(np.float32), (3, 5, 130), 64, 0.05, "global", np.float32),
    ]
    plans = _plans(vols)
    for off in (4, 12):
        plain = _run_plain(plans, vols, in_off=off)
        batched, _ = _run_batched(plans, vols, in_off=off)
        for i, (a, b) in enumerate(zip(batched, plain)):
            _same(a, b, i)
    for p, g, (x, ks, nb, clip, mode, od) in zip(plans, batched, vols):
        r = oracle_run(x, ks, nb, clip, mode, p.user_range, od)
        assert_parity(g, r, od, what=f"unaligned batched {x.shape}")


# ------------------------------------------------ the persistent launch
def _persist_phase_starts(plans):
    """First ticket of each pass, read from the table image the library writes."""
    import struct
    from paper_1906_11355_amd import _lib
    n = len(plans)
    img = _lib.batched_table(plans, [1 << 36] * n, [1 << 37] * n, 1 << 40)
    o = struct.unpack_from("<I", img, 8)[0]                 # McBatchHdr.o_persist
    total = struct.unpack_from("<I", img, o)[0]
    starts = struct.unpack_from("<5I", img, o + 16)         # McPersistHdr.phase_start
    return total, starts


def _run_persistent(plans, vols, ws=None, abort_ticket=None, max_spins=0):
    import torch
    from paper_1906_11355_amd import _lib
    ins, outs = [], []
    for x, *_r, od in vols:
        ins.append(to_device_bytes(x))
        outs.append(torch.zeros(x.size * np.dtype(od).itemsize + 64, dtype=torch.uint8, device="cuda"))
    need = _lib.batched_workspace_size(plans)
    if ws is None:
        ws = torch.full((need,), 0xEF, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    _lib.run_batched_persistent_ptr(plans, [p for _, p in ins], [o.data_ptr() for o in outs], ws.data_ptr(),
                                    ws.numel(), st, max_spins=max_spins, abort_ticket=abort_ticket)
    status = _lib.persistent_status(plans, ws.data_ptr(), st)
    torch.cuda.synchronize()
    offs = _lib.batched_workspace_offsets(plans)
    res = [collect(p, ws, off, o, o.data_ptr(), x.shape, od)
           for p, off, o, (x, *_r, od) in zip(plans, offs, outs, vols)]
    return res, ws, status


@pytest.mark.timeout(120)
def test_persistent_forced_give_up_ends_normally():
    """A ticket told to give up (from the host) sets the run's abort word:
    the kernel drains its tickets and ends, the status names that ticket."""
    vols = _volumes()
    plans = _plans(vols)
    total, starts = _persist_phase_starts(plans)
    for t in (starts[1], starts[3] + 1):
        print(f"persistent forced give-up at ticket {t} of {total}", flush=True)
        _, _, (aborted, tickets) = _run_persistent(plans, vols, abort_ticket=t)
        assert aborted == t + 1, (t, aborted)
        assert tickets >= total


@pytest.mark.timeout(120)
def test_persistent_single_launch_variant():
    """The whole batch in one persistent launch: every output and every
    intermediate array bit-identical to mclahe_run, on repeated calls (graph
    replays) with eager work between them, and within the oracle's bar."""
    import torch
    vols = _volumes()
    plans = _plans(vols)
    plain = _run_plain(plans, vols)
    ws = None
    for rep in range(3):
        print(f"persistent run {rep}", flush=True)
        res, ws, (aborted, _) = _run_persistent(plans, vols, ws)
        assert aborted == 0
        for i, (a, b) in enumerate(zip(res, plain)):
            _same(a, b, i)
        torch.zeros(1 << 20, device="cuda").add_(1.0)
        torch.cuda.synchronize()
    x, ks, nb, clip, mode, od = vols[2]
    assert_parity(res[2], oracle_run(x, ks, nb, clip, mode, None, od), od, what="persistent 4D")


@pytest.mark.timeout(300)
def test_persistent_mix_matches_per_pass_batched():
    """Sixteen volumes of the benchmark mix (2D uint16, 3D float per-kernel
    range, 4D float): persistent and per-pass batched runs agree bit for bit."""
    from paper_1906_11355_amd import synth
    items = [synth.gen_item(s) for s in synth.mix_spec(16, 4)]
    vols = [(it.x, it.kernel_size, it.n_bins, it.clip_limit, "kernel" if it.adaptive else "global", np.float32)
            for it in items]
    plans = _plans(vols)
    ref, _ = _run_batched(plans, vols)
    res, _, (aborted, _) = _run_persistent(plans, vols)
    assert aborted == 0
    for i, (a, b) in enumerate(zip(res, ref)):
        _same(a, b, i)
