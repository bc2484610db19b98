"""Host-side tests of the C-ABI library: no GPU needed.

The library loads and exports every symbol its header declares; plan
validation, geometry (against the oracle's Eq. 1-2), workspace layout, tuning
and the argument checks that run before any device call; and the shared
virtual-padding geometry code against numpy's symmetric padding.
"""
import ctypes
import os
import re
import subprocess
import sys
import tempfile

import numpy as np
import pytest

import oracle
from paper_1906_11355_amd import _lib
from paper_1906_11355_amd._lib import MclaheError, Plan
from exact_model import decimal_clip_count

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mclahe.h")


def test_library_exports_every_declared_symbol():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(mclahe_[a-z_]+)\s*\(", src))
    assert len(names) >= 20
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_version():
    for s in range(6):
        assert _lib.status_string(s).startswith("MCLAHE_")
    assert _lib.version() == "0.1.0"


@pytest.mark.parametrize("kw,status", [
    (dict(shape=(4,), kernel_size=(5,)), _lib.INVALID_VALUE),
    (dict(shape=(4,), kernel_size=(0,)), _lib.INVALID_VALUE),
    (dict(shape=(0,), kernel_size=(1,)), _lib.INVALID_VALUE),
    (dict(shape=(4, 4), kernel_size=(2,)), _lib.INVALID_VALUE),
    (dict(shape=(2,) * 9, kernel_size=(1,) * 9), _lib.INVALID_VALUE),
    (dict(n_bins=1), _lib.INVALID_VALUE),
    (dict(n_bins=8193), _lib.INVALID_VALUE),
    (dict(clip_limit=-0.1), _lib.INVALID_VALUE),
    (dict(clip_limit=float("inf")), _lib.INVALID_VALUE),
    (dict(clip_limit=float("nan")), _lib.INVALID_VALUE),
    (dict(mode="kernel", user_range=(0.0, 1.0)), _lib.INVALID_VALUE),
    (dict(user_range=(1.0, 1.0)), _lib.INVALID_VALUE),
    (dict(user_range=(0.0, float("inf"))), _lib.INVALID_VALUE),
])
def test_plan_validation(kw, status):
    args = dict(shape=(16, 16), kernel_size=(4, 4), n_bins=64, clip_limit=0.02)
    args.update(kw)
    with pytest.raises(MclaheError) as e:
        Plan(**args)
    assert e.value.status == status
    assert str(e.value)


def test_unsupported_dtype_rejected():
    with pytest.raises(TypeError):
        Plan((8, 8), (4, 4), in_dtype="float64")


def test_geometry_matches_oracle():
    rng = np.random.default_rng(0)
    for _ in range(200):
        D = int(rng.integers(1, 9))
        shape = [int(rng.integers(1, 40)) for _ in range(D)]
        ks = [int(rng.integers(1, s + 1)) for s in shape]
        p = Plan(shape, ks, 16, 0.3)
        g = p.geometry()
        pad, p0, p1, nk = oracle.geometry(shape, ks)
        assert g["pad"] == pad.tolist() and g["pad0"] == p0.tolist() and g["pad1"] == p1.tolist()
        assert g["n_kernels_axis"] == nk.tolist()
        assert g["n_kernels"] == int(np.prod(nk))
        assert g["kernel_voxels"] == int(np.prod(ks))
        assert g["clip_count"] == decimal_clip_count(0.3, int(np.prod(ks)))
        assert g["n_cells"] == int(np.prod(nk - 1))


@pytest.mark.parametrize("clip,ks,C", [
    (0.02, (30, 30, 15, 20), 5400),   # the photoemission experiment (Sec. IV.A)
    (0.01, (10, 10), 1),
    (0.29, (100,), 29),
    (2.0, (4, 4), 16),
])
def test_clip_count_of_decimal_limits(clip, ks, C):
    shape = tuple(2 * b for b in ks)
    assert Plan(shape, ks, 16, clip).geometry()["clip_count"] == C


def test_workspace_layout_and_tuning():
    p = Plan((256, 256, 128, 32), (32, 32, 16, 8), 512, 0.02)
    lay = p.layout()
    nk, nb = 3645, 512
    offs = [lay[k] for k in ("hist", "clipped", "lut", "range", "scale")]
    assert all(o % 256 == 0 for o in offs) and offs == sorted(offs)
    assert lay["clipped"] - lay["hist"] >= nk * nb * 4
    assert lay["lut"] - lay["clipped"] >= nk * nb * 8
    assert lay["range"] - lay["lut"] >= nk * nb * 4
    assert lay["total"] == p.workspace_size()
    t = p.tuning()
    assert t["hist_copies"] in (1, 2, 4, 8) and 1 <= t["hist_peel"] <= 3
    w0 = p.workspace_size()
    p.set_tuning(hist_rows_split=t["hist_rows_split"] * 2, hist_copies=4, hist_peel=1,
                 map_rows_split=7, map_group=1)
    t2 = p.tuning()
    assert t2["hist_rows_split"] == t["hist_rows_split"] * 2 and t2["hist_copies"] == 4
    assert t2["hist_peel"] == 1 and t2["map_group"] == 1 and t2["map_rows_split"] == 7
    assert 1 <= t2["map_unit_chunks"] <= 7
    p.set_tuning(**dict(t2, map_unit_chunks=3))
    assert p.tuning()["map_unit_chunks"] == 3
    p.set_tuning(**dict(t2, map_unit_chunks=99))          # clamped to the row split
    assert p.tuning()["map_unit_chunks"] == 7
    p.set_tuning(**t2)
    t2 = p.tuning()
    # a split too coarse for the per-unit row table is raised to the minimum
    q = Plan((256, 256, 128, 32), (32, 32, 16, 8), 512, 0.02)
    q.set_tuning(map_rows_split=1, hist_rows_split=1)
    assert q.tuning()["map_rows_split"] == 5 and q.tuning()["hist_rows_split"] == 5
    assert p.workspace_size() > w0          # more histogram partials
    with pytest.raises(MclaheError):
        p.set_tuning(hist_copies=3)
    assert p.tuning() == t2                 # a rejected tuning leaves the plan unchanged
    assert p.autotune_workspace_size() >= p.workspace_size()


def test_adaptive_layout_has_per_kernel_ranges():
    p = Plan((64, 64, 32), (16, 16, 8), 256, 0.02, "kernel")
    lay = p.layout()
    nk = p.geometry()["n_kernels"]
    assert lay["scale"] - lay["range"] >= nk * 2 * 4
    assert lay["total"] - lay["scale"] >= nk * 4


def test_run_argument_checks_before_device_calls():
    p = Plan((64, 64), (16, 16), 64, 0.02)
    need = p.workspace_size()
    with pytest.raises(MclaheError) as e:
        p.run_ptr(0, 256, 256, need)
    assert e.value.status == _lib.INVALID_VALUE
    with pytest.raises(MclaheError) as e:
        p.run_ptr(256, 512, 4096, need - 1)
    assert e.value.status == _lib.WORKSPACE
    with pytest.raises(MclaheError) as e:
        p.run_ptr(256, 512, 4096 + 4, need)
    assert e.value.status == _lib.WORKSPACE
    with pytest.raises(MclaheError) as e:
        p.run_ptr(258, 512, 4096, need)        # float input not 4-byte aligned
    assert e.value.status == _lib.INVALID_VALUE
    q = Plan((64, 64), (16, 16), 64, 0.02, in_dtype="uint8", out_dtype="float32")
    with pytest.raises(MclaheError):
        q.run_ptr(256, 256, 4096, q.workspace_size())   # in-place with different sizes


def test_batched_workspace_offsets():
    plans = [Plan((64, 64), (16, 16), 64, 0.02), Plan((32, 32, 16), (8, 8, 4), 128, 0.01, "kernel"),
             Plan((16, 16, 8, 8), (4, 4, 4, 4), 256, 0.05, in_dtype="uint16")]
    total = _lib.batched_workspace_size(plans)
    offs = _lib.batched_workspace_offsets(plans)
    assert all(o % 256 == 0 for o in offs) and offs == sorted(offs)
    for o, o2, p in zip(offs, offs[1:] + [total], plans):
        assert o2 - o >= p.workspace_size()


def test_batched_split_table_and_argument_checks():
    plans = [Plan((64, 64), (16, 16), 64, 0.02), Plan((32, 32, 16), (8, 8, 4), 128, 0.01, "kernel")]
    tb = _lib.batched_table_size(plans)
    assert tb == _lib.batched_workspace_offsets(plans)[0] and tb % 256 == 0
    ws = [p.workspace_size() for p in plans]
    ins, outs, wss = [1 << 20, 2 << 20], [3 << 20, 4 << 20], [5 << 20, 6 << 20]
    cases = [
        (dict(d_table=0), _lib.WORKSPACE),                        # no table buffer
        (dict(d_table=(7 << 20) + 64), _lib.WORKSPACE),           # misaligned table
        (dict(table_bytes=tb - 1), _lib.WORKSPACE),               # table too small
        (dict(ws_bytes=[ws[0], ws[1] - 1]), _lib.WORKSPACE),      # volume 1 workspace too small
        (dict(d_wss=[5 << 20, (6 << 20) + 8]), _lib.WORKSPACE),   # volume 1 workspace misaligned
        (dict(d_ins=[1 << 20, 0]), _lib.INVALID_VALUE),           # NULL input
    ]
    for kw, status in cases:
        a = dict(d_ins=ins, d_outs=outs, d_wss=wss, ws_bytes=ws, d_table=7 << 20, table_bytes=tb)
        a.update(kw)
        with pytest.raises(MclaheError) as e:
            _lib.run_batched_split_ptr(plans, a["d_ins"], a["d_outs"], a["d_wss"], a["ws_bytes"],
                                       a["d_table"], a["table_bytes"])
        assert e.value.status == status, (kw, e.value)


def test_chunked_sizes_and_argument_checks():
    p = Plan((64, 48, 40), (16, 12, 10), 128, 0.02)
    sizes = [p.chunked_workspace_size(L) for L in (1, 2, 3, 5, 50)]
    assert sizes == sorted(sizes) and sizes[-2] == sizes[-1]       # clamped to the 5 kernel layers
    assert sizes[0] < p.workspace_size() + 64 * 48 * 40 * 8         # a slab, not the volume
    need = sizes[1]
    for kw, status in [
        (dict(L=0), _lib.INVALID_VALUE),
        (dict(h_out=1 << 20), _lib.INVALID_VALUE),                 # in place
        (dict(h_in=0), _lib.INVALID_VALUE),
        (dict(ws=(4 << 20) + 8), _lib.WORKSPACE),
        (dict(wsb=need - 1), _lib.WORKSPACE),
    ]:
        a = dict(h_in=1 << 20, h_out=2 << 20, L=2, ws=4 << 20, wsb=need)
        a.update(kw)
        with pytest.raises(MclaheError) as e:
            p.run_chunked_ptr(a["h_in"], a["h_out"], a["L"], a["ws"], a["wsb"])
        assert e.value.status == status, (kw, e.value)
    q = Plan((1000,), (37,), 64, 0.1)
    with pytest.raises(MclaheError) as e:
        q.chunked_workspace_size(2)
    assert e.value.status == _lib.NOT_SUPPORTED


def test_tuning_cache_file_is_read_at_plan_creation(tmp_path):
    """A cache line written by the autotuner is applied to new plans of the
    same problem (fresh process: the file is read once per process)."""
    cache = tmp_path / "tune.txt"
    key = "D3_64x16_48x12_40x10_n128_m0_i2_o2_u0"
    cache.write_text(f"{key} 7 4 2 9 1 3\n")
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1906_11355_amd._lib import Plan\n"
            "print(Plan((64, 48, 40), (16, 12, 10), 128, 0.02).tuning())") % ROOT
    env = dict(os.environ, MCLAHE_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr
    t = eval(r.stdout.strip().splitlines()[-1])
    assert (t["hist_rows_split"], t["hist_copies"], t["hist_peel"]) == (7, 4, 2)
    assert (t["map_rows_split"], t["map_group"], t["map_unit_chunks"]) == (9, 1, 3)


def test_plan_count_limits():
    with pytest.raises(MclaheError):
        Plan((2 ** 20, 2 ** 20), (2 ** 19, 2 ** 19), 16, 0.1)   # kernel voxels >= 2^32


# ------------------------------------------ shared padding geometry (g++)
@pytest.fixture(scope="module")
def probe():
    d = tempfile.mkdtemp(prefix="mclahe_probe_")
    so = os.path.join(d, "probe.so")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC",
                           "-I", os.path.join(ROOT, "paper_1906_11355_amd", "csrc"),
                           os.path.join(ROOT, "tests", "geom_probe.cpp"), "-o", so])
    lib = ctypes.CDLL(so)
    for f in (lib.probe_kernel_box, lib.probe_cell_range):
        f.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_int)]
        f.restype = None
    return lib


def test_kernel_footprints_match_numpy_symmetric_padding(probe):
    """Every kernel's box and multiplicities equal the counts of original
    coordinates in its window of np.pad(arange(s), mode='symmetric')."""
    rng = np.random.default_rng(1)
    cases = [(s, b) for s in range(1, 30) for b in range(1, s + 1)]
    cases += [(int(s), int(rng.integers(1, s + 1))) for s in rng.integers(30, 3000, 200)]
    out = (ctypes.c_int * 4)()
    for s, b in cases:
        p = 2 * b - 1 - ((s - 1) % b)
        p0, p1 = p // 2, (p + 1) // 2
        padded = np.pad(np.arange(s), (p0, p1), mode="symmetric")
        n = padded.size // b
        for k in range(n):
            probe.probe_kernel_box(s, b, p0, p1, k, out)
            lo, hi, olo, ohi = out
            cnt = np.bincount(padded[k * b:(k + 1) * b], minlength=s)
            mult = np.zeros(s, int)
            mult[lo:hi] = 1
            mult[olo:ohi] += 1
            assert (cnt == mult).all(), (s, b, k, (lo, hi, olo, ohi))


def test_interpolation_cells_partition_the_axis(probe):
    rng = np.random.default_rng(2)
    cases = [(s, b) for s in range(1, 25) for b in range(1, s + 1)]
    cases += [(int(s), int(rng.integers(1, s + 1))) for s in rng.integers(25, 3000, 200)]
    out = (ctypes.c_int * 3)()
    for s, b in cases:
        p = 2 * b - 1 - ((s - 1) % b)
        p0, p1 = p // 2, (p + 1) // 2
        n = (s + p) // b
        owner = np.full(s, -1)
        for c in range(n - 1):
            probe.probe_cell_range(s, b, p0, p1, c, out)
            lo, hi, m0 = out
            if lo < hi:
                assert (owner[lo:hi] == -1).all()
                owner[lo:hi] = c
                assert 0 <= m0 < 2 * b
        x = np.arange(s)
        m = 2 * (x + p0) - (b - 1)
        assert (owner == m // (2 * b)).all(), (s, b)


# ------------------------------------------- batched descriptor table (g++)
def test_batched_table_decodes_every_unit_once():
    """Every work-group index of every batched pass maps to exactly one unit
    of one volume (decoded with the kernels' own functions), unit counts
    match the plans, and the descriptors point at the right buffers."""
    d = tempfile.mkdtemp(prefix="mclahe_batch_probe_")
    so = os.path.join(d, "probe.so")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC",
                           "-I", os.path.join(ROOT, "paper_1906_11355_amd", "csrc"),
                           os.path.join(ROOT, "tests", "batch_probe.cpp"), "-o", so])
    probe = ctypes.CDLL(so)
    probe.probe_batch.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint32),
                                  ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32)]
    probe.probe_batch.restype = ctypes.c_int
    from paper_1906_11355_amd import synth
    specs = synth.mix_spec(64, 4)
    plans = [Plan(s["shape"], s["kernel_size"], 256, s["clip_limit"],
                  "kernel" if s["adaptive"] else "global",
                  in_dtype="uint16" if s["kind"] == "2d" else "float32") for s in specs]
    plans.append(Plan((7, 5, 4, 3, 9), (3, 2, 2, 3, 4), 16, 0.1, "kernel"))     # generic path
    plans.append(Plan((1000,), (37,), 64, 0.1, user_range=(0.0, 10.0)))        # no range pass
    n = len(plans)
    ws = 1 << 40
    ins = [(1 << 36) + i * (1 << 30) for i in range(n)]
    outs = [(1 << 37) + i * (1 << 30) for i in range(n)]
    img = _lib.batched_table(plans, ins, outs, ws)
    counts = (ctypes.c_uint32 * (4 * n))()
    ptrs = (ctypes.c_uint64 * (3 * n))()
    nl = ctypes.c_uint32()
    assert probe.probe_batch(img, len(img), counts, ptrs, ctypes.byref(nl)) == 0
    # one launch per kernel class and pass: far fewer than 4 per volume
    assert 4 <= nl.value <= 4 * 6, nl.value
    offs = _lib.batched_workspace_offsets(plans)
    for i, p in enumerate(plans):
        g = p.geometry()
        assert counts[2 * n + i] == g["n_kernels"]                 # one clip unit per kernel
        if p.mode == _lib.KERNEL:
            assert counts[0 * n + i] == counts[1 * n + i]           # per-kernel range units
        assert counts[1 * n + i] > 0 and counts[3 * n + i] > 0
        assert ptrs[3 * i] == ins[i] and ptrs[3 * i + 1] == outs[i]
        assert ptrs[3 * i + 2] == ws + offs[i] + p.layout()["hist"]
    assert counts[0 * n + n - 1] == 0                              # user range: no range pass


@pytest.mark.parametrize("in_off,out_off", [(0, 0), (1, 0), (4, 0), (0, 8), (2, 2)])
def test_batched_units_fit_their_work_groups(in_off, out_off):
    """Buffers at any address keep wide chunks (rows shorter than one chunk
    take single elements); every unit's row segment must fit MC_T chunks
    (histogram) and the interpolation work-group (512 threads under a
    global range with LDS-staged LUTs, 256 otherwise)."""
    d = tempfile.mkdtemp(prefix="mclahe_batch_probe_")
    so = os.path.join(d, "probe.so")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC",
                           "-I", os.path.join(ROOT, "paper_1906_11355_amd", "csrc"),
                           os.path.join(ROOT, "tests", "batch_probe.cpp"), "-o", so])
    probe = ctypes.CDLL(so)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    probe.probe_batch_chunks.argtypes = [ctypes.c_char_p, ctypes.c_size_t, u32p, u32p, u32p]
    probe.probe_batch_chunks.restype = ctypes.c_int
    plans = [Plan((512, 512), (64, 64), 256, 0.01, in_dtype="uint8"),
             Plan((64, 2048), (16, 256), 256, 0.02, in_dtype="uint16"),
             Plan((40, 1040), (16, 260), 128, 0.03),
             Plan((40, 1040), (16, 260), 128, 0.03, "kernel"),
             Plan((6, 10, 520), (3, 5, 130), 64, 0.05),
             Plan((24, 1536), (8, 512), 256, 0.02, "kernel", out_dtype="uint8"),
             Plan((6, 4096), (3, 4096), 256, 0.01, in_dtype="uint8"),
             Plan((256, 256, 128, 32), (32, 32, 16, 8), 512, 0.02)]
    from paper_1906_11355_amd import synth
    plans += [Plan(s["shape"], s["kernel_size"], 256, s["clip_limit"], "kernel" if s["adaptive"] else "global",
                   in_dtype="uint16" if s["kind"] == "2d" else "float32") for s in synth.mix_spec(16, 4)]
    n = len(plans)
    ins = [(1 << 36) + i * (1 << 30) + in_off for i in range(n)]
    outs = [(1 << 37) + i * (1 << 30) + out_off for i in range(n)]
    img = _lib.batched_table(plans, ins, outs, 1 << 40)
    hm, mm, vec = ((ctypes.c_uint32 * n)() for _ in range(3))
    assert probe.probe_batch_chunks(img, len(img), hm, mm, vec) == 0
    for i, p in enumerate(plans):
        vmax = 4 if p.in_code == _lib.F32 else 8
        # wide chunks at any address; single elements only for rows shorter than a chunk
        assert vec[i] == (vmax if p.shape[-1] >= vmax else 1), i
        map_threads = 512 if p.mode == _lib.GLOBAL else 256
        assert 1 <= hm[i] <= 256, (i, hm[i])
        assert mm[i] <= map_threads, (i, mm[i])


# ---------------------------------------------------------------- metrics --
def test_metrics_workspace_size():
    small = _lib.metrics_workspace_size(1, 2)
    assert small > 0 and small % 256 == 0
    # grows with the bins (histogram counters) and with the work-groups, which
    # saturate for large volumes
    assert _lib.metrics_workspace_size(1, 8192) >= small + 2 * 8192 * 8 - 256
    big = _lib.metrics_workspace_size(1 << 28, 256)
    assert big == _lib.metrics_workspace_size(1 << 34, 256)
    assert big > _lib.metrics_workspace_size(1000, 256)


@pytest.mark.parametrize("nvox,nb", [(0, 256), (-5, 256), (100, 1), (100, 8193)])
def test_metrics_workspace_size_rejects(nvox, nb):
    with pytest.raises(MclaheError) as e:
        _lib.metrics_workspace_size(nvox, nb)
    assert e.value.status == _lib.INVALID_VALUE


@pytest.mark.parametrize("kw,status", [
    (dict(x=None), _lib.INVALID_VALUE),
    (dict(res=None), _lib.INVALID_VALUE),
    (dict(xdt=7), _lib.INVALID_VALUE),
    (dict(y=0x2000, ydt=9), _lib.INVALID_VALUE),
    (dict(peak=0.0), _lib.INVALID_VALUE),
    (dict(peak=float("inf")), _lib.INVALID_VALUE),
    (dict(peak=float("nan")), _lib.INVALID_VALUE),
    (dict(ws=None), _lib.WORKSPACE),
    (dict(ws=0x1010), _lib.WORKSPACE),
    (dict(wsb=16), _lib.WORKSPACE),
    (dict(nvox=0), _lib.INVALID_VALUE),
])
def test_metrics_argument_checks(kw, status):
    # every check runs before any device call: fake addresses are never touched
    a = dict(x=0x1000, xdt=2, y=None, ydt=2, nvox=1000, nb=256, peak=1.0, res=0x3000, ws=0x4000,
             wsb=1 << 20)
    a.update(kw)
    with pytest.raises(MclaheError) as e:
        _lib.metrics_ptr(a["x"], a["xdt"], a["y"], a["ydt"], a["nvox"], a["nb"], a["peak"], a["res"], None,
                         a["ws"], a["wsb"], 0)
    assert e.value.status == status


# -------------------------------------------------------------- denoising --
def test_gaussian_workspace_size():
    assert _lib.gaussian_workspace_size((10, 20), (0.0, 1.0)) == 0          # one pass: none
    assert _lib.gaussian_workspace_size((10, 20), (0.7, 1.0)) == 1024      # 200 floats, 256-aligned
    assert _lib.gaussian_workspace_size((256, 256, 128, 32), (0.7, 0.7, 0.9, 1.3)) == 4 * 256 * 256 * 128 * 32


@pytest.mark.parametrize("kw,status", [
    (dict(shape=(0, 4)), _lib.INVALID_VALUE),
    (dict(shape=(2,) * 9, sigma=(1.0,) * 9), _lib.INVALID_VALUE),
    (dict(sigma=(-1.0, 1.0)), _lib.INVALID_VALUE),
    (dict(sigma=(float("nan"), 1.0)), _lib.INVALID_VALUE),
    (dict(sigma=(20.0, 1.0)), _lib.NOT_SUPPORTED),
    (dict(truncate=0.0), _lib.INVALID_VALUE),
    (dict(code=5), _lib.INVALID_VALUE),
    (dict(src=None), _lib.INVALID_VALUE),
    (dict(dst=0x100010), _lib.INVALID_VALUE),          # overlaps the input
    (dict(ws=None), _lib.WORKSPACE),
    (dict(ws=0x900010), _lib.WORKSPACE),
    (dict(wsb=8), _lib.WORKSPACE),
])
def test_gaussian_argument_checks(kw, status):
    a = dict(shape=(16, 16), sigma=(0.7, 1.3), truncate=4.0, code=2, src=0x100000, dst=0x800000,
             ws=0x900000, wsb=1 << 20)
    a.update(kw)
    with pytest.raises(MclaheError) as e:
        _lib.gaussian_ptr(a["src"], a["code"], a["shape"], a["sigma"], a["truncate"], a["dst"], a["ws"],
                          a["wsb"], 0)
    assert e.value.status == status


@pytest.mark.parametrize("kw,status", [
    (dict(shape=(4, 0)), _lib.INVALID_VALUE),
    (dict(window=(0, 2)), _lib.INVALID_VALUE),
    (dict(window=(9, 8)), _lib.NOT_SUPPORTED),
    (dict(code=3), _lib.INVALID_VALUE),
    (dict(dst=0x100004), _lib.INVALID_VALUE),
    (dict(dst=None), _lib.INVALID_VALUE),
])
def test_median_argument_checks(kw, status):
    a = dict(shape=(16, 16), window=(2, 2), code=0, src=0x100000, dst=0x800000)
    a.update(kw)
    with pytest.raises(MclaheError) as e:
        _lib.median_ptr(a["src"], a["code"], a["shape"], a["window"], a["dst"], 0)
    assert e.value.status == status


# ---------------------------------------------------------------- variants --
def test_variant_roundtrip_and_checks():
    p = Plan((64, 64), (16, 16), 256, 0.02)
    assert p.variant() == {"redistribution": 0, "rounds": 1, "centre": 0}
    p.set_variant("repeated", 4, "half")
    assert p.variant() == {"redistribution": 1, "rounds": 4, "centre": 1}
    p.set_variant("integer", 7)                 # rounds only matter for "repeated"
    assert p.variant() == {"redistribution": 2, "rounds": 1, "centre": 0}
    ws = p.workspace_size()
    p.set_variant("equal")
    assert p.workspace_size() == ws
    for bad in (dict(redistribution=3), dict(redistribution="repeated", rounds=0),
                dict(redistribution="repeated", rounds=9), dict(centre=2)):
        with pytest.raises(MclaheError) as e:
            p.set_variant(**bad)
        assert e.value.status == _lib.INVALID_VALUE
    big = Plan((256, 256), (128, 128), 8192, 0.02)
    with pytest.raises(MclaheError) as e:
        big.set_variant("repeated", 5)          # 8192^5 * 16384 units overflow 64 bits
    assert e.value.status == _lib.NOT_SUPPORTED
    big.set_variant("repeated", 2)


def test_default_interpolation_groups_keep_256_unit_columns():
    """Under a global range the default interpolation group is the largest that
    fits the LDS while the volume keeps 256 unit columns (outer cells times
    last-axis groups); an explicit group is taken as given."""
    cases = [((512, 512), (64, 64), 256, 1),             # 8 x 8 cells: 8 columns per group of 1
             ((1024, 1024), (64, 64), 256, 1),           # 16 x 16 cells: 256 columns only with groups of 1
             ((256, 256, 128), (32, 32, 16), 256, 2),    # 64 outer cells x 4 groups of 2
             ((128, 128, 64), (16, 16, 8), 256, 2),
             ((256, 256, 128, 32), (32, 32, 16, 8), 512, 2)]   # LDS allows 2; 512 outer cells
    for shape, ks, nb, want in cases:
        p = Plan(shape, ks, nb, 0.02, "global")
        assert p.tuning()["map_group"] == want, (shape, p.tuning())
    p = Plan((512, 512), (64, 64), 256, 0.02, "global")
    t = p.tuning()
    t["map_group"] = 4
    p.set_tuning(**t)
    assert p.tuning()["map_group"] == 4
    # per-kernel ranges interpolate one cell at a time
    assert Plan((256, 256, 128), (32, 32, 16), 256, 0.02, "kernel").tuning()["map_group"] == 1


def test_noalloc_rejects_plans_beyond_its_scratch_before_any_device_call():
    """mclahe_run_noalloc refuses a plan whose workspace exceeds the static
    array, without touching a device (this host has none)."""
    big = Plan((1024, 1024), (8, 8), 8192, 0.02)
    assert big.workspace_size() > _lib.NOALLOC_SCRATCH_BYTES
    with pytest.raises(MclaheError) as e:
        big.run_noalloc_ptr(16 << 20, 32 << 20, 0)
    assert e.value.status == _lib.WORKSPACE
    assert "scratch" in str(e.value)
    with pytest.raises(MclaheError) as e:
        _lib._check(_lib.lib.mclahe_run_noalloc(None, None, None, None))
    assert e.value.status == _lib.INVALID_VALUE


def test_noalloc_scratch_size_matches_header():
    src = open(HEADER).read()
    m = re.search(r"#define\s+MCLAHE_NOALLOC_SCRATCH_BYTES\s+\((\d+)ull\s*<<\s*(\d+)\)", src)
    assert m, "MCLAHE_NOALLOC_SCRATCH_BYTES not found"
    assert int(m.group(1)) << int(m.group(2)) == _lib.NOALLOC_SCRATCH_BYTES


def test_batch_tuning_is_kept_apart_from_the_plain_tuning():
    p = Plan((64, 96, 40), (16, 16, 10), 128, 0.02)
    plain = p.tuning()
    b = p.batch_tuning()
    p.set_batch_tuning(hist_rows_split=1, map_unit_chunks=1, hist_copies=4)
    nb = p.batch_tuning()
    assert nb["hist_rows_split"] == 1 and nb["hist_copies"] == 4
    assert p.tuning() == plain                   # the plain decomposition did not move
    with pytest.raises(MclaheError):
        p.set_batch_tuning(hist_copies=-1)
    assert p.batch_tuning() == nb                # a refused setting changes nothing
    p.set_batch_tuning()                         # back to the defaults
    assert p.batch_tuning() == b


def test_autotune_batched_workspace_covers_the_default_batch():
    from paper_1906_11355_amd import synth
    plans = [Plan(s["shape"], s["kernel_size"], 256, s["clip_limit"], "kernel" if s["adaptive"] else "global",
                  in_dtype="uint16" if s["kind"] == "2d" else "float32") for s in synth.mix_spec(8, 4)]
    need = _lib.autotune_batched_workspace_size(plans)
    assert need == _lib.batched_workspace_size(plans)
    for p in plans:                              # fewer histogram units: a smaller batch workspace
        p.set_batch_tuning(hist_rows_split=1)
    assert _lib.batched_workspace_size(plans) <= need
    assert _lib.autotune_batched_workspace_size(plans) == need


def test_persistent_table_tickets_cover_every_unit_in_pass_order():
    """The persistent launch's table (in the batched table image): pass
    starts are the running sums of the per-pass unit prefix sums."""
    import struct
    from paper_1906_11355_amd import synth
    plans = [Plan(s["shape"], s["kernel_size"], 256, s["clip_limit"], "kernel" if s["adaptive"] else "global",
                  in_dtype="uint16" if s["kind"] == "2d" else "float32") for s in synth.mix_spec(12, 4)]
    n = len(plans)
    img = _lib.batched_table(plans, [1 << 36] * n, [1 << 37] * n, 1 << 40)
    o = struct.unpack_from("<I", img, 8)[0]
    total, nvol, spins, abort_at = struct.unpack_from("<4I", img, o)
    starts = struct.unpack_from("<5I", img, o + 16)
    pre_off = (o + 48 + 255) & ~255
    assert nvol == n and abort_at == 0xFFFFFFFF and spins > 0
    assert starts[0] == 0 and starts[4] == total
    for ph in range(4):
        pre = struct.unpack_from(f"<{n + 1}I", img, pre_off + 4 * ph * (n + 1))
        assert pre[0] == 0 and all(a <= b for a, b in zip(pre, pre[1:]))
        assert starts[ph + 1] - starts[ph] == pre[n]
