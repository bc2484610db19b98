"""Build libmclahe.so for gfx950 (in-tree, translation units in parallel).

    python -m paper_1906_11355_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmclahe.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = ["mclahe.hip", "k_plain_f32.hip", "k_plain_u16.hip", "k_plain_u8.hip", "mc_metrics.hip",
           "mc_denoise.hip", "k_persist.hip"]
# measurement tooling, a library of its own (not part of the MCLAHE ABI)
PROBE_SOURCE = os.path.join(CSRC, "probe", "lds_atomics.hip")
PROBE_LIB = os.path.join(HERE, "libmclahe_probe.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # binning must be bit-identical to the IEEE single-precision reading:
    # no contraction of (v - lo) * scale or of any other expression
    "-ffp-contract=off",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
    "-Wno-unused-result",
]


def _compile(src: str, csrc: str = CSRC, build_dir: str = BUILD) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-I", csrc, "-c", os.path.join(csrc, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"compile failed: {src}")
    return obj


def build_probe(lib: str = PROBE_LIB) -> str:
    """The LDS-atomic throughput probe used by the benchmark."""
    tmp = lib + ".tmp"
    cmd = [HIPCC, *FLAGS, "-shared", PROBE_SOURCE, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("compile failed: probe")
    os.replace(tmp, lib)
    return lib


def build(jobs: int | None = None, csrc: str = CSRC, build_dir: str = BUILD, lib: str = LIB,
          probe: bool = True) -> str:
    """Compile the sources in csrc into lib (defaults: this package, in-tree)."""
    os.makedirs(build_dir, exist_ok=True)
    jobs = jobs or min(len(SOURCES) + 1, max(1, os.cpu_count() or 1))
    with ThreadPoolExecutor(jobs) as ex:
        fp = ex.submit(build_probe) if probe else None
        objs = list(ex.map(lambda s: _compile(s, csrc, build_dir), SOURCES))
        if fp:
            fp.result()
    tmp = lib + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, lib)
    return lib


def build_host_asan(build_dir: str, jobs: int | None = None) -> tuple[str, str]:
    """A build of the same sources whose HOST code carries AddressSanitizer.

    Device code is compiled as usual (at -O1) and never instrumented: the
    sanitizer is passed to the host pass only.  Returns (library, runtime),
    where runtime is the sanitizer's shared runtime, which a process must
    preload before it loads the library.  For host-side checks on a machine
    without a GPU (plan validation, geometry, workspace layout, batched tables,
    tuning files).
    """
    os.makedirs(build_dir, exist_ok=True)
    flags = [f for f in FLAGS if f != "-O3"] + [
        "-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]

    def one(src):
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        r = subprocess.run([HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"compile failed: {src}")
        return obj

    jobs = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(one, SOURCES))
    lib = os.path.join(build_dir, "libmclahe_asan.so")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host",
                           "-fsanitize=address", *objs, "-o", lib + ".tmp"])
    os.replace(lib + ".tmp", lib)
    return lib, asan_runtime()


def asan_runtime() -> str:
    """Path of the AddressSanitizer shared runtime of hipcc's clang."""
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    return subprocess.check_output([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()


if __name__ == "__main__":
    print(build())
