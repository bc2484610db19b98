"""The host code of libmclahe under AddressSanitizer (no GPU needed).

The library's sources are built once more with the sanitizer on the host pass
only (device code is compiled but never instrumented), and the host-side ABI
tests run against that build in a child process that preloads the sanitizer's
runtime: plan validation and geometry, workspace layout, tuning and its cache
file, batched tables, the metric / filter / variant argument checks.  Any
sanitizer report makes the child exit non-zero.  The build is cached in the
system temporary directory, keyed by a hash of the sources.
"""
import hashlib
import os
import subprocess
import sys
import tempfile

import pytest

from paper_1906_11355_amd import build as libbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _source_hash() -> str:
    h = hashlib.sha256()
    for d in (libbuild.CSRC, libbuild.INCLUDE):
        for name in sorted(os.listdir(d)):
            p = os.path.join(d, name)
            if os.path.isfile(p):
                h.update(name.encode())
                h.update(open(p, "rb").read())
    h.update(open(libbuild.__file__, "rb").read())
    return h.hexdigest()[:16]


@pytest.fixture(scope="module")
def asan_lib():
    if not os.path.exists(libbuild.HIPCC):
        pytest.skip("hipcc not available")
    d = os.path.join(tempfile.gettempdir(), f"mclahe_host_asan_{_source_hash()}")
    lib = os.path.join(d, "libmclahe_asan.so")
    if os.path.exists(lib):
        return lib, libbuild.asan_runtime()
    return libbuild.build_host_asan(d)


def test_host_abi_tests_clean_under_asan(asan_lib):
    lib, rt = asan_lib
    assert os.path.exists(rt), rt
    # the build really is instrumented: its host code calls the sanitizer's checks
    syms = subprocess.check_output(["nm", "-D", "--undefined-only", lib], text=True)
    assert "__asan_report_load" in syms and "__asan_report_store" in syms
    env = dict(os.environ)
    env["LD_PRELOAD"] = rt
    env["MCLAHE_LIB"] = lib
    # leaks of the interpreter and of the HIP runtime are not the library's
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=23"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_host.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
