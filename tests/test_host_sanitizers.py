"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The sources are built a second time with the sanitizers on the host side only (the
device code is compiled as usual, without them), and the C-ABI checks of
test_abi_cpu.py, which run no GPU work, are repeated against that build in a child
process that preloads the sanitizer runtime: argument validation, error strings,
descriptor copies and the batch table must read and write only what they own.
"""

import os
import shutil
import subprocess
import sys

import pytest

from paper_2204_06489_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = B.HIPCC
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def _asan_runtime():
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = shutil.which("clang") or ""
    if not clang:
        return None
    r = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


@pytest.fixture(scope="module")
def sanitized_lib(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    runtime = _asan_runtime()
    if runtime is None:
        pytest.skip("AddressSanitizer runtime not found")
    out = tmp_path_factory.mktemp("kktfwi_san")
    flags = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-fPIC", "-fno-omit-frame-pointer", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
             "-Wno-unused-value", "-Wno-unused-result"] + SAN
    procs, objs = [], []
    for src in B.SOURCES:
        obj = str(out / src.replace(".hip", ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC] + flags + ["-c", os.path.join(B.CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    for p in procs:
        text = p.communicate()[0].decode(errors="replace")
        assert p.returncode == 0, text[-4000:]
    lib = str(out / "libkktfwi_san.so")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + SAN + ["-o", lib] + objs,
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return lib, runtime


def test_abi_checks_pass_under_address_and_undefined_sanitizers(sanitized_lib):
    lib, runtime = sanitized_lib
    code = ("import sys\n"
            "import paper_2204_06489_amd._lib as L\n"
            f"L.LIB_PATH = {lib!r}\n"
            "import pytest\n"
            "sys.exit(pytest.main(['-q', '-p', 'no:cacheprovider', 'tests/test_abi_cpu.py']))\n")
    env = dict(os.environ)
    env["LD_PRELOAD"] = runtime
    # the interpreter itself is not instrumented: its allocations are not reported as leaks
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    text = r.stdout + r.stderr
    assert "AddressSanitizer" not in text and "runtime error:" not in text, text[-4000:]
    assert r.returncode == 0, text[-4000:]
    assert " passed" in r.stdout
