"""Build libkktfwi.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2204_06489_amd.build [--jobs N]
"""

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["api.hip", "ops.hip", "blocklu.hip", "krylov.hip", "multigrid.hip"]
LIB = os.path.join(HERE, "libkktfwi.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are left to no one: the compiler must not form them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wno-unused-result", "-Wno-unused-value",
]


def _compile_one(src, obj):
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), cmd


def build(verbose=True):
    """Compile every source for gfx950 and link libkktfwi.so next to this file."""
    with tempfile.TemporaryDirectory(prefix="kktfwi_build_") as tmp:
        procs = []
        objs = []
        for src in SOURCES:
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            objs.append(obj)
            procs.append((src,) + _compile_one(src, obj))
        failed = False
        for src, proc, cmd in procs:
            out, _ = proc.communicate()
            text = out.decode(errors="replace")
            # hipcc's host pass does not know the packed-fp32 feature name; that is harmless
            lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
            if proc.returncode != 0:
                failed = True
                sys.stderr.write(f"[build] {src} failed:\n" + "\n".join(lines) + "\n")
            elif verbose and lines:
                sys.stderr.write(f"[build] {src}:\n" + "\n".join(lines[:40]) + "\n")
        if failed:
            raise RuntimeError("HIP compilation failed")
        tmp_lib = LIB + ".tmp"
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp_lib] + objs
        r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
        os.replace(tmp_lib, LIB)
    if verbose:
        sys.stderr.write(f"[build] wrote {LIB}\n")
    return LIB


if __name__ == "__main__":
    build()
