"""Build step of the HIP library (hipcc, gfx950) into the package directory.

The library is several translation units (the runtime and C ABI, and the
template instances of the wavefront kernels spread over a few files) compiled
in parallel and linked into one shared object."""
from __future__ import annotations

import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB_PATH = os.path.join(HERE, "libhalign.so")
SOURCES = ["halign.hip", "launch_stream_r1.hip", "launch_stream_r6.hip", "launch_stream_r11.hip",
           "launch_stream16_r2.hip", "launch_stream16_r10.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed fp32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    """Compile libhalign.so for gfx950 (always recompiles)."""
    with tempfile.TemporaryDirectory(prefix="halign_build_") as tmpdir:
        objs, procs = [], []
        for s in SOURCES:
            obj = os.path.join(tmpdir, os.path.splitext(s)[0] + ".o")
            cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-c", "-o", obj, os.path.join(CSRC, s)]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        errs = []
        for s, p in procs:
            out, _ = p.communicate()
            if p.returncode != 0:
                errs.append(f"hipcc failed on {s}:\n{out}")
            elif out.strip() and verbose:
                print(out, flush=True)
        if errs:
            raise RuntimeError("\n".join(errs))
        tmp = LIB_PATH + ".tmp"
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def stale() -> bool:
    if not os.path.exists(LIB_PATH):
        return True
    t = os.path.getmtime(LIB_PATH)
    return any(os.path.getmtime(os.path.join(CSRC, d)) > t for d in os.listdir(CSRC)) or \
        os.path.getmtime(os.path.join(ROOT, "include", "halign.h")) > t


if __name__ == "__main__":
    print(build(verbose=True))
