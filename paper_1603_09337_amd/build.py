"""Build libhasf.so for gfx950 with hipcc (in-tree, no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_lib", "libhasf.so")
SOURCES = ["hasf_api.hip", "hasf_filter.hip", "hasf_tile.hip", "hasf_edt.hip", "hasf_topo.hip", "hasf_serve.hip",
           "hasf_vol.hip", "hasf_wshed.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere (the library has no float math at all)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-value", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        sys.stderr.write(out + "\n")
        raise RuntimeError("hipcc failed (%d): %s" % (res.returncode, " ".join(cmd[-3:])))


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compiles every source to an object (in parallel), then links the
    shared library. Always compiles."""
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    objdir = os.path.join(os.path.dirname(OUT), "obj%d" % os.getpid())
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmds = [[hipcc()] + HIPCC_FLAGS + inc + ["-c", "-o", o, os.path.join(CSRC, s)] for s, o in zip(SOURCES, objs)]
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    tmp = OUT + ".tmp%d" % os.getpid()
    try:
        with ThreadPoolExecutor(jobs) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        _run([hipcc()] + HIPCC_FLAGS + ["-shared", "-o", tmp] + objs, verbose)
        os.replace(tmp, OUT)
    finally:
        # the object folder (and a half-written library) go whether or not
        # the build succeeded
        for f in objs + [tmp]:
            if os.path.exists(f):
                os.remove(f)
        if os.path.isdir(objdir):
            os.rmdir(objdir)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
