"""The C-ABI library loads, exports every entry point its header declares, and
its host-only parts behave as documented (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libhasf.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hasf_[a-z_0-9]+)\s*\(", src)))


def _lib():
    from paper_1603_09337_amd import hasf
    return hasf, hasf.lib()


def test_every_declared_symbol_is_exported():
    hasf, lib = _lib()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_simple_lut_matches_oracle_component_counting():
    # the library's table is its bit-sliced kernel formula evaluated on single
    # bits; the oracle's comes from counting components (Sec. 2)
    hasf, _ = _lib()
    assert hasf.simple_lut(8) == oracle.simple_lut(8).tolist()
    assert hasf.simple_lut(4) == oracle.simple_lut(4).tolist()


def test_simple_lut_rejects_bad_arguments():
    hasf, lib = _lib()
    bits = (ctypes.c_uint32 * 8)()
    assert lib.hasf_simple_lut(6, bits) == hasf.HASF_EINVAL
    assert lib.hasf_simple_lut(8, None) == hasf.HASF_EINVAL


def test_null_context_is_rejected_before_device_work():
    hasf, lib = _lib()
    p = ctypes.c_void_p(0x1000)
    assert lib.hasf_filter(None, p, None, 8, 8, 8, 1) == hasf.HASF_EINVAL
    assert lib.hasf_edt_sq(None, p, 8, 8, 8, 0, p, 8) == hasf.HASF_EINVAL
    assert lib.hasf_homotopic_thin(None, p, None, 8, 8, 8) == hasf.HASF_EINVAL
    assert lib.hasf_homotopic_thicken(None, p, p, 8, 8, 8) == hasf.HASF_EINVAL
    assert lib.hasf_filter3(None, p, None, 4, 4, 4, 1) == hasf.HASF_EINVAL
    assert lib.hasf_watershed(None, p, 8, 8, 8) == hasf.HASF_EINVAL
    assert lib.hasf_watershed_batch(None, None, 1) == hasf.HASF_EINVAL
    assert lib.hasf_set_stream(None, None) == hasf.HASF_EINVAL
    assert lib.hasf_sync(None) == hasf.HASF_EINVAL
    assert b"ctx" in lib.hasf_last_error(None)


def test_strerror():
    hasf, lib = _lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.hasf_strerror(code)
    assert lib.hasf_strerror(-99) == b"unknown status"


def test_serve_rejects_null_arguments():
    hasf, lib = _lib()
    t = ctypes.c_uint64()
    assert lib.hasf_serve(None, None, None) == hasf.HASF_EINVAL
    assert lib.hasf_serve_submit(None, None, ctypes.byref(t)) == hasf.HASF_EINVAL
    assert lib.hasf_serve_wait(None, 1, 0, None) == hasf.HASF_EINVAL
    assert lib.hasf_serve_stats(None, None) == hasf.HASF_EINVAL
    assert lib.hasf_serve_stop(None) == hasf.HASF_EINVAL


def test_binding_refuses_host_and_malformed_tensors():
    # checked before any device work, so this runs without a GPU
    import torch
    from paper_1603_09337_amd import hasf
    for t in (torch.zeros((4, 4), dtype=torch.uint8), torch.zeros((4, 4), dtype=torch.float32),
              torch.zeros((4, 4, 2), dtype=torch.uint8), None):
        with pytest.raises(ValueError):
            hasf._img(t, "X")
    with pytest.raises(ValueError):
        hasf._image((torch.zeros((4, 4), dtype=torch.uint8), None, 1))


C_PROGRAM = r"""
#include <stdio.h>
#include "libhasf.h"
int main(void)
{
    uint32_t bits[8];
    hasf_status st = hasf_simple_lut(8, bits);
    int n = 0;
    for (int m = 0; m < 256; ++m)
        n += (bits[m >> 5] >> (m & 31)) & 1u;
    hasf_image im = {0};
    hasf_serve_opts so = {0};
    hasf_opts o = {0};
    (void)im; (void)so; (void)o;
    printf("%d %d %s\n", (int)st, n, hasf_strerror(HASF_EINVAL));
    return st == HASF_OK && n == 116 && hasf_simple_lut(3, bits) == HASF_EINVAL ? 0 : 1;
}
"""


def test_header_is_plain_c_and_links(tmp_path):
    # the boundary is a C ABI: a C99 program compiles against the header with
    # -pedantic -Werror, links against the library and calls its host-only
    # entry points (no GPU needed)
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    hasf, _ = _lib()
    libdir = os.path.dirname(hasf.LIB_PATH)
    src = tmp_path / "use_hasf.c"
    src.write_text(C_PROGRAM)
    exe = tmp_path / "use_hasf"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                           os.path.join(ROOT, "include"), str(src), "-o", str(exe), "-L", libdir, "-lhasf",
                           "-Wl,-rpath," + libdir])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.split()[:2] == ["0", "116"]


def test_binding_constants_match_the_header():
    # every HASF_ constant the binding mirrors has the header's value
    import re
    hasf, _ = _lib()
    text = open(os.path.join(ROOT, "include", "libhasf.h")).read()
    defs = {}
    for name, expr in re.findall(r"^#define\s+(HASF_\w+)\s+(.+?)\s*(?:/\*.*)?$", text, re.M):
        expr = expr.replace("(size_t)", "")
        if re.fullmatch(r"[0-9()<>\s+\-*]+", expr):
            defs[name] = eval(expr)
    mirrored = [k for k in dir(hasf) if k.startswith("HASF_") and isinstance(getattr(hasf, k), int)]
    assert len(mirrored) > 10
    for k in mirrored:
        if k in defs:
            assert getattr(hasf, k) == defs[k], k
    for k in [k for k in defs if k.startswith("HASF_TILE_")]:
        assert getattr(hasf, k) == defs[k], k
    assert hasf.default_tile_shape(4096, 4096) == (defs["HASF_TILE_ROWS_LARGE"], defs["HASF_TILE_HALO_LARGE"])
    assert hasf.default_tile_shape(2048, 2048) == (defs["HASF_TILE_ROWS_DEFAULT"], defs["HASF_TILE_HALO_DEFAULT"])
    assert hasf.default_tile_shape(1024, 1024) == (defs["HASF_TILE_ROWS_SMALL"], defs["HASF_TILE_HALO_SMALL"])
