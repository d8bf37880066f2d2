"""CPU oracle for the homotopic alternating sequential filter (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package. It wraps ``hasf_oracle.c`` (plain C, one thread),
which shares nothing with the HIP library.

All arrays are numpy uint8 images (nonzero = object) or uint32 distance maps,
C-contiguous, shape (H, W).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hasf_oracle.c")
_SRC3 = os.path.join(_HERE, "hasf_oracle3d.c")
_SRCW = os.path.join(_HERE, "hasf_oracle_wshed.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

U8P = ctypes.POINTER(ctypes.c_uint8)
U32P = ctypes.POINTER(ctypes.c_uint32)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no threads)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, _SRC, _SRC3, _SRCW])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in (_SRC, _SRC3, _SRCW)):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    lib.oracle_simple_lut.argtypes = [ctypes.c_int, U8P]
    lib.oracle_topo_numbers.argtypes = [ctypes.c_int, ctypes.c_uint,
                                        ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    for name in ("oracle_edt_sq", "oracle_edt_sq_direct"):
        f = getattr(lib, name)
        f.argtypes = [U8P, ctypes.c_int, ctypes.c_int, ctypes.c_int, U32P]
        f.restype = ctypes.c_int
    for name in ("oracle_thin_p", "oracle_thicken_p", "oracle_thin_queue_p", "oracle_thicken_queue_p"):
        f = getattr(lib, name)
        f.argtypes = [U8P, U8P, U32P, ctypes.c_int, ctypes.c_int]
        f.restype = ctypes.c_long
    lib.oracle_thin_p_lut.argtypes = [U8P, U8P, U32P, ctypes.c_int, ctypes.c_int, U8P]
    lib.oracle_thin_p_lut.restype = ctypes.c_long
    for name in ("oracle_homotopic_thin", "oracle_homotopic_thicken"):
        f = getattr(lib, name)
        f.argtypes = [U8P, U8P, ctypes.c_int, ctypes.c_int]
        f.restype = ctypes.c_long
    for f in (lib.oracle_homotopic_thin_n, lib.oracle_homotopic_thicken_n):
        f.argtypes = [U8P, U8P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        f.restype = ctypes.c_long
    lib.oracle_hc.argtypes = [U8P, U8P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.oracle_hc.restype = ctypes.c_long
    lib.oracle_hf.argtypes = [U8P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.oracle_hf.restype = ctypes.c_long
    lib.oracle_hasf.argtypes = [U8P, U8P, ctypes.c_int, ctypes.c_int, ctypes.c_int, U8P]
    lib.oracle_hasf_cd.argtypes = [U8P, U8P, U8P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, U8P]
    lib.oracle_hasf_order.argtypes = [U8P, U8P, U8P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, U8P]
    lib.oracle_hasf.restype = ctypes.c_long
    lib.oracle_hasf_inf.argtypes = [U8P, U8P, U8P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.oracle_hasf_inf.restype = ctypes.c_long
    lib.oracle3_topo_numbers.argtypes = [ctypes.c_uint32, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.oracle3_simple.argtypes = [ctypes.c_uint32]
    lib.oracle3_edt_sq.argtypes = [U8P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, U32P]
    lib.oracle3_schedule.argtypes = [ctypes.c_int, U8P, U8P, U32P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.oracle3_schedule.restype = ctypes.c_long
    lib.oracle3_hasf.argtypes = [U8P, U8P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, U8P]
    lib.oracle3_hasf.restype = ctypes.c_long
    lib.oracle_wshed.argtypes = [U8P, ctypes.c_int, ctypes.c_int]
    lib.oracle_wshed.restype = ctypes.c_long
    lib.oracle_hasf_queue.argtypes = [U8P, U8P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.oracle_hasf_queue.restype = ctypes.c_long
    _lib = lib
    return lib


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(U8P)


def _opt_u8(a):
    if a is None:
        return None, None
    return _u8(a)


def _check(rc, what):
    if rc < 0:
        raise RuntimeError("%s failed with code %d" % (what, rc))
    return rc


def simple_lut(n: int = 8) -> np.ndarray:
    """256-entry table: 1 where the neighbourhood code is simple for (n, n-bar)."""
    lut = np.zeros(256, dtype=np.uint8)
    _check(_load().oracle_simple_lut(n, lut.ctypes.data_as(U8P)), "simple_lut")
    return lut


def topo_numbers(n: int, m: int):
    T = ctypes.c_int()
    Tb = ctypes.c_int()
    _check(_load().oracle_topo_numbers(n, m, ctypes.byref(T), ctypes.byref(Tb)), "topo_numbers")
    return T.value, Tb.value


def edt_sq(feat, frame: bool = False, direct: bool = False) -> np.ndarray:
    """Squared Euclidean distance to the nearest nonzero pixel (+ outside if frame)."""
    f, fp = _u8(feat)
    H, W = f.shape
    out = np.zeros((H, W), dtype=np.uint32)
    fn = _load().oracle_edt_sq_direct if direct else _load().oracle_edt_sq
    _check(fn(fp, H, W, int(bool(frame)), out.ctypes.data_as(U32P)), "edt_sq")
    return out


def thin_p(S, K, P, queue: bool = False):
    s, sp = _u8(S)
    s = s.copy()
    sp = s.ctypes.data_as(U8P)
    k, kp = _opt_u8(K)
    p = np.ascontiguousarray(P, dtype=np.uint32)
    fn = _load().oracle_thin_queue_p if queue else _load().oracle_thin_p
    rounds = _check(fn(sp, kp, p.ctypes.data_as(U32P), s.shape[0], s.shape[1]), "thin")
    return s, rounds


def thin_p_lut(S, K, P, lut):
    s = np.ascontiguousarray(S, dtype=np.uint8).copy()
    k, kp = _opt_u8(K)
    p = np.ascontiguousarray(P, dtype=np.uint32)
    l = np.ascontiguousarray(lut, dtype=np.uint8)
    rounds = _check(_load().oracle_thin_p_lut(s.ctypes.data_as(U8P), kp, p.ctypes.data_as(U32P),
                                              s.shape[0], s.shape[1], l.ctypes.data_as(U8P)),
                    "thin_lut")
    return s, rounds


def thicken_p(S, V, P, queue: bool = False):
    s = np.ascontiguousarray(S, dtype=np.uint8).copy()
    v, vp = _opt_u8(V)
    p = np.ascontiguousarray(P, dtype=np.uint32)
    fn = _load().oracle_thicken_queue_p if queue else _load().oracle_thicken_p
    rounds = _check(fn(s.ctypes.data_as(U8P), vp, p.ctypes.data_as(U32P), s.shape[0], s.shape[1]),
                    "thicken")
    return s, rounds


def homotopic_thin(X, K=None, n: int = 8) -> np.ndarray:
    """H(X, K) (Sec. 2) for the pair (n, n-bar) = (8, 4) or (4, 8)."""
    x = np.ascontiguousarray(X, dtype=np.uint8).copy()
    k, kp = _opt_u8(K)
    _check(_load().oracle_homotopic_thin_n(x.ctypes.data_as(U8P), kp, x.shape[0], x.shape[1], n),
           "homotopic_thin")
    return x


def homotopic_thicken(Y, V, n: int = 8) -> np.ndarray:
    """*H(Y, V) (Sec. 2) for the pair (n, n-bar) = (8, 4) or (4, 8)."""
    y = np.ascontiguousarray(Y, dtype=np.uint8).copy()
    v, vp = _opt_u8(V)
    _check(_load().oracle_homotopic_thicken_n(y.ctypes.data_as(U8P), vp, y.shape[0], y.shape[1], n),
           "homotopic_thicken")
    return y


def hc(X, C, i: int) -> np.ndarray:
    x = np.ascontiguousarray(X, dtype=np.uint8).copy()
    c, cp = _opt_u8(C)
    _check(_load().oracle_hc(x.ctypes.data_as(U8P), cp, x.shape[0], x.shape[1], i), "hc")
    return x


def hf(X, i: int) -> np.ndarray:
    x = np.ascontiguousarray(X, dtype=np.uint8).copy()
    _check(_load().oracle_hf(x.ctypes.data_as(U8P), x.shape[0], x.shape[1], i), "hf")
    return x


def hasf(X, C, r: int, stages: bool = False, queue: bool = False, D=None, n: int = 8, order: int = 0):
    """HASF of order r (Sec. 2) with constraint sets C (kept object) and D (kept
    background), for the connectivity pair (n, n-bar) = (8, 4) or (4, 8);
    order 0 applies HF_i o HC_i at every radius (the formula: cutting first),
    order 1 the dual HC_i o HF_i (filling first). With stages=True also
    returns an (r, 4, H, W) dump of the states in the order produced."""
    x = np.ascontiguousarray(X, dtype=np.uint8).copy()
    c, cp = _opt_u8(C)
    H, W = x.shape
    if queue:
        assert D is None and n == 8
        _check(_load().oracle_hasf_queue(x.ctypes.data_as(U8P), cp, H, W, r), "hasf_queue")
        return x
    st = np.zeros((max(r, 1), 4, H, W), dtype=np.uint8) if stages else None
    sp = st.ctypes.data_as(U8P) if st is not None else None
    if order != 0:
        assert not queue
        d, dp = _opt_u8(D)
        _check(_load().oracle_hasf_order(x.ctypes.data_as(U8P), cp, dp, H, W, r, n, order, sp), "hasf_order")
    elif D is None and n == 8:
        _check(_load().oracle_hasf(x.ctypes.data_as(U8P), cp, H, W, r, sp), "hasf")
    else:
        d, dp = _opt_u8(D)
        _check(_load().oracle_hasf_cd(x.ctypes.data_as(U8P), cp, dp, H, W, r, n, sp), "hasf_cd")
    return (x, st[:r]) if stages else x


def hasf_inf(X, C=None, D=None, n: int = 8, order: int = 0, r_max: int = 0):
    """"r = infinity": radii 1, 2, ... (order as in hasf) until the first
    radius that leaves the set unchanged, at most r_max (0: the saturation
    radius, the least i with i^2 >= (H-1)^2 + (W-1)^2). Returns (result,
    last radius applied)."""
    x = np.ascontiguousarray(X, dtype=np.uint8).copy()
    c, cp = _opt_u8(C)
    d, dp = _opt_u8(D)
    used = ctypes.c_int(0)
    _check(_load().oracle_hasf_inf(x.ctypes.data_as(U8P), cp, dp, x.shape[0], x.shape[1], n, order, r_max,
                                   ctypes.byref(used)), "hasf_inf")
    return x, used.value


# ---------------------------------------------------------------------------
# 3D: (26,6) connectivity, volumes of shape (D, H, W)
# ---------------------------------------------------------------------------
def topo_numbers3(code: int):
    """(T26, Tbar6) of a 26-neighbourhood code (bit b: offset b of
    {-1,0,1}^3 without the centre, lexicographic in (dz, dy, dx))."""
    T, Tb = ctypes.c_int(0), ctypes.c_int(0)
    _load().oracle3_topo_numbers(code, ctypes.byref(T), ctypes.byref(Tb))
    return T.value, Tb.value


def simple3(code: int) -> bool:
    return bool(_load().oracle3_simple(code))


def _u8v(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    assert a.ndim == 3
    return a, a.ctypes.data_as(U8P)


def edt_sq3(F, frame: bool = False) -> np.ndarray:
    """Squared distance to the nearest nonzero voxel (+ outside the box if frame)."""
    f, fp = _u8v(F)
    out = np.zeros(f.shape, dtype=np.uint32)
    _check(_load().oracle3_edt_sq(fp, *f.shape, int(bool(frame)), out.ctypes.data_as(U32P)), "edt_sq3")
    return out


def schedule3(mode: int, S, B, P):
    """mode 0: thin S keeping B; mode 1: thicken S inside B; priority P."""
    s = np.ascontiguousarray(S, dtype=np.uint8).copy()
    b = None if B is None else np.ascontiguousarray(B, dtype=np.uint8)
    p = np.ascontiguousarray(P, dtype=np.uint32)
    rc = _load().oracle3_schedule(mode, s.ctypes.data_as(U8P), None if b is None else b.ctypes.data_as(U8P),
                                  p.ctypes.data_as(U32P), *s.shape)
    if rc < 0:
        raise RuntimeError("schedule3 failed (%d)" % rc)
    return s


def hasf3(X, C, r: int, stages: bool = False):
    """3D HASF of order r, (26,6), constraint set C; with stages=True also an
    (r, 4, D, H, W) dump as in hasf()."""
    x = np.ascontiguousarray(X, dtype=np.uint8).copy()
    c = None if C is None else np.ascontiguousarray(C, dtype=np.uint8)
    st = np.zeros((max(r, 1), 4) + x.shape, dtype=np.uint8) if stages else None
    _check(_load().oracle3_hasf(x.ctypes.data_as(U8P), None if c is None else c.ctypes.data_as(U8P), *x.shape, r,
                                None if st is None else st.ctypes.data_as(U8P)), "hasf3")
    return (x, st[:r]) if stages else x


def hasf_labels(Lab, values, r: int):
    """Per-label smoothing: for each label value v, HASF of order r (C and D
    empty, (8,4), cutting first) of the object set {p : Lab[p] == v}, as its
    own binary image (Sec. 2 applied label by label). Returns an (n, H, W)
    array of 0/1 planes, one per value, in the order given."""
    lab = np.ascontiguousarray(Lab, dtype=np.uint8)
    return np.stack([hasf((lab == np.uint8(v)).astype(np.uint8), None, r) for v in values])


def wshed(F):
    """The topological watershed's lowering (grey-level W-thinning, lower
    sections 4-connected) of the uint8 grey-level image F, to stability, on the
    subfield schedule: returns the lowered image."""
    f = np.ascontiguousarray(F, dtype=np.uint8).copy()
    n = _load().oracle_wshed(f.ctypes.data_as(U8P), *f.shape)
    if n < 0:
        raise ValueError("oracle wshed: bad arguments")
    return f
