"""ctypes binding of libhasf (argument marshalling only).

Images are torch uint8 CUDA tensors of shape (H, W) with unit column stride;
the row pitch is taken from ``stride(0)``. Every call is enqueued on the
current torch stream of the context's device. No computation happens here:
each function forwards to the C entry point of the same name.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libhasf.so")

HASF_OK = 0
HASF_EINVAL = -1
HASF_ENOMEM = -2
HASF_EDEVICE = -3
HASF_EAGAIN = -4
HASF_ETIMEDOUT = -5
HASF_EINTERNAL = -6
HASF_R_MAX = 15
HASF_SERVE_LANES_MAX = 16
HASF_SERVE_PERSISTENT = 1
HASF_NOALLOC_SCRATCH_BYTES = 16 << 20
HASF_INF_COMPOSED = 1
# the tile shape by image size (as the header's HASF_TILE_* defaults)
HASF_TILE_SMALL_PIXELS = 1 << 21
HASF_TILE_ROWS_SMALL = 32
HASF_TILE_HALO_SMALL = 12
HASF_TILE_ROWS_DEFAULT = 64
HASF_TILE_HALO_DEFAULT = 16
HASF_TILE_LARGE_PIXELS = 1 << 23
HASF_TILE_ROWS_LARGE = 128
HASF_TILE_HALO_LARGE = 24


def default_tile_shape(H: int, W: int):
    """(tile rows, halo rows) the library takes for an H x W image when
    tile_rows and tile_halo are 0."""
    px = H * W
    if px >= HASF_TILE_LARGE_PIXELS:
        return HASF_TILE_ROWS_LARGE, HASF_TILE_HALO_LARGE
    if px < HASF_TILE_SMALL_PIXELS:
        return HASF_TILE_ROWS_SMALL, HASF_TILE_HALO_SMALL
    return HASF_TILE_ROWS_DEFAULT, HASF_TILE_HALO_DEFAULT

if not os.path.exists(LIB_PATH):
    raise ImportError("libhasf.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)

# torch first: the library then binds to the HIP runtime torch has already
# loaded, so the process has one runtime (two runtimes do not share the GPU)
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)


class _Opts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("hbm_budget", ctypes.c_size_t), ("flags", ctypes.c_uint),
                ("grid_min_pixels", ctypes.c_size_t), ("batch_grid_min_pixels", ctypes.c_size_t),
                ("tile_rows", ctypes.c_int), ("tile_halo", ctypes.c_int), ("tune_cache", ctypes.c_char_p),
                ("tile_cols", ctypes.c_int)]


class _Image(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("C", ctypes.c_void_p), ("H", ctypes.c_int), ("W", ctypes.c_int),
                ("ld", ctypes.c_int64), ("r", ctypes.c_int), ("D", ctypes.c_void_p), ("conn", ctypes.c_int),
                ("order", ctypes.c_int)]


class _Volume(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("C", ctypes.c_void_p), ("D", ctypes.c_int), ("H", ctypes.c_int),
                ("W", ctypes.c_int), ("r", ctypes.c_int)]


class _GImage(ctypes.Structure):
    _fields_ = [("F", ctypes.c_void_p), ("H", ctypes.c_int), ("W", ctypes.c_int), ("ld", ctypes.c_int64)]


class _ServeOpts(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_size_t), ("lanes", ctypes.c_int), ("max_batch", ctypes.c_int),
                ("max_pending", ctypes.c_int), ("flags", ctypes.c_uint), ("express_lanes", ctypes.c_int),
                ("express_max_pixels", ctypes.c_int)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("ticket", ctypes.c_uint64), ("submit_s", ctypes.c_double),
                ("done_s", ctypes.c_double), ("latency_ms", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("pending", ctypes.c_uint64), ("in_flight", ctypes.c_uint64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("frames_per_s", ctypes.c_double),
                ("mpixel_per_s", ctypes.c_double), ("pool_bytes", ctypes.c_size_t),
                ("pool_peak_bytes", ctypes.c_size_t), ("kernel_launches", ctypes.c_uint64),
                ("frames_per_launch", ctypes.c_double), ("batch_max", ctypes.c_uint64)]


_vp = ctypes.c_void_p
_lib.hasf_serve.argtypes = [_vp, ctypes.POINTER(_ServeOpts), ctypes.POINTER(_vp)]
_lib.hasf_serve_submit.argtypes = [_vp, ctypes.POINTER(_Image), ctypes.POINTER(ctypes.c_uint64)]
_lib.hasf_serve_submit_host.argtypes = [_vp, ctypes.POINTER(_Image), ctypes.POINTER(ctypes.c_uint64)]
_lib.hasf_serve_wait.argtypes = [_vp, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(_Result)]
_lib.hasf_serve_stats.argtypes = [_vp, ctypes.POINTER(_Stats)]
_lib.hasf_serve_stop.argtypes = [_vp]
for _f in ("hasf_serve", "hasf_serve_submit", "hasf_serve_submit_host", "hasf_serve_wait", "hasf_serve_stats",
           "hasf_serve_stop"):
    getattr(_lib, _f).restype = ctypes.c_int
_lib.hasf_create.argtypes = [ctypes.POINTER(_Opts), ctypes.POINTER(_vp)]
_lib.hasf_destroy.argtypes = [_vp]
_lib.hasf_destroy.restype = None
_lib.hasf_set_stream.argtypes = [_vp, _vp]
_lib.hasf_sync.argtypes = [_vp]
_lib.hasf_strerror.argtypes = [ctypes.c_int]
_lib.hasf_strerror.restype = ctypes.c_char_p
_lib.hasf_last_error.argtypes = [_vp]
_lib.hasf_last_error.restype = ctypes.c_char_p
_lib.hasf_simple_lut.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_uint32)]
_lib.hasf_edt_sq.argtypes = [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int, _vp,
                             ctypes.c_int64]
_lib.hasf_edt_sq_noalloc.argtypes = _lib.hasf_edt_sq.argtypes
_lib.hasf_homotopic_thin.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int64]
_lib.hasf_homotopic_thicken.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int64]
_lib.hasf_homotopic_thin_conn.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int]
_lib.hasf_homotopic_thicken_conn.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                             ctypes.c_int]
_lib.hasf_filter.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int]
_lib.hasf_filter_cd.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                ctypes.c_int]
_lib.hasf_filter_batch.argtypes = [_vp, ctypes.POINTER(_Image), ctypes.c_int]
_lib.hasf_filter3_batch.argtypes = [_vp, ctypes.POINTER(_Volume), ctypes.c_int]
_lib.hasf_watershed_batch.argtypes = [_vp, ctypes.POINTER(_GImage), ctypes.c_int]
_lib.hasf_watershed.argtypes = [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int64]
_lib.hasf_filter3.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
_lib.hasf_filter_inf.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_uint, ctypes.POINTER(ctypes.c_int)]
_lib.hasf_filter_labels.argtypes = [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_uint8), ctypes.c_int, ctypes.c_int, _vp,
                                    ctypes.c_int64, ctypes.c_int64]
for _f in ("hasf_create", "hasf_set_stream", "hasf_sync", "hasf_simple_lut", "hasf_edt_sq", "hasf_edt_sq_noalloc",
           "hasf_homotopic_thin", "hasf_homotopic_thicken", "hasf_homotopic_thin_conn",
           "hasf_homotopic_thicken_conn", "hasf_filter", "hasf_filter_cd",
           "hasf_filter_batch", "hasf_filter_labels", "hasf_filter_inf", "hasf_filter3", "hasf_filter3_batch",
           "hasf_watershed", "hasf_watershed_batch"):
    getattr(_lib, _f).restype = ctypes.c_int


class _GridCounts(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("rounds", ctypes.c_uint64), ("levels", ctypes.c_uint64),
                ("barriers", ctypes.c_uint64)]


_lib.hasf_get_grid_counts.argtypes = [_vp, ctypes.POINTER(_GridCounts), ctypes.c_int]
_lib.hasf_get_grid_counts.restype = ctypes.c_int


class HasfError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__("%s (%d): %s" % (_lib.hasf_strerror(status).decode(), status, detail))
        self.status = status


def lib():
    return _lib


def simple_lut(n: int = 8):
    """256-entry simple-point table as a list of 0/1 (host-only)."""
    bits = (ctypes.c_uint32 * 8)()
    st = _lib.hasf_simple_lut(n, bits)
    if st != HASF_OK:
        raise HasfError(st, _lib.hasf_last_error(None).decode())
    return [(bits[m >> 5] >> (m & 31)) & 1 for m in range(256)]


def _image(item, tag="", device=None):
    """hasf_image for (X, C, r), (X, C, r, D, conn) or (X, C, r, D, conn, order)."""
    X, C, r = item[0], item[1], item[2]
    D = item[3] if len(item) > 3 else None
    conn = item[4] if len(item) > 4 else 0
    order = item[5] if len(item) > 5 else 0
    H, W, ld = _img(X, "X" + tag, device)
    _companion(C, X, "C" + tag)
    _companion(D, X, "D" + tag)
    return _Image(X.data_ptr(), C.data_ptr() if C is not None else None, H, W, ld, r,
                  D.data_ptr() if D is not None else None, conn, order)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _img(t, name, device=None):
    """(H, W, pitch) of a 2D uint8 CUDA tensor with unit column stride (and,
    when device is given, on that device)."""
    if t is None or t.dtype != torch.uint8 or t.dim() != 2 or t.stride(1) != 1 or not t.is_cuda:
        raise ValueError("%s must be a 2D uint8 CUDA tensor with unit column stride" % name)
    if t.shape[0] > 1 and t.stride(0) < t.shape[1]:
        raise ValueError("%s: rows overlap (pitch %d < width %d)" % (name, t.stride(0), t.shape[1]))
    if device is not None and t.device.index != device:
        raise ValueError("%s is on cuda:%s, the context on cuda:%d" % (name, t.device.index, device))
    return t.shape[0], t.shape[1], t.stride(0)


def _companion(T, X, name):
    """A plane that shares X's layout (C, D, K, V): same dtype, device, shape and pitch."""
    if T is None:
        return
    _img(T, name, X.device.index)
    if T.shape != X.shape or T.stride(0) != X.stride(0):
        raise ValueError("%s must match X's shape and pitch" % name)


class Context:
    def __init__(self, device: int = 0, hbm_budget: int = 0, grid_min_pixels: int = 0,
                 batch_grid_min_pixels: int = 0, tile_rows: int = 0, tile_halo: int = 0,
                 tune_cache: str = None, tile_cols: int = 0):
        import torch
        self._torch = torch
        self.device = device
        self.tile_rows = tile_rows
        self.tile_halo = tile_halo
        h = _vp()
        opts = _Opts(device, hbm_budget, 0, grid_min_pixels, batch_grid_min_pixels, tile_rows, tile_halo,
                     tune_cache.encode() if tune_cache else None, tile_cols)
        st = _lib.hasf_create(ctypes.byref(opts), ctypes.byref(h))
        if st != HASF_OK:
            raise HasfError(st, _lib.hasf_last_error(None).decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.hasf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != HASF_OK:
            raise HasfError(st, _lib.hasf_last_error(self._h).decode())

    def _stream(self):
        s = self._torch.cuda.current_stream(self.device).cuda_stream
        self._check(_lib.hasf_set_stream(self._h, _vp(s)))

    def sync(self):
        self._check(_lib.hasf_sync(self._h))

    def grid_counts(self, reset: bool = False):
        """hasf_get_grid_counts: launches, rounds, levels, barriers of the
        grid-filtered images since creation or the last reset."""
        c = _GridCounts()
        self._check(_lib.hasf_get_grid_counts(self._h, ctypes.byref(c), int(bool(reset))))
        return {k: int(getattr(c, k)) for k, _ in _GridCounts._fields_}

    def edt_sq(self, feat, border_is_feature: bool = False, out=None, noalloc: bool = False):
        """hasf_edt_sq, or hasf_edt_sq_noalloc when noalloc is set (then give
        `out`: allocating it here would defeat the purpose)."""
        H, W, ld = _img(feat, "feat", self.device)
        if out is None:
            out = self._torch.empty((H, W), dtype=self._torch.int32, device=feat.device)
        elif (out.dtype not in (torch.int32, torch.uint32) or out.dim() != 2 or tuple(out.shape) != (H, W)
              or out.stride(1) != 1 or not out.is_cuda or out.device.index != self.device
              or (H > 1 and out.stride(0) < W)):
            raise ValueError("out must be an (H, W) int32 or uint32 tensor with unit column stride on cuda:%d"
                             % self.device)
        self._stream()
        fn = _lib.hasf_edt_sq_noalloc if noalloc else _lib.hasf_edt_sq
        self._check(fn(self._h, _ptr(feat), H, W, ld, int(bool(border_is_feature)), _ptr(out), out.stride(0)))
        return out

    def homotopic_thin(self, X, K=None, conn: int = 8):
        H, W, ld = _img(X, "X", self.device)
        _companion(K, X, "K")
        self._stream()
        if conn == 8:
            self._check(_lib.hasf_homotopic_thin(self._h, _ptr(X), _ptr(K), H, W, ld))
        else:
            self._check(_lib.hasf_homotopic_thin_conn(self._h, _ptr(X), _ptr(K), H, W, ld, conn))
        return X

    def homotopic_thicken(self, Y, V, conn: int = 8):
        H, W, ld = _img(Y, "Y", self.device)
        if V is None:
            raise ValueError("V must not be None")
        _companion(V, Y, "V")
        self._stream()
        if conn == 8:
            self._check(_lib.hasf_homotopic_thicken(self._h, _ptr(Y), _ptr(V), H, W, ld))
        else:
            self._check(_lib.hasf_homotopic_thicken_conn(self._h, _ptr(Y), _ptr(V), H, W, ld, conn))
        return Y

    def filter(self, X, C=None, r: int = 1, D=None, conn: int = 8, order: int = 0):
        """hasf_filter (D None, conn 8, order 0), hasf_filter_cd (order 0) or,
        for the dual order (filling first), hasf_filter_batch of this one image."""
        if order != 0:
            self.filter_batch([(X, C, r, D, conn, order)])
            return X
        H, W, ld = _img(X, "X", self.device)
        _companion(C, X, "C")
        _companion(D, X, "D")
        self._stream()
        if D is None and conn == 8:
            self._check(_lib.hasf_filter(self._h, _ptr(X), _ptr(C), H, W, ld, r))
        else:
            self._check(_lib.hasf_filter_cd(self._h, _ptr(X), _ptr(C), _ptr(D), H, W, ld, r, conn))
        return X

    def filter_inf(self, X, C=None, D=None, conn: int = 8, order: int = 0, r_max: int = 0,
                   composed: bool = False) -> int:
        """hasf_filter_inf: radii 1, 2, ... until a radius leaves X unchanged
        (at most r_max; 0: the saturation radius). Returns the last radius
        applied; the context's stream is idle on return."""
        H, W, ld = _img(X, "X", self.device)
        _companion(C, X, "C")
        _companion(D, X, "D")
        self._stream()
        used = ctypes.c_int(0)
        self._check(_lib.hasf_filter_inf(self._h, _ptr(X), _ptr(C), _ptr(D), H, W, ld, conn, order, r_max,
                                         HASF_INF_COMPOSED if composed else 0, ctypes.byref(used)))
        return used.value

    @staticmethod
    def _vol(X, name):
        if (X is None or X.dtype != torch.uint8 or X.dim() != 3 or not X.is_cuda or not X.is_contiguous()):
            raise ValueError("%s must be a contiguous 3D uint8 CUDA tensor" % name)
        return tuple(X.shape)

    def filter3_batch(self, items):
        """3D HASF, (26,6): items are (X, C or None, r) with X a contiguous
        (D, H, W) uint8 CUDA tensor, filtered in place in one launch."""
        arr = (_Volume * max(1, len(items)))()
        for k, (X, C, r) in enumerate(items):
            D, H, W = self._vol(X, "X[%d]" % k)
            if C is not None and (self._vol(C, "C[%d]" % k) != (D, H, W)):
                raise ValueError("C[%d] must match X's shape" % k)
            if X.device.index != self.device:
                raise ValueError("X[%d] is on another device" % k)
            arr[k] = _Volume(X.data_ptr(), C.data_ptr() if C is not None else None, D, H, W, r)
        self._stream()
        self._check(_lib.hasf_filter3_batch(self._h, arr, len(items)))
        return [it[0] for it in items]

    def filter3(self, X, C=None, r: int = 1):
        return self.filter3_batch([(X, C, r)])[0]

    def watershed_batch(self, images):
        """The topological watershed's lowering (grey-level W-thinning) of each
        2D uint8 CUDA tensor (row pitch allowed), in place, in one launch."""
        arr = (_GImage * max(1, len(images)))()
        for k, F in enumerate(images):
            H, W, ld = _img(F, "F[%d]" % k, self.device)
            arr[k] = _GImage(F.data_ptr(), H, W, ld)
        self._stream()
        self._check(_lib.hasf_watershed_batch(self._h, arr, len(images)))
        return images

    def watershed(self, F):
        return self.watershed_batch([F])[0]

    def plan_batch(self, items):
        """Prepare the descriptor array of a batch once (the tensors must stay alive).
        items: (X, C or None, r), (X, C or None, r, D or None, conn) or
        (X, C or None, r, D or None, conn, order)."""
        arr = (_Image * max(1, len(items)))()
        for k, it in enumerate(items):
            arr[k] = _image(it, "[%d]" % k, self.device)
        return (arr, len(items), list(items))

    def run_plan(self, plan):
        arr, n, _ = plan
        self._stream()
        self._check(_lib.hasf_filter_batch(self._h, arr, n))

    def filter_batch(self, items):
        """items: sequence of (X, C or None, r), (X, C or None, r, D or None, conn)
        or (X, C or None, r, D or None, conn, order)."""
        arr = (_Image * max(1, len(items)))()
        for k, it in enumerate(items):
            arr[k] = _image(it, "[%d]" % k, self.device)
        self._stream()
        self._check(_lib.hasf_filter_batch(self._h, arr, len(items)))
        return [it[0] for it in items]

    def filter_labels(self, L, values, r: int = 1, out=None):
        """hasf_filter_labels: plane k of the result is HASF of order r of the
        pixels of L equal to values[k], as 0/1. out: None (an (n, H, W) uint8
        tensor is allocated) or an (n, H, W) uint8 CUDA tensor with unit column
        stride whose planes do not overlap."""
        H, W, ld = _img(L, "L", self.device)
        vals = bytes(int(v) for v in values)  # ValueError outside 0..255
        n = len(vals)
        if out is None:
            out = self._torch.empty((max(n, 1), H, W), dtype=self._torch.uint8, device=L.device)
        elif (out.dtype != self._torch.uint8 or out.dim() != 3 or tuple(out.shape) != (n, H, W)
              or out.stride(2) != 1 or not out.is_cuda or out.device.index != self.device):
            raise ValueError("out must be an (n, H, W) uint8 tensor with unit column stride on cuda:%d"
                             % self.device)
        buf = (ctypes.c_uint8 * max(n, 1)).from_buffer_copy(vals if n else b"\0")
        self._stream()
        self._check(_lib.hasf_filter_labels(self._h, _ptr(L), H, W, ld, buf, n, r, _ptr(out), out.stride(1),
                                            out.stride(0)))
        return out


class Server:
    """Served stream on a context's device (hasf_serve). Frames are device
    tensors filtered in place (submit_host: host tensors, copied in and out);
    keep them alive until wait() returns."""

    def __init__(self, ctx: Context, pool_bytes: int = 0, lanes: int = 0, max_batch: int = 0,
                 max_pending: int = 0, persistent: bool = False, express_lanes: int = -1,
                 express_max_pixels: int = 0):
        self._ctx = ctx
        h = _vp()
        flags = HASF_SERVE_PERSISTENT if persistent else 0
        opts = _ServeOpts(pool_bytes, lanes, max_batch, max_pending, flags, express_lanes, express_max_pixels)
        st = _lib.hasf_serve(ctx._h, ctypes.byref(opts), ctypes.byref(h))
        if st != HASF_OK:
            raise HasfError(st, _lib.hasf_last_error(ctx._h).decode())
        self._h = h
        self._keep = {}

    def submit(self, X, C=None, r: int = 1, check: bool = True, D=None, conn: int = 0, order: int = 0):
        """Queue a frame; returns its ticket (or the status when check=False and it fails)."""
        im = _image((X, C, r, D, conn, order), device=self._ctx.device)
        t = ctypes.c_uint64()
        st = _lib.hasf_serve_submit(self._h, ctypes.byref(im), ctypes.byref(t))
        if st != HASF_OK:
            if check:
                raise HasfError(st, "hasf_serve_submit")
            return st
        self._keep[t.value] = (X, C, D)
        return t.value

    def submit_host(self, X, C=None, r: int = 1, check: bool = True, D=None, conn: int = 0, order: int = 0):
        """Queue a frame in host memory (hasf_serve_submit_host): X, C, D are 2D
        uint8 CPU tensors with unit column stride and one pitch (pinned memory
        keeps the copies asynchronous); X receives the result. Returns the
        ticket (or the status when check=False and it fails)."""
        for name, T in (("X", X), ("C", C), ("D", D)):
            if T is None and name != "X":
                continue
            if (T is None or T.dtype != torch.uint8 or T.dim() != 2 or T.stride(1) != 1 or T.is_cuda
                    or (T.shape[0] > 1 and T.stride(0) < T.shape[1])):
                raise ValueError("%s must be a 2D uint8 CPU tensor with unit column stride" % name)
            if name != "X" and (T.shape != X.shape or T.stride(0) != X.stride(0)):
                raise ValueError("%s must have X's shape and pitch" % name)
        im = _Image(X.data_ptr(), C.data_ptr() if C is not None else None, X.shape[0], X.shape[1], X.stride(0), r,
                    D.data_ptr() if D is not None else None, conn, order)
        t = ctypes.c_uint64()
        st = _lib.hasf_serve_submit_host(self._h, ctypes.byref(im), ctypes.byref(t))
        if st != HASF_OK:
            if check:
                raise HasfError(st, "hasf_serve_submit_host")
            return st
        self._keep[t.value] = (X, C, D)
        return t.value

    def submit_raw(self, ptr, H, W, ld, r, cptr=None, dptr=None, conn=0, order=0):
        """Queue a frame given by device pointer (the caller keeps it alive); returns (status, ticket)."""
        im = _Image(ptr, cptr, H, W, ld, r, dptr, conn, order)
        t = ctypes.c_uint64()
        st = _lib.hasf_serve_submit(self._h, ctypes.byref(im), ctypes.byref(t))
        return st, t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        res = _Result()
        st = _lib.hasf_serve_wait(self._h, ticket, timeout_ms, ctypes.byref(res))
        if st == HASF_ETIMEDOUT:
            return None
        self._keep.pop(ticket, None)
        if st != HASF_OK:
            raise HasfError(st, "hasf_serve_wait")
        return {"ticket": res.ticket, "submit_s": res.submit_s, "done_s": res.done_s,
                "latency_ms": res.latency_ms}

    def stats(self):
        s = _Stats()
        st = _lib.hasf_serve_stats(self._h, ctypes.byref(s))
        if st != HASF_OK:
            raise HasfError(st, "hasf_serve_stats")
        return {k: getattr(s, k) for k, _ in _Stats._fields_}

    def stop(self):
        if getattr(self, "_h", None):
            st = _lib.hasf_serve_stop(self._h)
            self._h = None
            self._keep.clear()
            if st != HASF_OK:
                raise HasfError(st, "hasf_serve_stop")

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass
