"""Python binding of libcomposite.so (include/composite.h).

Argument marshalling only: every step of the compositing path runs in the HIP
library.  The functions carry the C names; ``Composite`` is a small owner
object over one context.  If the library is missing the import of this module
fails loudly; there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os
import re
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# COMPOSITE_LIBRARY names another build of the same sources (the host-side
# sanitizer build of the CPU tests); by default the in-tree library is loaded.
LIB_PATH = os.environ.get("COMPOSITE_LIBRARY") or os.path.join(_HERE, "libcomposite.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "composite.h")

CMP_OK, CMP_EINVAL, CMP_ENOMEM, CMP_ERANGE, CMP_ENOTMEMBER = 0, -1, -2, -3, -4
CMP_EUNSUPPORTED, CMP_EDEVICE, CMP_EBUSY, CMP_ETIMEDOUT, CMP_ECANCELED = -5, -6, -7, -8, -9
CMP_COUNT, CMP_SUM, CMP_MAX = 1, 2, 4
CMP_LINEAR, CMP_TILED = 0, 1
CMP_DST_HOST, CMP_DST_DEVICE, CMP_DST_PINNED = 0, 1, 2
OUTPUT_BITS = {"count": CMP_COUNT, "sum": CMP_SUM, "max": CMP_MAX}


# cmp_opts.dev_alloc / dev_free: device allocator hooks.
DEV_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEV_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class cmp_opts(C.Structure):
    _fields_ = [("nbuf", C.c_int32), ("chunk_depth", C.c_int32), ("layout", C.c_int32),
                ("tile_w", C.c_int32), ("tile_h", C.c_int32), ("device", C.c_int32),
                ("copy_stream", C.c_void_p), ("compute_stream", C.c_void_p),
                ("dev_alloc", DEV_ALLOC_FN), ("dev_free", DEV_FREE_FN), ("alloc_ctx", C.c_void_p),
                ("retain_members", C.c_int32), ("debug_poison", C.c_int32),
                ("profile", C.c_int32), ("pageable_host", C.c_int32),
                ("host_paced", C.c_int32), ("verify_members", C.c_int32),
                ("pingpong", C.c_int32), ("copy_streams", C.c_int32)]


class cmp_request(C.Structure):
    _fields_ = [("ids", C.POINTER(C.c_int32)), ("n", C.c_int32), ("x0", C.c_int32),
                ("y0", C.c_int32), ("w", C.c_int32), ("h", C.c_int32),
                ("dev_count", C.c_void_p), ("out_pitch", C.c_int64)]


class cmp_tune(C.Structure):
    _fields_ = [("mode", C.c_int32), ("tile_vecs", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("use_graph", C.c_int32), ("order", C.c_int32), ("stream_loads", C.c_int32),
                ("slots", C.c_int32), ("reserved", C.c_int32 * 1)]


CMP_ORDER_COST, CMP_ORDER_ROWS = 0, 1


CMP_BATCH_PERSISTENT, CMP_BATCH_PER_REQUEST, CMP_BATCH_SHARED, CMP_BATCH_MATRIX = 0, 1, 2, 3
CMP_OP_ADD, CMP_OP_REMOVE = 0, 1


class cmp_server_opts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_sessions", C.c_int32),
                ("max_batch", C.c_int32), ("max_view_pixels", C.c_int32),
                ("tile_vecs", C.c_int32), ("blocks_per_cu", C.c_int32), ("overlap", C.c_int32),
                ("remat_max_members", C.c_int32), ("count_bits", C.c_int32),
                ("oversubscribe_pct", C.c_int32), ("max_queue", C.c_int32),
                ("view_group", C.c_int32), ("reserved", C.c_int32 * 1)]


class cmp_server_stats(C.Structure):
    _fields_ = [("requests", C.c_int64), ("steps", C.c_int64), ("max_step", C.c_int64),
                ("spills", C.c_int64), ("restores", C.c_int64), ("resident_slots", C.c_int64),
                ("device_ms", C.c_double), ("drops", C.c_int64), ("rebuilds", C.c_int64),
                ("refused_sessions", C.c_int64), ("refused_busy", C.c_int64),
                ("queue_peak", C.c_int64), ("wait_ms", C.c_double), ("host_ms", C.c_double),
                ("flight_ms", C.c_double), ("view_ms", C.c_double)]


class cmp_replay_req(C.Structure):
    _fields_ = [("t_ns", C.c_int64), ("sid", C.c_int64), ("ids_off", C.c_int64),
                ("op", C.c_int32), ("n", C.c_int32), ("vx0", C.c_int32), ("vy0", C.c_int32),
                ("vw", C.c_int32), ("vh", C.c_int32)]


class CompositeError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {composite_strerror(status)} ({status})")


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "or python -m paper_2104_14667_amd.build")
    return C.CDLL(LIB_PATH)


lib = _load()

_vp, _i32, _i64, _u32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32
_P = C.POINTER
_SIGS = {
    "composite_default_opts": (None, [_P(cmp_opts)]),
    "composite_init": (C.c_int, [_P(_vp), _i32, _i32, _u32, _i32, _P(cmp_opts)]),
    "composite_clear": (C.c_int, [_vp]),
    "composite_add": (C.c_int, [_vp, _P(_vp), _P(_i64), _i32]),
    "composite_add_device": (C.c_int, [_vp, _P(_vp), _P(_i64), _i32]),
    "composite_remove": (C.c_int, [_vp, _P(_vp), _P(_i64), _i32, _i32]),
    "composite_read": (C.c_int, [_vp, _u32, _i32, _i32, _i32, _i32, _vp, _i64, _i32]),
    "composite_sync": (C.c_int, [_vp]),
    "composite_members": (C.c_int, [_vp, _P(_i64)]),
    "composite_device_buffer": (C.c_int, [_vp, _u32, _P(_vp)]),
    "composite_kernel_stats": (C.c_int, [_vp, _P(_i64), _P(C.c_double), _i32]),
    "composite_pool_create": (C.c_int, [_P(_vp), _vp, _i64, _i32, _i32, _i64, _i64, _i32]),
    "composite_pool_free": (None, [_vp]),
    "composite_default_tune": (None, [_P(cmp_tune)]),
    "composite_batch_run": (C.c_int, [_vp, _P(cmp_request), _i32, _P(cmp_tune)]),
    "composite_batch_last": (C.c_int, [_vp, _P(C.c_double), _P(_i64), _P(_i32)]),
    "composite_default_server_opts": (None, [_P(cmp_server_opts)]),
    "composite_server_create": (C.c_int, [_P(_vp), _vp, _P(cmp_server_opts)]),
    "composite_server_free": (None, [_vp]),
    "composite_session_open": (C.c_int, [_vp, _P(_i64)]),
    "composite_session_close": (C.c_int, [_vp, _i64]),
    "composite_session_submit": (C.c_int, [_vp, _i64, _i32, _P(_i32), _i32, _i32, _i32, _i32,
                                           _i32, _vp, _i64, _P(C.c_uint64)]),
    "composite_session_wait": (C.c_int, [_vp, C.c_uint64, _i64, _P(_i64), _P(_i64)]),
    "composite_server_stats": (C.c_int, [_vp, _P(cmp_server_stats)]),
    "composite_server_replay": (C.c_int, [_vp, _P(cmp_replay_req), _i64, _P(_i32), _P(_vp),
                                          _i32, _i64, _P(_i64), _P(_i32)]),
    "composite_server_pause": (C.c_int, [_vp, _i32]),
    "composite_histogram": (C.c_int, [_vp, _P(_i64), _i32, _P(_i64)]),
    "composite_repack_tiled": (C.c_int, [_vp, _i64, _vp, _i64, _i32, _i32, _i32, _i32, _i32, _vp]),
    "composite_tiled_bytes": (C.c_int64, [_i32, _i32, _i32, _i32]),
    "composite_accumulate_static": (C.c_int, [_P(_vp), _i32, _i32, _i32, _u32, _i32, _vp, _vp, _vp,
                                              _i32, _vp]),
    "composite_strerror": (C.c_char_p, [C.c_int]),
    "composite_free": (None, [_vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def header_functions(path: str = HEADER) -> list:
    """Names of the functions include/composite.h declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(composite_\w+)\s*\(", text)))


def composite_strerror(status: int) -> str:
    return lib.composite_strerror(int(status)).decode()


def _check(rc: int, what: str) -> None:
    if rc != CMP_OK:
        raise CompositeError(rc, what)


def composite_default_opts() -> cmp_opts:
    o = cmp_opts()
    lib.composite_default_opts(C.byref(o))
    return o


def _ptr(x) -> int:
    """Address of a torch tensor, numpy array or integer."""
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    if isinstance(x, np.ndarray):
        return int(x.ctypes.data)
    raise TypeError(f"cannot take the address of {type(x)}")


def _ptr_array(maps) -> C.Array:
    return (C.c_void_p * len(maps))(*[_ptr(m) for m in maps])


def _ids_array(ids, n):
    if ids is None:
        return None
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.int64))
    if ids.size != n:
        raise ValueError("one id per map")
    return (C.c_int64 * n)(*ids.tolist())


def composite_init(W: int, H: int, outputs: int, count_bits: int = 32,
                   opts: Optional[cmp_opts] = None) -> int:
    h = C.c_void_p()
    _check(lib.composite_init(C.byref(h), int(W), int(H), int(outputs), int(count_bits),
                              C.byref(opts) if opts is not None else None), "composite_init")
    return h.value


def composite_clear(ctx: int) -> None:
    _check(lib.composite_clear(ctx), "composite_clear")


def composite_add(ctx: int, host_maps: Sequence, ids=None) -> None:
    n = len(host_maps)
    _check(lib.composite_add(ctx, _ptr_array(host_maps), _ids_array(ids, n), n), "composite_add")


def composite_add_device(ctx: int, dev_maps: Sequence, ids=None) -> None:
    n = len(dev_maps)
    _check(lib.composite_add_device(ctx, _ptr_array(dev_maps), _ids_array(ids, n), n),
           "composite_add_device")


def composite_remove(ctx: int, maps: Optional[Sequence], ids=None, n: Optional[int] = None,
                     maps_on_device: bool = False) -> None:
    if maps is not None:
        n = len(maps)
    elif n is None:
        n = len(ids)
    arr = _ptr_array(maps) if maps is not None else None
    _check(lib.composite_remove(ctx, arr, _ids_array(ids, n), n, int(bool(maps_on_device))),
           "composite_remove")


def composite_read(ctx: int, which: int, x0: int, y0: int, w: int, h: int, dst,
                   dst_pitch_bytes: int, dst_kind: int = CMP_DST_HOST) -> None:
    _check(lib.composite_read(ctx, int(which), int(x0), int(y0), int(w), int(h), _ptr(dst),
                              int(dst_pitch_bytes), int(dst_kind)), "composite_read")


def composite_sync(ctx: int) -> None:
    _check(lib.composite_sync(ctx), "composite_sync")


def composite_members(ctx: int) -> int:
    n = C.c_int64()
    _check(lib.composite_members(ctx, C.byref(n)), "composite_members")
    return n.value


def composite_device_buffer(ctx: int, which: int) -> int:
    p = C.c_void_p()
    _check(lib.composite_device_buffer(ctx, int(which), C.byref(p)), "composite_device_buffer")
    return p.value


def composite_kernel_stats(ctx: int, reset: bool = False):
    n = C.c_int64()
    ms = C.c_double()
    _check(lib.composite_kernel_stats(ctx, C.byref(n), C.byref(ms), int(bool(reset))),
           "composite_kernel_stats")
    return n.value, ms.value


def composite_histogram(ctx: int, nbins: int):
    bins = np.zeros(int(nbins), dtype=np.int64)
    over = C.c_int64()
    _check(lib.composite_histogram(ctx, bins.ctypes.data_as(C.POINTER(C.c_int64)), int(nbins),
                                   C.byref(over)), "composite_histogram")
    return bins, over.value


def composite_tiled_bytes(W: int, H: int, tile_w: int, tile_h: int) -> int:
    return int(lib.composite_tiled_bytes(int(W), int(H), int(tile_w), int(tile_h)))


def composite_repack_tiled(src, src_stride: int, dst, dst_stride: int, n: int, W: int, H: int,
                           tile_w: int, tile_h: int, stream=None) -> None:
    st = None if stream is None else (stream if isinstance(stream, int) else int(stream.cuda_stream))
    _check(lib.composite_repack_tiled(_ptr(src), int(src_stride), _ptr(dst), int(dst_stride),
                                      int(n), int(W), int(H), int(tile_w), int(tile_h), st),
           "composite_repack_tiled")


CMP_STATIC_MAX_MEMBERS = 8192


def composite_accumulate_static(dev_maps: Sequence, W: int, H: int, outputs: int, count_bits: int,
                                dev_count=None, dev_sum=None, dev_max=None, set: bool = True,
                                stream=None) -> int:
    """Returns the status (no raise): callers check refusals by code."""
    st = None if stream is None else (stream if isinstance(stream, int) else int(stream.cuda_stream))
    n = len(dev_maps)
    arr = _ptr_array(dev_maps) if n else None
    return int(lib.composite_accumulate_static(
        arr, n, int(W), int(H), int(outputs), int(count_bits),
        None if dev_count is None else _ptr(dev_count), None if dev_sum is None else _ptr(dev_sum),
        None if dev_max is None else _ptr(dev_max), 1 if set else 0, st))


def composite_free(ctx: int) -> None:
    lib.composite_free(ctx)


_DT = {CMP_SUM: np.uint32, CMP_MAX: np.uint8}


def torch_allocator(device: int = 0):
    """(alloc, free) over torch's caching allocator, for Composite(allocator=...).
    Blocks are associated with torch's current stream of `device`; the library
    frees them only once its own streams no longer use them."""
    import torch

    def alloc(nbytes: int) -> int:
        return int(torch.cuda.caching_allocator_alloc(int(nbytes), device))

    def free(ptr: int) -> None:
        torch.cuda.caching_allocator_delete(int(ptr))

    return alloc, free


class Composite:
    """One compositing context (owner of a device composite).

    allocator: None (hipMalloc), "torch" (torch's caching allocator), or a pair
    of callables alloc(nbytes) -> device address and free(address)."""

    def __init__(self, W: int, H: int, outputs=("count",), count_bits: int = 32, allocator=None,
                 **opts):
        self.W, self.H = int(W), int(H)
        self.outputs = tuple(outputs)
        self.count_bits = int(count_bits)
        o = composite_default_opts()
        if allocator is not None:
            a, f = torch_allocator(int(opts.get("device", 0))) if allocator == "torch" else allocator
            # the callbacks must outlive the context
            self._hooks = (DEV_ALLOC_FN(lambda n, _ctx: a(n) or None),
                           DEV_FREE_FN(lambda ptr, _ctx: f(ptr)))
            o.dev_alloc, o.dev_free = self._hooks
        fields = {f[0] for f in cmp_opts._fields_}
        for k, v in opts.items():
            if k not in fields or k in ("reserved", "dev_alloc", "dev_free", "alloc_ctx"):
                raise TypeError(f"unknown option {k!r}")
            if k in ("copy_stream", "compute_stream") and v is not None and not isinstance(v, int):
                v = int(v.cuda_stream)          # torch.cuda.Stream
            setattr(o, k, v)
        self.opts = o
        bits = 0
        for name in self.outputs:
            bits |= OUTPUT_BITS[name]
        self.ctx = composite_init(W, H, bits, count_bits, o)

    def close(self) -> None:
        if self.ctx:
            composite_free(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clear(self):
        composite_clear(self.ctx)

    def add(self, host_maps, ids=None):
        composite_add(self.ctx, host_maps, ids)

    def add_device(self, dev_maps, ids=None):
        composite_add_device(self.ctx, dev_maps, ids)

    def remove(self, maps=None, ids=None, on_device=False):
        composite_remove(self.ctx, maps, ids, None, on_device)

    def sync(self):
        composite_sync(self.ctx)

    def members(self) -> int:
        return composite_members(self.ctx)

    def kernel_stats(self, reset=False):
        return composite_kernel_stats(self.ctx, reset)

    def dtype(self, name: str):
        if name == "count":
            return np.uint16 if self.count_bits == 16 else np.uint32
        return _DT[OUTPUT_BITS[name]]

    def read(self, name: str, window=None, out: Optional[np.ndarray] = None,
             pinned: bool = False) -> np.ndarray:
        """Window (x0, y0, w, h) of one output into host memory (numpy); pass
        pinned=True when `out` views page-locked memory."""
        x0, y0, w, h = window if window is not None else (0, 0, self.W, self.H)
        dt = self.dtype(name)
        if out is None:
            out = np.empty((h, w), dtype=dt)
        if out.dtype != dt or out.shape != (h, w) or not out.flags.c_contiguous:
            raise ValueError("out must be a C-contiguous (h, w) array of the output's dtype")
        composite_read(self.ctx, OUTPUT_BITS[name], x0, y0, w, h, out, w * out.itemsize,
                       CMP_DST_PINNED if pinned else CMP_DST_HOST)
        return out

    def read_device(self, name: str, dst, window=None, pitch_bytes: Optional[int] = None):
        """Window of one output into device memory (a torch tensor or address)."""
        x0, y0, w, h = window if window is not None else (0, 0, self.W, self.H)
        eb = np.dtype(self.dtype(name)).itemsize
        composite_read(self.ctx, OUTPUT_BITS[name], x0, y0, w, h, dst,
                       pitch_bytes if pitch_bytes is not None else w * eb, CMP_DST_DEVICE)

    def device_buffer(self, name: str) -> int:
        return composite_device_buffer(self.ctx, OUTPUT_BITS[name])

    def histogram(self, nbins: int):
        """(bins[nbins] of overlap classes, pixels with count >= nbins)."""
        return composite_histogram(self.ctx, nbins)


# ---------------------------------------------------------------- batched pool

def composite_default_tune() -> cmp_tune:
    t = cmp_tune()
    lib.composite_default_tune(C.byref(t))
    return t


def composite_pool_create(dev_base, count: int, W: int, H: int, stride_bytes: int,
                          pool_bytes: int, device: int = 0) -> int:
    h = C.c_void_p()
    _check(lib.composite_pool_create(C.byref(h), _ptr(dev_base), int(count), int(W), int(H),
                                     int(stride_bytes), int(pool_bytes), int(device)),
           "composite_pool_create")
    return h.value


def composite_pool_free(pool: int) -> None:
    lib.composite_pool_free(pool)


def make_requests(requests) -> tuple:
    """ctypes array of cmp_request from dicts with ids, x0, y0, w, h, out (a
    device tensor or address) and optional pitch (elements).  Returns the array
    and the id buffers it points into (keep both alive)."""
    arr = (cmp_request * len(requests))()
    keep = []
    for i, r in enumerate(requests):
        ids = np.ascontiguousarray(np.asarray(r["ids"], dtype=np.int32))
        keep.append(ids)
        arr[i].ids = ids.ctypes.data_as(C.POINTER(C.c_int32)) if ids.size else None
        arr[i].n = ids.size
        arr[i].x0, arr[i].y0, arr[i].w, arr[i].h = int(r["x0"]), int(r["y0"]), int(r["w"]), int(r["h"])
        arr[i].dev_count = _ptr(r["out"])
        arr[i].out_pitch = int(r.get("pitch", r["w"]))
    return arr, keep


def composite_batch_run(pool: int, requests, tune: Optional[cmp_tune] = None) -> None:
    arr, keep = make_requests(requests)
    _check(lib.composite_batch_run(pool, arr, len(requests),
                                   C.byref(tune) if tune is not None else None),
           "composite_batch_run")
    del keep


def composite_batch_last(pool: int):
    """(device ms, work items, mode that ran) of the last batch."""
    ms = C.c_double()
    items = C.c_int64()
    mode = C.c_int32()
    _check(lib.composite_batch_last(pool, C.byref(ms), C.byref(items), C.byref(mode)),
           "composite_batch_last")
    return ms.value, items.value, mode.value


def make_tune(mode=CMP_BATCH_PERSISTENT, tile_vecs=1024, blocks_per_cu=8, use_graph=1,
              order=CMP_ORDER_ROWS, stream_loads=0, slots=0) -> cmp_tune:
    t = composite_default_tune()
    t.mode, t.tile_vecs, t.blocks_per_cu, t.use_graph = mode, tile_vecs, blocks_per_cu, use_graph
    t.order, t.stream_loads, t.slots = order, stream_loads, slots
    return t


class Pool:
    """Device-resident pool of rasters for batched crop requests."""

    def __init__(self, dev_base, count: int, W: int, H: int, stride_bytes: int,
                 pool_bytes: int, device: int = 0):
        self.count, self.W, self.H = int(count), int(W), int(H)
        self.handle = composite_pool_create(dev_base, count, W, H, stride_bytes, pool_bytes, device)

    def run(self, requests, tune: Optional[cmp_tune] = None) -> None:
        composite_batch_run(self.handle, requests, tune)

    def last(self):
        return composite_batch_last(self.handle)

    def close(self):
        if self.handle:
            composite_pool_free(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- served sessions

def composite_default_server_opts() -> cmp_server_opts:
    o = cmp_server_opts()
    lib.composite_default_server_opts(C.byref(o))
    return o


class Server:
    """Continuous-batching server of add/remove/viewport requests over a pool."""

    def __init__(self, pool: Pool, **opts):
        o = composite_default_server_opts()
        fields = {f[0] for f in cmp_server_opts._fields_}
        for k, v in opts.items():
            if k not in fields or k == "reserved":
                raise TypeError(f"unknown server option {k!r}")
            setattr(o, k, v)
        self.opts = o
        self.pool = pool
        h = C.c_void_p()
        _check(lib.composite_server_create(C.byref(h), pool.handle, C.byref(o)),
               "composite_server_create")
        self.handle = h.value

    @property
    def count_dtype(self):
        """numpy dtype of the returned viewport counts: the session
        composites' width (uint16 with count_bits = 16, else uint32)."""
        return np.uint16 if self.opts.count_bits == 16 else np.uint32

    def open(self) -> int:
        sid = C.c_int64()
        _check(lib.composite_session_open(self.handle, C.byref(sid)), "composite_session_open")
        return sid.value

    def try_open(self) -> Optional[int]:
        """A session id, or None when admission refuses it (CMP_ENOMEM)."""
        sid = C.c_int64()
        rc = lib.composite_session_open(self.handle, C.byref(sid))
        if rc == CMP_ENOMEM:
            return None
        _check(rc, "composite_session_open")
        return sid.value

    def pause(self, paused: bool = True) -> None:
        _check(lib.composite_server_pause(self.handle, int(bool(paused))), "composite_server_pause")

    def close_session(self, sid: int) -> None:
        _check(lib.composite_session_close(self.handle, int(sid)), "composite_session_close")

    def submit(self, sid: int, op: int, ids, viewport, dst, pitch: Optional[int] = None) -> int:
        """dst: page-locked host memory (a pinned torch tensor or its address)
        of counts of the width count_dtype gives."""
        ids = np.ascontiguousarray(np.asarray(ids, dtype=np.int32))
        vx0, vy0, vw, vh = viewport
        t = C.c_uint64()
        _check(lib.composite_session_submit(
            self.handle, int(sid), int(op),
            ids.ctypes.data_as(C.POINTER(C.c_int32)) if ids.size else None, int(ids.size),
            int(vx0), int(vy0), int(vw), int(vh), _ptr(dst),
            int(pitch if pitch is not None else vw), C.byref(t)), "composite_session_submit")
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1):
        ts, td = C.c_int64(), C.c_int64()
        _check(lib.composite_session_wait(self.handle, C.c_uint64(ticket), int(timeout_us),
                                          C.byref(ts), C.byref(td)), "composite_session_wait")
        return ts.value, td.value

    def stats(self) -> dict:
        st = cmp_server_stats()
        _check(lib.composite_server_stats(self.handle, C.byref(st)), "composite_server_stats")
        return {k: getattr(st, k) for k, _ in cmp_server_stats._fields_}

    def replay(self, schedule, sid_of, dst_ring, pitch: int, with_status: bool = False):
        """Open-loop replay of requests (dicts t, sid, op, ids, vx0, vy0, vw, vh,
        as made by synth.ServeWorkload.schedule); sid_of maps the schedule's
        session index to a server session id.  Returns latency in ns per
        request (completion time minus scheduled arrival, -1 if it did not
        complete); with_status, also each request's status (refused requests
        are recorded and the replay goes on)."""
        n = len(schedule)
        reqs = (cmp_replay_req * n)()
        ids_all = []
        off = 0
        for i, r in enumerate(schedule):
            q = reqs[i]
            q.t_ns = int(round(r["t"] * 1e9))
            q.sid = int(sid_of[r["sid"]])
            q.op = CMP_OP_ADD if r["op"] == "add" else CMP_OP_REMOVE
            q.n = len(r["ids"])
            q.ids_off = off
            q.vx0, q.vy0, q.vw, q.vh = int(r["vx0"]), int(r["vy0"]), int(r["vw"]), int(r["vh"])
            ids_all.append(np.asarray(r["ids"], dtype=np.int32))
            off += q.n
        ids = np.ascontiguousarray(np.concatenate(ids_all) if ids_all else np.zeros(1, np.int32))
        ring = (C.c_void_p * len(dst_ring))(*[_ptr(d) for d in dst_ring])
        lat = np.zeros(n, dtype=np.int64)
        status = np.zeros(n, dtype=np.int32)
        rc = lib.composite_server_replay(self.handle, reqs, n, ids.ctypes.data_as(C.POINTER(C.c_int32)),
                                         ring, len(dst_ring), int(pitch),
                                         lat.ctypes.data_as(C.POINTER(C.c_int64)),
                                         status.ctypes.data_as(C.POINTER(C.c_int32))
                                         if with_status else None)
        _check(rc, "composite_server_replay")
        return (lat, status) if with_status else lat

    def close(self):
        if self.handle:
            lib.composite_server_free(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
