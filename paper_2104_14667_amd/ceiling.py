"""Binding of libceiling.so, the same-traffic reference kernel used by the
benchmark and the experiments (measurement only; the compositing library
never loads it).

Modes (`rmw`): 0 member reads only; 1 plus a 9 B/px read-modify-write of
uint32 count, uint32 sum and uint8 max; 2 plus a 4 B/px uint32 count
read-modify-write; 3 plus a 2 B/px uint16 count read-modify-write; 4 plus the
9 B/px written without being read; 5 plus the 9 B/px read without being
written."""

from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libceiling.so")


def same_traffic_ceiling(torch, ptr, stride, n, npix, modes=((1, "rmw_ms"), (0, "read_only_ms")),
                         reps=6):
    """Best time in ms, per mode, of the reference kernel over n device rasters
    at ptr + i * stride of npix bytes each."""
    lib = C.CDLL(LIB_PATH)
    lib.traffic_ceiling.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_int64, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                    C.POINTER(C.c_float)]
    cnt = torch.zeros(npix, dtype=torch.int32, device="cuda:0")
    sm = torch.zeros(npix, dtype=torch.int32, device="cuda:0")
    mx = torch.zeros(npix, dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    out = {}
    for rmw, name in modes:
        ms = C.c_float()
        rc = lib.traffic_ceiling(ptr, stride, n, npix, cnt.data_ptr(), sm.data_ptr(),
                                 mx.data_ptr(), rmw, reps, torch.cuda.current_stream().cuda_stream,
                                 C.byref(ms))
        if rc != 0:
            raise RuntimeError(f"traffic_ceiling failed: hip error {rc}")
        out[name] = ms.value
    del cnt, sm, mx
    return out


def tile_read_ceiling(torch, ptr, stride, pitch, count, W, H, blocks, reps=6, write_segments=0):
    """Best time in ms of the batched matrix kernel's read pattern with trivial
    arithmetic over a pool of count rasters, raster k's row y at
    ptr + k * stride + y * pitch; with write_segments > 0 each 512-pixel tile
    also writes that many 2 KiB pieces of u32 (the batch's output volume)."""
    lib = C.CDLL(LIB_PATH)
    lib.tile_read_ceiling.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int32, C.c_int32,
                                      C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                      C.c_int32, C.c_void_p, C.POINTER(C.c_float)]
    ntiles = H * ((W + 511) // 512)
    sink = torch.empty(ntiles * 256, dtype=torch.int32, device="cuda:0")
    wout = (torch.empty(ntiles * write_segments * 512, dtype=torch.int32, device="cuda:0")
            if write_segments > 0 else None)
    torch.cuda.synchronize()
    ms = C.c_float()
    rc = lib.tile_read_ceiling(ptr, stride, pitch, count, W, H, sink.data_ptr(),
                               wout.data_ptr() if wout is not None else None, int(write_segments),
                               blocks, reps, torch.cuda.current_stream().cuda_stream, C.byref(ms))
    if rc != 0:
        raise RuntimeError(f"tile_read_ceiling failed: hip error {rc}")
    return ms.value


def two_phase_ceiling(torch, ptr, stride, n, npix, V, blocks_per_cu, reps=6):
    """Best time in ms of the two-phase reference (reads of a band by the whole
    grid, a grid-wide barrier, the band's writes, a barrier) over n device
    rasters at ptr + i * stride of npix bytes each."""
    lib = C.CDLL(LIB_PATH)
    lib.two_phase_ceiling.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_int64, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                      C.c_int32, C.c_void_p, C.POINTER(C.c_float)]
    cnt = torch.zeros(npix, dtype=torch.int32, device="cuda:0")
    sm = torch.zeros(npix, dtype=torch.int32, device="cuda:0")
    mx = torch.zeros(npix, dtype=torch.uint8, device="cuda:0")
    scratch = torch.zeros(2, dtype=torch.int32, device="cuda:0")
    torch.cuda.synchronize()
    ms = C.c_float()
    rc = lib.two_phase_ceiling(ptr, stride, n, npix, cnt.data_ptr(), sm.data_ptr(), mx.data_ptr(), V,
                               blocks_per_cu, scratch.data_ptr(), reps,
                               torch.cuda.current_stream().cuda_stream, C.byref(ms))
    if rc != 0:
        raise RuntimeError(f"two_phase_ceiling failed: {rc}")
    return ms.value
