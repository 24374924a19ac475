"""The C-ABI library loads and exports what include/composite.h declares (CPU).

No compute calls: this box has no GPU."""

import ctypes as C

import pytest
import torch

from paper_2104_14667_amd import composite as cb


def test_header_declares_the_boundary():
    names = cb.header_functions()
    for must in ("composite_init", "composite_add", "composite_add_device",
                 "composite_remove", "composite_read", "composite_free"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(cb.LIB_PATH)
    missing = [n for n in cb.header_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding wraps every one of them under the same name
    for n in cb.header_functions():
        assert hasattr(cb, n) or n in cb._SIGS, n


def test_strerror_is_total():
    for s in range(-10, 2):
        assert isinstance(cb.composite_strerror(s), str) and cb.composite_strerror(s)
    assert cb.composite_strerror(cb.CMP_ERANGE).startswith("composite value")


def test_default_opts():
    o = cb.composite_default_opts()
    assert (o.nbuf, o.chunk_depth, o.layout, o.tile_w, o.tile_h) == (2, 8, cb.CMP_LINEAR, 64, 64)
    assert o.copy_stream is None and o.compute_stream is None
    assert C.sizeof(cb.cmp_opts) == 96
    assert o.host_paced == 0 and o.pageable_host == 0 and o.verify_members == 0 and o.pingpong == 0


def test_argument_checks_before_any_device_call():
    h = C.c_void_p()
    assert cb.lib.composite_init(None, 4, 4, 1, 32, None) == cb.CMP_EINVAL
    assert cb.lib.composite_init(C.byref(h), 0, 4, 1, 32, None) == cb.CMP_EINVAL
    assert cb.lib.composite_init(C.byref(h), 4, 4, 0, 32, None) == cb.CMP_EINVAL
    assert cb.lib.composite_init(C.byref(h), 4, 4, 8, 32, None) == cb.CMP_EINVAL
    assert cb.lib.composite_init(C.byref(h), 4, 4, 1, 8, None) == cb.CMP_EINVAL
    assert cb.lib.composite_init(C.byref(h), 1 << 20, 1 << 12, 1, 32, None) == cb.CMP_EINVAL
    o = cb.composite_default_opts()
    o.nbuf = 3
    assert cb.lib.composite_init(C.byref(h), 4, 4, 1, 32, C.byref(o)) == cb.CMP_EINVAL
    o = cb.composite_default_opts()
    o.layout = cb.CMP_TILED
    assert cb.lib.composite_init(C.byref(h), 24, 4, 1, 32, C.byref(o)) == cb.CMP_EUNSUPPORTED
    o = cb.composite_default_opts()
    o.copy_streams = 3
    assert cb.lib.composite_init(C.byref(h), 16, 4, 1, 32, C.byref(o)) == cb.CMP_EINVAL
    o = cb.composite_default_opts()
    o.copy_streams, o.nbuf = 2, 1                           # two copy streams need two slots
    assert cb.lib.composite_init(C.byref(h), 16, 4, 1, 32, C.byref(o)) == cb.CMP_EINVAL
    o = cb.composite_default_opts()
    o.pingpong = 2
    assert cb.lib.composite_init(C.byref(h), 16, 4, 1, 32, C.byref(o)) == cb.CMP_EINVAL
    o = cb.composite_default_opts()
    o.dev_alloc = cb.DEV_ALLOC_FN(lambda n, ctx: None)        # without dev_free
    assert cb.lib.composite_init(C.byref(h), 16, 4, 1, 32, C.byref(o)) == cb.CMP_EINVAL
    o = cb.composite_default_opts()
    o.verify_members = 2
    assert cb.lib.composite_init(C.byref(h), 16, 4, 1, 32, C.byref(o)) == cb.CMP_EINVAL
    with pytest.raises(TypeError):
        cb.Composite(16, 4, ("count",), 32, verify_member=1)    # misspelt option
    for fn in ("composite_clear", "composite_sync"):
        assert getattr(cb.lib, fn)(None) == cb.CMP_EINVAL
    cb.lib.composite_free(None)   # NULL-safe


@pytest.mark.skipif(torch.cuda.device_count() > 0, reason="a GPU is present")
def test_init_without_gpu_reports_edevice():
    h = C.c_void_p()
    assert cb.lib.composite_init(C.byref(h), 16, 16, 1, 32, None) == cb.CMP_EDEVICE
    assert h.value is None


def test_pool_and_batch_argument_checks():
    h = C.c_void_p()
    assert cb.lib.composite_pool_create(None, 1, 1, 4, 4, 16, 32, 0) == cb.CMP_EINVAL
    assert cb.lib.composite_pool_create(C.byref(h), None, 1, 4, 4, 16, 32, 0) == cb.CMP_EINVAL
    assert cb.lib.composite_pool_create(C.byref(h), 4096, 2, 4, 4, 16, 40, 0) == cb.CMP_EINVAL
    assert cb.lib.composite_pool_create(C.byref(h), 4096, 2, 4, 4, 8, 64, 0) == cb.CMP_EINVAL
    assert cb.lib.composite_batch_run(None, None, 0, None) == cb.CMP_EINVAL
    t = cb.composite_default_tune()
    assert (t.mode, t.tile_vecs, t.blocks_per_cu, t.use_graph) == (cb.CMP_BATCH_MATRIX, 1024, 4, 1)
    assert (t.order, t.stream_loads, t.slots) == (cb.CMP_ORDER_ROWS, 1, 24)
    assert C.sizeof(cb.cmp_request) == 48 and C.sizeof(cb.cmp_tune) == 32
    cb.lib.composite_pool_free(None)


@pytest.mark.skipif(torch.cuda.device_count() > 0, reason="a GPU is present")
def test_pool_without_gpu_reports_edevice():
    h = C.c_void_p()
    assert cb.lib.composite_pool_create(C.byref(h), 4096, 2, 4, 4, 16, 64, 0) == cb.CMP_EDEVICE


def test_tiled_bytes_and_repack_argument_checks():
    assert cb.composite_tiled_bytes(64, 64, 64, 64) == 4096
    assert cb.composite_tiled_bytes(65, 1, 64, 64) == 2 * 64 * 64
    assert cb.composite_tiled_bytes(4096, 9, 128, 4) == 32 * 3 * 128 * 4
    assert cb.lib.composite_tiled_bytes(0, 1, 16, 1) == -1
    assert cb.lib.composite_repack_tiled(None, 16, 4096, 16, 1, 16, 1, 16, 1, None) == cb.CMP_EINVAL
    assert cb.lib.composite_repack_tiled(4096, 16, 8192, 16, 1, 16, 1, 24, 1, None) == cb.CMP_EINVAL
    assert cb.lib.composite_repack_tiled(4096, 24, 8192, 16, 1, 24, 1, 16, 1, None) == cb.CMP_EINVAL
    assert cb.lib.composite_repack_tiled(4096, 8, 8192, 16, 1, 16, 1, 16, 1, None) == cb.CMP_EINVAL
    assert cb.lib.composite_repack_tiled(4096, 16, 8192, 16, 0, 16, 1, 16, 1, None) == cb.CMP_OK
    assert cb.lib.composite_histogram(None, None, 4, None) == cb.CMP_EINVAL


def test_server_opts_and_stats_layout():
    o = cb.composite_default_server_opts()
    assert C.sizeof(cb.cmp_server_opts) == 56 and C.sizeof(cb.cmp_server_stats) == 128
    assert (o.max_batch, o.tile_vecs, o.blocks_per_cu, o.overlap) == (64, 256, 0, 1)
    assert o.remat_max_members == 2048 and o.hbm_budget_bytes == 16 << 30
    assert (o.count_bits, o.oversubscribe_pct, o.max_queue) == (32, 0, 1024)
    assert cb.lib.composite_server_create(None, None, None) == cb.CMP_EINVAL
    h = C.c_void_p()
    assert cb.lib.composite_server_create(C.byref(h), None, C.byref(o)) == cb.CMP_EINVAL


def test_server_argument_checks_before_any_device_call():
    """Options are checked before the pool is touched, and every served call
    refuses a NULL server or bad arguments without side effects."""
    h = C.c_void_p(1234)
    fake_pool = C.c_void_p(8)          # never dereferenced: the options fail first
    for field, bad in (("count_bits", 24), ("count_bits", 0), ("oversubscribe_pct", -1),
                       ("max_queue", 0), ("max_batch", 0), ("max_batch", 4097),
                       ("hbm_budget_bytes", 0), ("overlap", 2), ("remat_max_members", 65536),
                       ("tile_vecs", 63), ("blocks_per_cu", 17), ("view_group", -1), ("view_group", 65)):
        o = cb.composite_default_server_opts()
        setattr(o, field, bad)
        assert cb.lib.composite_server_create(C.byref(h), fake_pool, C.byref(o)) == cb.CMP_EINVAL, field
        assert h.value is None
        h = C.c_void_p(1234)
    o = cb.composite_default_server_opts()
    o.reserved[0] = 1
    assert cb.lib.composite_server_create(C.byref(h), fake_pool, C.byref(o)) == cb.CMP_EINVAL
    sid = C.c_int64()
    t = C.c_uint64()
    assert cb.lib.composite_session_open(None, C.byref(sid)) == cb.CMP_EINVAL
    assert cb.lib.composite_session_close(None, 1) == cb.CMP_EINVAL
    assert cb.lib.composite_session_submit(None, 1, 0, None, 0, 0, 0, 1, 1, None, 1,
                                           C.byref(t)) == cb.CMP_EINVAL
    assert cb.lib.composite_session_wait(None, 1, 0, None, None) == cb.CMP_EINVAL
    assert cb.lib.composite_server_pause(None, 1) == cb.CMP_EINVAL
    assert cb.lib.composite_server_stats(None, None) == cb.CMP_EINVAL
    lat = (C.c_int64 * 1)()
    assert cb.lib.composite_server_replay(None, None, 1, None, None, 1, 16, lat, None) == cb.CMP_EINVAL
    cb.lib.composite_server_free(None)
    assert cb.composite_strerror(cb.CMP_ECANCELED).startswith("not attempted")


def test_ceiling_library_checks_arguments():
    """The benchmark's same-traffic reference kernel (libceiling.so) rejects
    bad arguments before any device call."""
    from paper_2104_14667_amd import ceiling
    lib = C.CDLL(ceiling.LIB_PATH)
    f = lib.traffic_ceiling
    f.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p,
                  C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.POINTER(C.c_float)]
    ms = C.c_float()
    ok = dict(members=16, stride=64, n=2, npix=64, count=16, sum=16, max=16, rmw=1, reps=3)
    bads = [dict(members=None), dict(n=0), dict(npix=40), dict(stride=32), dict(reps=1),
            dict(count=None), dict(npix=1 << 33, stride=1 << 33), dict(rmw=14), dict(rmw=-1)]
    for bad in bads:
        a = dict(ok, **bad)
        rc = f(a["members"], a["stride"], a["n"], a["npix"], a["count"], a["sum"], a["max"],
               a["rmw"], a["reps"], None, C.byref(ms))
        assert rc == 1, bad                                  # hipErrorInvalidValue


def test_tile_read_reference_checks_arguments():
    """The batched kernel's read-pattern reference (libceiling.so) rejects bad
    arguments, a write volume without its buffer among them, before any
    device call."""
    from paper_2104_14667_amd import ceiling
    lib = C.CDLL(ceiling.LIB_PATH)
    f = lib.tile_read_ceiling
    f.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                  C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.POINTER(C.c_float)]
    ms = C.c_float()
    ok = dict(base=16, stride=4096, pitch=64, count=32, W=64, H=4, sink=16, wout=None, wsegs=0,
              blocks=2, reps=3)
    bads = [dict(base=None), dict(sink=None), dict(count=31), dict(W=7), dict(H=0), dict(blocks=0),
            dict(reps=1), dict(stride=0), dict(pitch=63), dict(wsegs=-1), dict(wsegs=2)]
    for bad in bads:
        a = dict(ok, **bad)
        rc = f(a["base"], a["stride"], a["pitch"], a["count"], a["W"], a["H"], a["sink"], a["wout"],
               a["wsegs"], a["blocks"], a["reps"], None, C.byref(ms))
        assert rc == 1, bad                                  # hipErrorInvalidValue
