"""Python binding of the C ABI in include/gxbpf.h (ctypes; argument marshalling
only).  Device buffers are torch tensors; streams are torch CUDA/HIP streams.
Every step of the path runs in libgxbpf.so: there is no fallback, and
importing this module without the built library raises."""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgxbpf.so")

MAP_HASH, MAP_ARRAY, MAP_RINGBUF = 1, 2, 27
F_SHARED, F_READ_ONLY = 1, 2
HOOK_MEM_ACCESS, HOOK_KERNEL_TIMING, HOOK_WAVE_MEM, HOOK_SIMT_MEM, HOOK_SCHED = 1, 2, 3, 4, 5
MODE_EVENT_PARALLEL, MODE_STREAM_SEQUENTIAL = 0, 1
RECORD_SIZE = {HOOK_MEM_ACCESS: 24, HOOK_KERNEL_TIMING: 16, HOOK_WAVE_MEM: 24, HOOK_SIMT_MEM: 24, HOOK_SCHED: 32}


class GxError(OSError):
    pass


class ProgInfo(C.Structure):
    _fields_ = [("mode", C.c_uint32), ("hook", C.c_uint32), ("n_insns", C.c_uint32),
                ("stack_bytes", C.c_uint32), ("max_insns", C.c_uint64), ("max_calls", C.c_uint64),
                ("max_ring_bytes", C.c_uint64)]


class Stats(C.Structure):
    _fields_ = [("launches", C.c_uint64), ("events", C.c_uint64), ("ring_drops", C.c_uint64),
                ("hash_e2big", C.c_uint64), ("vm_errors", C.c_uint64), ("bytes_drained", C.c_uint64)]


class Batch(C.Structure):
    _fields_ = [("prog_fd", C.c_int32), ("record_size", C.c_uint32), ("d_events", C.c_void_p),
                ("n_events", C.c_uint64), ("d_rc", C.c_void_p)]


EXPORTS = ["gx_open", "gx_close", "gx_create_map", "gx_map_update", "gx_map_lookup", "gx_map_delete",
           "gx_map_dump", "gx_map_clear", "gx_load_program", "gx_prog_info_get", "gx_verify", "gx_run_batch", "gx_run_batch_noalloc", "gx_run_app_vadd", "gx_run_sched",
           "gx_run_batches", "gx_autotune_batches", "gx_drain_ringbuf_view", "gx_drain_ringbuf_start", "gx_drain_ringbuf_finish", "gx_graph_create", "gx_graph_launch", "gx_graph_destroy", "gx_autotune", "gx_jit_program", "gx_jit_program_set", "gx_jit_source",
           "gx_jit_set_source", "gx_drain_ringbuf", "gx_ringbuf_pos", "gx_snapshot_start", "gx_snapshot_read",
           "gx_snapshot_flush", "gx_snapshot_stop", "gx_stats_get", "gx_profile_enable", "gx_profile_read",
           "gx_server_create", "gx_server_submit", "gx_server_submit_borrowed", "gx_server_poll",
           "gx_server_release", "gx_server_drain", "gx_server_destroy"]
SERVE_CONTINUOUS, SERVE_PER_REQUEST = 0, 1


class Tune(C.Structure):
    _fields_ = [("lanes", C.c_uint32), ("qbits", C.c_uint32), ("blocks", C.c_uint32), ("trials", C.c_uint32),
                ("best_ms", C.c_double), ("default_ms", C.c_double)]


class ServerCfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("streams", C.c_uint32), ("mode", C.c_uint32),
                ("max_group", C.c_uint32), ("pad", C.c_uint32)]


class Completion(C.Structure):
    _fields_ = [("req_id", C.c_uint64), ("tenant", C.c_int32), ("status", C.c_int32), ("n_events", C.c_uint64),
                ("rc", C.POINTER(C.c_uint32)), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("priv", C.c_void_p)]

_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run paper_2512_12615_amd/build.py "
                           "(or __graft_entry__.build()) first")
    # Share torch's HIP runtime: torch loads its own libamdhip64 at import, and
    # our library's libamdhip64.so.7 dependency then binds to that copy
    # instead of loading a second runtime into the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, u32, u64, i64 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int64
    L.gx_open.argtypes = [C.c_int, C.POINTER(vp)]
    L.gx_close.argtypes = [vp]
    L.gx_close.restype = None
    L.gx_create_map.argtypes = [vp, u32, u32, u32, u32, u32]
    L.gx_map_update.argtypes = [vp, C.c_int, vp, vp, u64]
    L.gx_map_lookup.argtypes = [vp, C.c_int, vp, vp]
    L.gx_map_delete.argtypes = [vp, C.c_int, vp]
    L.gx_map_dump.argtypes = [vp, C.c_int, vp, vp, u64]
    L.gx_map_dump.restype = i64
    L.gx_map_clear.argtypes = [vp, C.c_int]
    L.gx_load_program.argtypes = [vp, vp, u32, u32, vp, u32, C.c_char_p, u32]
    L.gx_prog_info_get.argtypes = [vp, C.c_int, C.POINTER(ProgInfo)]
    L.gx_verify.argtypes = [vp, u32, u32, vp, u32, C.c_char_p, u32, C.POINTER(ProgInfo)]
    L.gx_run_batch.argtypes = [vp, C.c_int, vp, u64, u32, vp, vp]
    L.gx_run_batch_noalloc.argtypes = [vp, C.c_int, vp, u64, u32, vp, vp]
    L.gx_run_app_vadd.argtypes = [vp, C.c_int, vp, vp, vp, u64, u64, vp, vp]
    L.gx_run_sched.argtypes = [vp, C.c_int, vp, u32, u32, vp, vp, vp, u32, vp, vp]
    L.gx_run_batches.argtypes = [vp, C.POINTER(Batch), u32, vp]
    L.gx_autotune.argtypes = [vp, C.c_int, vp, u64, u32, vp, vp, C.POINTER(Tune)]
    L.gx_graph_create.argtypes = [vp, C.POINTER(Batch), u32, C.POINTER(vp)]
    L.gx_autotune_batches.argtypes = [vp, C.POINTER(Batch), u32, vp, C.POINTER(Tune)]
    L.gx_drain_ringbuf_view.argtypes = [vp, C.c_int, C.POINTER(vp), C.POINTER(u64), C.POINTER(u64)]
    L.gx_drain_ringbuf_view.restype = C.c_int64
    L.gx_drain_ringbuf_start.argtypes = [vp, C.c_int]
    L.gx_drain_ringbuf_start.restype = C.c_int
    L.gx_drain_ringbuf_finish.argtypes = [vp, C.c_int, C.POINTER(vp), C.POINTER(u64), C.POINTER(u64)]
    L.gx_drain_ringbuf_finish.restype = C.c_int64
    L.gx_graph_launch.argtypes = [vp, vp]
    L.gx_graph_destroy.argtypes = [vp]
    L.gx_graph_destroy.restype = None
    L.gx_jit_program.argtypes = [vp, C.c_int, C.c_char_p, u32]
    L.gx_jit_program_set.argtypes = [vp, vp, u32, C.c_char_p, u32]
    L.gx_jit_source.argtypes = [vp, u32, u32, vp, u32, C.c_int, C.c_char_p, u64]
    L.gx_jit_source.restype = i64
    L.gx_jit_set_source.argtypes = [vp, vp, vp, vp, vp, u32, C.c_int, C.c_char_p, u64]
    L.gx_jit_set_source.restype = i64
    L.gx_drain_ringbuf.argtypes = [vp, C.c_int, vp, u64, C.POINTER(u64)]
    L.gx_drain_ringbuf.restype = i64
    L.gx_ringbuf_pos.argtypes = [vp, C.c_int, C.POINTER(u64), C.POINTER(u64)]
    L.gx_snapshot_start.argtypes = [vp, vp, u32, u64, vp]
    L.gx_snapshot_read.argtypes = [vp, C.c_int, vp, vp, u64, C.POINTER(u64)]
    L.gx_snapshot_read.restype = i64
    L.gx_snapshot_flush.argtypes = [vp]
    L.gx_snapshot_stop.argtypes = [vp]
    L.gx_snapshot_stop.restype = None
    L.gx_stats_get.argtypes = [vp, C.POINTER(Stats)]
    L.gx_profile_enable.argtypes = [vp, C.c_int]
    L.gx_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(u64)]
    L.gx_server_create.argtypes = [vp, C.POINTER(ServerCfg), C.POINTER(vp)]
    L.gx_server_submit.argtypes = [vp, C.c_int32, C.c_int, vp, u64, u32, u64]
    L.gx_server_submit_borrowed.argtypes = [vp, C.c_int32, C.c_int, vp, u64, u32, u64]
    L.gx_server_poll.argtypes = [vp, C.POINTER(Completion), u32, C.c_int]
    L.gx_server_release.argtypes = [vp, C.POINTER(Completion)]
    L.gx_server_release.restype = None
    L.gx_server_drain.argtypes = [vp]
    L.gx_server_destroy.argtypes = [vp]
    L.gx_server_destroy.restype = None
    _lib = L
    return L


def _check(r, what):
    if r < 0:
        raise GxError(-r, f"{what}: {os.strerror(-r)}")
    return r


def _words(code: bytes) -> np.ndarray:
    if len(code) % 8:
        raise ValueError("bytecode length must be a multiple of 8")
    return np.frombuffer(code, dtype="<u8").copy() if code else np.zeros(1, "<u8")


def verify(code: bytes, hook: int, shapes):
    """Verify without a device.  ``shapes``: (type, key_size, value_size,
    max_entries, flags) per map, in the program's map-table order.
    Returns (ok, log, ProgInfo)."""
    sh = np.array(shapes, dtype=np.uint32).reshape(-1, 5) if shapes else np.zeros((0, 5), np.uint32)
    w = _words(code)
    log = C.create_string_buffer(512)
    info = ProgInfo()
    r = lib().gx_verify(w.ctypes.data_as(C.c_void_p), len(code) // 8, hook, sh.ctypes.data_as(C.c_void_p),
                        len(sh), log, 512, C.byref(info))
    return r == 0, log.value.decode(), info


def jit_source(code: bytes, hook: int, shapes, compile: bool = False, app: bool = False) -> str:
    """HIP source the JIT generates for a program (no device needed); with
    ``compile`` it is also compiled for gfx950; with ``app`` it is the
    instrumented vector add's kernel.  Raises GxError on rejection or
    compile failure (message holds the log)."""
    sh = np.array(shapes, dtype=np.uint32).reshape(-1, 5) if shapes else np.zeros((0, 5), np.uint32)
    w = _words(code)
    cap = 1 << 22
    out = C.create_string_buffer(cap)
    r = lib().gx_jit_source(w.ctypes.data_as(C.c_void_p), len(code) // 8, hook, sh.ctypes.data_as(C.c_void_p),
                            len(sh), int(compile) | (2 if app else 0), out, cap)
    if r < 0:
        raise GxError(-r, f"gx_jit_source: {os.strerror(-r)}: {out.value.decode(errors='replace')}")
    return out.value.decode()


def jit_set_source(programs, compile: bool = False) -> str:
    """Source of a program set; ``programs``: list of (code, hook, shapes)."""
    words = [_words(c) for c, _, _ in programs]
    insns = np.concatenate(words) if words else np.zeros(1, "<u8")
    n_insns = np.array([len(c) // 8 for c, _, _ in programs], np.uint32)
    hooks = np.array([h for _, h, _ in programs], np.uint32)
    shapes = [np.array(sh, np.uint32).reshape(-1, 5) if sh else np.zeros((0, 5), np.uint32) for _, _, sh in programs]
    n_maps = np.array([len(x) for x in shapes], np.uint32)
    flat = np.concatenate([x.reshape(-1) for x in shapes] + [np.zeros(1, np.uint32)])
    cap = 1 << 24
    out = C.create_string_buffer(cap)
    r = lib().gx_jit_set_source(insns.ctypes.data_as(C.c_void_p), n_insns.ctypes.data_as(C.c_void_p),
                                hooks.ctypes.data_as(C.c_void_p), flat.ctypes.data_as(C.c_void_p),
                                n_maps.ctypes.data_as(C.c_void_p), len(programs), int(compile), out, cap)
    if r < 0:
        raise GxError(-r, f"gx_jit_set_source: {os.strerror(-r)}: {out.value.decode(errors='replace')[:4000]}")
    return out.value.decode()


def _dptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


@dataclass
class MapInfo:
    type: int
    key_size: int
    value_size: int
    max_entries: int
    flags: int


class Runtime:
    """One gx_rt on one HIP device."""

    def __init__(self, device: int = 0):
        self._h = C.c_void_p()
        _check(lib().gx_open(device, C.byref(self._h)), "gx_open")
        self.maps: dict[int, MapInfo] = {}
        self._drain_bufs: dict[int, np.ndarray] = {}
        self.device = device

    def close(self):
        if self._h:
            lib().gx_close(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # maps -----------------------------------------------------------------
    def create_map(self, type_, key_size, value_size, max_entries, flags=0) -> int:
        fd = _check(lib().gx_create_map(self._h, type_, key_size, value_size, max_entries, flags), "gx_create_map")
        self.maps[fd] = MapInfo(type_, key_size, value_size, max_entries, flags)
        return fd

    def map_update(self, fd, key: bytes, val: bytes, flags=0) -> int:
        return lib().gx_map_update(self._h, fd, C.c_char_p(bytes(key)), C.c_char_p(bytes(val)), flags)

    def map_lookup(self, fd, key: bytes):
        buf = C.create_string_buffer(self.maps[fd].value_size)
        r = lib().gx_map_lookup(self._h, fd, C.c_char_p(bytes(key)), buf)
        return None if r else buf.raw

    def map_delete(self, fd, key: bytes) -> int:
        return lib().gx_map_delete(self._h, fd, C.c_char_p(bytes(key)))

    def map_clear(self, fd):
        _check(lib().gx_map_clear(self._h, fd), "gx_map_clear")

    def map_dump(self, fd):
        """(keys, values) as uint8 arrays of shape (n, key_size) / (n, value_size)."""
        m = self.maps[fd]
        n = _check(lib().gx_map_dump(self._h, fd, None, None, 0), "gx_map_dump")
        keys = np.zeros((max(n, 1), m.key_size), np.uint8)
        vals = np.zeros((max(n, 1), m.value_size), np.uint8)
        _check(lib().gx_map_dump(self._h, fd, keys.ctypes.data_as(C.c_void_p), vals.ctypes.data_as(C.c_void_p), n),
               "gx_map_dump")
        return keys[:n], vals[:n]

    # programs ---------------------------------------------------------------
    def load_program(self, code: bytes, hook: int, map_fds) -> int:
        w = _words(code)
        fds = np.array(list(map_fds), dtype=np.int32)
        log = C.create_string_buffer(512)
        r = lib().gx_load_program(self._h, w.ctypes.data_as(C.c_void_p), len(code) // 8, hook,
                                  fds.ctypes.data_as(C.c_void_p) if len(fds) else None, len(fds), log, 512)
        if r < 0:
            raise GxError(-r, f"gx_load_program: {os.strerror(-r)}: {log.value.decode()}")
        return r

    def autotune(self, prog_fd, events, n_events=None, record_size=None, rc=None, stream=None) -> dict:
        """Time the candidate launch shapes of a program on a sample batch
        (map contents restored afterwards) and keep the fastest."""
        if record_size is None:
            record_size = RECORD_SIZE[self.prog_info(prog_fd).hook]
        if n_events is None:
            n_events = events.numel() * events.element_size() // record_size
        t = Tune()
        _check(lib().gx_autotune(self._h, prog_fd, _dptr(events), n_events, record_size, _dptr(rc),
                                 _stream_handle(stream), C.byref(t)), "gx_autotune")
        return {k: getattr(t, k) for k, _ in Tune._fields_}

    def jit_program(self, fd):
        """Compile a loaded program to native gfx950 code (later run_batch
        calls of it launch the compiled kernels)."""
        log = C.create_string_buffer(1 << 16)
        r = lib().gx_jit_program(self._h, fd, log, 1 << 16)
        if r < 0:
            raise GxError(-r, f"gx_jit_program: {os.strerror(-r)}: {log.value.decode(errors='replace')}")

    def jit_program_set(self, fds) -> int:
        """Compile several programs into one module whose persistent kernel
        runs all their runs of a batched phase in one launch."""
        arr = np.array(list(fds), dtype=np.int32)
        log = C.create_string_buffer(1 << 16)
        r = lib().gx_jit_program_set(self._h, arr.ctypes.data_as(C.c_void_p), len(arr), log, 1 << 16)
        if r < 0:
            raise GxError(-r, f"gx_jit_program_set: {os.strerror(-r)}: {log.value.decode(errors='replace')}")
        return r

    def prog_info(self, fd) -> ProgInfo:
        info = ProgInfo()
        _check(lib().gx_prog_info_get(self._h, fd, C.byref(info)), "gx_prog_info_get")
        return info

    def run_batch(self, prog_fd, events, n_events=None, record_size=None, rc=None, stream=None):
        """events: uint8 device tensor of records; rc: uint32/int32 device tensor or None."""
        if record_size is None:
            record_size = RECORD_SIZE[self.prog_info(prog_fd).hook]
        if n_events is None:
            n_events = events.numel() * events.element_size() // record_size
        r = lib().gx_run_batch(self._h, prog_fd, _dptr(events), n_events, record_size, _dptr(rc),
                               _stream_handle(stream))
        _check(r, "gx_run_batch")

    def run_batch_noalloc(self, prog_fd, events, n_events=None, record_size=None, rc=None, stream=None):
        """run_batch on the device's fixed scratch array: allocates nothing
        (gx_run_batch_noalloc); calls on one device must not overlap."""
        if record_size is None:
            record_size = RECORD_SIZE[self.prog_info(prog_fd).hook]
        if n_events is None:
            n_events = events.numel() * events.element_size() // record_size
        r = lib().gx_run_batch_noalloc(self._h, prog_fd, _dptr(events), n_events, record_size, _dptr(rc),
                                       _stream_handle(stream))
        _check(r, "gx_run_batch_noalloc")

    def run_app_vadd(self, prog_fd, a, b, c, stride=1, rc=None, stream=None):
        """The instrumented vector add (gx_run_app_vadd): c[j] = a[j] + b[j],
        j = i stride mod n, with prog_fd (or none if < 0) at its load of a[j].
        a, b, c: float64 device tensors of n elements; rc: uint32/int32
        device tensor of n or None."""
        n = a.numel()
        if b.numel() != n or c.numel() != n or a.dtype != b.dtype or a.dtype != c.dtype:
            raise ValueError("a, b and c must hold the same number of doubles")
        if rc is not None and rc.numel() < n:
            raise ValueError("rc holds fewer than n elements")
        r = lib().gx_run_app_vadd(self._h, prog_fd, _dptr(a), _dptr(b), _dptr(c), n, stride, _dptr(rc),
                                  _stream_handle(stream))
        _check(r, "gx_run_app_vadd")

    def run_sched(self, prog_fd, cost, workers, out, log=None, log_rc=None, log_n=None, stream=None):
        """The device block scheduler (gx_run_sched): cost: uint32 device
        tensor of units; out: 64 x units uint64 (int64) device words; log:
        (cap, 4) uint64 words, log_rc: cap uint32, log_n: one uint32 (device
        tensors or None)."""
        n_units = cost.numel()
        if out.numel() < 64 * n_units:
            raise ValueError("out holds fewer than 64 words per unit")
        cap = 0 if log is None else log.numel() // 4
        if log is not None and (log_rc is None or log_rc.numel() < cap):
            raise ValueError("log_rc must hold one code per logged decision")
        r = lib().gx_run_sched(self._h, prog_fd, _dptr(cost), n_units, workers, _dptr(out), _dptr(log),
                               _dptr(log_rc), cap, _dptr(log_n), _stream_handle(stream))
        _check(r, "gx_run_sched")

    def run_batches(self, descs, stream=None):
        """descs: list of (prog_fd, events tensor, n_events, record_size, rc tensor or None)."""
        _check(lib().gx_run_batches(self._h, _batch_array(descs), len(descs), _stream_handle(stream)), "gx_run_batches")

    def autotune_batches(self, descs, stream=None) -> dict:
        """Choose the batched launch's waves per CU by timing ``descs`` (map
        contents restored afterwards)."""
        t = Tune()
        _check(lib().gx_autotune_batches(self._h, _batch_array(descs), len(descs), _stream_handle(stream),
                                         C.byref(t)), "gx_autotune_batches")
        return {"waves_per_cu": t.blocks, "trials": t.trials, "best_ms": t.best_ms, "default_ms": t.default_ms}

    def graph_create(self, descs) -> "Graph":
        """Capture a batch (descs as for run_batches) into a replayable graph."""
        return Graph(self, descs)

    # ring buffers -----------------------------------------------------------
    def drain_ringbuf_view(self, fd):
        """Drain without a host copy (gx_drain_ringbuf_view): returns (view,
        kept_bytes, n_records), view a uint8 array over the runtime's pinned
        staging buffer, valid until the next drain of this ring, which also
        holds discard records (parse_ring skips them)."""
        view, vb, n = C.c_void_p(), C.c_uint64(0), C.c_uint64(0)
        kept = _check(lib().gx_drain_ringbuf_view(self._h, fd, C.byref(view), C.byref(vb), C.byref(n)),
                      "gx_drain_ringbuf_view")
        if not vb.value:
            return np.empty(0, np.uint8), kept, n.value
        return np.ctypeslib.as_array(C.cast(view, C.POINTER(C.c_uint8)), shape=(vb.value,)), kept, n.value

    def drain_ringbuf_start(self, fd):
        """First half of drain_ringbuf_view (gx_drain_ringbuf_start): the
        copy to the host is queued and overlaps the next launches."""
        _check(lib().gx_drain_ringbuf_start(self._h, fd), "gx_drain_ringbuf_start")

    def drain_ringbuf_finish(self, fd):
        """Second half (gx_drain_ringbuf_finish): (view, kept_bytes,
        n_records) as drain_ringbuf_view returns them."""
        view, vb, n = C.c_void_p(), C.c_uint64(0), C.c_uint64(0)
        kept = _check(lib().gx_drain_ringbuf_finish(self._h, fd, C.byref(view), C.byref(vb), C.byref(n)),
                      "gx_drain_ringbuf_finish")
        if not vb.value:
            return np.empty(0, np.uint8), kept, n.value
        return np.ctypeslib.as_array(C.cast(view, C.POINTER(C.c_uint8)), shape=(vb.value,)), kept, n.value

    def drain_ringbuf(self, fd, cap=None, copy=True):
        """Returns (records, n_records): the committed records as bytes, or
        (copy=False) as a view of a buffer the next drain of this ring
        reuses."""
        if cap is None:
            cap = self.maps[fd].max_entries
        buf = self._drain_bufs.get(fd)
        if buf is None or len(buf) < max(cap, 8):
            buf = np.empty(max(cap, 8), np.uint8)
            self._drain_bufs[fd] = buf
        n = C.c_uint64(0)
        nb = _check(lib().gx_drain_ringbuf(self._h, fd, buf.ctypes.data_as(C.c_void_p), cap, C.byref(n)),
                    "gx_drain_ringbuf")
        return (buf[:nb].tobytes() if copy else buf[:nb]), n.value

    def ringbuf_pos(self, fd):
        """(head, tail): bytes the ring's writers reserved and the host
        drained since the ring was created (gx_ringbuf_pos)."""
        h, t = C.c_uint64(0), C.c_uint64(0)
        _check(lib().gx_ringbuf_pos(self._h, fd, C.byref(h), C.byref(t)), "gx_ringbuf_pos")
        return h.value, t.value

    # host snapshots ---------------------------------------------------------
    def snapshot_start(self, fds, interval_us=1000, stream=None):
        """Start the snapshot daemon over maps ``fds`` (gx_snapshot_start)."""
        arr = np.array(list(fds), dtype=np.int32)
        _check(lib().gx_snapshot_start(self._h, arr.ctypes.data_as(C.c_void_p), len(arr), int(interval_us),
                                       _stream_handle(stream)), "gx_snapshot_start")

    def snapshot_read(self, fd):
        """(keys, values, version) of the latest host snapshot of a map,
        without touching the device (shapes as map_dump)."""
        m = self.maps[fd]
        ver = C.c_uint64(0)
        n = _check(lib().gx_snapshot_read(self._h, fd, None, None, 0, C.byref(ver)), "gx_snapshot_read")
        keys = np.zeros((max(n, 1), m.key_size), np.uint8)
        vals = np.zeros((max(n, 1), m.value_size), np.uint8)
        n2 = _check(lib().gx_snapshot_read(self._h, fd, keys.ctypes.data_as(C.c_void_p),
                                           vals.ctypes.data_as(C.c_void_p), n, C.byref(ver)), "gx_snapshot_read")
        n = min(n, n2)
        return keys[:n], vals[:n], ver.value

    def snapshot_flush(self):
        _check(lib().gx_snapshot_flush(self._h), "gx_snapshot_flush")

    def snapshot_stop(self):
        lib().gx_snapshot_stop(self._h)

    def profile_enable(self, on=True):
        _check(lib().gx_profile_enable(self._h, int(on)), "gx_profile_enable")

    def profile_read(self):
        """(summed VM-kernel milliseconds, bracketed launches) since the last read."""
        ms, n = C.c_double(0), C.c_uint64(0)
        _check(lib().gx_profile_read(self._h, C.byref(ms), C.byref(n)), "gx_profile_read")
        return ms.value, n.value

    def stats(self) -> dict:
        s = Stats()
        _check(lib().gx_stats_get(self._h, C.byref(s)), "gx_stats_get")
        return {k: getattr(s, k) for k, _ in Stats._fields_}


def _batch_array(descs):
    arr = (Batch * max(len(descs), 1))()
    for i, (p, ev, n, rs, rc) in enumerate(descs):
        arr[i].prog_fd = p
        arr[i].record_size = rs
        arr[i].d_events = ev.data_ptr()
        arr[i].n_events = n
        arr[i].d_rc = rc.data_ptr() if rc is not None else None
    return arr


class Graph:
    """A batch captured into a HIP graph (gx_graph_*): launch() replays it."""

    def __init__(self, rt: "Runtime", descs):
        self.rt = rt
        self._keep = list(descs)  # the device buffers must outlive the graph
        self._h = C.c_void_p()
        _check(lib().gx_graph_create(rt._h, _batch_array(descs), len(descs), C.byref(self._h)), "gx_graph_create")

    def launch(self, stream=None):
        _check(lib().gx_graph_launch(self._h, _stream_handle(stream)), "gx_graph_launch")

    def close(self):
        if self._h:
            lib().gx_graph_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def parse_ring(buf: bytes):
    """Payloads of the records {u32 len; u32 flags; payload padded to 8};
    discard records (flags bit 0) are skipped."""
    out, pos = [], 0
    while pos + 8 <= len(buf):
        ln = int.from_bytes(buf[pos:pos + 4], "little")
        flags = int.from_bytes(buf[pos + 4:pos + 8], "little")
        if not flags & 1:
            out.append(bytes(buf[pos + 8:pos + 8 + ln]))
        pos += 8 + ((ln + 7) & ~7)
    return out


class Server:
    """Continuous-batching request loop on a Runtime (see gx_server_* in the header)."""

    def __init__(self, rt: "Runtime", budget_bytes: int, streams: int = 4, mode: int = SERVE_CONTINUOUS,
                 max_group: int = 0):
        self.rt = rt
        cfg = ServerCfg(budget_bytes, streams, mode, max_group, 0)
        self._h = C.c_void_p()
        _check(lib().gx_server_create(rt._h, C.byref(cfg), C.byref(self._h)), "gx_server_create")

    def submit(self, tenant, prog_fd, events: np.ndarray, req_id: int):
        ev = np.ascontiguousarray(events)
        _check(lib().gx_server_submit(self._h, tenant, prog_fd, ev.ctypes.data_as(C.c_void_p), len(ev),
                                      ev.dtype.itemsize, req_id), "gx_server_submit")

    def submit_borrowed(self, tenant, prog_fd, host_ptr: int, n_events: int, record_size: int, req_id: int):
        """Queue a request whose events stay at ``host_ptr`` (caller-owned,
        ideally pinned) until its completion has been polled."""
        _check(lib().gx_server_submit_borrowed(self._h, tenant, prog_fd, C.c_void_p(host_ptr), n_events,
                                               record_size, req_id), "gx_server_submit_borrowed")

    def poll(self, max_n=256, wait_ms=0, keep_rc=True):
        """List of dicts (req_id, tenant, status, rc copy or None, t_submit, t_admit, t_done)."""
        arr = (Completion * max_n)()
        n = lib().gx_server_poll(self._h, arr, max_n, wait_ms)
        out = []
        for i in range(max(n, 0)):
            c = arr[i]
            rc = np.ctypeslib.as_array(c.rc, shape=(c.n_events,)).copy() if keep_rc and c.rc else None
            out.append({"req_id": c.req_id, "tenant": c.tenant, "status": c.status, "n_events": c.n_events,
                        "rc": rc, "t_submit": c.t_submit, "t_admit": c.t_admit, "t_done": c.t_done})
            lib().gx_server_release(self._h, C.byref(c))
        return out

    def drain(self):
        _check(lib().gx_server_drain(self._h), "gx_server_drain")

    def close(self):
        if self._h:
            lib().gx_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
