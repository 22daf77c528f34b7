"""Python handle on the CPU oracle (ctypes).  Test infrastructure only.

The oracle is the definition of the result the GPU runtime must reproduce:
events executed one at a time in index order, maps and ring buffer updated
immediately.  Only the tests, the smoke check and the benchmark's CPU baseline
use this module; the product path never imports it.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = ["interp.cpp", "checker.cpp", "capi.cpp"]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["g++", "-O2", "-std=c++17", "-Wall", "-shared", "-fPIC", "-o", LIB_PATH]
        cmd += [os.path.join(_HERE, s) for s in SOURCES]
        subprocess.run(cmd, check=True)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        vp, u32, u64, i64 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int64
        L.gxo_new.restype = vp
        L.gxo_free.argtypes = [vp]
        L.gxo_create_map.argtypes = [vp, C.c_int, u32, u32, u32, u32]
        L.gxo_map_update.argtypes = [vp, C.c_int, vp, vp, u64]
        L.gxo_map_lookup.argtypes = [vp, C.c_int, vp, vp]
        L.gxo_map_delete.argtypes = [vp, C.c_int, vp]
        L.gxo_map_dump.argtypes = [vp, C.c_int, vp, vp, u64]
        L.gxo_map_dump.restype = i64
        L.gxo_ring_drain.argtypes = [vp, C.c_int, vp, u64, C.POINTER(u64)]
        L.gxo_ring_drain.restype = i64
        L.gxo_set_tracking.argtypes = [vp, C.c_int]
        L.gxo_run.argtypes = [vp, vp, u32, C.c_int, vp, u32, vp, u64, C.c_int, u64, vp]
        L.gxo_stats.argtypes = [vp, vp, C.c_char_p, u32]
        L.gxo_reset_stats.argtypes = [vp]
        L.gxo_check.argtypes = [vp, u32, C.c_int, vp, u32, vp, u32, C.c_char_p, u32, vp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


@dataclass
class CheckResult:
    ok: bool
    log: str
    stack_bytes: int
    max_insns: int
    max_calls: int
    max_ring_bytes: int
    event_parallel: bool


def check(code: bytes, hook: int, shapes, table=None) -> CheckResult:
    """Run the oracle's checker.  ``shapes``: list of (type, key_size,
    value_size, max_entries, flags); ``table``: the program's map table
    (indices into ``shapes``; default identity)."""
    L = lib()
    sh = np.array(shapes, dtype=np.uint32).reshape(-1, 5) if shapes else np.zeros((0, 5), np.uint32)
    tb = np.array(list(range(len(sh))) if table is None else table, dtype=np.int32)
    log = C.create_string_buffer(512)
    facts = np.zeros(6, dtype=np.uint64)
    codeb = np.frombuffer(code, dtype=np.uint8).copy() if code else np.zeros(8, np.uint8)
    L.gxo_check(_ptr(codeb), len(code) // 8, hook, _ptr(sh), len(sh), _ptr(tb), len(tb), log, 512, _ptr(facts))
    return CheckResult(bool(facts[0]), log.value.decode(), int(facts[1]), int(facts[2]),
                       int(facts[3]), int(facts[4]), bool(facts[5]))


class Oracle:
    """One oracle instance: a set of maps and accumulated statistics."""

    def __init__(self):
        self._h = lib().gxo_new()
        self.shapes = []

    def __del__(self):
        try:
            lib().gxo_free(self._h)
        except Exception:
            pass

    def create_map(self, type_, key_size, value_size, max_entries, flags=0) -> int:
        r = lib().gxo_create_map(self._h, type_, key_size, value_size, max_entries, flags)
        if r >= 0:
            self.shapes.append((type_, key_size, value_size, max_entries, flags))
        return r

    def update(self, mid, key: bytes, val: bytes, flags=0) -> int:
        k = np.frombuffer(key, np.uint8).copy()
        v = np.frombuffer(val, np.uint8).copy()
        return lib().gxo_map_update(self._h, mid, _ptr(k), _ptr(v), flags)

    def lookup(self, mid, key: bytes):
        vsz = self.shapes[mid][2]
        k = np.frombuffer(key, np.uint8).copy()
        v = np.zeros(vsz, np.uint8)
        r = lib().gxo_map_lookup(self._h, mid, _ptr(k), _ptr(v))
        return None if r else v.tobytes()

    def delete(self, mid, key: bytes) -> int:
        k = np.frombuffer(key, np.uint8).copy()
        return lib().gxo_map_delete(self._h, mid, _ptr(k))

    def dump(self, mid):
        """(keys, values) as uint8 arrays of shape (n, key_size) / (n, value_size)."""
        _, ksz, vsz, _, _ = self.shapes[mid]
        n = lib().gxo_map_dump(self._h, mid, None, None, 0)
        keys = np.zeros((max(n, 1), ksz), np.uint8)
        vals = np.zeros((max(n, 1), vsz), np.uint8)
        lib().gxo_map_dump(self._h, mid, _ptr(keys), _ptr(vals), n)
        return keys[:n], vals[:n]

    def drain(self, mid, cap=1 << 30):
        """Ring records as a list of payload bytes (commit order)."""
        buf = np.zeros(cap if cap < (1 << 30) else self.shapes[mid][3], np.uint8)
        nrec = C.c_uint64(0)
        nb = lib().gxo_ring_drain(self._h, mid, _ptr(buf), len(buf), C.byref(nrec))
        return parse_ring(buf[:nb].tobytes())

    def set_tracking(self, on: bool):
        lib().gxo_set_tracking(self._h, int(on))

    def run(self, code: bytes, hook: int, events: np.ndarray, table=None, order=0, seed=0):
        """Run over ``events`` (structured record array); returns rc (uint32)."""
        tb = np.array(list(range(len(self.shapes))) if table is None else table, dtype=np.int32)
        ev = np.ascontiguousarray(events)
        rc = np.zeros(len(ev), np.uint32)
        codeb = np.frombuffer(code, np.uint8).copy()
        r = lib().gxo_run(self._h, _ptr(codeb), len(code) // 8, hook, _ptr(tb), len(tb),
                          ev.ctypes.data_as(C.c_void_p), len(ev), order, seed, _ptr(rc))
        if r:
            raise ValueError(f"oracle run failed: {r}")
        return rc

    def stats(self) -> dict:
        out = np.zeros(6, np.uint64)
        msg = C.create_string_buffer(256)
        lib().gxo_stats(self._h, _ptr(out), msg, 256)
        keys = ["insns", "helper_calls", "drops", "e2big", "violations", "faults"]
        d = {k: int(v) for k, v in zip(keys, out)}
        d["fault_msg"] = msg.value.decode()
        return d

    def reset_stats(self):
        lib().gxo_reset_stats(self._h)


def parse_ring(buf: bytes):
    """Split drained ring bytes ``{u32 len, u32 flags, payload padded to 8}``."""
    out, pos = [], 0
    while pos + 8 <= len(buf):
        ln = int.from_bytes(buf[pos:pos + 4], "little")
        out.append(bytes(buf[pos + 8:pos + 8 + ln]))
        pos += 8 + ((ln + 7) & ~7)
    return out
