"""The oracle on several host threads at once (test infrastructure: the
benchmark's CPU baseline and the tests that check it against one thread).

Each thread runs its own oracle instance, with its own maps, over a
disjoint part of the work; the arithmetic is the oracle's own, untouched.
The ctypes calls release the interpreter lock, so the threads run in
parallel.

* Stream-sequential programs split by stream key (key mod T): each
  stream's events stay in order in one thread, owned state (hash keys carry
  the stream) stays with it, so the per-thread hash maps hold disjoint keys
  and the union of the rings is a single thread's ring.
* Event-parallel programs split the batch into T contiguous ranges (at
  64-record tile boundaries for warp-leader hooks): events are independent
  and shared maps take one commutative operation, so the per-thread maps
  combine with that operation into the single-threaded result.
* Independent runs (a batch of programs, a request trace) go to threads
  whole (the largest first, to the least-loaded thread).
"""

from __future__ import annotations

import math
import os
import threading
import time

import numpy as np

from oracle.oracle import Oracle

STREAM_FIELD = {1: "stream", 2: "kernel_id", 3: "stream"}  # hook -> stream key field


def host_threads(cap: int = 16) -> int:
    """Threads for the baseline: the CPUs this process may use, at most ``cap``."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, cap))


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def split(events: np.ndarray, hook: int, event_parallel: bool, T: int):
    """Index arrays of the T parts (each in index order)."""
    n = len(events)
    if event_parallel:
        align = 64 if hook == 3 else 1
        step = math.ceil(math.ceil(n / T) / align) * align
        return [np.arange(min(t * step, n), min((t + 1) * step, n)) for t in range(T)]
    key = events[STREAM_FIELD[hook]].astype(np.int64)
    part = key % T
    order = np.argsort(part, kind="stable")
    bounds = np.searchsorted(part[order], np.arange(T + 1))
    return [order[bounds[t]:bounds[t + 1]] for t in range(T)]


def new_oracle(shapes, init=None, tracking=False) -> Oracle:
    o = Oracle()
    o.set_tracking(tracking)
    for sh in shapes:
        assert o.create_map(*sh) >= 0
    for mi, k, v in init or []:
        assert o.update(mi, k, v) == 0
    return o


def run_threads(jobs):
    """Run callables on one thread each; returns their results."""
    out = [None] * len(jobs)
    err = []

    def work(i, f):
        try:
            out[i] = f()
        except BaseException as e:  # re-raised below
            err.append(e)

    th = [threading.Thread(target=work, args=(i, f)) for i, f in enumerate(jobs)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    if err:
        raise err[0]
    return out


def run_parallel(code: bytes, hook: int, shapes, events: np.ndarray, event_parallel: bool, T: int, init=None):
    """One batch on T threads.  Returns (seconds, oracles, parts, rcs): the
    wall time of splitting and running, each thread's oracle, its event
    indices and its return codes."""
    oracles = [new_oracle(shapes, init) for _ in range(T)]
    t0 = time.perf_counter()
    parts = split(events, hook, event_parallel, T)
    subs = [np.ascontiguousarray(events[p]) for p in parts]
    rcs = run_threads([lambda o=o, s=s: o.run(code, hook, s) for o, s in zip(oracles, subs)])
    dt = time.perf_counter() - t0
    return dt, oracles, parts, rcs


def gather_rc(n: int, parts, rcs) -> np.ndarray:
    rc = np.zeros(n, np.uint32)
    for p, r in zip(parts, rcs):
        rc[p] = r
    return rc


def merge_array(oracles, mid: int, op: str | None, init_vals: np.ndarray | None = None) -> bytes:
    """A map's final values: an owned map's (op None: the threads touched
    disjoint slots, so each slot is taken from the thread that changed it),
    or a shared map's combined with its commutative operation (word size
    from the map's value size: 4 or 8 bytes)."""
    vals = [o.dump(mid)[1] for o in oracles]
    vsz = vals[0].shape[1] if vals[0].ndim == 2 else 0
    dt = "<u4" if vsz % 8 else "<u8"
    w = [np.frombuffer(v.tobytes(), dt) for v in vals]
    base = np.zeros_like(w[0]) if init_vals is None else np.frombuffer(init_vals.tobytes(), dt)
    if op is None:
        out = base.copy()
        for x in w:
            ch = x != base
            out[ch] = x[ch]
    elif op == "add":
        out = base + sum((x - base for x in w), np.zeros_like(base))
    elif op == "or":
        out = base.copy()
        for x in w:
            out |= x
    elif op == "and":
        out = base.copy()
        for x in w:
            out &= x
    else:
        out = base.copy()
        for x in w:
            out ^= x ^ base
    return out.tobytes()


def merge_hash(oracles, mid: int):
    """Union of the threads' (key, value) pairs (disjoint key sets)."""
    items = []
    for o in oracles:
        k, v = o.dump(mid)
        items += [(bytes(a), bytes(b)) for a, b in zip(k, v)]
    return sorted(items)


def merge_ring(oracles, mid: int):
    out = []
    for o in oracles:
        out += o.drain(mid)
    return sorted(out)


def insns(oracles) -> int:
    return sum(o.stats()["insns"] for o in oracles)


def trials(fn, k: int = 10, budget_s: float | None = None):
    """fn() -> (seconds, units, insns) per trial; returns the median and
    geometric mean of the units/s and insns/s over k trials (fewer, but at
    least 3, once ``budget_s`` seconds have passed)."""
    rates, irates = [], []
    t0 = time.perf_counter()
    for i in range(k):
        dt, units, ins = fn()
        rates.append(units / dt)
        irates.append(ins / dt)
        if budget_s is not None and i >= 2 and time.perf_counter() - t0 > budget_s:
            break
    gm = lambda xs: float(math.exp(sum(math.log(x) for x in xs) / len(xs)))  # noqa: E731
    return {"median": float(np.median(rates)), "geomean": gm(rates),
            "insns_median": float(np.median(irates)), "insns_geomean": gm(irates), "trials": len(rates)}
