"""Seeded synthetic inputs: hook-event batches, the policy programs, and the
random program generator.

This module produces *inputs only* -- event records, program text and map
shapes.  It holds none of the eBPF semantics; both the CPU oracle and the GPU
runtime consume what it produces.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) in its counter form:
``x_i = mix(seed + (i + 1) * GAMMA)``, which vectorises over ``i``.

The paper (section 6) measures its policies on applications and datasets that
are not available here; these generators are synthetic stand-ins with the
shapes described in the workload recipe (region = 2 MiB, pages = 4 KiB as in
section 4.3.1; sequential-run / random access mixes as in Figure 1's
patterns; per-kernel latency histograms as in the observability tools of
Table 2).
"""

from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

from . import asm

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)

# hook types and record layouts (little endian, packed)
HOOK_MEM_ACCESS = 1
HOOK_KERNEL_TIMING = 2
# warp-leader hook: one invocation per tile of 64 memory-access records, on
# the tile's aggregate {u64 lo @0, u64 hi @8, u32 n @16, u32 stream @20}
HOOK_WAVE_MEM = 3
# SIMT hook: one invocation per memory-access record, on the record followed
# by its tile's aggregate at byte 24 (warp-uniform); the verifier holds the
# program to warp-uniform branches, keys and side effects
HOOK_SIMT_MEM = 4
# device block scheduler: one invocation per steal decision of a persistent
# worker, on {u32 worker, u32 done, u64 elapsed_ns, u64 steal_ns, u32 stolen,
# u32 left}; a non-zero return code means "take one more unit"
HOOK_SCHED = 5
MEM_DTYPE = np.dtype([("addr", "<u8"), ("stream", "<u4"), ("pad", "<u4"), ("ts", "<u8")])
TIMING_DTYPE = np.dtype([("kernel_id", "<u4"), ("pad", "<u4"), ("lat", "<u8")])
SCHED_DTYPE = np.dtype([("worker", "<u4"), ("done", "<u4"), ("elapsed_ns", "<u8"), ("steal_ns", "<u8"),
                        ("stolen", "<u4"), ("left", "<u4")])
assert MEM_DTYPE.itemsize == 24 and TIMING_DTYPE.itemsize == 16 and SCHED_DTYPE.itemsize == 32

# map types (Linux numbering) and flags
MAP_HASH, MAP_ARRAY, MAP_RINGBUF = 1, 2, 27
F_SHARED, F_READ_ONLY = 1, 2


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * M1
    z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def splitmix(seed: int, n: int, start: int = 0) -> np.ndarray:
    """``n`` SplitMix64 outputs of the sequence seeded by ``seed``."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + n + 1, dtype=np.uint64)
        return _mix(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * GAMMA)


def subseed(seed: int, tag: int) -> int:
    """Seed of an independent sub-sequence (a SplitMix64 output of ``seed ^ tag``)."""
    return int(splitmix(seed ^ (tag * 0x632BE59BD9B4E019 & 0xFFFFFFFFFFFFFFFF), 1)[0])


def u01(x: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits."""
    return (x >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def zipf_table(s: float, n: int) -> np.ndarray:
    w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    c = np.cumsum(w)
    return c / c[-1]


def zipf_ranks(u: np.ndarray, table: np.ndarray) -> np.ndarray:
    """Inverse-CDF Zipf draw: ranks in [1, n]."""
    r = np.searchsorted(table, u, side="right") + 1
    return np.minimum(r, len(table)).astype(np.uint64)


def manifest(arrays: dict) -> dict:
    return {k: hashlib.sha256(np.ascontiguousarray(v).tobytes()).hexdigest() for k, v in arrays.items()}


# ---------------------------------------------------------------------------
# event generators

def gen_mem_uniform(n: int, seed: int, streams: int = 1024) -> np.ndarray:
    """Memory-access records: addr uniform over [0, 8 GiB), stream uniform in
    [0, streams), timestamps strictly increasing."""
    ev = np.zeros(n, dtype=MEM_DTYPE)
    ev["addr"] = splitmix(subseed(seed, 1), n) >> np.uint64(31)
    ev["stream"] = (u01(splitmix(subseed(seed, 2), n)) * streams).astype(np.uint32)
    ev["ts"] = np.cumsum(np.uint64(1) + (splitmix(subseed(seed, 3), n) >> np.uint64(58)))
    return ev


def gen_mem_stride(n: int, seed: int, streams: int = 1024, pages_log2: int = 18,
                   run_frac: float = 0.4, zipf_s: float = 1.1) -> np.ndarray:
    """Memory-access records for the stride-prefetch policy.

    Each event picks its stream uniformly.  Per stream, accesses come in
    segments: with probability q a sequential run (length U[8, 64], stride
    U[1, 16] pages, uniform start page), otherwise one random access whose page
    is a Zipf(zipf_s) rank scattered by an odd multiplier.  q is set so that
    ``run_frac`` of the events fall in runs (mean run length 36).
    """
    npages = 1 << pages_log2
    pmask = np.uint64(npages - 1)
    mean_run = 36.0
    q = run_frac / (mean_run * (1 - run_frac) + run_frac)  # P(segment is a run)
    ztab = zipf_table(zipf_s, npages)
    ev = np.zeros(n, dtype=MEM_DTYPE)
    sid = (u01(splitmix(subseed(seed, 1), n)) * streams).astype(np.uint32)
    ev["stream"] = sid
    ev["ts"] = np.cumsum(np.uint64(1) + (splitmix(subseed(seed, 2), n) >> np.uint64(58)))
    lowbits = splitmix(subseed(seed, 3), n) & np.uint64(0xFFF)
    order = np.argsort(sid, kind="stable")
    counts = np.bincount(sid, minlength=streams)
    pages = np.empty(n, dtype=np.uint64)
    pos = 0
    for s in range(streams):
        ns = int(counts[s])
        if ns == 0:
            continue
        ss = subseed(seed, 1000 + s)
        m = ns  # every segment yields >= 1 event, so ns segments always suffice
        is_run = u01(splitmix(subseed(ss, 1), m)) < q
        run_len = 8 + (u01(splitmix(subseed(ss, 2), m)) * 57).astype(np.int64)
        stride = np.uint64(1) + (u01(splitmix(subseed(ss, 3), m)) * 16).astype(np.uint64)
        start = splitmix(subseed(ss, 4), m) & pmask
        rank = zipf_ranks(u01(splitmix(subseed(ss, 5), m)), ztab)
        with np.errstate(over="ignore"):
            rnd_page = ((rank - np.uint64(1)) * np.uint64(0x9E3779B1)) & pmask
        seg_len = np.where(is_run, run_len, 1)
        ends = np.cumsum(seg_len)
        j = np.arange(ns, dtype=np.int64)
        seg = np.searchsorted(ends, j, side="right")
        k = (j - (ends[seg] - seg_len[seg])).astype(np.uint64)
        with np.errstate(over="ignore"):
            run_page = (start[seg] + k * stride[seg]) & pmask
        pages[order[pos:pos + ns]] = np.where(is_run[seg], run_page, rnd_page[seg])
        pos += ns
    ev["addr"] = (pages << np.uint64(12)) | lowbits
    return ev


def gen_mem_wave(n: int, seed: int, coalesced: float = 0.75, streams: int = 1024) -> np.ndarray:
    """Memory-access records as the lanes of waves issue them: records come
    in tiles of 64 (one wave's access); a fraction ``coalesced`` of the
    tiles read consecutive 8-byte words from a uniform base (u64-aligned in
    [0, 8 GiB)), the others 64 uniform addresses.  The tile's stream is
    uniform in [0, streams); timestamps strictly increase."""
    ev = np.zeros(n, dtype=MEM_DTYPE)
    tiles = (n + 63) // 64
    tile = np.arange(n, dtype=np.uint64) // np.uint64(64)
    lane = np.arange(n, dtype=np.uint64) % np.uint64(64)
    co = u01(splitmix(subseed(seed, 1), tiles)) < coalesced
    base = (splitmix(subseed(seed, 2), tiles) >> np.uint64(31)) & ~np.uint64(7)
    rand = (splitmix(subseed(seed, 3), n) >> np.uint64(31))
    ev["addr"] = np.where(co[tile.astype(np.int64)], base[tile.astype(np.int64)] + lane * np.uint64(8), rand)
    ev["stream"] = (u01(splitmix(subseed(seed, 4), tiles)) * streams).astype(np.uint32)[tile.astype(np.int64)]
    ev["ts"] = np.cumsum(np.uint64(1) + (splitmix(subseed(seed, 5), n) >> np.uint64(58)))
    return ev


def gen_timing(n: int, seed: int, kernels: int = 4096, zipf_s: float = 1.2,
               mu: float = 10.0, sigma: float = 1.5) -> np.ndarray:
    """Kernel-timing records: kernel_id = Zipf(zipf_s) rank scattered by an odd
    multiplier over ``kernels``; latency = floor(exp(mu + sigma * z)) ns with z
    a Box-Muller standard normal."""
    ev = np.zeros(n, dtype=TIMING_DTYPE)
    rank = zipf_ranks(u01(splitmix(subseed(seed, 1), n)), zipf_table(zipf_s, kernels))
    with np.errstate(over="ignore"):
        ev["kernel_id"] = (((rank - np.uint64(1)) * np.uint64(2654435761)) % np.uint64(kernels)).astype(np.uint32)
    u1 = 1.0 - u01(splitmix(subseed(seed, 2), n))  # (0, 1]
    u2 = u01(splitmix(subseed(seed, 3), n))
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    ev["lat"] = np.floor(np.exp(mu + sigma * z)).astype(np.uint64)
    return ev


def p99_threshold(lat: np.ndarray) -> int:
    """Nearest-rank empirical 99th percentile: sorted[ceil(0.99 N) - 1]."""
    k = math.ceil(0.99 * len(lat)) - 1
    return int(np.partition(lat, k)[k])


# ---------------------------------------------------------------------------
# map specifications and the three policy programs

@dataclass
class MapSpec:
    name: str
    type: int
    key_size: int
    value_size: int
    max_entries: int
    flags: int = 0


@dataclass
class Policy:
    name: str
    hook: int
    text: str
    maps: list = field(default_factory=list)

    @property
    def code(self) -> bytes:
        return asm.assemble(self.text, [m.name for m in self.maps])

    @property
    def record_size(self) -> int:
        return {HOOK_KERNEL_TIMING: 16, HOOK_SCHED: 32}.get(self.hook, 24)


# Access counter: per 2 MiB region counts in a shared array; rc = region & 1.
ACCESS_COUNTER = """
    ldxdw r6, [r1+0]          ; addr
    rsh64 r6, 21              ; region = addr >> 21
    mov64 r0, 0
    jge r6, 4096, out         ; bounds check (never taken for addr < 8 GiB)
    stxw [r10-4], r6
    lddw r1, map:hist
    mov64 r2, r10
    add64 r2, -4
    call map_lookup_elem
    jeq r0, 0, out0
    mov64 r1, 1
    aadd64 [r0+0], r1         ; commutative atomic add, no fetch
    mov64 r0, r6
    and64 r0, 1               ; rc = region & 1
    exit
out0:
    mov64 r0, 0
out:
    exit
"""


def access_counter_policy() -> Policy:
    return Policy("access_counter", HOOK_MEM_ACCESS, ACCESS_COUNTER,
                  [MapSpec("hist", MAP_ARRAY, 4, 8, 4096, F_SHARED)])


# Stride prefetch: per (stream, region-tag) state in a hash map; emits a
# prefetch decision record when the same non-zero stride repeats.
STRIDE_PREFETCH = """
    ldxdw r6, [r1+0]          ; a = addr
    ldxw r7, [r1+8]           ; s = stream_id
    ldxdw r8, [r1+16]         ; ts
    stxdw [r10-48], r8
    stxw [r10-52], r7
    mov64 r2, r7
    lsh64 r2, 32
    mov64 r3, r6
    rsh64 r3, 21
    and64 r3, 31
    or64 r2, r3               ; key = s << 32 | (region & 31)
    stxdw [r10-8], r2
    lddw r1, map:state
    mov64 r2, r10
    add64 r2, -8
    call map_lookup_elem
    jne r0, 0, found
    stxdw [r10-32], r6        ; new entry {a, 0, 0}
    stdw [r10-24], 0
    stdw [r10-16], 0
    lddw r1, map:state
    mov64 r2, r10
    add64 r2, -8
    mov64 r3, r10
    add64 r3, -32
    mov64 r4, 0
    call map_update_elem
    mov64 r0, 0
    exit
found:
    mov64 r9, r0              ; v
    ldxdw r1, [r9+0]          ; last_addr
    mov64 r2, r1
    rsh64 r2, 21
    mov64 r3, r6
    rsh64 r3, 21
    jeq r2, r3, tag_hit
    stxdw [r9+0], r6          ; tag miss: v = {a, 0, 0}
    stdw [r9+8], 0
    stw [r9+16], 0
    mov64 r0, 0
    exit
tag_hit:
    mov64 r7, r6
    rsh64 r7, 12              ; pg = a >> 12
    rsh64 r1, 12
    mov64 r8, r7
    sub64 r8, r1              ; d = pg - (last_addr >> 12)
    stxdw [r9+0], r6          ; last_addr = a
    mov64 r0, 0
    jeq r8, 0, ret
    ldxdw r1, [r9+8]
    jne r1, r8, newstride
    ldxw r1, [r9+16]
    add32 r1, 1               ; conf += 1
    stxw [r9+16], r1
    ja check
newstride:
    stxdw [r9+8], r8          ; stride = d
    stw [r9+16], 0            ; conf = 0
    mov64 r1, 0
check:
    jlt r1, 2, ret0
    mov64 r2, r1
    and64 r2, 7
    jne r2, 2, ret0
    jsgt r8, 16, ret0
    jslt r8, -16, ret0
    mov64 r6, 0               ; n
    mov64 r2, 1               ; k (loop counter)
    mov64 r3, r7              ; p
loop:
    add64 r3, r8              ; p = pg + k * d
    jslt r3, 0, loop_end
    jsge r3, 262144, loop_end
    mov64 r4, r3
    rsh64 r4, 9
    mov64 r5, r7
    rsh64 r5, 9
    jne r4, r5, loop_end      ; stay inside the current 2 MiB region
    mov64 r6, r2              ; n = k
    add64 r2, 1
    jle r2, 8, loop
loop_end:
    jeq r6, 0, ret0
    ldxw r1, [r10-52]
    stxw [r10-40], r1         ; record {u32 s, u32 n, u64 (pg+d)<<12, i64 d<<12, u64 ts}
    stxw [r10-36], r6
    mov64 r1, r7
    add64 r1, r8
    lsh64 r1, 12
    stxdw [r10-32], r1
    mov64 r1, r8
    lsh64 r1, 12
    stxdw [r10-24], r1
    ldxdw r1, [r10-48]
    stxdw [r10-16], r1
    lddw r1, map:ring
    mov64 r2, r10
    add64 r2, -40
    mov64 r3, 32
    mov64 r4, 0
    call ringbuf_output
    mov64 r0, r6
    exit
ret0:
    mov64 r0, 0
ret:
    exit
"""


def stride_prefetch_policy(hash_entries: int = 1 << 16, ring_bytes: int = 64 << 20) -> Policy:
    return Policy("stride_prefetch", HOOK_MEM_ACCESS, STRIDE_PREFETCH, [
        MapSpec("state", MAP_HASH, 8, 24, hash_entries, 0),
        MapSpec("ring", MAP_RINGBUF, 0, 0, ring_bytes, 0),
    ])


# Observability: per-kernel log2 latency histogram plus tail trace records.
LATENCY_HIST = """
    ldxw r6, [r1+0]           ; k = kernel_id
    ldxdw r7, [r1+8]          ; l = latency_ns
    mov64 r8, r7
    mov64 r9, 0               ; b = floor(log2 l), 0 for l = 0
    mov64 r1, r8
    rsh64 r1, 32
    jeq r1, 0, s16
    mov64 r8, r1
    add64 r9, 32
s16:
    mov64 r1, r8
    rsh64 r1, 16
    jeq r1, 0, s8
    mov64 r8, r1
    add64 r9, 16
s8:
    mov64 r1, r8
    rsh64 r1, 8
    jeq r1, 0, s4
    mov64 r8, r1
    add64 r9, 8
s4:
    mov64 r1, r8
    rsh64 r1, 4
    jeq r1, 0, s2
    mov64 r8, r1
    add64 r9, 4
s2:
    mov64 r1, r8
    rsh64 r1, 2
    jeq r1, 0, s1
    mov64 r8, r1
    add64 r9, 2
s1:
    mov64 r1, r8
    rsh64 r1, 1
    jeq r1, 0, sdone
    add64 r9, 1
sdone:
    stxw [r10-4], r6
    lddw r1, map:hist
    mov64 r2, r10
    add64 r2, -4
    call map_lookup_elem
    jeq r0, 0, nohist
    mov64 r1, r9
    lsh64 r1, 3
    add64 r0, r1              ; &hist[k][b]
    mov64 r1, 1
    aadd64 [r0+0], r1
nohist:
    stw [r10-8], 0
    lddw r1, map:cfg
    mov64 r2, r10
    add64 r2, -8
    call map_lookup_elem
    jeq r0, 0, done
    ldxdw r1, [r0+0]          ; T (read-only config)
    jle r7, r1, done
    stxw [r10-40], r6         ; record {u32 k, u32 b, u64 l, u64 T, u64 0}
    stxw [r10-36], r9
    stxdw [r10-32], r7
    stxdw [r10-24], r1
    stdw [r10-16], 0
    lddw r1, map:ring
    mov64 r2, r10
    add64 r2, -40
    mov64 r3, 32
    mov64 r4, 0
    call ringbuf_output
done:
    mov64 r0, r9
    exit
"""


# Warp-leader access monitor: once per wave tile, on the tile's aggregate.
# A tile within one 4 KiB page counts its records in the page's 2 MiB region
# (coalesced); a wider tile counts once as scattered, and a tile spanning
# more than 4 GiB also sends {lo, hi, n | stream << 32} to the ring.  The
# return code is the number of 4 KiB pages the tile spans.
WAVE_MONITOR = """
    ldxdw r6, [r1+0]          ; lo
    ldxdw r7, [r1+8]          ; hi
    ldxw r8, [r1+16]          ; n
    ldxw r9, [r1+20]          ; stream of the first record
    mov64 r2, r6
    rsh64 r2, 21
    and64 r2, 4095            ; region of lo
    stxw [r10-4], r2
    mov64 r3, r7
    sub64 r3, r6
    jgt r3, 4095, wide
    lddw r1, map:coal
    mov64 r2, r10
    add64 r2, -4
    call map_lookup_elem
    jeq r0, 0, pages
    aadd64 [r0+0], r8
    ja pages
wide:
    lddw r1, map:scat
    mov64 r2, r10
    add64 r2, -4
    call map_lookup_elem
    jeq r0, 0, far
    mov64 r1, 1
    aadd64 [r0+0], r1
far:
    mov64 r3, r7
    sub64 r3, r6
    rsh64 r3, 32
    jeq r3, 0, pages
    stxdw [r10-32], r6
    stxdw [r10-24], r7
    mov64 r1, r9
    lsh64 r1, 32
    or64 r1, r8
    stxdw [r10-16], r1
    lddw r1, map:ring
    mov64 r2, r10
    add64 r2, -32
    mov64 r3, 24
    mov64 r4, 0
    call ringbuf_output
pages:
    mov64 r0, r7
    rsh64 r0, 12
    mov64 r1, r6
    rsh64 r1, 12
    sub64 r0, r1
    add64 r0, 1
    exit
"""


def wave_monitor_policy(ring_bytes: int = 64 << 20) -> Policy:
    return Policy("wave_monitor", HOOK_WAVE_MEM, WAVE_MONITOR, [
        MapSpec("coal", MAP_ARRAY, 4, 8, 4096, F_SHARED),
        MapSpec("scat", MAP_ARRAY, 4, 8, 4096, F_SHARED),
        MapSpec("ring", MAP_RINGBUF, 0, 0, ring_bytes, 0),
    ])


# The wave monitor's counting part, as a warp-leader handler and as the same
# handler run by every lane under the SIMT hook: tiles whose addresses span
# at most 4 KiB count their records into coal[region of lo], the others
# into scat[region of lo]; rc = the tile's highest address.  Once per tile
# the leader adds n; per lane each record adds 1 (the device combines the
# wave's lanes into one update), so both give the same maps and rc.
WAVE_COUNTS_LEADER = """
    ldxdw r6, [r1+0]          ; lo
    ldxdw r7, [r1+8]          ; hi
    ldxw r8, [r1+16]          ; n
    mov64 r2, r6
    rsh64 r2, 21
    and64 r2, 4095
    stxw [r10-4], r2
    mov64 r3, r7
    sub64 r3, r6
    jgt r3, 4095, wide
    lddw r1, map:coal
    mov64 r2, r10
    add64 r2, -4
    call map_lookup_elem
    jeq r0, 0, out
    aadd64 [r0+0], r8
    ja out
wide:
    lddw r1, map:scat
    mov64 r2, r10
    add64 r2, -4
    call map_lookup_elem
    jeq r0, 0, out
    aadd64 [r0+0], r8
out:
    mov64 r0, r7
    exit
"""

WAVE_COUNTS_SIMT = """
    ldxdw r6, [r1+24]         ; lo of the tile (uniform)
    ldxdw r7, [r1+32]         ; hi of the tile (uniform)
    mov64 r2, r6
    rsh64 r2, 21
    and64 r2, 4095
    stxw [r10-4], r2
    mov64 r3, r7
    sub64 r3, r6
    mov64 r8, 1
    jgt r3, 4095, wide
    lddw r1, map:coal
    mov64 r2, r10
    add64 r2, -4
    call map_lookup_elem
    jeq r0, 0, out
    aadd64 [r0+0], r8
    ja out
wide:
    lddw r1, map:scat
    mov64 r2, r10
    add64 r2, -4
    call map_lookup_elem
    jeq r0, 0, out
    aadd64 [r0+0], r8
out:
    mov64 r0, r7
    exit
"""


def wave_counts_policy(simt: bool) -> Policy:
    maps = [MapSpec("coal", MAP_ARRAY, 4, 8, 4096, F_SHARED), MapSpec("scat", MAP_ARRAY, 4, 8, 4096, F_SHARED)]
    if simt:
        return Policy("wave_counts_simt", HOOK_SIMT_MEM, WAVE_COUNTS_SIMT, maps)
    return Policy("wave_counts_leader", HOOK_WAVE_MEM, WAVE_COUNTS_LEADER, maps)


def latency_hist_policy(kernels: int = 4096, ring_bytes: int = 64 << 20) -> Policy:
    return Policy("latency_hist", HOOK_KERNEL_TIMING, LATENCY_HIST, [
        MapSpec("hist", MAP_ARRAY, 4, 512, kernels, F_SHARED),
        MapSpec("cfg", MAP_ARRAY, 4, 8, 1, F_READ_ONLY),
        MapSpec("ring", MAP_RINGBUF, 0, 0, ring_bytes, 0),
    ])


# ---------------------------------------------------------------------------
# policies for hooks inside application kernels

# L2 stride prefetch for the instrumented vector add (warp leader, section
# 6.2.1's device prefetch policy): the tile's lane-to-lane stride, estimated
# from its address range, is counted into stride[min(stride in elements,
# 4095)], and the return code asks the trampoline to prefetch, in every
# lane, the element one tile of iterations ahead (stride x records);
# tiles of one record return 0 (no prefetch).
STRIDE_L2 = """
    ldxdw r6, [r1+0]          ; lo
    ldxdw r7, [r1+8]          ; hi
    ldxw r8, [r1+16]          ; n
    mov64 r0, 0
    jlt r8, 2, out
    mov64 r9, r7
    sub64 r9, r6
    mov64 r3, r8
    sub64 r3, 1
    div64 r9, r3              ; bytes from lane to lane
    rsh64 r9, 3               ; in elements
    mov64 r2, r9
    jlt r2, 4096, keep
    mov64 r2, 4095
keep:
    stxw [r10-4], r2
    lddw r1, map:stride
    mov64 r2, r10
    add64 r2, -4
    call map_lookup_elem
    jeq r0, 0, dist
    mov64 r1, 1
    aadd64 [r0+0], r1
dist:
    mov64 r0, r9
    mul64 r0, r8
out:
    exit
"""


def stride_l2_policy() -> Policy:
    return Policy("stride_l2", HOOK_WAVE_MEM, STRIDE_L2, [MapSpec("stride", MAP_ARRAY, 4, 8, 4096, F_SHARED)])


# Block-scheduler policies (section 4.3.2's should_try_steal; section
# 6.2.1's Greedy and LatencyBudget, the support matrix's MaxSteals).  Each
# counts its yes-decisions per worker in steals[worker mod 4096]; cfg[0] is
# the policy's parameter.
_SCHED_COUNT = """
    ldxw r6, [r9+0]           ; worker
    and64 r6, 4095
    stxw [r10-8], r6
    lddw r1, map:steals
    mov64 r2, r10
    add64 r2, -8
    call map_lookup_elem
    jeq r0, 0, yes
    mov64 r1, 1
    aadd64 [r0+0], r1
yes:
    mov64 r0, 1
    exit
"""

_SCHED_CFG = """
    mov64 r9, r1
    stw [r10-4], 0
    lddw r1, map:cfg
    mov64 r2, r10
    add64 r2, -4
    call map_lookup_elem
    jeq r0, 0, no
    ldxdw r7, [r0+0]          ; the parameter
"""

# always steal while another worker has units left
SCHED_GREEDY = "    mov64 r9, r1\n" + _SCHED_COUNT

# steal while this worker has stolen fewer than cfg[0] units
SCHED_MAX_STEALS = _SCHED_CFG + """
    ldxw r6, [r9+24]          ; stolen
    jge r6, r7, no
""" + _SCHED_COUNT + """
no:
    mov64 r0, 0
    exit
"""

# steal while this worker has spent less than cfg[0] ns stealing
SCHED_LATENCY_BUDGET = _SCHED_CFG + """
    ldxdw r6, [r9+16]         ; steal_ns
    jge r6, r7, no
""" + _SCHED_COUNT + """
no:
    mov64 r0, 0
    exit
"""


def sched_policy(kind: str) -> Policy:
    text = {"greedy": SCHED_GREEDY, "max_steals": SCHED_MAX_STEALS, "latency_budget": SCHED_LATENCY_BUDGET}[kind]
    maps = [MapSpec("steals", MAP_ARRAY, 4, 8, 4096, F_SHARED)]
    if kind != "greedy":
        maps.append(MapSpec("cfg", MAP_ARRAY, 4, 8, 1, F_READ_ONLY))
    return Policy("sched_" + kind, HOOK_SCHED, text, maps)


def sched_costs(workers: int, units_per_worker: int, regime: str, base: int, seed: int) -> np.ndarray:
    """Work-unit costs (iterations per unit) of the block-scheduler workload,
    in the unit order the workers' ranges split (worker w owns units
    [w n / W, (w + 1) n / W)).  "moderate": the cost grows linearly from
    base to 2 base over the units, so the last workers' ranges hold twice
    the work of the first's; "heavy_tail": a contiguous 10 % of the workers
    own units 100-200 x costlier (section 6.2.1's clustered heavy tail), the
    rest cost base; "uniform": every unit costs base."""
    n = workers * units_per_worker
    if regime == "uniform":
        return np.full(n, base, np.uint32)
    if regime == "moderate":
        return (base + (np.arange(n, dtype=np.uint64) * base) // max(n - 1, 1)).astype(np.uint32)
    if regime == "heavy_tail":
        u = u01(splitmix(subseed(seed, 9), n))
        cost = np.full(n, base, np.float64)
        w = np.arange(n) * workers // n  # the owning worker
        h0 = int(u01(splitmix(subseed(seed, 10), 1))[0] * (workers - workers // 10))
        heavy = (w >= h0) & (w < h0 + max(1, workers // 10))
        cost[heavy] = base * (100 + 100 * u[heavy])
        return np.minimum(cost, 2**32 - 1).astype(np.uint32)
    raise ValueError(regime)


# ---------------------------------------------------------------------------
# seeded random program generator (the batched and served workloads)

class _Gen:
    """Builds one verifier-friendly random program.

    Conventions: r6, r7, r8 (and r9 outside loops) carry the program's state;
    r0-r5 are temporaries; the event's addr / stream / ts live on the stack at
    fp-16 / fp-24 / fp-32.  Owned state follows the stream: the owned array is
    indexed by stream, hash keys carry the stream in their upper 32 bits, and
    the shared array only receives commutative atomic adds.
    """

    ALU = ["add", "sub", "mul", "div", "sdiv", "or", "and", "lsh", "rsh", "mod",
           "smod", "xor", "mov", "arsh"]
    JOPS = list(asm.JMP_OPS)
    MAX_CALLS = 48

    def __init__(self, seed: int, target_len: int, own_words: int):
        self.x = int(seed) & 0xFFFFFFFFFFFFFFFF
        self.target = target_len
        self.own_words = own_words
        self.lines: list[str] = []
        self.n = 0
        self.label = 0
        self.calls = 0
        # one commutative operation per shared map (mixed operations on a
        # slot would not commute across streams)
        self.shared_op = ["aadd64", "aadd64", "aadd64", "aor64", "aand64", "axor64", "aadd32"][self.below(7)]

    def rnd(self) -> int:
        self.x = (self.x + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
        z = self.x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
        return z ^ (z >> 31)

    def below(self, k: int) -> int:
        return self.rnd() % k

    def emit(self, line: str, slots: int = 1):
        self.lines.append(line)
        self.n += slots

    def lab(self) -> str:
        self.label += 1
        return f"L{self.label}"

    def state_regs(self, in_loop: bool):
        return ["r6", "r7", "r8"] if in_loop else ["r6", "r7", "r8", "r9"]

    def imm(self) -> int:
        c = self.below(6)
        if c == 0:
            return self.below(64)
        if c == 1:
            return -1 - self.below(64)
        if c == 2:
            return [0, 1, -1, 0x7FFFFFFF, -0x80000000, 0xFFFF][self.below(6)]
        return int(self.rnd() & 0xFFFFFFFF) - (1 << 31)

    def alu(self, in_loop: bool):
        regs = self.state_regs(in_loop)
        dst = regs[self.below(len(regs))]
        w = "64" if self.below(3) else "32"
        kind = self.below(20)
        if kind == 0:
            self.emit(f"neg{w} {dst}")
            return
        if kind == 1:
            e = ["le16", "le32", "le64", "be16", "be32", "be64", "bswap16", "bswap32", "bswap64"]
            self.emit(f"{e[self.below(len(e))]} {dst}")
            return
        if kind == 2:
            src = regs[self.below(len(regs))]
            if w == "64":
                self.emit(f"movsx{[8, 16, 32][self.below(3)]}_64 {dst}, {src}")
            else:
                self.emit(f"movsx{[8, 16][self.below(2)]}_32 {dst}, {src}")
            return
        op = self.ALU[self.below(len(self.ALU))]
        if self.below(2):
            src = regs[self.below(len(regs))]
            self.emit(f"{op}{w} {dst}, {src}")
        else:
            if op in ("lsh", "rsh", "arsh"):
                k = self.below(64 if w == "64" else 32)
            elif op in ("div", "mod", "sdiv", "smod"):
                k = self.imm() or 7
            else:
                k = self.imm()
            self.emit(f"{op}{w} {dst}, {k}")

    def cond(self, in_loop: bool) -> str:
        regs = self.state_regs(in_loop)
        a = regs[self.below(len(regs))]
        op = self.JOPS[self.below(len(self.JOPS))] + ("32" if self.below(4) == 0 else "")
        b = regs[self.below(len(regs))] if self.below(2) else str(self.imm())
        return f"{op} {a}, {b}"

    def reload_key_stream(self):
        self.emit("ldxdw r1, [r10-24]")

    def own_array(self, in_loop: bool):
        skip = self.lab()
        w = self.below(self.own_words)
        self.emit("ldxdw r1, [r10-24]")
        self.emit("and64 r1, 1023")
        self.emit("stxw [r10-4], r1")
        self.emit("lddw r1, map:own", 2)
        self.emit("mov64 r2, r10")
        self.emit("add64 r2, -4")
        self.emit("call map_lookup_elem")
        self.emit(f"jeq r0, 0, {skip}")
        regs = self.state_regs(in_loop)
        r = regs[self.below(len(regs))]
        c = self.below(4)
        if c == 0:
            self.emit(f"ldxdw r1, [r0+{8 * w}]")
            self.emit(f"add64 r1, {r}")
            self.emit(f"stxdw [r0+{8 * w}], r1")
            self.emit(f"xor64 {r}, r1")
        elif c == 1:
            self.emit(f"mov64 r1, {r}")
            self.emit(f"afadd64 [r0+{8 * w}], r1")
            self.emit(f"add64 {r}, r1")
        elif c == 2:
            self.emit(f"ldxw {r}, [r0+{8 * w + 4 * self.below(2)}]")
        else:
            self.emit(f"mov64 r1, {r}")
            self.emit(f"axchg64 [r0+{8 * w}], r1")
            self.emit(f"sub64 {r}, r1")
        self.emit(f"{skip}:", 0)
        self.calls += 1

    def hash_op(self, in_loop: bool):
        found, done = self.lab(), self.lab()
        regs = self.state_regs(in_loop)
        r = regs[self.below(len(regs))]
        self.emit("ldxdw r1, [r10-24]")
        self.emit("lsh64 r1, 32")
        self.emit(f"mov64 r2, {r}")
        self.emit("and64 r2, 7")
        self.emit("or64 r1, r2")
        self.emit("stxdw [r10-8], r1")
        if self.below(8) == 0:
            self.emit("lddw r1, map:hh", 2)
            self.emit("mov64 r2, r10")
            self.emit("add64 r2, -8")
            self.emit("call map_delete_elem")
            self.emit(f"add64 {r}, r0")
            self.calls += 1
            return
        self.emit("lddw r1, map:hh", 2)
        self.emit("mov64 r2, r10")
        self.emit("add64 r2, -8")
        self.emit("call map_lookup_elem")
        self.emit(f"jne r0, 0, {found}")
        self.emit(f"stxdw [r10-48], {r}")
        self.emit("ldxdw r1, [r10-32]")
        self.emit("stxdw [r10-40], r1")
        self.emit("lddw r1, map:hh", 2)
        self.emit("mov64 r2, r10")
        self.emit("add64 r2, -8")
        self.emit("mov64 r3, r10")
        self.emit("add64 r3, -48")
        self.emit(f"mov64 r4, {self.below(2)}")
        self.emit("call map_update_elem")
        self.emit(f"add64 {r}, r0")
        self.emit(f"ja {done}")
        self.emit(f"{found}:", 0)
        self.emit("ldxdw r1, [r0+0]")
        self.emit(f"add64 r1, {r}")
        self.emit("stxdw [r0+0], r1")
        self.emit("ldxdw r1, [r0+8]")
        self.emit(f"xor64 {r}, r1")
        self.emit(f"{done}:", 0)
        self.calls += 2

    def shared(self, in_loop: bool):
        skip = self.lab()
        regs = self.state_regs(in_loop)
        r = regs[self.below(len(regs))]
        self.emit(f"mov64 r1, {r}")
        self.emit("and64 r1, 255")
        self.emit("stxw [r10-4], r1")
        self.emit("lddw r1, map:sh", 2)
        self.emit("mov64 r2, r10")
        self.emit("add64 r2, -4")
        self.emit("call map_lookup_elem")
        self.emit(f"jeq r0, 0, {skip}")
        self.emit(f"mov64 r1, {r}")
        self.emit("and64 r1, 0xffff")
        self.emit(f"{self.shared_op} [r0+0], r1")
        self.emit(f"{skip}:", 0)
        self.calls += 1

    def block(self, depth: int, in_loop: bool, budget: int, mult: int):
        while self.n < budget:
            c = self.below(16)
            if c < 8:
                self.alu(in_loop)
            elif c < 10 and depth < 3:
                skip = self.lab()
                self.emit(f"{self.cond(in_loop)}, {skip}")
                self.block(depth + 1, in_loop, min(budget, self.n + 2 + self.below(8)), mult)
                self.emit(f"{skip}:", 0)
            elif c == 10 and not in_loop and depth < 2:
                trips = 1 + self.below(16)
                top = self.lab()
                self.emit("mov64 r9, 0")
                self.emit(f"{top}:", 0)
                self.block(depth + 1, True, min(budget, self.n + 3 + self.below(12)), mult * trips)
                self.emit("add64 r9, 1")
                self.emit(f"jlt r9, {trips}, {top}")
            elif c >= 11 and self.calls + 2 * mult <= self.MAX_CALLS:
                k = c - 11
                if k < 2:
                    self.own_array(in_loop)
                    self.calls += mult - 1
                elif k < 4:
                    self.hash_op(in_loop)
                    self.calls += 2 * (mult - 1)
                else:
                    self.shared(in_loop)
                    self.calls += mult - 1
            else:
                self.alu(in_loop)

    def build(self) -> str:
        self.emit("ldxdw r6, [r1+0]")
        self.emit("ldxw r7, [r1+8]")
        self.emit("ldxdw r8, [r1+16]")
        self.emit("stxdw [r10-16], r6")
        self.emit("stxdw [r10-24], r7")
        self.emit("stxdw [r10-32], r8")
        self.emit("mov64 r9, r6")
        self.emit("xor64 r9, r8")
        self.block(0, False, max(self.target - 4, self.n + 1), 1)
        self.emit("mov64 r0, r6")
        self.emit("xor64 r0, r7")
        self.emit("add64 r0, r9")
        self.emit("exit")
        return "\n".join(self.lines) + "\n"


def gen_program(seed: int) -> Policy:
    """One random, verifier-accepted program with its private maps.

    Length is floor(16 * 32**u) slots (log-uniform over [16, 512)); the body
    mixes ALU64/ALU32 operations (division and shifts by register included),
    forward branches, counted loops of at most 16 trips, owned array and hash
    lookups/updates/deletes, and commutative atomics on a shared array.
    """
    g0 = _Gen(subseed(seed, 7), 0, 1)
    u = u01(np.array([g0.rnd()], dtype=np.uint64))[0]
    target = int(math.floor(16 * 32 ** u))
    own_words = 1 + g0.below(4)
    g = _Gen(subseed(seed, 8), target, own_words)
    text = g.build()
    maps = [
        MapSpec("own", MAP_ARRAY, 4, 8 * own_words, 1024, 0),
        MapSpec("hh", MAP_HASH, 8, 16, 16384, 0),
        MapSpec("sh", MAP_ARRAY, 4, 8, 256, F_SHARED),
    ]
    return Policy(f"gen{seed}", HOOK_MEM_ACCESS, text, maps)


def batched_workload(n_programs: int = 256, seed: int = 1003, min_log2: int = 10,
                     max_log2: int = 20):
    """Programs and per-program event counts floor(2**(min + (max-min) u))."""
    progs = [gen_program(subseed(seed, 100 + i)) for i in range(n_programs)]
    u = u01(splitmix(subseed(seed, 5), n_programs))
    sizes = np.floor(2.0 ** (min_log2 + (max_log2 - min_log2) * u)).astype(np.int64)
    return progs, sizes


def serving_trace(n_requests: int, seed: int = 1004, tenants: int = 64,
                  programs: int = 32, rate_per_s: float = 20000.0,
                  min_log2: int = 8, max_log2: int = 18):
    """Open-loop Poisson arrivals: (arrival_s, tenant, program, n_events)."""
    gaps = -np.log(1.0 - u01(splitmix(subseed(seed, 1), n_requests))) / rate_per_s
    arrival = np.cumsum(gaps)
    tenant = (u01(splitmix(subseed(seed, 2), n_requests)) * tenants).astype(np.int64)
    u = u01(splitmix(subseed(seed, 3), n_requests))
    n_ev = np.floor(2.0 ** (min_log2 + (max_log2 - min_log2) * u)).astype(np.int64)
    return arrival, tenant, tenant % programs, n_ev
