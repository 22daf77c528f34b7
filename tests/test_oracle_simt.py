"""SIMT-aware verification (section 4.4): under the SIMT hook every value is
warp-uniform (the tile aggregate's fields at byte 24 and what is computed
from them) or lane-varying (the record's own fields and what they touch);
branch conditions and loop exits, map keys, ring records and flags and the
addresses of map updates must be uniform.  Both checkers (the oracle's and
the runtime's, written separately) must reject every program of the
corpus and accept the uniform ones, and the oracle's execution of the hook
is pinned to a plain Python model of the per-record context."""

import numpy as np
import pytest

from runners import oracle_run

from oracle import oracle as O
from paper_2512_12615_amd import gxbpf as G
from paper_2512_12615_amd import workloads as W

SH = (W.MAP_ARRAY, 4, 8, 4096, W.F_SHARED)
RO = (W.MAP_ARRAY, 4, 8, 4096, W.F_READ_ONLY)
RING = (W.MAP_RINGBUF, 0, 0, 1 << 22, 0)
OWN = (W.MAP_HASH, 8, 8, 1024, 0)

LOOKUP_UNIFORM = """
    ldxw r6, [r1+44]
    and64 r6, 4095
    stxw [r10-4], r6
    lddw r1, map:m
    mov64 r2, r10
    add64 r2, -4
    call map_lookup_elem
    jeq r0, 0, out
"""

REJECTS = {
    # a branch on the record's address
    "branch_on_lane_field": ("""
        ldxdw r6, [r1+0]
        mov64 r0, 0
        jgt r6, 100, out
        mov64 r0, 1
    out:
        exit
    """, [SH]),
    # lane variance flows through arithmetic, even when the result is constant
    "branch_through_arithmetic": ("""
        ldxdw r6, [r1+16]
        and64 r6, 0
        mov64 r0, 0
        jeq r6, 0, out
        mov64 r0, 1
    out:
        exit
    """, [SH]),
    # through a stack slot
    "branch_through_stack": ("""
        ldxw r6, [r1+8]
        stxdw [r10-8], r6
        ldxdw r7, [r10-8]
        mov64 r0, 0
        jne r7, 3, out
        mov64 r0, 1
    out:
        exit
    """, [SH]),
    # a counted loop left early on a lane-varying condition
    "loop_exit_on_lane_field": ("""
        ldxdw r6, [r1+0]
        mov64 r0, 0
        mov64 r2, 0
    head:
        jgt r6, r2, out
        add64 r0, 1
        add64 r2, 1
        jlt r2, 8, head
    out:
        exit
    """, [SH]),
    # a map key made from the record
    "map_key_from_lane_field": ("""
        ldxdw r6, [r1+0]
        rsh64 r6, 21
        and64 r6, 4095
        stxw [r10-4], r6
        lddw r1, map:m
        mov64 r2, r10
        add64 r2, -4
        call map_lookup_elem
        jeq r0, 0, out
        mov64 r1, 1
        aadd64 [r0+0], r1
    out:
        mov64 r0, 0
        exit
    """, [SH]),
    # a map update at a lane-varying address (uniform key, varying offset)
    "atomic_at_lane_varying_address": ("""
        ldxdw r8, [r1+0]
""" + LOOKUP_UNIFORM + """
        and64 r8, 0
        add64 r0, r8
        mov64 r1, 1
        aadd64 [r0+0], r1
    out:
        mov64 r0, 0
        exit
    """, [SH]),
    # a ring record holding a lane-varying value
    "ring_record_from_lane_field": ("""
        ldxdw r6, [r1+0]
        stxdw [r10-8], r6
        lddw r1, map:m
        mov64 r2, r10
        add64 r2, -8
        mov64 r3, 8
        mov64 r4, 0
        call ringbuf_output
        mov64 r0, 0
        exit
    """, [RING]),
    # ringbuf_output flags computed from the record
    "ring_flags_from_lane_field": ("""
        ldxdw r6, [r1+24]
        stxdw [r10-8], r6
        ldxdw r7, [r1+0]
        and64 r7, 0
        lddw r1, map:m
        mov64 r2, r10
        add64 r2, -8
        mov64 r3, 8
        mov64 r4, r7
        call ringbuf_output
        mov64 r0, 0
        exit
    """, [RING]),
    # a read-only map value read at a lane-varying offset decides a branch
    "branch_on_value_read_at_lane_offset": ("""
        ldxdw r8, [r1+16]
""" + LOOKUP_UNIFORM + """
        and64 r8, 0
        add64 r0, r8
        ldxdw r6, [r0+0]
        jeq r6, 0, out
    out:
        mov64 r0, 0
        exit
    """, [RO]),
    # owned state: the SIMT hook runs a wave's events at once
    "owned_map": ("""
        ldxw r6, [r1+44]
        stxdw [r10-8], r6
        stdw [r10-16], 1
        lddw r1, map:m
        mov64 r2, r10
        add64 r2, -8
        mov64 r3, r10
        add64 r3, -16
        mov64 r4, 0
        call map_update_elem
        mov64 r0, 0
        exit
    """, [OWN]),
}

ACCEPTS = {
    # branches, keys and records from the tile aggregate; varying addend and rc
    "uniform_control_varying_addend": ("""
        ldxdw r8, [r1+0]
        ldxdw r9, [r1+32]
        ldxdw r7, [r1+24]
        sub64 r9, r7
""" + LOOKUP_UNIFORM + """
        mov64 r1, r8
        and64 r1, 4095
        aadd64 [r0+0], r1
    out:
        mov64 r0, r8
        and64 r0, 7
        jgt r9, 4095, wide
        exit
    wide:
        add64 r0, 8
        exit
    """, [SH]),
    "uniform_ring_record": ("""
        mov64 r9, r1
        ldxdw r6, [r1+24]
        stxdw [r10-16], r6
        ldxw r7, [r1+40]
        stxdw [r10-8], r7
        mov64 r0, 0
        jlt r7, 64, out
        lddw r1, map:m
        mov64 r2, r10
        add64 r2, -16
        mov64 r3, 16
        mov64 r4, 0
        call ringbuf_output
    out:
        ldxdw r0, [r9+0]
        exit
    """, [RING]),
}


def _both(text, shapes):
    names = ["m", "n", "r"][:len(shapes)]
    pol = W.Policy("t", W.HOOK_SIMT_MEM, text, [W.MapSpec(nm, *sh) for nm, sh in zip(names, shapes)])
    ok, log, _ = G.verify(pol.code, pol.hook, shapes)
    r = O.check(pol.code, pol.hook, shapes)
    return pol, ok, log, r


@pytest.mark.parametrize("name", sorted(REJECTS))
def test_both_checkers_reject(name):
    text, shapes = REJECTS[name]
    _, ok, log, r = _both(text, shapes)
    assert not ok, f"runtime verifier accepted {name}"
    assert not r.ok, f"oracle checker accepted {name}"
    if name != "owned_map":
        assert "SIMT" in log and "SIMT" in r.log, (log, r.log)


@pytest.mark.parametrize("name", sorted(REJECTS))
def test_the_same_programs_pass_as_per_record_hooks(name):
    """Every rejection above is the SIMT rule's: as a plain per-record
    program (no uniformity rules) each is accepted, except the ones that
    read the aggregate's fields, which the per-record context lacks."""
    text, shapes = REJECTS[name]
    names = ["m", "n", "r"][:len(shapes)]
    pol = W.Policy("t", W.HOOK_MEM_ACCESS, text, [W.MapSpec(nm, *sh) for nm, sh in zip(names, shapes)])
    uses_aggregate = any(f"[r1+{o}]" in text for o in (24, 32, 40, 44))
    assert O.check(pol.code, pol.hook, shapes).ok == (not uses_aggregate)
    assert G.verify(pol.code, pol.hook, shapes)[0] == (not uses_aggregate)


@pytest.mark.parametrize("name", sorted(ACCEPTS))
def test_both_checkers_accept(name):
    text, shapes = ACCEPTS[name]
    _, ok, log, r = _both(text, shapes)
    assert ok, log
    assert r.ok, r.log
    assert r.event_parallel


def test_wave_count_handlers_are_accepted_and_agree():
    for simt in (False, True):
        pol = W.wave_counts_policy(simt)
        shapes = [(m.type, m.key_size, m.value_size, m.max_entries, m.flags) for m in pol.maps]
        assert G.verify(pol.code, pol.hook, shapes)[0] and O.check(pol.code, pol.hook, shapes).ok
    ev = W.gen_mem_wave(64 * 50 + 7, 11)
    a = oracle_run(W.wave_counts_policy(False), ev)
    b = oracle_run(W.wave_counts_policy(True), ev)
    assert np.array_equal(a.rc, b.rc) and a.maps == b.maps
    total = sum(int(np.frombuffer(m, "<u8").sum()) for m in b.maps)
    assert total == len(ev)


CTX_ECHO = """
    ldxdw r6, [r1+{off}]
    mov64 r0, r6
    exit
"""


@pytest.mark.parametrize("off,size", [(0, 8), (8, 4), (16, 8), (24, 8), (32, 8), (40, 4), (44, 4)])
def test_context_is_record_then_tile_aggregate(off, size):
    """Each record's context: its own fields, then its tile's aggregate
    (lowest and highest address of the tile's records, their count, the
    first record's stream), computed here from the records directly."""
    op = "ldxdw" if size == 8 else "ldxw"
    text = CTX_ECHO.replace("ldxdw", op).format(off=off)
    pol = W.Policy("echo", W.HOOK_SIMT_MEM, text, [])
    ev = W.gen_mem_wave(64 * 9 + 21, 12)
    got = oracle_run(pol, ev).rc
    n = len(ev)
    tile = np.arange(n) // 64
    lo = np.array([ev["addr"][t * 64:t * 64 + 64].min() for t in range(tile.max() + 1)])[tile]
    hi = np.array([ev["addr"][t * 64:t * 64 + 64].max() for t in range(tile.max() + 1)])[tile]
    cnt = np.array([len(ev[t * 64:t * 64 + 64]) for t in range(tile.max() + 1)])[tile]
    s0 = ev["stream"][(tile * 64)]
    want = {0: ev["addr"], 8: ev["stream"], 16: ev["ts"], 24: lo, 32: hi, 40: cnt, 44: s0}[off]
    assert np.array_equal(got, (np.asarray(want).astype(np.uint64) & np.uint64(0xFFFFFFFF)).astype(np.uint32))
