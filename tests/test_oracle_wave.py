"""The warp-leader hook in the oracle (section 4.4's warp-level execution:
one invocation per wave on the wave's aggregate), pinned to plain Python
models: the aggregate of every tile, the return code given to every record
of its tile, the monitor policy's maps and ring, and the rule that such a
program may only touch shared, read-only or ring maps (both checkers)."""

import numpy as np
import pytest

import policy_models as PM
from runners import oracle_run

from paper_2512_12615_amd import workloads as W

EMIT = """
    ldxdw r6, [r1+0]
    ldxdw r7, [r1+8]
    ldxw r8, [r1+16]
    ldxw r9, [r1+20]
    stxdw [r10-24], r6
    stxdw [r10-16], r7
    stxw [r10-8], r8
    stxw [r10-4], r9
    lddw r1, map:ring
    mov64 r2, r10
    add64 r2, -24
    mov64 r3, 24
    mov64 r4, 0
    call ringbuf_output
    mov64 r0, r8
    exit
"""


def _emit_policy():
    return W.Policy("wave_emit", W.HOOK_WAVE_MEM, EMIT, [W.MapSpec("ring", W.MAP_RINGBUF, 0, 0, 1 << 20, 0)])


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 130, 1000])
def test_tile_context_and_broadcast(n):
    ev = W.gen_mem_wave(n, 10 + n, coalesced=0.5, streams=7)
    o = oracle_run(_emit_policy(), ev)
    tiles = PM.wave_tiles(ev)
    want = sorted(int(lo).to_bytes(8, "little") + int(hi).to_bytes(8, "little") + int(k).to_bytes(4, "little") +
                  int(s).to_bytes(4, "little") for lo, hi, k, s in tiles)
    assert o.rings[0] == want
    expect_rc = np.concatenate([np.full(k, k, np.uint32) for _, _, k, _ in tiles]) if tiles else np.zeros(0, np.uint32)
    assert np.array_equal(o.rc, expect_rc)
    assert o.stats["insns"] == 16 * len(tiles)  # one invocation per tile


def test_tile_order_does_not_matter():
    ev = W.gen_mem_wave(5000, 3)
    pol = W.wave_monitor_policy()
    a = oracle_run(pol, ev)
    b = oracle_run(pol, ev, order=2, seed=9)
    assert np.array_equal(a.rc, b.rc) and a.maps == b.maps and a.rings == b.rings


@pytest.mark.parametrize("n,co", [(64 * 37, 0.75), (100003, 0.3), (5, 1.0)])
def test_wave_monitor_matches_model(n, co):
    ev = W.gen_mem_wave(n, 21, coalesced=co)
    # some tiles span more than 4 GiB, some coalesced tiles cross a page
    o = oracle_run(W.wave_monitor_policy(), ev)
    coal, scat, ring, rc = PM.wave_monitor(ev)
    assert o.maps[0] == coal.tobytes() and o.maps[1] == scat.tobytes()
    assert o.rings[2] == ring
    assert np.array_equal(o.rc, rc)


def test_warp_leader_needs_event_parallel_maps():
    from oracle import oracle as O
    from paper_2512_12615_amd import gxbpf as G
    text = """
        ldxdw r6, [r1+0]
        stxdw [r10-8], r6
        lddw r1, map:h
        mov64 r2, r10
        add64 r2, -8
        call map_lookup_elem
        mov64 r0, 0
        exit
    """
    own = W.Policy("wave_hash", W.HOOK_WAVE_MEM, text, [W.MapSpec("h", W.MAP_HASH, 8, 8, 64, 0)])
    shapes = [(m.type, m.key_size, m.value_size, m.max_entries, m.flags) for m in own.maps]
    assert not O.check(own.code, own.hook, shapes).ok
    assert not G.verify(own.code, own.hook, shapes)[0]
    ro = [(W.MAP_HASH, 8, 8, 64, W.F_READ_ONLY)]
    assert O.check(own.code, own.hook, ro).ok and G.verify(own.code, own.hook, ro)[0]
    # per-record field offsets of the memory hook are not the wave context's
    bad = W.Policy("wave_bad", W.HOOK_WAVE_MEM, "ldxw r0, [r1+8]\n exit", [])
    assert not O.check(bad.code, bad.hook, []).ok and not G.verify(bad.code, bad.hook, [])[0]
