"""Pins for the oracle on the three policies and on the map/ring semantics.

* Access counter and latency histogram: closed forms (numpy bincount of the
  region / of kernel_id*64 + floor(log2 latency); return codes; ring records
  are exactly the events above the threshold).
* Stride prefetch: an independent Python model of the policy (no eBPF).
* Determinism: other serialisations that keep each stream's order give the
  same result (and, for event-parallel programs, any permutation does).
* Map helper error codes, ring overflow, hash capacity, ownership tracking.
"""

import numpy as np
import pytest

import policy_models as PM
from runners import assert_same, normalise_hash, oracle_run

from paper_2512_12615_amd import asm
from paper_2512_12615_amd import workloads as W


def test_access_counter_closed_form():
    pol = W.access_counter_policy()
    ev = W.gen_mem_uniform(1 << 18, 1000)
    res = oracle_run(pol, ev)
    hist, rc = PM.access_counter(ev)
    assert np.array_equal(np.frombuffer(res.maps[0], "<u8"), hist)
    assert np.array_equal(res.rc, rc)
    assert int(hist.sum()) == len(ev)
    assert res.stats["faults"] == 0 and res.stats["violations"] == 0


def test_latency_hist_closed_form():
    pol = W.latency_hist_policy()
    ev = W.gen_timing(1 << 17, 1002)
    T = W.p99_threshold(ev["lat"])
    assert T == PM.percentile_threshold(ev["lat"])
    res = oracle_run(pol, ev, init=[(1, b"\0\0\0\0", np.uint64(T).tobytes())])
    hist, b, records = PM.latency_hist(ev, T)
    assert np.array_equal(np.frombuffer(res.maps[0], "<u8").reshape(4096, 64), hist)
    assert np.array_equal(res.rc, b)
    got = sorted(tuple(np.frombuffer(r, "<u4,<u4,<u8,<u8,<u8")[0].tolist()) for r in res.rings[2])
    assert got == records
    assert len(records) == int((ev["lat"] > T).sum()) > 0
    assert res.stats["drops"] == 0 and res.stats["faults"] == 0


def test_stride_prefetch_model():
    pol = W.stride_prefetch_policy()
    ev = W.gen_mem_stride(1 << 15, 1001, streams=64)
    res = oracle_run(pol, ev)
    rc, state, records = PM.stride_prefetch(ev)
    assert np.array_equal(res.rc, rc)
    want = sorted((np.uint64(k).tobytes(),
                   np.array([v[0], v[1]], "<u8").tobytes() + np.array([v[2], 0], "<u4").tobytes())
                  for k, v in state.items())
    assert res.maps[0] == want
    got = sorted(tuple(np.frombuffer(r, "<u4,<u4,<u8,<u8,<u8")[0].tolist()) for r in res.rings[1])
    assert got == sorted(records)
    assert len(records) > 10 and rc.max() <= 8
    st = res.stats
    assert st["faults"] == 0 and st["violations"] == 0 and st["e2big"] == 0 and st["drops"] == 0


def test_stride_prefetch_records_stay_in_region():
    ev = W.gen_mem_stride(1 << 14, 77, streams=16)
    _, _, records = PM.stride_prefetch(ev)
    for s, n, first, dpage, ts in records:
        d = dpage if dpage < (1 << 63) else dpage - (1 << 64)
        pages = [(first >> 12) + k * (d >> 12) for k in range(n)]
        assert len({p >> 9 for p in pages}) == 1 and all(0 <= p < (1 << 18) for p in pages)


@pytest.mark.parametrize("order", [1, 3])
def test_stream_serialisations_agree(order):
    pol = W.stride_prefetch_policy()
    ev = W.gen_mem_stride(1 << 14, 5, streams=32)
    assert_same(oracle_run(pol, ev), oracle_run(pol, ev, order=order), f"order {order}")


@pytest.mark.parametrize("order", [1, 2, 3])
def test_event_parallel_orders_agree(order):
    for pol, ev, init in [
        (W.access_counter_policy(), W.gen_mem_uniform(1 << 14, 3), None),
        (W.latency_hist_policy(), W.gen_timing(1 << 14, 4), [(1, b"\0\0\0\0", np.uint64(50000).tobytes())]),
    ]:
        assert_same(oracle_run(pol, ev, init), oracle_run(pol, ev, init, order=order, seed=99), pol.name)


def test_generated_programs_deterministic_and_clean():
    for i in range(12):
        pol = W.gen_program(W.subseed(1003, 100 + i))
        ev = W.gen_mem_uniform(2048, 500 + i)
        a = oracle_run(pol, ev)
        st = a.stats
        assert st["faults"] == 0, (i, st["fault_msg"])
        assert st["violations"] == 0 and st["e2big"] == 0, (i, st)
        for order in (1, 3):
            assert_same(a, oracle_run(pol, ev, order=order), f"program {i} order {order}")


# ---------------------------------------------------------------------------
# helper semantics (Linux errno values)

def _helper_prog(body, maps):
    return asm.assemble(body + "\nexit", maps)


def _run1(body, shapes, init=()):
    from oracle import oracle as O
    o = O.Oracle()
    for s in shapes:
        assert o.create_map(*s) >= 0
    for mi, k, v in init:
        o.update(mi, k, v)
    rc = o.run(_helper_prog(body, ["m", "r"][:len(shapes)]), W.HOOK_MEM_ACCESS, np.zeros(1, W.MEM_DTYPE))
    st = o.stats()
    assert st["faults"] == 0, st["fault_msg"]
    return np.int32(rc[0]).item(), o


UPD = """
    stdw [r10-8], {key}
    stdw [r10-24], 7
    stdw [r10-16], 9
    lddw r1, map:m
    mov64 r2, r10
    add64 r2, -8
    mov64 r3, r10
    add64 r3, -24
    mov64 r4, {flags}
    call map_update_elem
    mov64 r0, r0
"""
HASH16 = (W.MAP_HASH, 8, 16, 2, 0)


@pytest.mark.parametrize("flags,present,want", [
    (0, False, 0), (0, True, 0), (1, False, 0), (1, True, -17), (2, False, -2), (2, True, 0), (3, False, -22),
])
def test_hash_update_flags(flags, present, want):
    init = [(0, np.uint64(5).tobytes(), bytes(16))] if present else []
    rc, o = _run1(UPD.format(key=5, flags=flags), [HASH16], init)
    assert rc == want


def test_hash_full_gives_e2big():
    init = [(0, np.uint64(1).tobytes(), bytes(16)), (0, np.uint64(2).tobytes(), bytes(16))]
    rc, o = _run1(UPD.format(key=5, flags=0), [HASH16], init)
    assert rc == -7 and o.stats()["e2big"] == 1
    rc, o = _run1(UPD.format(key=2, flags=0), [HASH16], init)  # existing key still updates
    assert rc == 0


@pytest.mark.parametrize("key,flags,want", [(0, 0, 0), (0, 2, 0), (0, 1, -17), (16, 0, -7), (0, 5, -22)])
def test_array_update(key, flags, want):
    body = UPD.replace("stdw [r10-8], {key}", "stw [r10-8], {key}")
    rc, _ = _run1(body.format(key=key, flags=flags), [(W.MAP_ARRAY, 4, 16, 16, 0)])
    assert rc == want


def test_delete_semantics():
    body = """
        stdw [r10-8], {key}
        lddw r1, map:m
        mov64 r2, r10
        add64 r2, -8
        call map_delete_elem
        mov64 r0, r0
    """
    rc, o = _run1(body.format(key=5), [HASH16], [(0, np.uint64(5).tobytes(), bytes(16))])
    assert rc == 0 and len(o.dump(0)[0]) == 0
    rc, _ = _run1(body.format(key=6), [HASH16], [(0, np.uint64(5).tobytes(), bytes(16))])
    assert rc == -2
    rc, _ = _run1(body.replace("stdw [r10-8]", "stw [r10-8]").format(key=0), [(W.MAP_ARRAY, 4, 8, 4, 0)])
    assert rc == -22


def test_array_lookup_out_of_range_is_null():
    body = """
        stw [r10-4], {idx}
        lddw r1, map:m
        mov64 r2, r10
        add64 r2, -4
        call map_lookup_elem
        mov64 r1, r0
        mov64 r0, 1
        jne r1, 0, out
        mov64 r0, 0
    out:
    """
    assert _run1(body.format(idx=3), [(W.MAP_ARRAY, 4, 8, 4, 0)])[0] == 1
    assert _run1(body.format(idx=4), [(W.MAP_ARRAY, 4, 8, 4, 0)])[0] == 0


RING_OUT = """
    stdw [r10-8], {v}
    lddw r1, map:m
    mov64 r2, r10
    add64 r2, -{sz}
    mov64 r3, {sz}
    mov64 r4, {flags}
    call ringbuf_output
    mov64 r0, r0
"""


def test_ring_overflow_counts_drops_and_stays_parseable():
    from oracle import oracle as O
    o = O.Oracle()
    o.create_map(W.MAP_RINGBUF, 0, 0, 4096, 0)
    code = asm.assemble("ldxdw r6, [r1+16]\n" + RING_OUT.format(v=0, sz=8, flags=0).replace("stdw [r10-8], 0", "stxdw [r10-8], r6") + "\nexit", ["m"])
    ev = np.zeros(300, W.MEM_DTYPE)
    ev["ts"] = np.arange(300)
    rc = o.run(code, W.HOOK_MEM_ACCESS, ev)
    # each record takes 8 + 8 bytes: 256 fit in 4096 bytes
    assert int((rc == 0).sum()) == 256 and int((rc.view(np.int32) == -11).sum()) == 44
    assert o.stats()["drops"] == 44
    recs = o.drain(0)
    assert [int(np.frombuffer(r, "<u8")[0]) for r in recs] == list(range(256))


def test_ring_flags_must_be_zero():
    from oracle import oracle as O
    rc, _ = _run1(RING_OUT.format(v=1, sz=8, flags=1), [(W.MAP_RINGBUF, 0, 0, 4096, 0)])
    assert rc == -22


def test_ring_odd_size_payload():
    body = RING_OUT.format(v=0, sz=5, flags=0).replace("add64 r2, -5", "add64 r2, -8")
    body = body.replace("stdw [r10-8], 0", "lddw r6, 0x0102030405060708\nstxdw [r10-8], r6")
    rc, o = _run1(body, [(W.MAP_RINGBUF, 0, 0, 4096, 0)])
    assert rc == 0
    assert o.drain(0) == [bytes([8, 7, 6, 5, 4])]


def test_ownership_violation_detected():
    # every event writes array slot 0: two streams touching a written slot
    text = """
        stw [r10-4], 0
        lddw r1, map:m
        mov64 r2, r10
        add64 r2, -4
        call map_lookup_elem
        jeq r0, 0, out
        stdw [r0+0], 1
    out:
        mov64 r0, 0
        exit
    """
    pol = W.Policy("racy", W.HOOK_MEM_ACCESS, text, [W.MapSpec("m", W.MAP_ARRAY, 4, 8, 4, 0)])
    ev = np.zeros(4, W.MEM_DTYPE)
    ev["stream"] = [0, 1, 0, 1]
    assert oracle_run(pol, ev).stats["violations"] == 1
    ev["stream"] = 3
    assert oracle_run(pol, ev).stats["violations"] == 0


def test_host_map_ops_and_dump():
    from oracle import oracle as O
    o = O.Oracle()
    o.create_map(W.MAP_HASH, 8, 8, 4, 0)
    for k in [5, 1, 3]:
        assert o.update(0, np.uint64(k).tobytes(), np.uint64(k * 10).tobytes()) == 0
    assert o.lookup(0, np.uint64(3).tobytes()) == np.uint64(30).tobytes()
    assert o.delete(0, np.uint64(3).tobytes()) == 0
    assert o.lookup(0, np.uint64(3).tobytes()) is None
    keys, vals = o.dump(0)
    assert normalise_hash(keys, vals) == sorted((np.uint64(k).tobytes(), np.uint64(k * 10).tobytes()) for k in [1, 5])
    assert o.create_map(W.MAP_ARRAY, 8, 8, 4, 0) < 0          # array keys are u32
    assert o.create_map(W.MAP_RINGBUF, 0, 0, 5000, 0) < 0     # ring size power of two
    assert o.create_map(W.MAP_ARRAY, 4, 8, 4, W.F_SHARED | W.F_READ_ONLY) < 0
