"""The multi-threaded CPU baseline computes what one thread computes: the
oracle split over threads (by stream for stream-sequential programs, by
event range for event-parallel ones, merged with each shared map's
commutative operation) gives the single-threaded oracle's return codes, maps
and ring multiset."""

import numpy as np
import pytest

from runners import normalise_hash, oracle_run

from oracle import parallel as P
from paper_2512_12615_amd import workloads as W


def _shapes(pol):
    return [(m.type, m.key_size, m.value_size, m.max_entries, m.flags) for m in pol.maps]


def _check(pol, ev, event_parallel, merge_ops, init=None, T=4):
    one = oracle_run(pol, ev, init, tracking=False)
    dt, oracles, parts, rcs = P.run_parallel(pol.code, pol.hook, _shapes(pol), ev, event_parallel, T, init)
    assert dt > 0
    assert sorted(np.concatenate(parts).tolist()) == list(range(len(ev)))
    assert np.array_equal(P.gather_rc(len(ev), parts, rcs), one.rc)
    for mi, m in enumerate(pol.maps):
        if m.type == W.MAP_RINGBUF:
            assert P.merge_ring(oracles, mi) == one.rings[mi], f"ring {mi}"
        elif m.type == W.MAP_HASH:
            assert P.merge_hash(oracles, mi) == one.maps[mi], f"hash {mi}"
        else:
            init_vals = None
            if init:
                init_vals = np.zeros((m.max_entries, m.value_size), np.uint8)
                for k, key, val in init:
                    if k == mi:
                        init_vals[int.from_bytes(key, "little")] = np.frombuffer(val, np.uint8)
            assert P.merge_array(oracles, mi, merge_ops.get(mi), init_vals) == one.maps[mi], f"array {mi}"
    assert P.insns(oracles) > 0


@pytest.mark.parametrize("T", [1, 3, 8])
def test_access_counter_split_by_range(T):
    ev = W.gen_mem_uniform(20011, 5)
    _check(W.access_counter_policy(), ev, True, {0: "add"}, T=T)


def test_latency_hist_split_by_range():
    ev = W.gen_timing(30001, 6)
    init = [(1, b"\0\0\0\0", np.uint64(W.p99_threshold(ev["lat"])).tobytes())]
    _check(W.latency_hist_policy(kernels=256), ev, True, {0: "add", 1: None}, init=init, T=5)


@pytest.mark.parametrize("T", [2, 7])
def test_stride_prefetch_split_by_stream(T):
    ev = W.gen_mem_stride(40000, 7, streams=64)
    _check(W.stride_prefetch_policy(), ev, False, {}, T=T)


def test_wave_monitor_split_at_tiles():
    ev = W.gen_mem_wave(64 * 300 + 17, 8)
    _check(W.wave_monitor_policy(), ev, True, {0: "add", 1: "add"}, T=6)


def test_split_keeps_each_stream_in_one_part_in_order():
    ev = W.gen_mem_uniform(5000, 9, streams=100)
    parts = P.split(ev, W.HOOK_MEM_ACCESS, False, 7)
    for p in parts:
        assert np.all(np.diff(p) > 0)
        assert len(set((ev["stream"][p] % 7).tolist())) <= 1
    assert P.host_threads() >= 1 and P.host_cpu_model()
