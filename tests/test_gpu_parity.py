"""GPU parity: the HIP runtime against the oracle, bit for bit (return codes,
final map contents, ring-record multisets), through the C ABI.

Small cases span several waves and a ragged tail and are compared with the
oracle element by element.  Full-size workloads are compared with the oracle
on sampled streams / events and with the closed forms that hold at any size.
"""

import numpy as np
import pytest

import policy_models as PM
from gpu_runner import gpu_run
from runners import assert_same, oracle_run

from paper_2512_12615_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture
def rt():
    from paper_2512_12615_amd import gxbpf as G
    r = G.Runtime(0)
    yield r
    r.close()


def _log(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 10007, 1 << 16])
def test_access_counter_vs_oracle(rt, n):
    _log(f"access_counter n={n}")
    pol = W.access_counter_policy()
    ev = W.gen_mem_uniform(n, 1000 + n)
    g = gpu_run(rt, pol, ev)
    assert_same(g, oracle_run(pol, ev), "access_counter")
    assert g.stats["vm_errors"] == 0


def test_access_counter_empty(rt):
    pol = W.access_counter_policy()
    g = gpu_run(rt, pol, np.zeros(0, W.MEM_DTYPE))
    assert np.frombuffer(g.maps[0], "<u8").sum() == 0


@pytest.mark.parametrize("n", [1, 100, 4099, 1 << 16])
def test_latency_hist_vs_oracle(rt, n):
    _log(f"latency_hist n={n}")
    pol = W.latency_hist_policy()
    ev = W.gen_timing(n, 1002 + n)
    T = W.p99_threshold(ev["lat"])
    init = [(1, b"\0\0\0\0", np.uint64(T).tobytes())]
    g = gpu_run(rt, pol, ev, init)
    assert_same(g, oracle_run(pol, ev, init), "latency_hist")
    assert g.stats["ring_drops"] == 0 and g.stats["vm_errors"] == 0


@pytest.mark.parametrize("n,streams", [(1, 1), (777, 8), (1 << 14, 64), (1 << 16, 1024)])
def test_stride_prefetch_vs_oracle(rt, n, streams):
    _log(f"stride_prefetch n={n} streams={streams}")
    pol = W.stride_prefetch_policy()
    ev = W.gen_mem_stride(n, 1001 + n, streams=streams)
    g = gpu_run(rt, pol, ev)
    o = oracle_run(pol, ev)
    assert_same(g, o, "stride_prefetch")
    assert g.stats["hash_e2big"] == 0 and g.stats["ring_drops"] == 0 and g.stats["vm_errors"] == 0


@pytest.mark.parametrize("i", range(8))
def test_generated_programs_vs_oracle(rt, i):
    pol = W.gen_program(W.subseed(1003, 100 + i))
    n = [100, 1000, 4096, 5000, 20000, 64, 3000, 777][i]
    _log(f"generated program {i} ({len(pol.code) // 8} slots) n={n}")
    ev = W.gen_mem_uniform(n, 700 + i)
    g = gpu_run(rt, pol, ev)
    assert_same(g, oracle_run(pol, ev), f"program {i}")
    assert g.stats["vm_errors"] == 0


def test_host_map_ops(rt):
    fd = rt.create_map(W.MAP_HASH, 8, 16, 4, 0)
    for k in [5, 1, 3]:
        assert rt.map_update(fd, np.uint64(k).tobytes(), np.array([k, 2 * k], "<u8").tobytes()) == 0
    assert rt.map_update(fd, np.uint64(5).tobytes(), bytes(16), 1) == -17
    assert rt.map_update(fd, np.uint64(9).tobytes(), bytes(16), 2) == -2
    assert rt.map_lookup(fd, np.uint64(3).tobytes()) == np.array([3, 6], "<u8").tobytes()
    assert rt.map_delete(fd, np.uint64(3).tobytes()) == 0
    assert rt.map_delete(fd, np.uint64(3).tobytes()) == -2
    assert rt.map_lookup(fd, np.uint64(3).tobytes()) is None
    assert rt.map_update(fd, np.uint64(7).tobytes(), bytes(16)) == 0
    assert rt.map_update(fd, np.uint64(8).tobytes(), bytes(16)) == 0
    assert rt.map_update(fd, np.uint64(10).tobytes(), bytes(16)) == -7   # full
    keys, vals = rt.map_dump(fd)
    assert sorted(int(x) for x in keys.view("<u8").ravel()) == [1, 5, 7, 8]
    afd = rt.create_map(W.MAP_ARRAY, 4, 8, 4, 0)
    assert rt.map_update(afd, np.uint32(2).tobytes(), np.uint64(42).tobytes()) == 0
    assert rt.map_update(afd, np.uint32(4).tobytes(), np.uint64(42).tobytes()) == -7
    assert rt.map_delete(afd, np.uint32(0).tobytes()) == -22
    assert rt.map_dump(afd)[1].view("<u8").ravel().tolist() == [0, 0, 42, 0]


def test_ring_overflow_counts_drops(rt):
    from paper_2512_12615_amd import asm
    text = """
        ldxdw r6, [r1+16]
        stxdw [r10-8], r6
        lddw r1, map:ring
        mov64 r2, r10
        add64 r2, -8
        mov64 r3, 8
        mov64 r4, 0
        call ringbuf_output
        exit
    """
    pol = W.Policy("ring", W.HOOK_MEM_ACCESS, text, [W.MapSpec("ring", W.MAP_RINGBUF, 0, 0, 4096, 0)])
    ev = np.zeros(1000, W.MEM_DTYPE)
    ev["ts"] = np.arange(1000)
    g = gpu_run(rt, pol, ev)
    ok = g.rc == 0
    assert int(ok.sum()) <= 256 and int(ok.sum()) >= 192
    assert g.stats["ring_drops"] == 1000 - int(ok.sum())
    got = sorted(int(np.frombuffer(r, "<u8")[0]) for r in g.rings[0])
    assert got == sorted(np.nonzero(ok)[0].tolist())


def test_hash_full_counts_e2big(rt):
    pol = W.stride_prefetch_policy(hash_entries=8)
    ev = W.gen_mem_stride(1000, 3, streams=64)
    g = gpu_run(rt, pol, ev)
    keys = g.maps[0]
    assert len(keys) == 8
    assert g.stats["hash_e2big"] > 0


# ---------------------------------------------------------------------------
# full-size workloads (the configurations the benchmark times)

def _floor_log2(lat):
    b = np.floor(np.log2(np.maximum(lat, 1).astype(np.float64))).astype(np.int64)
    one = np.uint64(1)
    b = np.where((b < 63) & ((one << (b + 1).astype(np.uint64)) <= lat), b + 1, b)
    b = np.where((b > 0) & ((one << b.astype(np.uint64)) > lat), b - 1, b)
    return np.where(lat == 0, 0, b)


def test_access_counter_full_size(rt):
    n = 1 << 20
    _log(f"access_counter full n={n}")
    pol = W.access_counter_policy()
    ev = W.gen_mem_uniform(n, 1000)
    g = gpu_run(rt, pol, ev)
    hist, rc = PM.access_counter(ev)
    assert np.array_equal(np.frombuffer(g.maps[0], "<u8"), hist)
    assert np.array_equal(g.rc, rc)


def test_latency_hist_full_size(rt):
    n = 1 << 26
    _log(f"latency_hist full n={n}")
    pol = W.latency_hist_policy()
    ev = W.gen_timing(n, 1002)
    T = W.p99_threshold(ev["lat"])
    g = gpu_run(rt, pol, ev, [(1, b"\0\0\0\0", np.uint64(T).tobytes())])
    b = _floor_log2(ev["lat"])
    k = ev["kernel_id"].astype(np.int64)
    hist = np.bincount(k * 64 + b, minlength=4096 * 64).astype(np.uint64)
    assert np.array_equal(np.frombuffer(g.maps[0], "<u8"), hist)
    assert np.array_equal(g.rc, b.astype(np.uint32))
    sel = ev["lat"] > np.uint64(T)
    rec = np.frombuffer(b"".join(g.rings[2]), dtype=[("k", "<u4"), ("b", "<u4"), ("l", "<u8"), ("t", "<u8"), ("z", "<u8")])
    got = np.sort(rec, order=["k", "l", "b"])
    want = np.zeros(int(sel.sum()), rec.dtype)
    want["k"], want["b"], want["l"], want["t"] = k[sel], b[sel], ev["lat"][sel], T
    want = np.sort(want, order=["k", "l", "b"])
    assert np.array_equal(got, want)
    # oracle on a sample of events (event-parallel: any subset is a valid run)
    idx = np.sort(np.random.default_rng(5).choice(n, 20000, replace=False))
    o = oracle_run(pol, ev[idx], [(1, b"\0\0\0\0", np.uint64(T).tobytes())])
    assert np.array_equal(o.rc, g.rc[idx])


def test_stride_prefetch_full_size_sampled_streams(rt):
    n = 1 << 24
    _log(f"stride_prefetch full n={n}")
    pol = W.stride_prefetch_policy()
    ev = W.gen_mem_stride(n, 1001)
    g = gpu_run(rt, pol, ev)
    assert g.stats["hash_e2big"] == 0 and g.stats["ring_drops"] == 0 and g.stats["vm_errors"] == 0
    # streams are independent: the oracle on a subset of streams reproduces
    # exactly that subset of the GPU result
    streams = np.array([0, 1, 7, 100, 511, 512, 1000, 1023], dtype=np.uint32)
    sel = np.isin(ev["stream"], streams)
    o = oracle_run(pol, ev[sel])
    assert np.array_equal(o.rc, g.rc[sel])
    keep = {int(s) for s in streams}
    gh = [(k, v) for k, v in g.maps[0] if (int.from_bytes(k, "little") >> 32) in keep]
    assert gh == o.maps[0]
    gr = sorted(r for r in g.rings[1] if int.from_bytes(r[:4], "little") in keep)
    assert gr == o.rings[1]
    # whole-run properties
    assert int(g.rc.max()) <= 8
    assert len(g.maps[0]) <= 1024 * 32


DIVERGE = """
    ldxdw r6, [r1+0]
    ldxdw r7, [r1+16]
    mov64 r0, 0
    mov64 r8, r6
    and64 r8, 7
    jeq r8, 0, early          ; 1/8 of the lanes leave at once
    mov64 r9, 0
loop:
    mov64 r2, r6
    rsh64 r2, 3
    and64 r2, 15
    jgt r2, 12, brk            ; data-dependent break out of the counted loop
    add64 r0, r2
    jset r6, 0x100, odd
    add64 r0, 3
    ja next
odd:
    xor64 r0, r7
next:
    rsh64 r6, 4
    add64 r9, 1
    jlt r9, 6, loop
brk:
    jsgt32 r0, 100, big
    mov64 r0, 1
    exit
big:
    and64 r0, 0xfff
    exit
early:
    mov64 r0, 77
    exit
"""


@pytest.mark.parametrize("n", [64, 1000, 65536])
def test_divergence_stress_vs_oracle(rt, n):
    _log(f"divergence n={n}")
    pol = W.Policy("diverge", W.HOOK_MEM_ACCESS, DIVERGE, [])
    ev = W.gen_mem_uniform(n, 31 + n)
    ev["addr"] = W.splitmix(5, n)
    g = gpu_run(rt, pol, ev)
    assert_same(g, oracle_run(pol, ev), "divergence")


CHURN = """
    ldxw r6, [r1+8]           ; stream
    ldxdw r7, [r1+0]
    mov64 r8, r6
    lsh64 r8, 32
    mov64 r2, r7
    and64 r2, 3
    or64 r8, r2               ; key = stream << 32 | (addr & 3)
    stxdw [r10-8], r8
    lddw r1, map:h
    mov64 r2, r10
    add64 r2, -8
    call map_lookup_elem
    jeq r0, 0, insert
    ldxdw r1, [r0+0]
    add64 r1, r7
    stxdw [r0+0], r1
    jset r7, 0x30, keep
    lddw r1, map:h            ; delete on a data-dependent quarter of the hits
    mov64 r2, r10
    add64 r2, -8
    call map_delete_elem
    mov64 r0, 2
    exit
keep:
    mov64 r0, 1
    exit
insert:
    stxdw [r10-16], r7
    lddw r1, map:h
    mov64 r2, r10
    add64 r2, -8
    mov64 r3, r10
    add64 r3, -16
    mov64 r4, 1
    call map_update_elem
    exit
"""


def test_hash_churn_across_launches(rt):
    """Inserts, updates and deletes on per-stream keys over several launches:
    tombstones of a launch are reclaimed only by later launches."""
    import torch
    from gpu_runner import collect, setup, to_device
    pol = W.Policy("churn", W.HOOK_MEM_ACCESS, CHURN, [W.MapSpec("h", W.MAP_HASH, 8, 8, 512, 0)])
    fds, prog = setup(rt, pol)
    from oracle import oracle as O
    o = O.Oracle()
    o.create_map(W.MAP_HASH, 8, 8, 512, 0)
    for b in range(4):
        ev = W.gen_mem_uniform(20000, 90 + b, streams=128)
        rc = torch.zeros(len(ev), dtype=torch.int32, device="cuda")
        rt.run_batch(prog, to_device(ev), n_events=len(ev), record_size=24, rc=rc)
        torch.cuda.synchronize()
        orc = o.run(pol.code, pol.hook, ev)
        assert np.array_equal(rc.cpu().numpy().view(np.uint32), orc), f"launch {b}"
        g = collect(rt, pol, fds, None)
        k, v = o.dump(0)
        from runners import normalise_hash
        assert g.maps[0] == normalise_hash(k, v), f"launch {b}"
    st = rt.stats()
    assert st["hash_e2big"] == 0 and st["vm_errors"] == 0
