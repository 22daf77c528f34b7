"""Hierarchical maps (section 4.4): the host tier (read-only maps in pinned
host memory that the device reads through their mapped address) gives the
oracle's results on both engines; host snapshots taken by the daemon thread
between runs are always the map's state after some prefix of the runs, and
after a flush equal the exact map."""

import numpy as np
import pytest

from gpu_runner import gpu_run, setup, to_device
from runners import assert_same, normalise_hash, oracle_run

from paper_2512_12615_amd import workloads as W

pytestmark = pytest.mark.gpu

F_HOST = 4


@pytest.fixture
def rt():
    from paper_2512_12615_amd import gxbpf as G
    r = G.Runtime(0)
    yield r
    r.close()


@pytest.mark.parametrize("jit", [False, True], ids=["interpreted", "compiled"])
def test_latency_hist_with_host_tier_threshold(rt, jit):
    print(f"host tier threshold jit={jit}", flush=True)
    pol = W.latency_hist_policy()
    pol.maps[1] = W.MapSpec("cfg", W.MAP_ARRAY, 4, 8, 1, W.F_READ_ONLY | F_HOST)
    ev = W.gen_timing(50001, 77)
    init = [(1, b"\0\0\0\0", np.uint64(W.p99_threshold(ev["lat"])).tobytes())]
    g = gpu_run(rt, pol, ev, init, jit=jit)
    assert_same(g, oracle_run(pol, ev, init), "latency_hist")


HOST_HASH = """
    ldxdw r6, [r1+0]
    rsh64 r6, 30
    stxdw [r10-8], r6
    lddw r1, map:cold
    mov64 r2, r10
    add64 r2, -8
    call map_lookup_elem
    mov64 r7, 0
    jeq r0, 0, out
    ldxdw r7, [r0+0]
out:
    mov64 r0, r7
    exit
"""


@pytest.mark.parametrize("jit", [False, True], ids=["interpreted", "compiled"])
def test_host_tier_hash_lookups(rt, jit):
    print(f"host tier hash jit={jit}", flush=True)
    pol = W.Policy("cold", W.HOOK_MEM_ACCESS, HOST_HASH,
                   [W.MapSpec("cold", W.MAP_HASH, 8, 8, 1024, W.F_READ_ONLY | F_HOST)])
    init = [(0, int(k).to_bytes(8, "little"), int(k * 7919 + 3).to_bytes(8, "little")) for k in range(0, 8, 2)]
    ev = W.gen_mem_uniform(20000, 78)
    g = gpu_run(rt, pol, ev, init, jit=jit)
    assert_same(g, oracle_run(pol, ev, init), "cold hash")
    assert (g.rc != 0).any() and (g.rc == 0).any()


def test_snapshots_are_prefixes_of_the_runs(rt):
    """40 access-counter runs over distinct batches on one stream, with the
    daemon copying every 200 us: every snapshot read meanwhile equals the
    histogram after some number of whole runs (never a torn or partial one),
    versions never go back, and after a flush the snapshot is the final map."""
    import torch
    print("snapshots are prefixes", flush=True)
    pol = W.access_counter_policy()
    fds, prog = setup(rt, pol, jit=True)
    stream = torch.cuda.current_stream()
    hosts = [W.gen_mem_uniform(1 << 18, 900 + k) for k in range(40)]
    dev = [to_device(h) for h in hosts]
    prefix = [np.zeros(4096, np.uint64)]
    for h in hosts:
        prefix.append(prefix[-1] + np.bincount((h["addr"] >> np.uint64(21)).astype(np.int64), minlength=4096).astype(np.uint64))
    index = {p.tobytes(): j for j, p in enumerate(prefix)}
    rt.snapshot_start([fds[0]], interval_us=200, stream=stream)
    seen, last_ver, last_j = 0, 0, 0
    for k in range(40):
        rt.run_batch(prog, dev[k], n_events=len(hosts[k]), record_size=24, stream=stream)
        _, vals, ver = rt.snapshot_read(fds[0])
        if ver:
            j = index.get(np.frombuffer(vals.tobytes(), "<u8").tobytes())
            assert j is not None, f"snapshot {ver} is not the state after whole runs"
            assert ver >= last_ver and j >= last_j
            last_ver, last_j, seen = ver, j, seen + 1
    rt.snapshot_flush()
    _, vals, ver = rt.snapshot_read(fds[0])
    assert np.array_equal(np.frombuffer(vals.tobytes(), "<u8"), prefix[-1])
    assert ver > last_ver
    rt.snapshot_stop()
    torch.cuda.synchronize()
    _, vals = rt.map_dump(fds[0])
    assert np.array_equal(np.frombuffer(vals.tobytes(), "<u8"), prefix[-1])


def test_snapshot_of_a_hash_map_after_flush(rt):
    import torch
    print("snapshot of the stride policy's hash map", flush=True)
    pol = W.stride_prefetch_policy()
    fds, prog = setup(rt, pol, jit=True)
    stream = torch.cuda.current_stream()
    rt.snapshot_start([fds[0]], interval_us=500, stream=stream)
    for b in range(4):
        ev = W.gen_mem_stride(1 << 16, 60 + b, streams=256)
        rt.run_batch(prog, to_device(ev), n_events=len(ev), record_size=24, stream=stream)
    rt.snapshot_flush()
    k, v, ver = rt.snapshot_read(fds[0])
    assert ver >= 1
    rt.snapshot_stop()
    kd, vd = rt.map_dump(fds[0])
    assert normalise_hash(k, v) == normalise_hash(kd, vd) and len(kd) > 0
