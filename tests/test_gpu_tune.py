"""Autotuner: trials leave no trace (maps, rings and counters as before),
and runs with the chosen launch shape still match the oracle."""

import numpy as np
import pytest

from gpu_runner import collect, setup, to_device
from runners import assert_same, oracle_run

from paper_2512_12615_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture
def rt():
    from paper_2512_12615_amd import gxbpf as G
    r = G.Runtime(0)
    yield r
    r.close()


@pytest.mark.parametrize("jit", [False, True])
def test_autotune_stream_sequential(rt, jit):
    import torch
    print(f"autotune stride prefetch jit={jit}", flush=True)
    pol = W.stride_prefetch_policy()
    fds, prog = setup(rt, pol, jit=jit)
    warm = W.gen_mem_stride(1 << 14, 5, streams=256)
    ev = W.gen_mem_stride(1 << 16, 6, streams=256)
    # some state before tuning
    rc0 = torch.zeros(len(warm), dtype=torch.int32, device="cuda")
    rt.run_batch(prog, to_device(warm), n_events=len(warm), record_size=24, rc=rc0)
    torch.cuda.synchronize()
    before = [rt.map_dump(fds[0])]
    stats0 = rt.stats()
    d = to_device(ev)
    rc = torch.zeros(len(ev), dtype=torch.int32, device="cuda")
    t = rt.autotune(prog, d, n_events=len(ev), record_size=24, rc=rc)
    assert t["trials"] == 22 and 1 <= t["lanes"] <= 64 and 10 <= t["qbits"] <= 14
    assert t["best_ms"] <= t["default_ms"] + 1e-9
    after = [rt.map_dump(fds[0])]
    assert all(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) for a, b in zip(before, after))
    assert rt.stats() == stats0
    # the ring holds exactly the warm-up's records; then a real run with the tuned shape
    rt.run_batch(prog, d, n_events=len(ev), record_size=24, rc=rc)
    torch.cuda.synchronize()
    g = collect(rt, pol, fds, rc.cpu().numpy().view(np.uint32))
    from oracle import oracle as O
    o = O.Oracle()
    for m in pol.maps:
        o.create_map(m.type, m.key_size, m.value_size, m.max_entries, m.flags)
    o.run(pol.code, pol.hook, warm)
    orc = o.run(pol.code, pol.hook, ev)
    assert np.array_equal(g.rc, orc)
    from runners import normalise_hash
    k, v = o.dump(0)
    assert g.maps[0] == normalise_hash(k, v)
    assert g.rings[1] == sorted(o.drain(1))


def test_autotune_event_parallel_compiled(rt):
    import torch
    print("autotune access counter compiled", flush=True)
    pol = W.access_counter_policy()
    fds, prog = setup(rt, pol, jit=True)
    ev = W.gen_mem_uniform(1 << 18, 9)
    d = to_device(ev)
    t = rt.autotune(prog, d, n_events=len(ev), record_size=24)
    assert t["trials"] == 9  # the default and 64..8192 blocks
    assert np.frombuffer(rt.map_dump(fds[0])[1].tobytes(), "<u8").sum() == 0
    rc = torch.zeros(len(ev), dtype=torch.int32, device="cuda")
    rt.run_batch(prog, d, n_events=len(ev), record_size=24, rc=rc)
    torch.cuda.synchronize()
    g = collect(rt, pol, fds, rc.cpu().numpy().view(np.uint32))
    assert_same(g, oracle_run(pol, ev), "access_counter tuned")


def test_autotune_batches_leaves_no_trace(rt):
    """The batched form's tuner times the batch with each waves-per-CU
    candidate; the maps are as before it, and the next batched run (with the
    choice) matches the oracle."""
    import torch
    print("autotune batches", flush=True)
    progs, sizes = W.batched_workload(12, seed=77, min_log2=8, max_log2=13)
    runs = [(p, W.gen_mem_uniform(int(n), 700 + i)) for i, (p, n) in enumerate(zip(progs, sizes))]
    runs.append((W.access_counter_policy(), W.gen_mem_uniform(9000, 71)))
    descs, keep = [], []
    for pol, ev in runs:
        fds, prog = setup(rt, pol)
        rc = torch.zeros(len(ev), dtype=torch.int32, device="cuda")
        descs.append((prog, to_device(ev), len(ev), pol.record_size, rc))
        keep.append((pol, ev, fds, rc))
    before = [[rt.map_dump(fd) if m.type != W.MAP_RINGBUF else None for fd, m in zip(fds, pol.maps)]
              for pol, ev, fds, rc in keep]
    t = rt.autotune_batches(descs)
    assert t["waves_per_cu"] in (2, 4, 8, 16, 32) and t["trials"] == 5 and t["best_ms"] > 0
    after = [[rt.map_dump(fd) if m.type != W.MAP_RINGBUF else None for fd, m in zip(fds, pol.maps)]
             for pol, ev, fds, rc in keep]
    for b, a in zip(before, after):
        for x, y in zip(b, a):
            if x is not None:
                assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
    rt.run_batches(descs)
    torch.cuda.synchronize()
    for pol, ev, fds, rc in keep:
        g = collect(rt, pol, fds, rc.cpu().numpy().view(np.uint32))
        assert_same(g, oracle_run(pol, ev), pol.name)
