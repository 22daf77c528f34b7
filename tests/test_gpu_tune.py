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
    assert t["trials"] == 7
    assert np.frombuffer(rt.map_dump(fds[0])[1].tobytes(), "<u8").sum() == 0
    rc = torch.zeros(len(ev), dtype=torch.int32, device="cuda")
    rt.run_batch(prog, d, n_events=len(ev), record_size=24, rc=rc)
    torch.cuda.synchronize()
    g = collect(rt, pol, fds, rc.cpu().numpy().view(np.uint32))
    assert_same(g, oracle_run(pol, ev), "access_counter tuned")
