"""GPU parity of programs compiled to native gfx950 code: the same cases as
the interpreter's parity tests, with the program compiled at load time, must
give exactly the oracle's results."""

import numpy as np
import pytest

from gpu_runner import collect, gpu_run, setup, to_device
from runners import assert_same, normalise_hash, oracle_run
from test_gpu_parity import CHURN, DIVERGE

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


@pytest.mark.parametrize("n", [1, 65, 10007, 1 << 16])
def test_jit_access_counter(rt, n):
    _log(f"jit access_counter n={n}")
    pol = W.access_counter_policy()
    ev = W.gen_mem_uniform(n, 1000 + n)
    g = gpu_run(rt, pol, ev, jit=True)
    assert_same(g, oracle_run(pol, ev), "access_counter")
    assert g.stats["vm_errors"] == 0


@pytest.mark.parametrize("n", [1, 4099, 1 << 16])
def test_jit_latency_hist(rt, n):
    _log(f"jit latency_hist n={n}")
    pol = W.latency_hist_policy()
    ev = W.gen_timing(n, 1002 + n)
    init = [(1, b"\0\0\0\0", np.uint64(W.p99_threshold(ev["lat"])).tobytes())]
    g = gpu_run(rt, pol, ev, init, jit=True)
    assert_same(g, oracle_run(pol, ev, init), "latency_hist")
    assert g.stats["ring_drops"] == 0 and g.stats["vm_errors"] == 0


@pytest.mark.parametrize("n,streams", [(1, 1), (777, 8), (1 << 16, 1024)])
def test_jit_stride_prefetch(rt, n, streams):
    _log(f"jit stride_prefetch n={n} streams={streams}")
    pol = W.stride_prefetch_policy()
    ev = W.gen_mem_stride(n, 1001 + n, streams=streams)
    g = gpu_run(rt, pol, ev, jit=True)
    assert_same(g, oracle_run(pol, ev), "stride_prefetch")
    assert g.stats["hash_e2big"] == 0 and g.stats["ring_drops"] == 0 and g.stats["vm_errors"] == 0


@pytest.mark.parametrize("i", range(8))
def test_jit_generated_programs(rt, i):
    pol = W.gen_program(W.subseed(1003, 100 + i))
    n = [100, 1000, 4096, 5000, 20000, 64, 3000, 777][i]
    _log(f"jit generated program {i} ({len(pol.code) // 8} slots) n={n}")
    ev = W.gen_mem_uniform(n, 700 + i)
    g = gpu_run(rt, pol, ev, jit=True)
    assert_same(g, oracle_run(pol, ev), f"program {i}")
    assert g.stats["vm_errors"] == 0


@pytest.mark.parametrize("n", [64, 65536])
def test_jit_divergence(rt, n):
    _log(f"jit divergence n={n}")
    pol = W.Policy("diverge", W.HOOK_MEM_ACCESS, DIVERGE, [])
    ev = W.gen_mem_uniform(n, 31 + n)
    ev["addr"] = W.splitmix(5, n)
    g = gpu_run(rt, pol, ev, jit=True)
    assert_same(g, oracle_run(pol, ev), "divergence")


def test_jit_hash_churn(rt):
    import torch
    from oracle import oracle as O
    _log("jit churn")
    pol = W.Policy("churn", W.HOOK_MEM_ACCESS, CHURN, [W.MapSpec("h", W.MAP_HASH, 8, 8, 512, 0)])
    fds, prog = setup(rt, pol, jit=True)
    o = O.Oracle()
    o.create_map(W.MAP_HASH, 8, 8, 512, 0)
    for b in range(3):
        ev = W.gen_mem_uniform(20000, 90 + b, streams=128)
        rc = torch.zeros(len(ev), dtype=torch.int32, device="cuda")
        rt.run_batch(prog, to_device(ev), n_events=len(ev), record_size=24, rc=rc)
        torch.cuda.synchronize()
        assert np.array_equal(rc.cpu().numpy().view(np.uint32), o.run(pol.code, pol.hook, ev)), f"launch {b}"
        g = collect(rt, pol, fds, None)
        k, v = o.dump(0)
        assert g.maps[0] == normalise_hash(k, v), f"launch {b}"
    assert rt.stats()["vm_errors"] == 0
