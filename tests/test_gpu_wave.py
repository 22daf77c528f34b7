"""GPU parity of the warp-leader hook: one invocation per wave tile on the
tile's aggregate, return code given to every record of the tile, in the
interpreter, compiled, and in a batched launch beside per-record programs."""

import numpy as np
import pytest

from gpu_runner import collect, gpu_run, setup, to_device
from runners import assert_same, oracle_run
from test_oracle_wave import _emit_policy

from paper_2512_12615_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture
def rt():
    from paper_2512_12615_amd import gxbpf as G
    r = G.Runtime(0)
    yield r
    r.close()


@pytest.mark.parametrize("jit", [False, True])
@pytest.mark.parametrize("n", [1, 63, 64, 65, 130, 100003])
def test_wave_context_parity(rt, jit, n):
    print(f"wave emit jit={jit} n={n}", flush=True)
    pol = _emit_policy()
    ev = W.gen_mem_wave(n, 500 + n, coalesced=0.5, streams=9)
    g = gpu_run(rt, pol, ev, jit=jit)
    assert_same(g, oracle_run(pol, ev), f"emit n={n}")
    assert g.stats["vm_errors"] == 0 and g.stats["ring_drops"] == 0


@pytest.mark.parametrize("jit", [False, True])
@pytest.mark.parametrize("n,co", [(64 * 1000, 0.75), (1 << 20, 0.3)])
def test_wave_monitor_parity(rt, jit, n, co):
    print(f"wave monitor jit={jit} n={n}", flush=True)
    pol = W.wave_monitor_policy()
    ev = W.gen_mem_wave(n, 600 + n, coalesced=co)
    g = gpu_run(rt, pol, ev, jit=jit)
    assert_same(g, oracle_run(pol, ev), f"monitor n={n}")
    assert g.stats["vm_errors"] == 0


def test_wave_monitor_batched(rt):
    """A warp-leader program in a batched launch beside per-record ones."""
    import torch
    print("wave monitor batched", flush=True)
    runs = [(W.wave_monitor_policy(), W.gen_mem_wave(70001, 31)),
            (W.access_counter_policy(), W.gen_mem_uniform(50000, 32)),
            (W.wave_monitor_policy(), W.gen_mem_wave(333, 33)),
            (W.stride_prefetch_policy(), W.gen_mem_stride(40000, 34, streams=64))]
    descs, keep = [], []
    for j, (pol, ev) in enumerate(runs):
        fds, prog = setup(rt, pol, jit=(j == 2))
        rc = torch.zeros(len(ev), dtype=torch.int32, device="cuda")
        descs.append((prog, to_device(ev), len(ev), pol.record_size, rc))
        keep.append((pol, ev, fds, rc))
    rt.run_batches(descs)
    torch.cuda.synchronize()
    for pol, ev, fds, rc in keep:
        g = collect(rt, pol, fds, rc.cpu().numpy().view(np.uint32))
        assert_same(g, oracle_run(pol, ev), pol.name)
    assert rt.stats()["vm_errors"] == 0
