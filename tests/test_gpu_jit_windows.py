"""GPU parity of compiled programs whose map values are reached through
several pointers (map-value windows): two lookups of one key, an array
update under a live pointer, atomics, partial stores through an offset
pointer, deletes and lookups in a loop.  Each runs with one queue per wave
(wave-uniform kernel) and with 64 queues per wave, alone and as members of
a program set, and must give exactly the oracle's results."""

import numpy as np
import pytest

import jit_window_programs as P
from gpu_runner import collect, gpu_run, setup, to_device
from runners import assert_same, oracle_run

from paper_2512_12615_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture
def rt():
    from paper_2512_12615_amd import gxbpf as G
    r = G.Runtime(0)
    yield r
    r.close()


@pytest.mark.parametrize("lanes", [1, 64])
@pytest.mark.parametrize("name", sorted(P.PROGRAMS))
def test_window_programs_match_oracle(rt, monkeypatch, name, lanes):
    print(f"window program {name} lanes={lanes}", flush=True)
    monkeypatch.setenv("GX_SEQ_LANES", str(lanes))
    pol = P.policy(name)
    for n, streams, seed in [(1, 1, 3), (5000, 16, 4), (1 << 15, 128, 5)]:  # keys are per stream up to 128 streams
        ev = W.gen_mem_uniform(n, seed, streams=streams)
        g = gpu_run(rt, pol, ev, jit=True)
        assert_same(g, oracle_run(pol, ev), f"{name} n={n}")
        assert g.stats["vm_errors"] == 0 and g.stats["hash_e2big"] == 0


def test_window_programs_in_a_set(rt):
    import torch
    print("window programs as a program set", flush=True)
    descs, keep, fds_all = [], [], []
    for i, name in enumerate(sorted(P.PROGRAMS)):
        pol = P.policy(name)
        ev = W.gen_mem_uniform(4000 + 777 * i, 40 + i, streams=64)
        fds, prog = setup(rt, pol)
        rc = torch.zeros(len(ev), dtype=torch.int32, device="cuda")
        descs.append((prog, to_device(ev), len(ev), pol.record_size, rc))
        keep.append((pol, ev, fds, rc))
        fds_all.append(prog)
    assert rt.jit_program_set(fds_all) >= 0
    rt.run_batches(descs)
    torch.cuda.synchronize()
    for pol, ev, fds, rc in keep:
        g = collect(rt, pol, fds, rc.cpu().numpy().view(np.uint32))
        assert_same(g, oracle_run(pol, ev), pol.name)
    assert rt.stats()["vm_errors"] == 0


@pytest.mark.parametrize("name", sorted(P.PROGRAMS))
def test_window_programs_with_shared_queues(rt, monkeypatch, name):
    """One queue per wave over 64 queues: streams s and s + 64 share a queue,
    and their keys (stream << 32 | page & 7) fall on the same entry of the
    64-entry lookup memo, so entries are evicted by a colliding key and the
    first key is looked up again after stores through its window."""
    print(f"window program {name} on shared queues", flush=True)
    monkeypatch.setenv("GX_SEQ_LANES", "1")
    monkeypatch.setenv("GX_QUEUE_BITS", "6")
    pol = P.policy(name)
    ev = W.gen_mem_uniform(1 << 15, 9, streams=128)
    g = gpu_run(rt, pol, ev, jit=True)
    assert_same(g, oracle_run(pol, ev), name)
    assert g.stats["vm_errors"] == 0 and g.stats["hash_e2big"] == 0
