"""GPU parity of the batched form: many programs over their own event batches
in one persistent launch must give exactly the results of running them one
after another (checked against the oracle run in that order)."""

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


def _mixed_runs(k, seed):
    progs, sizes = W.batched_workload(k, seed=seed, min_log2=6, max_log2=14)
    runs = [(p, W.gen_mem_uniform(int(n), 300 + i), None) for i, (p, n) in enumerate(zip(progs, sizes))]
    # event-parallel policies in the same launch
    runs.append((W.access_counter_policy(), W.gen_mem_uniform(5000, 1), None))
    ev = W.gen_timing(3000, 2)
    runs.append((W.latency_hist_policy(), ev, [(1, b"\0\0\0\0", np.uint64(W.p99_threshold(ev["lat"])).tobytes())]))
    runs.append((W.stride_prefetch_policy(), W.gen_mem_stride(7000, 3, streams=128), None))
    return runs


@pytest.mark.parametrize("k", [1, 24])
def test_batched_matches_oracle(rt, k):
    import torch
    print(f"batched k={k}", flush=True)
    runs = _mixed_runs(k, 1003 + k)
    descs, keep = [], []
    for pol, ev, init in runs:
        fds, prog = setup(rt, pol, init)
        dev = to_device(ev)
        rc = torch.zeros(max(len(ev), 1), dtype=torch.int32, device="cuda")
        descs.append((prog, dev, len(ev), pol.record_size, rc))
        keep.append((pol, ev, init, fds, rc))
    rt.run_batches(descs)
    torch.cuda.synchronize()
    for i, (pol, ev, init, fds, rc) in enumerate(keep):
        g = collect(rt, pol, fds, rc[:len(ev)].cpu().numpy().view(np.uint32))
        assert_same(g, oracle_run(pol, ev, init), f"run {i} ({pol.name})")
    assert rt.stats()["vm_errors"] == 0


def test_batched_same_program_twice_runs_in_order(rt):
    """Two batches of one program share its maps: they form two phases and
    the second sees the first's updates."""
    import torch
    pol = W.stride_prefetch_policy()
    fds, prog = setup(rt, pol)
    ev1 = W.gen_mem_stride(6000, 11, streams=64)
    ev2 = W.gen_mem_stride(6000, 12, streams=64)
    rc1 = torch.zeros(len(ev1), dtype=torch.int32, device="cuda")
    rc2 = torch.zeros(len(ev2), dtype=torch.int32, device="cuda")
    rt.run_batches([(prog, to_device(ev1), len(ev1), 24, rc1), (prog, to_device(ev2), len(ev2), 24, rc2)])
    torch.cuda.synchronize()
    both = np.concatenate([ev1, ev2])
    o = oracle_run(pol, both)
    g = collect(rt, pol, fds, np.concatenate([rc1.cpu().numpy(), rc2.cpu().numpy()]).view(np.uint32))
    assert_same(g, o, "two phases")


def test_batched_mixed_compiled_and_interpreted(rt):
    """Compiled programs in a batch run as their own kernels beside the
    persistent interpreter (after the shared partition); every run still
    matches the oracle."""
    import torch
    print("batched mixed compiled/interpreted", flush=True)
    runs = _mixed_runs(6, 2024)
    descs, keep = [], []
    for j, (pol, ev, init) in enumerate(runs):
        fds, prog = setup(rt, pol, init, jit=(j % 2 == 1) or j >= 6)
        dev = to_device(ev)
        rc = torch.zeros(max(len(ev), 1), dtype=torch.int32, device="cuda")
        descs.append((prog, dev, len(ev), pol.record_size, rc))
        keep.append((pol, ev, init, fds, rc))
    want = [oracle_run(pol, ev, init) for pol, ev, init, _, _ in keep]
    for rep in range(2):  # the second batch reuses the staging ring and side streams
        rt.run_batches(descs)
        torch.cuda.synchronize()
        for i, (pol, ev, init, fds, rc) in enumerate(keep):
            g = collect(rt, pol, fds, rc[:len(ev)].cpu().numpy().view(np.uint32))
            assert_same(g, want[i], f"rep {rep} run {i} ({pol.name})")
        if rep == 0:
            for pol, ev, init, fds, rc in keep:
                for fd, m in zip(fds, pol.maps):
                    rt.map_clear(fd)
                for mi, k, v in init or []:
                    assert rt.map_update(fds[mi], k, v) == 0
    assert rt.stats()["vm_errors"] == 0


def test_batched_program_set(rt):
    """Runs of programs compiled as one set share one persistent launch
    (beside a compiled single program and an interpreted one); two instances
    of one program share a slot and keep their own maps."""
    import torch
    print("batched program set", flush=True)
    runs = _mixed_runs(5, 3031)
    # a second instance of the first generated program, on its own maps and events
    runs.append((runs[0][0], W.gen_mem_uniform(3333, 919), None))
    descs, keep, set_fds = [], [], []
    for j, (pol, ev, init) in enumerate(runs):
        fds, prog = setup(rt, pol, init, jit=(j == 1))
        if j != 2:
            set_fds.append(prog)
        dev = to_device(ev)
        rc = torch.zeros(max(len(ev), 1), dtype=torch.int32, device="cuda")
        descs.append((prog, dev, len(ev), pol.record_size, rc))
        keep.append((pol, ev, init, fds, rc))
    sid = rt.jit_program_set(set_fds)
    assert sid >= 0
    rt.run_batches(descs)
    torch.cuda.synchronize()
    for i, (pol, ev, init, fds, rc) in enumerate(keep):
        g = collect(rt, pol, fds, rc[:len(ev)].cpu().numpy().view(np.uint32))
        assert_same(g, oracle_run(pol, ev, init), f"run {i} ({pol.name})")
    assert rt.stats()["vm_errors"] == 0
