"""GPU parity of a batch captured into a HIP graph: every replay must leave
exactly what one eager gx_run_batches call over identical programs, maps and
events leaves (and the first replay what the oracle leaves).  Replays are
interleaved with eager work and synchronizations, and the event buffers are
rewritten between replays."""

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


def _runs(k, seed):
    progs, sizes = W.batched_workload(k, seed=seed, min_log2=6, max_log2=13)
    runs = [(p, W.gen_mem_uniform(int(n), 500 + i), None) for i, (p, n) in enumerate(zip(progs, sizes))]
    runs.append((W.access_counter_policy(), W.gen_mem_uniform(5000, 7), None))
    ev = W.gen_timing(3000, 8)
    runs.append((W.latency_hist_policy(), ev, [(1, b"\0\0\0\0", np.uint64(W.p99_threshold(ev["lat"])).tobytes())]))
    runs.append((W.stride_prefetch_policy(), W.gen_mem_stride(7000, 9, streams=128), None))
    return runs


def _side(rt, runs, jit_of):
    import torch
    descs, keep = [], []
    for j, (pol, ev, init) in enumerate(runs):
        fds, prog = setup(rt, pol, init, jit=jit_of(j))
        dev = to_device(ev)
        rc = torch.zeros(max(len(ev), 1), dtype=torch.int32, device="cuda")
        descs.append((prog, dev, len(ev), pol.record_size, rc))
        keep.append((pol, fds, rc, dev))
    return descs, keep


def _collect_all(rt, keep, runs):
    return [collect(rt, pol, fds, rc[:len(ev)].cpu().numpy().view(np.uint32))
            for (pol, fds, rc, _), (_, ev, _) in zip(keep, runs)]


@pytest.mark.parametrize("mode", ["interp", "mixed"])
def test_graph_replays_match_eager(rt, mode):
    import torch
    print(f"graph replays mode={mode}", flush=True)
    runs = _runs(10, 4242)
    jit_of = (lambda j: False) if mode == "interp" else (lambda j: j % 2 == 1 or j >= 10)
    g_descs, g_keep = _side(rt, runs, jit_of)
    e_descs, e_keep = _side(rt, runs, jit_of)

    graph = rt.graph_create(g_descs)
    torch.cuda.synchronize()
    # creating the graph runs the batch once and puts the maps back
    for i, (a, b) in enumerate(zip(_collect_all(rt, g_keep, runs), _collect_all(rt, e_keep, runs))):
        assert a.maps == b.maps and a.rings == b.rings, f"create left a trace in run {i}"

    want0 = [oracle_run(pol, ev, init) for pol, ev, init in runs]
    assert sum(ev.dtype == W.MEM_DTYPE for _, ev, _ in (runs[0], runs[3], runs[-1])) >= 2
    for rep in range(3):
        if rep == 2:
            # new contents in the same device buffers: the graph reads them
            for j in (0, 3, len(runs) - 1):
                pol, ev, init = runs[j]
                if ev.dtype != W.MEM_DTYPE:
                    continue
                new = W.gen_mem_uniform(len(ev), 77 + j, streams=128)
                b = torch.from_numpy(np.ascontiguousarray(new).view(np.uint8).reshape(-1))
                g_keep[j][3].copy_(b)
                e_keep[j][3].copy_(b)
        graph.launch()
        torch.cuda.synchronize()
        # eager work of the same runtime between replays
        rt.run_batches(e_descs)
        torch.cuda.synchronize()
        got = _collect_all(rt, g_keep, runs)
        ref = _collect_all(rt, e_keep, runs)
        for i, (a, b) in enumerate(zip(got, ref)):
            assert_same(a, b, f"replay {rep} run {i} ({runs[i][0].name}) vs eager")
            if rep == 0:
                assert_same(a, want0[i], f"replay 0 run {i} ({runs[i][0].name}) vs oracle")
    graph.close()
    assert rt.stats()["vm_errors"] == 0


def test_graph_program_set(rt):
    """A batch whose compiled programs run as one program set replays like
    its eager run."""
    import torch
    print("graph program set", flush=True)
    runs = _runs(4, 5151)
    g_descs, g_keep = _side(rt, runs, lambda j: False)
    e_descs, e_keep = _side(rt, runs, lambda j: False)
    assert rt.jit_program_set([d[0] for d in g_descs] + [d[0] for d in e_descs]) >= 0
    graph = rt.graph_create(g_descs)
    for rep in range(2):
        graph.launch()
        torch.cuda.synchronize()
        rt.run_batches(e_descs)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(_collect_all(rt, g_keep, runs), _collect_all(rt, e_keep, runs))):
            assert_same(a, b, f"replay {rep} run {i} ({runs[i][0].name}) vs eager")
            if rep == 0:
                assert_same(a, oracle_run(*runs[i]), f"replay 0 run {i} vs oracle")
    graph.close()
    assert rt.stats()["vm_errors"] == 0
