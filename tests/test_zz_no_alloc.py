"""The allocation-free run entry point (gx_run_batch_noalloc) against
gx_run_batch: the same program over the same inputs on twin maps, two calls
in a row (the second smaller, so stale workspace contents of the first call
would show), must give identical return codes, maps and ring records.  The
stream-sequential cases use the scratch array for the partition; the
compiled latency histogram runs once with its cache spill in the array and
once flushing directly."""

import errno

import numpy as np
import pytest

from gpu_runner import setup, to_device
from runners import normalise_hash

from paper_2512_12615_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture
def rt():
    from paper_2512_12615_amd import gxbpf as G
    r = G.Runtime(0)
    yield r
    r.close()


def _events(kind, n, seed):
    if kind == "stride":
        return W.gen_mem_stride(n, seed)
    if kind == "latency":
        return W.gen_timing(n, seed)
    return W.gen_mem_uniform(n, seed)


def _policy(kind):
    return {"stride": W.stride_prefetch_policy, "latency": W.latency_hist_policy,
            "access": W.access_counter_policy}[kind]()


def _state(rt, pol, fds):
    from paper_2512_12615_amd import gxbpf as G
    out = []
    for fd, m in zip(fds, pol.maps):
        if m.type == W.MAP_RINGBUF:
            buf, _ = rt.drain_ringbuf(fd)
            out.append(sorted(G.parse_ring(buf)))
        elif m.type == W.MAP_HASH:
            out.append(normalise_hash(*rt.map_dump(fd)))
        else:
            out.append(rt.map_dump(fd)[1].tobytes())
    return out


@pytest.mark.parametrize("kind,jit,blocks", [
    ("stride", True, None), ("stride", False, None),
    ("latency", True, "64"), ("latency", True, None),
    ("access", False, None), ("access", True, None),
])
def test_noalloc_matches_run_batch(rt, monkeypatch, kind, jit, blocks):
    import torch
    print(f"noalloc {kind} jit={jit} blocks={blocks}", flush=True)
    if blocks:
        monkeypatch.setenv("GX_JIT_BLOCKS", blocks)
    pol = _policy(kind)
    fa, pa = setup(rt, pol, jit=jit)
    fb, pb = setup(rt, pol, jit=jit)
    if kind == "latency":
        for fds in (fa, fb):
            assert rt.map_update(fds[1], b"\0\0\0\0", np.uint64(40000).tobytes()) == 0
    for call, n in enumerate([300007, 70001]):
        ev = _events(kind, n, 900 + call)
        d = to_device(ev)
        ra = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        rb = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        rt.run_batch(pa, d, n_events=n, record_size=pol.record_size, rc=ra)
        rt.run_batch_noalloc(pb, d, n_events=n, record_size=pol.record_size, rc=rb)
        torch.cuda.synchronize()
        assert torch.equal(ra, rb), f"call {call}: return codes differ"
        sa, sb = _state(rt, pol, fa), _state(rt, pol, fb)
        for i, (x, y) in enumerate(zip(sa, sb)):
            assert x == y, f"call {call}: map {i} differs"
    st = rt.stats()
    assert st["hash_e2big"] == 0 and st["ring_drops"] == 0 and st["vm_errors"] == 0


def test_noalloc_rejects_runs_beyond_the_scratch_array(rt):
    import torch
    from paper_2512_12615_amd import gxbpf as G
    print("noalloc oversized run", flush=True)
    pol = W.stride_prefetch_policy()
    _, prog = setup(rt, pol)
    n = 600000
    d = torch.zeros(n * 24, dtype=torch.uint8, device="cuda")
    with pytest.raises(G.GxError) as e:
        rt.run_batch_noalloc(prog, d, n_events=n, record_size=24)
    assert e.value.errno == errno.E2BIG
    torch.cuda.synchronize()
