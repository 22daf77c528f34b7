"""Drains in two halves (gx_drain_ringbuf_start / _finish): the copy of a
launch's ring records runs while the next launch is queued, whose VM kernel
waits for it.  Over eight launches into a 64 KiB ring that the writers go
round several times, every record reaches the host exactly once (the
multiset of all payloads as the oracle's over the concatenated batches),
the histogram and return codes are the oracle's, no record is dropped, and
the interpreter's uncounted records take the synchronous fallback.  Both
engines."""

import errno

import numpy as np
import pytest

from gpu_runner import setup, to_device
from runners import oracle_run

from paper_2512_12615_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    from paper_2512_12615_amd import gxbpf as G
    r = G.Runtime(0)
    yield r
    r.close()


@pytest.mark.parametrize("jit", [False, True])
def test_started_drains_overlap_launches(rt, jit):
    import torch
    from paper_2512_12615_amd import gxbpf as G
    print(f"started drains jit={jit}", flush=True)
    pol = W.latency_hist_policy(ring_bytes=1 << 16)
    batches = [W.gen_timing(1 << 13, 3100 + k) for k in range(8)]
    allev = np.concatenate(batches)
    thr = np.uint64(np.percentile(allev["lat"], 90))  # about 10 % tail records, 33 KB per launch
    init = [(1, b"\0\0\0\0", thr.tobytes())]
    fds, prog = setup(rt, pol, init=init, jit=jit)
    ring = fds[2]
    rc = torch.zeros(1 << 13, dtype=torch.int32, device="cuda")
    recs, rcs, nrec = [], [], 0
    with pytest.raises(G.GxError) as e:
        rt.drain_ringbuf_finish(ring)
    assert e.value.errno == errno.EINVAL
    pending = False
    for b in batches:
        rt.run_batch(prog, to_device(b), n_events=len(b), record_size=pol.record_size, rc=rc)
        if pending:
            view, _, n = rt.drain_ringbuf_finish(ring)
            recs += G.parse_ring(view.tobytes())
            nrec += n
        rt.drain_ringbuf_start(ring)
        pending = True
        for call in (lambda: rt.drain_ringbuf_start(ring), lambda: rt.drain_ringbuf_view(ring)):
            with pytest.raises(G.GxError) as e:
                call()
            assert e.value.errno == errno.EBUSY
        rcs.append(rc.cpu().numpy().copy())
    view, _, n = rt.drain_ringbuf_finish(ring)
    recs += G.parse_ring(view.tobytes())
    nrec += n
    # the oracle runs the concatenated batches in one go, with a ring that
    # holds them all (same program: the ring's size is the map's)
    want = oracle_run(W.latency_hist_policy(ring_bytes=1 << 22), allev, init)
    assert want.stats["drops"] == 0
    assert np.array_equal(np.concatenate(rcs).view(np.uint32), want.rc)
    assert rt.map_dump(fds[0])[1].tobytes() == want.maps[0]
    assert len(recs) == nrec == len(want.rings[2]) > 5000
    assert sorted(recs) == want.rings[2]
    head, tail = rt.ringbuf_pos(ring)
    assert head == tail and head > 3 * (1 << 16), "the writers went round the ring several times"
    assert rt.stats()["ring_drops"] == 0
