"""Ring buffers that wrap: records that straddle the end of the data area
must be written (word by word, masked) and drained (two-segment copy)
intact.  A 64 KiB ring takes several launches of records, with a drain
after each, until the writers have gone round it at least twice; record
sizes of 24, 40 and 48 bytes do not divide the capacity, so records and the
discard records that close unused chunk space land across the end.  Every
launch's drained multiset and return codes equal the oracle's, for the
interpreter and compiled programs, with the copying drain and the view
drain, for an event-parallel and a stream-sequential program."""

import numpy as np
import pytest

from gpu_runner import setup, to_device

from paper_2512_12615_amd import workloads as W

pytestmark = pytest.mark.gpu

CAP = 1 << 16

# a quarter of the events emit a 12- or 36-byte record (24 or 48 bytes with
# the header and padding); rc is the helper's result, 1 for the others
TWO_SIZES = """
    ldxdw r6, [r1+16]
    ldxdw r7, [r1+0]
    mov64 r0, 1
    mov64 r8, r7
    and64 r8, 3
    jne r8, 0, out
    stxdw [r10-48], r6
    stxdw [r10-40], r7
    stxdw [r10-32], r6
    stxdw [r10-24], r7
    stxdw [r10-16], r6
    mov64 r8, r7
    rsh64 r8, 2
    and64 r8, 1
    lddw r1, map:ring
    mov64 r2, r10
    add64 r2, -48
    mov64 r4, 0
    jeq r8, 0, small
    mov64 r3, 36
    call ringbuf_output
    ja out
small:
    mov64 r3, 12
    call ringbuf_output
out:
    exit
"""


def _policy(kind):
    if kind == "two_sizes":
        return W.Policy("two_sizes", W.HOOK_MEM_ACCESS, TWO_SIZES, [W.MapSpec("ring", W.MAP_RINGBUF, 0, 0, CAP, 0)])
    return W.stride_prefetch_policy(ring_bytes=CAP)


def _events(kind, launch):
    if kind == "two_sizes":
        ev = W.gen_mem_uniform(2900 + 37 * launch, 500 + launch)
        ev["ts"] += np.uint64(launch << 40)  # payloads differ between launches
        return ev
    return W.gen_mem_stride(12000 + 101 * launch, 77 + launch, streams=64)


@pytest.fixture
def rt():
    from paper_2512_12615_amd import gxbpf as G
    r = G.Runtime(0)
    yield r
    r.close()


@pytest.mark.parametrize("drain", ["copy", "view"])
@pytest.mark.parametrize("jit", [False, True], ids=["interpreted", "compiled"])
@pytest.mark.parametrize("kind", ["two_sizes", "stride"])
def test_ring_wraps_and_drains_intact(rt, kind, jit, drain):
    import torch
    from oracle import oracle as O
    from paper_2512_12615_amd import gxbpf as G
    print(f"ring wrap {kind} jit={jit} drain={drain}", flush=True)
    pol = _policy(kind)
    fds, prog = setup(rt, pol, jit=jit)
    ring = len(pol.maps) - 1
    o = O.Oracle()
    for m in pol.maps:
        o.create_map(m.type, m.key_size, m.value_size, m.max_entries, m.flags)
    laps = 0
    for launch in range(8):
        ev = _events(kind, launch)
        rc = torch.zeros(len(ev), dtype=torch.int32, device="cuda")
        rt.run_batch(prog, to_device(ev), n_events=len(ev), record_size=24, rc=rc)
        torch.cuda.synchronize()
        if drain == "copy":
            buf, nrec = rt.drain_ringbuf(fds[ring])
            got = G.parse_ring(buf)
        else:
            view, kept, nrec = rt.drain_ringbuf_view(fds[ring])
            got = G.parse_ring(view.tobytes())
        assert len(got) == nrec
        want_rc = o.run(pol.code, pol.hook, ev)
        assert np.array_equal(rc.cpu().numpy().view(np.uint32), want_rc), f"launch {launch}: rc"
        want = o.drain(ring)
        assert sorted(got) == sorted(want), f"launch {launch}: {len(got)} records vs {len(want)}"
        head, tail = rt.ringbuf_pos(fds[ring])
        assert head == tail
        laps = head // CAP
    assert laps >= 2, f"the writers went round the ring {laps} times"
    st = rt.stats()
    assert st["ring_drops"] == 0 and st["hash_e2big"] == 0 and st["vm_errors"] == 0
