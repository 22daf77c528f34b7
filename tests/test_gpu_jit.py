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


@pytest.mark.parametrize("ahead", [0, 1, 3, 7])
def test_jit_tiles_loaded_ahead(rt, monkeypatch, ahead):
    """The event-parallel kernel with the records of 0 (one tile at a
    time), 1, 3 and 7 tiles loaded ahead of the running one: every depth
    unrolls the tile loop differently, and runs that end inside an unrolled
    round or leave waves without tiles must still give the oracle's rc,
    maps and ring records."""
    monkeypatch.setenv("GX_EP_AHEAD", str(ahead))
    for n in (64 * 4099 + 37, 64 * 3 + 1):
        _log(f"jit latency_hist ahead={ahead} n={n}")
        pol = W.latency_hist_policy()
        ev = W.gen_timing(n, 1202 + n)
        init = [(1, b"\0\0\0\0", np.uint64(W.p99_threshold(ev["lat"])).tobytes())]
        g = gpu_run(rt, pol, ev, init, jit=True)
        assert_same(g, oracle_run(pol, ev, init), f"latency_hist ahead={ahead} n={n}")
        assert g.stats["ring_drops"] == 0 and g.stats["vm_errors"] == 0


@pytest.mark.parametrize("n,streams", [(1, 1), (777, 8), (1 << 16, 1024)])
def test_jit_stride_prefetch(rt, n, streams):
    _log(f"jit stride_prefetch n={n} streams={streams}")
    pol = W.stride_prefetch_policy()
    ev = W.gen_mem_stride(n, 1001 + n, streams=streams)
    g = gpu_run(rt, pol, ev, jit=True)
    assert_same(g, oracle_run(pol, ev), "stride_prefetch")
    assert g.stats["hash_e2big"] == 0 and g.stats["ring_drops"] == 0 and g.stats["vm_errors"] == 0


def test_jit_stride_prefetch_shared_queues(rt, monkeypatch):
    """64 queues for 1024 streams: 16 streams per queue, whose keys collide
    in the lookup memo of the one-queue kernel."""
    _log("jit stride_prefetch on 64 queues")
    monkeypatch.setenv("GX_SEQ_LANES", "1")
    monkeypatch.setenv("GX_QUEUE_BITS", "6")
    pol = W.stride_prefetch_policy()
    ev = W.gen_mem_stride(1 << 17, 4242)
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


def test_jit_ring_overflow_counts_drops(rt):
    """A 4 KiB ring takes 256 records of 16 B: the rest are dropped, counted,
    and reported as -EAGAIN to exactly the events whose records are missing."""
    text = """
        ldxdw r6, [r1+16]
        stxdw [r10-8], r6
        lddw r1, map:ring
        mov64 r2, r10
        add64 r2, -8
        mov64 r3, 8
        mov64 r4, 0
        call ringbuf_output
        exit
    """
    _log("jit ring overflow")
    pol = W.Policy("ring", W.HOOK_MEM_ACCESS, text, [W.MapSpec("ring", W.MAP_RINGBUF, 0, 0, 4096, 0)])
    ev = np.zeros(1000, W.MEM_DTYPE)
    ev["ts"] = np.arange(1000)
    g = gpu_run(rt, pol, ev, jit=True)
    ok = g.rc == 0
    assert int(ok.sum()) <= 256 and int(ok.sum()) >= 192
    assert g.stats["ring_drops"] == 1000 - int(ok.sum())
    got = sorted(int(np.frombuffer(r, "<u8")[0]) for r in g.rings[0])
    assert got == sorted(np.nonzero(ok)[0].tolist())


def test_jit_ring_records_across_drains(rt):
    """Many waves, each carving records from its own chunk, over several
    launches with a drain after each: every record arrives exactly once."""
    import torch
    text = """
        ldxdw r6, [r1+16]
        mov64 r0, r6
        and64 r0, 3
        jne r0, 0, out
        stxdw [r10-16], r6
        ldxdw r7, [r1+0]
        stxdw [r10-8], r7
        lddw r1, map:ring
        mov64 r2, r10
        add64 r2, -16
        mov64 r3, 16
        mov64 r4, 0
        call ringbuf_output
    out:
        exit
    """
    _log("jit ring across drains")
    pol = W.Policy("ring2", W.HOOK_MEM_ACCESS, text, [W.MapSpec("ring", W.MAP_RINGBUF, 0, 0, 1 << 22, 0)])
    fds, prog = setup(rt, pol, jit=True)
    for b in range(3):
        n = 200003 + b
        ev = W.gen_mem_uniform(n, 60 + b)
        ev["ts"] = np.arange(n, dtype=np.uint64) * 7 + b
        rc = torch.zeros(n, dtype=torch.int32, device="cuda")
        rt.run_batch(prog, to_device(ev), n_events=n, record_size=24, rc=rc)
        torch.cuda.synchronize()
        buf, nrec = rt.drain_ringbuf(fds[0])
        from paper_2512_12615_amd import gxbpf as G
        recs = G.parse_ring(buf)
        want = ev[(ev["ts"] & 3) == 0]
        assert nrec == len(want) == len(recs)
        got = sorted((int.from_bytes(r[:8], "little"), int.from_bytes(r[8:16], "little")) for r in recs)
        assert got == sorted(zip(want["ts"].tolist(), want["addr"].tolist()))
        assert np.array_equal(rc.cpu().numpy().view(np.uint32), (ev["ts"] & 3).astype(np.uint32))
    assert rt.stats()["ring_drops"] == 0


def _shared_prog(op, width, entries, operand="and64 r1, 0xffff"):
    """Event-parallel program: one commutative atomic per event on a shared
    array of ``entries`` words, index and operand from the record."""
    mn = {"add": "aadd", "or": "aor", "and": "aand", "xor": "axor"}[op] + ("64" if width == 8 else "32")
    st = "stxdw" if width == 8 else "stxw"
    text = f"""
        ldxdw r6, [r1+0]
        ldxdw r7, [r1+16]
        mov64 r1, r6
        rsh64 r1, 12
        and64 r1, {entries - 1}
        stxw [r10-4], r1
        lddw r1, map:sh
        mov64 r2, r10
        add64 r2, -4
        call map_lookup_elem
        jeq r0, 0, out
        mov64 r1, r7
        {'xor64 r1, -1' if op == 'and' else operand}
        {mn} [r0+0], r1
    out:
        mov64 r0, r6
        and64 r0, 7
        exit
    """
    return W.Policy(f"shared_{op}{width}_{len(operand)}", W.HOOK_MEM_ACCESS, text,
                    [W.MapSpec("sh", W.MAP_ARRAY, 4, width, entries, W.F_SHARED)])


@pytest.mark.parametrize("op,width,entries", [("add", 8, 4096), ("or", 4, 1024), ("and", 8, 2048),
                                              ("xor", 4, 4096), ("add", 8, 1 << 16), ("xor", 8, 1 << 18),
                                              ("add", 8, 1 << 21)])
def test_jit_shared_map_lds_accumulation(rt, op, width, entries):
    """Shared-map atomics summed in LDS per block (whole-map mirror for small
    maps, tagged cache with direct misses for large ones: 8-bit tags up to
    2^18 words here, 32-bit tags for the 2^21-word map, whose word index
    divided by the set count exceeds a byte) give the oracle's map
    exactly."""
    _log(f"jit shared {op}{width} entries={entries}")
    pol = _shared_prog(op, width, entries)
    n = 300007
    ev = W.gen_mem_uniform(n, 77 + entries)
    # skew: a quarter of the events hit 8 hot words
    hot = W.splitmix(5, n) % np.uint64(4) == 0
    ev["addr"] = np.where(hot, (W.splitmix(6, n) % np.uint64(8)) << np.uint64(12), ev["addr"])
    ev["ts"] = W.splitmix(7, n)
    init = None
    if op == "and":  # start from all-ones words so that AND has something to clear
        ones = (b"\xff" * width)
        init = [(0, np.uint32(k).tobytes(), ones) for k in range(entries)]
    g = gpu_run(rt, pol, ev, init, jit=True)
    assert_same(g, oracle_run(pol, ev, init), pol.name)
    assert g.stats["vm_errors"] == 0


@pytest.mark.parametrize("operand", ["rsh64 r1, 32", "mov64 r1, r1", "rsh64 r1, 31"])
def test_jit_shared_add_partial_sums_wrap(rt, operand):
    """64-bit sums cached as 32-bit partial sums: only addends small enough
    that no partial sum can wrap are summed in LDS; operands near or above
    2^32 go to the map directly, mixed ones take both paths."""
    _log(f"jit shared add64 operand={operand}")
    pol = _shared_prog("add", 8, 1 << 16, operand)
    n = 400009
    ev = W.gen_mem_uniform(n, 91)
    hot = W.splitmix(15, n) % np.uint64(2) == 0
    ev["addr"] = np.where(hot, (W.splitmix(16, n) % np.uint64(16)) << np.uint64(12), ev["addr"])
    ev["ts"] = W.splitmix(17, n)
    g = gpu_run(rt, pol, ev, jit=True)
    assert_same(g, oracle_run(pol, ev), pol.name)
    assert g.stats["vm_errors"] == 0


RING_RECORD = """
    ldxdw r6, [r1+0]
    ldxdw r7, [r1+16]
    mov64 r0, r6
    and64 r0, 7
    jne r0, 0, out
    stxdw [r10-24], r7
    stxdw [r10-16], r6
    stxdw [r10-8], r7
    lddw r1, map:ring
    mov64 r2, r10
    add64 r2, {off}
    mov64 r3, {size}
    mov64 r4, 0
    call ringbuf_output
    mov64 r0, r6
    and64 r0, 3
out:
    exit
"""


@pytest.mark.parametrize("off,size", [(-24, 24), (-24, 12), (-16, 13), (-20, 12), (-13, 5)])
def test_jit_ring_records_from_the_frame(rt, off, size):
    """Ring records built in the private frame: word-aligned ones go to the
    helper by value (whole words, or a last word cut to the record's size),
    unaligned ones through the LDS frames; every payload byte as the
    oracle's."""
    _log(f"jit ring record off={off} size={size}")
    text = RING_RECORD.format(off=off, size=size)
    pol = W.Policy(f"ringrec{-off}_{size}", W.HOOK_MEM_ACCESS, text,
                   [W.MapSpec("ring", W.MAP_RINGBUF, 0, 0, 1 << 22, 0)])
    n = 64 * 311 + 17
    ev = W.gen_mem_uniform(n, 131 + size)
    ev["ts"] = W.splitmix(19, n)
    g = gpu_run(rt, pol, ev, jit=True)
    want = oracle_run(pol, ev)
    assert len(want.rings[0]) > 1000
    assert_same(g, want, pol.name)


def test_jit_ring_partial_drains(rt):
    """Draining into a buffer smaller than the committed records hands out
    whole records in order across calls, each exactly once, skipping the
    discarded chunk tails."""
    import torch
    from paper_2512_12615_amd import gxbpf as G
    text = """
        ldxdw r6, [r1+16]
        mov64 r0, r6
        and64 r0, 7
        jne r0, 0, out
        stxdw [r10-8], r6
        lddw r1, map:ring
        mov64 r2, r10
        add64 r2, -8
        mov64 r3, 8
        mov64 r4, 0
        call ringbuf_output
    out:
        exit
    """
    _log("jit ring partial drains")
    pol = W.Policy("ring3", W.HOOK_MEM_ACCESS, text, [W.MapSpec("ring", W.MAP_RINGBUF, 0, 0, 1 << 20, 0)])
    fds, prog = setup(rt, pol, jit=True)
    n = 50000
    ev = W.gen_mem_uniform(n, 61)
    ev["ts"] = np.arange(n, dtype=np.uint64)
    rc = torch.zeros(n, dtype=torch.int32, device="cuda")
    rt.run_batch(prog, to_device(ev), n_events=n, record_size=24, rc=rc)
    torch.cuda.synchronize()
    got, total = [], 0
    for _ in range(1000):
        buf, nrec = rt.drain_ringbuf(fds[0], cap=1000)
        if nrec == 0:
            break
        assert len(buf) <= 1000 and len(buf) == 16 * nrec
        got += [int.from_bytes(r, "little") for r in G.parse_ring(buf)]
        total += nrec
    assert sorted(got) == list(range(0, n, 8))
    assert rt.stats()["ring_drops"] == 0


def test_jit_instances_share_code_keep_their_maps(rt):
    """Two instances of one program on separate maps (one compiled module)
    run in one batch; each matches the oracle on its own events."""
    import torch
    _log("jit two instances")
    pol = W.stride_prefetch_policy()
    runs = []
    for j in range(2):
        fds, prog = setup(rt, pol, jit=True)
        ev = W.gen_mem_stride(30000 + 7 * j, 400 + j, streams=64)
        rc = torch.zeros(len(ev), dtype=torch.int32, device="cuda")
        runs.append((fds, prog, ev, to_device(ev), rc))
    rt.run_batches([(prog, d, len(ev), 24, rc) for fds, prog, ev, d, rc in runs])
    torch.cuda.synchronize()
    for j, (fds, prog, ev, d, rc) in enumerate(runs):
        g = collect(rt, pol, fds, rc.cpu().numpy().view(np.uint32))
        assert_same(g, oracle_run(pol, ev), f"instance {j}")


def test_jit_ring_drain_view(rt):
    """The drain without a host copy hands out the pinned range with its
    discard records; the records in it are the oracle's, and the range is
    released like a copying drain's."""
    import torch
    from paper_2512_12615_amd import gxbpf as G
    _log("jit ring drain view")
    pol = W.stride_prefetch_policy()
    fds, prog = setup(rt, pol, jit=True)
    seen, want = [], []
    o_ev = []
    for b in range(2):
        ev = W.gen_mem_stride(40000, 91 + b, streams=64)
        o_ev.append(ev)
        rc = torch.zeros(len(ev), dtype=torch.int32, device="cuda")
        rt.run_batch(prog, to_device(ev), n_events=len(ev), record_size=24, rc=rc)
        view, kept, n = rt.drain_ringbuf_view(fds[1])
        recs = G.parse_ring(bytes(view))
        assert n == len(recs)
        assert kept == sum(8 + ((len(r) + 7) & ~7) for r in recs)
        seen += recs
    want = oracle_run(pol, np.concatenate(o_ev)).rings[1]
    assert sorted(seen) == want
    view, kept, n = rt.drain_ringbuf_view(fds[1])
    assert kept == 0 and n == 0 and len(view) == 0


def _combined_prog(op, width, words):
    """Stream-sequential program (an owned hash entry per stream) whose loop
    updates a shared array six times per event, cycling over ``words``
    words: one-lane compiled runs combine these updates in registers (four
    words, replaced round robin), so more than four words force
    replacements within an event."""
    mn = {"add": "aadd", "or": "aor", "and": "aand", "xor": "axor"}[op] + ("64" if width == 8 else "32")
    text = f"""
        ldxw r6, [r1+8]
        ldxdw r7, [r1+16]
        stxdw [r10-8], r6
        stdw [r10-16], 1
        lddw r1, map:own
        mov64 r2, r10
        add64 r2, -8
        mov64 r3, r10
        add64 r3, -16
        mov64 r4, 0
        call map_update_elem
        mov64 r9, 0
    loop:
        mov64 r1, r7
        add64 r1, r9
        mod64 r1, {words}
        stxw [r10-4], r1
        lddw r1, map:sh
        mov64 r2, r10
        add64 r2, -4
        call map_lookup_elem
        jeq r0, 0, next
        mov64 r1, r7
        rsh64 r1, 7
        {'xor64 r1, -1' if op == 'and' else 'and64 r1, 0xfffff'}
        {mn} [r0+0], r1
    next:
        add64 r9, 1
        jlt r9, 6, loop
        mov64 r0, r6
        and64 r0, 7
        exit
    """
    return W.Policy(f"combined_{op}{width}_{words}", W.HOOK_MEM_ACCESS, text,
                    [W.MapSpec("own", W.MAP_HASH, 8, 8, 4096, 0),
                     W.MapSpec("sh", W.MAP_ARRAY, 4, width, 16, W.F_SHARED)])


@pytest.mark.parametrize("op,width,words", [("add", 8, 1), ("add", 4, 3), ("or", 8, 5), ("xor", 4, 9),
                                            ("and", 8, 16), ("add", 8, 7)])
@pytest.mark.parametrize("batched", [False, True])
def test_jit_one_lane_combiner(rt, op, width, words, batched):
    """Every stream hits the same few shared words from the one-queue kernel
    (and from a compiled program set): maps and return codes equal the
    oracle's."""
    import torch
    _log(f"jit combiner {op}{width} words={words} batched={batched}")
    pol = _combined_prog(op, width, words)
    n = 1 << 14
    ev = W.gen_mem_uniform(n, 300 + words)
    ev["ts"] = W.splitmix(301 + words, n)
    init = [(1, np.uint32(k).tobytes(), b"\xff" * width) for k in range(16)] if op == "and" else None
    want = oracle_run(pol, ev, init)
    if not batched:
        g = gpu_run(rt, pol, ev, init, jit=True)
        assert_same(g, want, pol.name)
        assert g.stats["vm_errors"] == 0
        return
    fds, prog = setup(rt, pol, init)
    rt.jit_program_set([prog])
    rc = torch.zeros(n, dtype=torch.int32, device="cuda")
    rt.run_batches([(prog, to_device(ev), n, 24, rc)])
    torch.cuda.synchronize()
    g = collect(rt, pol, fds, rc.cpu().numpy().view(np.uint32))
    assert_same(g, want, pol.name + " set")
