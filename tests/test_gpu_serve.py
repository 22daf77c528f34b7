"""Served form: every request's result is the same alone and in the mix.

"Alone" is the request's tenant's sequence replayed by itself in the oracle
(a tenant's requests run in submission order on the tenant's own maps); "in
the mix" is the server admitting many tenants' requests concurrently."""

import numpy as np
import pytest

from runners import normalise_hash

from paper_2512_12615_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture
def rt():
    from paper_2512_12615_amd import gxbpf as G
    r = G.Runtime(0)
    yield r
    r.close()


def _tenants(rt, k_tenants, k_programs, jit=False):
    progs = [W.gen_program(W.subseed(1004, 100 + p)) for p in range(k_programs)]
    ten = []
    for t in range(k_tenants):
        pol = progs[t % k_programs]
        fds = [rt.create_map(m.type, m.key_size, m.value_size, m.max_entries, m.flags) for m in pol.maps]
        prog = rt.load_program(pol.code, pol.hook, fds)
        if jit:
            rt.jit_program(prog)
        ten.append((pol, fds, prog))
    return ten


@pytest.mark.parametrize("mode,borrow,jit", [(0, False, False), (1, False, False), (0, True, False), (0, True, True),
                                             (1, False, True)])
def test_serve_same_alone_and_in_mix(rt, mode, borrow, jit):
    import torch
    from paper_2512_12615_amd import gxbpf as G
    from oracle import oracle as O
    print(f"serve mode={mode} borrow={borrow} jit={jit}", flush=True)
    ten = _tenants(rt, 8, 4, jit)
    arrival, tenant, _, n_ev = W.serving_trace(80, seed=77, tenants=8, min_log2=6, max_log2=12)
    reqs = [(i, int(t), W.gen_mem_uniform(int(n), 5000 + i)) for i, (t, n) in enumerate(zip(tenant, n_ev))]
    srv = G.Server(rt, budget_bytes=1 << 22, streams=3, mode=mode)
    pinned = []
    for i, t, ev in reqs:
        if borrow:
            h = torch.from_numpy(ev.view(np.uint8)).pin_memory()
            pinned.append(h)
            srv.submit_borrowed(t, ten[t][2], h.data_ptr(), len(ev), ev.dtype.itemsize, i)
        else:
            srv.submit(t, ten[t][2], ev, i)
    srv.drain()
    done = {}
    while len(done) < len(reqs):
        for c in srv.poll(64, wait_ms=100):
            assert c["status"] == 0
            done[c["req_id"]] = c
    srv.close()
    # alone: each tenant's requests in submission order, through the oracle
    for t in range(8):
        pol = ten[t][0]
        o = O.Oracle()
        for m in pol.maps:
            o.create_map(m.type, m.key_size, m.value_size, m.max_entries, m.flags)
        for i, tt, ev in reqs:
            if tt != t:
                continue
            rc = o.run(pol.code, pol.hook, ev)
            assert np.array_equal(done[i]["rc"], rc), f"request {i} of tenant {t}"
        for mi, (m, fd) in enumerate(zip(pol.maps, ten[t][1])):
            keys, vals = rt.map_dump(fd)
            okeys, ovals = o.dump(mi)
            if m.type == W.MAP_ARRAY:
                assert vals.tobytes() == ovals.tobytes(), f"tenant {t} map {mi}"
            else:
                assert normalise_hash(keys, vals) == normalise_hash(okeys, ovals), f"tenant {t} map {mi}"
    lat = [c["t_done"] - c["t_submit"] for c in done.values()]
    assert all(x > 0 for x in lat)


def test_serve_at_the_benchmark_scale(rt):
    """The served form's configuration: 64 tenants over the 32 generated
    programs (compiled; four program sets for the continuous path), hash maps
    of 2^22 entries (256 MiB of map per tenant, 16 GiB resident), a 4 GiB
    admission budget, four streams, and the first 240 requests of the
    Poisson trace (2^8..2^18 events each, all submitted at once, so the
    server batches and queues as under overload).  Every request's return
    codes equal its tenant's requests replayed in order by the oracle; the
    maps of eight sampled tenants equal the oracle's."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from paper_2512_12615_amd import gxbpf as G
    from oracle import oracle as O
    print("serve at the benchmark scale", flush=True)
    progs = [W.gen_program(W.subseed(1004, 100 + p)) for p in range(32)]
    ten = []
    for t in range(64):
        pol = progs[t % 32]
        fds = [rt.create_map(m.type, m.key_size, m.value_size, (1 << 22) if m.type == W.MAP_HASH else m.max_entries,
                             m.flags) for m in pol.maps]
        ten.append((pol, fds, rt.load_program(pol.code, pol.hook, fds)))
    with ThreadPoolExecutor(8) as ex:
        list(ex.map(lambda t: rt.jit_program(ten[t][2]), range(32)))
    for t in range(32, 64):
        rt.jit_program(ten[t][2])
    with ThreadPoolExecutor(4) as ex:
        list(ex.map(lambda k: rt.jit_program_set([ten[t][2] for t in range(64) if (t % 32) % 4 == k]), range(4)))
    print("serve at scale: compiled", flush=True)
    n_req = 240
    _, tenant, _, n_ev = W.serving_trace(n_req)
    reqs = [(i, int(t), W.gen_mem_uniform(int(n), 9000 + i)) for i, (t, n) in enumerate(zip(tenant, n_ev))]
    pinned = [torch.from_numpy(ev.view(np.uint8)).pin_memory() for _, _, ev in reqs]
    srv = G.Server(rt, budget_bytes=4 << 30, streams=4, mode=G.SERVE_CONTINUOUS)
    for (i, t, ev), h in zip(reqs, pinned):
        srv.submit_borrowed(t, ten[t][2], h.data_ptr(), len(ev), 24, i)
    srv.drain()
    done = {}
    while len(done) < n_req:
        for c in srv.poll(256, wait_ms=100):
            assert c["status"] == 0
            done[c["req_id"]] = c
    srv.close()
    print(f"serve at scale: {sum(len(ev) for _, _, ev in reqs)} events served", flush=True)
    sampled = set(sorted(set(int(t) for t in tenant))[::max(1, len(set(tenant.tolist())) // 8)][:8])

    def replay(t):
        pol = ten[t][0]
        o = O.Oracle()
        o.set_tracking(False)
        for m in pol.maps:
            o.create_map(m.type, m.key_size, m.value_size, (1 << 22) if m.type == W.MAP_HASH else m.max_entries,
                         m.flags)
        bad = []
        for i, tt, ev in reqs:
            if tt == t and not np.array_equal(done[i]["rc"], o.run(pol.code, pol.hook, ev)):
                bad.append(i)
        dumps = [o.dump(mi) for mi in range(len(pol.maps))] if t in sampled else None
        return t, bad, dumps

    with ThreadPoolExecutor(16) as ex:
        results = list(ex.map(replay, sorted(set(int(t) for t in tenant))))
    for t, bad, dumps in results:
        assert not bad, f"tenant {t}: requests {bad[:5]} differ from the oracle"
        if dumps is None:
            continue
        pol = ten[t][0]
        for mi, (m, fd) in enumerate(zip(pol.maps, ten[t][1])):
            keys, vals = rt.map_dump(fd)
            okeys, ovals = dumps[mi]
            if m.type == W.MAP_ARRAY:
                assert vals.tobytes() == ovals.tobytes(), f"tenant {t} map {mi}"
            else:
                assert normalise_hash(keys, vals) == normalise_hash(okeys, ovals), f"tenant {t} map {mi}"
    print(f"serve at scale: {len(results)} tenants replayed, {len(sampled)} tenants' maps compared", flush=True)
