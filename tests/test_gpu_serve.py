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
