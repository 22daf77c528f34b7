"""Run a policy through the GPU runtime (C ABI via the binding) and normalise
the result exactly like runners.oracle_run does."""

import numpy as np

from runners import Result, normalise_hash

from paper_2512_12615_amd import workloads as W


def to_device(events):
    import torch
    return torch.from_numpy(np.ascontiguousarray(events).view(np.uint8).reshape(-1)).cuda()


def setup(rt, policy, init=None, jit=False):
    fds = [rt.create_map(m.type, m.key_size, m.value_size, m.max_entries, m.flags) for m in policy.maps]
    for mi, k, v in init or []:
        assert rt.map_update(fds[mi], k, v) == 0
    prog = rt.load_program(policy.code, policy.hook, fds)
    if jit:
        rt.jit_program(prog)
    return fds, prog


def collect(rt, policy, fds, rc):
    res = Result(rc=rc)
    from paper_2512_12615_amd import gxbpf as G
    for fd, m in zip(fds, policy.maps):
        if m.type == W.MAP_RINGBUF:
            buf, _ = rt.drain_ringbuf(fd)
            res.maps.append(None)
            res.rings.append(sorted(G.parse_ring(buf)))
        else:
            keys, vals = rt.map_dump(fd)
            res.maps.append(vals.tobytes() if m.type == W.MAP_ARRAY else normalise_hash(keys, vals))
            res.rings.append(None)
    res.stats = rt.stats()
    return res


def gpu_run(rt, policy, events, init=None, d_events=None, jit=False):
    import torch
    fds, prog = setup(rt, policy, init, jit)
    n = len(events)
    ev = to_device(events) if d_events is None else d_events
    rc = torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")
    rt.run_batch(prog, ev, n_events=n, record_size=policy.record_size, rc=rc)
    torch.cuda.synchronize()
    return collect(rt, policy, fds, rc[:n].cpu().numpy().view(np.uint32))
