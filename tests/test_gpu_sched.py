"""The device block scheduler (section 4.3.2's work-stealing scheduler with
persistent workers; section 6.2.1's policies).  Whatever the policy, every
work unit runs exactly once (all outputs equal the generator's closed
form); the logged decisions replayed through the oracle give the same
return codes and the same steal counts in the policy's map; and each
policy's rule holds on its own log (FixedWork never asks, Greedy always
steals, MaxSteals stops at K, LatencyBudget at B ns).  Both engines."""

import errno

import numpy as np
import pytest

from app_model import lcg_results
from gpu_runner import setup
from runners import oracle_run

from paper_2512_12615_amd import workloads as W

pytestmark = pytest.mark.gpu

PARAM = {"greedy": None, "max_steals": 2, "latency_budget": 20000}


@pytest.fixture(scope="module")
def rt():
    from paper_2512_12615_amd import gxbpf as G
    r = G.Runtime(0)
    yield r
    r.close()


def _sched(rt, kind, cost, workers, jit, log_cap=1 << 16):
    import torch
    print(f"sched {kind} units={len(cost)} workers={workers} jit={jit}", flush=True)
    pol = None
    fds, prog = [], -1
    if kind != "fixed":
        pol = W.sched_policy(kind)
        init = [] if PARAM[kind] is None else [(1, b"\0\0\0\0", np.uint64(PARAM[kind]).tobytes())]
        fds, prog = setup(rt, pol, init=init, jit=jit)
    d_cost = torch.from_numpy(cost.view(np.int32)).cuda()
    out = torch.zeros(64 * len(cost), dtype=torch.int64, device="cuda")
    log = torch.zeros((log_cap, 4), dtype=torch.int64, device="cuda")
    log_rc = torch.zeros(log_cap, dtype=torch.int32, device="cuda")
    log_n = torch.zeros(1, dtype=torch.int32, device="cuda")
    rt.run_sched(prog, d_cost, workers, out, log=log, log_rc=log_rc, log_n=log_n)
    torch.cuda.synchronize()
    n = int(log_n.item())
    k = min(n, log_cap)
    ctx = np.ascontiguousarray(log[:k].cpu().numpy()).view(np.uint64).reshape(-1).view(W.SCHED_DTYPE)
    steals = np.frombuffer(rt.map_dump(fds[0])[1].tobytes(), "<u8") if fds else None
    return out.cpu().numpy().view(np.uint64), ctx, log_rc[:k].cpu().numpy().view(np.uint32), n, steals, pol


def _check_policy(kind, ctx, rc):
    if kind == "greedy":
        assert rc.all()
    elif kind == "max_steals":
        assert np.array_equal(rc, (ctx["stolen"] < PARAM[kind]).astype(np.uint32))
        assert ctx["stolen"].max(initial=0) <= PARAM[kind]
    elif kind == "latency_budget":
        assert np.array_equal(rc, (ctx["steal_ns"] < PARAM[kind]).astype(np.uint32))
    # per worker, decisions keep their order: done and stolen never decrease
    for w in np.unique(ctx["worker"]):
        mine = ctx[ctx["worker"] == w]
        assert np.all(np.diff(mine["stolen"].astype(np.int64)) >= 0)
        assert np.all(np.diff(mine["done"].astype(np.int64)) >= 0)
        assert np.all(np.diff(mine["steal_ns"].astype(np.int64)) >= 0)
        assert np.all(mine["elapsed_ns"] >= mine["steal_ns"])
        # a "no" ends the worker's stealing
        assert not np.any(rc[ctx["worker"] == w][:-1] == 0)


@pytest.mark.parametrize("jit", [False, True])
@pytest.mark.parametrize("kind", ["fixed", "greedy", "max_steals", "latency_budget"])
@pytest.mark.parametrize("regime,workers,upw,base", [("moderate", 96, 8, 200), ("heavy_tail", 200, 4, 20),
                                                      ("uniform", 37, 3, 50)])
def test_scheduler_runs_every_unit_once_and_replays(rt, kind, jit, regime, workers, upw, base):
    cost = W.sched_costs(workers, upw, regime, base, 7)
    out, ctx, rc, n, steals, pol = _sched(rt, kind, cost, workers, jit)
    assert np.array_equal(out, lcg_results(cost)), "a unit ran twice, never, or wrongly"
    if kind == "fixed":
        assert n == 0
        return
    assert n == len(ctx), "log overflow"
    if regime != "uniform":
        assert n > 0, "the early workers never asked to steal"
    _check_policy(kind, ctx, rc)
    init = [] if PARAM[kind] is None else [(1, b"\0\0\0\0", np.uint64(PARAM[kind]).tobytes())]
    want = oracle_run(pol, ctx, init=init)
    assert np.array_equal(want.rc, rc), "the oracle decides otherwise on the logged contexts"
    assert want.maps[0] == steals.tobytes(), "steal counts differ from the oracle's"
    assert want.stats["faults"] == 0


@pytest.mark.parametrize("jit", [False, True])
def test_edges(rt, jit):
    # one worker: no victim, so no decision; more workers than units:
    # empty ranges steal at once; one unit
    for workers, units in [(1, 5), (64, 10), (130, 1)]:
        cost = np.full(units, 30, np.uint32)
        out, ctx, rc, n, _, _ = _sched(rt, "greedy", cost, workers, jit)
        assert np.array_equal(out, lcg_results(cost))
        if workers == 1:
            assert n == 0
        assert rc.all()


def test_log_overflow_keeps_the_first_decisions(rt):
    # worker 0's eight units are heavy: the others finish first and steal
    cost = np.full(64 * 8, 5, np.uint32)
    cost[:8] = 20000
    out, ctx, rc, n, _, _ = _sched(rt, "greedy", cost, 64, False, log_cap=4)
    assert np.array_equal(out, lcg_results(cost))
    assert len(ctx) == 4 and n >= 4
    assert rc.all()


def test_rejections(rt):
    import torch
    from paper_2512_12615_amd import gxbpf as G
    cost = torch.ones(8, dtype=torch.int32, device="cuda")
    out = torch.zeros(64 * 8, dtype=torch.int64, device="cuda")
    _, mem = setup(rt, W.access_counter_policy())
    fds, sched = setup(rt, W.sched_policy("greedy"))
    for prog, workers in [(mem, 4), (sched, 0), (sched, 1 << 17)]:
        with pytest.raises(G.GxError) as e:
            rt.run_sched(prog, cost, workers, out)
        assert e.value.errno == errno.EINVAL
    # a scheduling program cannot run over records
    ev = torch.zeros(32 * 10, dtype=torch.uint8, device="cuda")
    with pytest.raises(G.GxError) as e:
        rt.run_batch(sched, ev, n_events=10, record_size=32)
    assert e.value.errno == errno.EINVAL
    torch.cuda.synchronize()
