"""The device block scheduler's hook (section 4.3.2's should_try_steal) on
the oracle: both checkers accept the three policies and hold the hook to
shared, read-only or ring maps and to its context layout, and the oracle's
decisions over synthetic contexts are pinned to each policy's plain rule
(Greedy: always; MaxSteals: while fewer than K units were stolen;
LatencyBudget: while less than B ns were spent stealing), with the steal
counts they leave in their map.  Also pins the workload's helpers: the
work unit's closed form against direct iteration, the cost regimes' shape,
and the instrumented vector add's access records."""

import numpy as np
import pytest

from app_model import lcg_results, vadd_records
from runners import oracle_run

from oracle import oracle as O
from paper_2512_12615_amd import gxbpf as G
from paper_2512_12615_amd import workloads as W

SH_STEALS = (W.MAP_ARRAY, 4, 8, 4096, W.F_SHARED)


def _shapes(pol):
    return [(m.type, m.key_size, m.value_size, m.max_entries, m.flags) for m in pol.maps]


def _contexts(n, seed):
    rng = np.random.default_rng(seed)
    ev = np.zeros(n, W.SCHED_DTYPE)
    ev["worker"] = rng.integers(0, 6000, n)
    ev["done"] = rng.integers(0, 100, n)
    ev["elapsed_ns"] = rng.integers(0, 10**7, n)
    ev["steal_ns"] = rng.integers(0, 10**5, n)
    ev["stolen"] = rng.integers(0, 8, n)
    ev["left"] = rng.integers(1, 50, n)
    return ev


@pytest.mark.parametrize("kind", ["greedy", "max_steals", "latency_budget"])
def test_policies_accepted_by_both_checkers(kind):
    pol = W.sched_policy(kind)
    r = O.check(pol.code, pol.hook, _shapes(pol))
    assert r.ok and r.event_parallel, r.log
    ok, log, _ = G.verify(pol.code, pol.hook, _shapes(pol))
    assert ok, log


REJECTS = {
    # owned state: every worker decides at once
    "owned_hash": ("""
        ldxw r6, [r1+0]
        stxdw [r10-8], r6
        stdw [r10-16], 1
        lddw r1, map:m
        mov64 r2, r10
        add64 r2, -8
        mov64 r3, r10
        add64 r3, -16
        mov64 r4, 0
        call map_update_elem
        mov64 r0, 1
        exit
    """, [(W.MAP_HASH, 8, 8, 64, 0)]),
    # past the 32-byte context
    "ctx_past_end": ("ldxw r0, [r1+32]\nexit", []),
    # a field read at the wrong width
    "ctx_wrong_width": ("ldxdw r0, [r1+24]\nexit", []),
    # a write to the context
    "ctx_write": ("stw [r1+0], 1\nmov64 r0, 1\nexit", []),
}


@pytest.mark.parametrize("name", sorted(REJECTS))
def test_both_checkers_reject(name):
    text, shapes = REJECTS[name]
    pol = W.Policy("t", W.HOOK_SCHED, text, [W.MapSpec("m", *s) for s in shapes])
    assert not O.check(pol.code, pol.hook, shapes).ok
    assert not G.verify(pol.code, pol.hook, shapes)[0]


@pytest.mark.parametrize("off,size", [(0, 4), (4, 4), (8, 8), (16, 8), (24, 4), (28, 4)])
def test_every_context_field_reads_back(off, size):
    op = {4: "ldxw", 8: "ldxdw"}[size]
    pol = W.Policy("echo", W.HOOK_SCHED, f"{op} r0, [r1+{off}]\nexit", [])
    assert O.check(pol.code, pol.hook, []).ok and G.verify(pol.code, pol.hook, [])[0]
    ev = _contexts(300, 3)
    got = oracle_run(pol, ev).rc
    name = {0: "worker", 4: "done", 8: "elapsed_ns", 16: "steal_ns", 24: "stolen", 28: "left"}[off]
    assert np.array_equal(got, (ev[name].astype(np.uint64) & np.uint64(0xFFFFFFFF)).astype(np.uint32))


@pytest.mark.parametrize("kind,param", [("greedy", None), ("max_steals", 3), ("latency_budget", 40000)])
def test_decisions_follow_the_policy_rule(kind, param):
    pol = W.sched_policy(kind)
    ev = _contexts(5000, 4)
    init = [] if param is None else [(1, b"\0\0\0\0", np.uint64(param).tobytes())]
    res = oracle_run(pol, ev, init=init)
    if kind == "greedy":
        want = np.ones(len(ev), bool)
    elif kind == "max_steals":
        want = ev["stolen"] < param
    else:
        want = ev["steal_ns"] < param
    assert np.array_equal(res.rc, want.astype(np.uint32))
    steals = np.frombuffer(res.maps[0], "<u8")
    expect = np.bincount(ev["worker"][want] & 4095, minlength=4096)
    assert np.array_equal(steals, expect.astype(np.uint64))


def test_missing_parameter_means_no_steal():
    """An unset cfg[0] is 0: MaxSteals and LatencyBudget then never steal."""
    for kind in ("max_steals", "latency_budget"):
        res = oracle_run(W.sched_policy(kind), _contexts(100, 5))
        assert not res.rc.any()


def test_lcg_closed_form_matches_iteration():
    cost = np.array([0, 1, 2, 7, 64, 1000, 3], np.uint32)
    got = lcg_results(cost)
    for u, k in enumerate(cost):
        for lane in (0, 1, 63):
            x = 64 * u + lane
            for _ in range(int(k)):
                x = (x * 6364136223846793005 + 1442695040888963407) % 2**64
            assert int(got[64 * u + lane]) == x


def test_cost_regimes():
    c = W.sched_costs(100, 8, "moderate", 1000, 1)
    assert c[0] == 1000 and c[-1] == 2000 and np.all(np.diff(c.astype(np.int64)) >= 0)
    h = W.sched_costs(100, 8, "heavy_tail", 1000, 1)
    owner = np.arange(800) * 100 // 800
    heavy = np.unique(owner[h > 1000])
    assert len(heavy) == 10 and np.all(np.diff(heavy) == 1)  # 10 % of the workers, contiguous
    assert h[h > 1000].min() >= 100_000 and h.max() <= 200_000
    assert np.all(W.sched_costs(7, 3, "uniform", 5, 0) == 5)


def test_vadd_records_are_a_permutation():
    n, s = 64 * 5 + 13, 97
    ev = vadd_records(n, s)
    assert np.array_equal(np.sort(ev["addr"] // 8), np.arange(n))
    assert np.array_equal(ev["stream"], np.arange(n) // 64) and np.array_equal(ev["ts"], np.arange(n))
    assert int(ev["addr"][3]) == 8 * (3 * s % n)
