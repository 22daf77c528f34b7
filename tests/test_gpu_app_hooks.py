"""A device hook inside an application kernel (section 5.3's trampolines at
a kernel's memory instructions): the instrumented vector add must compute
c[j] = a[j] + b[j] for every element and leave return codes, maps and ring
records bit-identical to the oracle's run of the same program over the
access records the kernel makes (the plain model in app_model), for the
per-lane, warp-leader and SIMT hooks on both engines, at small ragged
sizes and at 2^24 elements with a wide stride."""

import errno

import numpy as np
import pytest

from app_model import vadd_records
from gpu_runner import collect, setup
from runners import assert_same, oracle_run

from paper_2512_12615_amd import workloads as W

pytestmark = pytest.mark.gpu

POLICIES = {
    "access_counter": W.access_counter_policy,
    "wave_counts_leader": lambda: W.wave_counts_policy(False),
    "wave_counts_simt": lambda: W.wave_counts_policy(True),
    "stride_l2": W.stride_l2_policy,
}


@pytest.fixture(scope="module")
def rt():
    from paper_2512_12615_amd import gxbpf as G
    r = G.Runtime(0)
    yield r
    r.close()


def _arrays(n, seed):
    import torch
    g = torch.Generator().manual_seed(seed)
    a = torch.randn(n, generator=g, dtype=torch.float64)
    b = torch.randn(n, generator=g, dtype=torch.float64)
    return a, b, a.cuda(), b.cuda(), torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")


def _run(rt, pol, n, stride, jit, seed=1):
    import torch
    print(f"app vadd {pol.name} n={n} stride={stride} jit={jit}", flush=True)
    fds, prog = setup(rt, pol, jit=jit)
    a, b, da, db, dc = _arrays(n, seed)
    rc = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    rt.run_app_vadd(prog, da, db, dc, stride=stride, rc=rc)
    torch.cuda.synchronize()
    assert torch.equal(dc.cpu(), a + b), "the application's own result changed"
    return collect(rt, pol, fds, rc.cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("jit", [False, True])
@pytest.mark.parametrize("name", sorted(POLICIES))
@pytest.mark.parametrize("n,stride", [(64 * 37 + 5, 1), (64 * 41 + 19, 97), (1, 0), (63, 62)])
def test_app_hook_matches_oracle(rt, name, jit, n, stride):
    pol = POLICIES[name]()
    got = _run(rt, pol, n, stride, jit)
    want = oracle_run(pol, vadd_records(n, stride))
    assert_same(want, got, f"{name} n={n} stride={stride} jit={jit}")
    assert got.stats["vm_errors"] == 0


@pytest.mark.parametrize("jit", [False, True])
@pytest.mark.parametrize("name", ["stride_l2", "wave_counts_simt"])
def test_app_hook_at_full_size(rt, name, jit):
    """2^24 elements (2^18 tiles) with a stride of 4099 elements: the tiles'
    address ranges wrap around the array, so the strides the prefetch
    policy sees vary."""
    pol = POLICIES[name]()
    n, stride = 1 << 24, 4099
    got = _run(rt, pol, n, stride, jit, seed=2)
    want = oracle_run(pol, vadd_records(n, stride))
    assert_same(want, got, f"{name} full jit={jit}")


def test_app_without_hook(rt):
    import torch
    for n, stride in [(1, 0), (64 * 1000 + 3, 12345), (1 << 22, 1)]:
        a, b, da, db, dc = _arrays(n, 3)
        rt.run_app_vadd(-1, da, db, dc, stride=stride)
        torch.cuda.synchronize()
        assert torch.equal(dc.cpu(), a + b)


def test_app_rejections(rt):
    import torch
    from paper_2512_12615_amd import gxbpf as G
    a, b, da, db, dc = _arrays(640, 4)
    seq_fds, seq = setup(rt, W.stride_prefetch_policy(hash_entries=1024, ring_bytes=1 << 16))
    timing_fds, timing = setup(rt, W.latency_hist_policy(ring_bytes=1 << 16))
    sched_fds, sched = setup(rt, W.sched_policy("greedy"))
    _, ok = setup(rt, W.access_counter_policy())
    for prog, stride in [(seq, 1), (timing, 1), (sched, 1), (ok, 640), (ok, 10), (ok, 0)]:
        with pytest.raises(G.GxError) as e:
            rt.run_app_vadd(prog, da, db, dc, stride=stride)
        assert e.value.errno == errno.EINVAL, (prog, stride)
    torch.cuda.synchronize()
