"""The SIMT hook on the GPU (section 4.4): every lane runs its record with
its wave tile's aggregate; verified programs branch only on uniform values,
so waves never split, and their shared-map updates go to one word per wave,
combined before the atomic.  Results equal the oracle's on both engines,
and the per-lane handler equals the warp-leader handler that does the same
counting once per tile."""

import numpy as np
import pytest

import test_oracle_simt as S
from gpu_runner import gpu_run
from runners import assert_same, oracle_run

from paper_2512_12615_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture
def rt():
    from paper_2512_12615_amd import gxbpf as G
    r = G.Runtime(0)
    yield r
    r.close()


@pytest.mark.parametrize("jit", [False, True], ids=["interpreted", "compiled"])
@pytest.mark.parametrize("name", sorted(S.ACCEPTS))
def test_simt_programs_match_oracle(rt, jit, name):
    print(f"simt {name} jit={jit}", flush=True)
    text, shapes = S.ACCEPTS[name]
    names = ["m", "n", "r"][:len(shapes)]
    pol = W.Policy(name, W.HOOK_SIMT_MEM, text, [W.MapSpec(nm, *sh) for nm, sh in zip(names, shapes)])
    for n, seed in [(1, 1), (64 * 37 + 5, 2), (100003, 3)]:
        ev = W.gen_mem_wave(n, seed)
        g = gpu_run(rt, pol, ev, jit=jit)
        assert_same(g, oracle_run(pol, ev), f"{name} n={n}")
        assert g.stats["vm_errors"] == 0 and g.stats["ring_drops"] == 0


@pytest.mark.parametrize("jit", [False, True], ids=["interpreted", "compiled"])
def test_per_lane_handler_equals_warp_leader(rt, jit):
    print(f"simt wave counts jit={jit}", flush=True)
    ev = W.gen_mem_wave((1 << 18) + 33, 9)
    lead = gpu_run(rt, W.wave_counts_policy(False), ev, jit=jit)
    lane = gpu_run(rt, W.wave_counts_policy(True), ev, jit=jit)
    assert_same(lane, oracle_run(W.wave_counts_policy(True), ev), "per lane")
    assert np.array_equal(lead.rc, lane.rc) and lead.maps == lane.maps
