"""Wave aggregation of commutative map updates by distinct address, on both
engines: every lane of a wave updates one word, or the lanes of each wave
spread over 2, 4 or 8 hot words, or over (mostly) distinct words; addends
equal (closed form) or different per lane (DPP reduction over a full wave,
lane-by-lane reads otherwise, including partial waves at a ragged end);
ADD, OR, AND and XOR at 32 and 64 bits.  The shared maps are 64 KiB, beyond
the interpreter's LDS mirror (its updates go through the wave aggregation
to device atomics) and inside the compiled kernel's LDS cache (aggregated
before it).  Maps and return codes must equal the oracle's."""

import numpy as np
import pytest

from gpu_runner import gpu_run
from runners import assert_same, oracle_run

from paper_2512_12615_amd import workloads as W

pytestmark = pytest.mark.gpu

WORDS = 8192

OPS = {"add": "aadd", "or": "aor", "and": "aand", "xor": "axor"}


def _program(op, width, addend):
    w = "64" if width == 8 else "32"
    val = "mov64 r3, 1" if addend == "one" else "mov64 r3, r6\n    rsh64 r3, 3\n    and64 r3, 0xffff"
    if op == "and":
        val += "\n    xor64 r3, -1" if addend != "one" else "\n    mov64 r3, -2"
    text = f"""
    ldxdw r6, [r1+0]
    mov64 r7, r6
    rsh64 r7, 40
    and64 r7, {WORDS - 1}
    stxw [r10-4], r7
    lddw r1, map:m
    mov64 r2, r10
    add64 r2, -4
    call map_lookup_elem
    mov64 r8, r0
    mov64 r0, 0
    jeq r8, 0, out
    {val}
    {OPS[op]}{w} [r8+0], r3
    mov64 r0, r7
out:
    exit
"""
    return W.Policy(f"agg_{op}{w}_{addend}", W.HOOK_MEM_ACCESS, text,
                    [W.MapSpec("m", W.MAP_ARRAY, 4, width, WORDS, W.F_SHARED)])


def _events(n, hot, seed):
    """n records; the 64 records of each wave tile update ``hot`` words (0:
    random words over the whole map)."""
    x = W.splitmix(seed, 2 * n)
    tile = np.arange(n) // 64
    if hot:
        word = (tile * 37 + (x[:n] % np.uint64(hot)).astype(np.int64)) % WORDS
    else:
        word = (x[:n] % np.uint64(WORDS)).astype(np.int64)
    ev = np.zeros(n, W.MEM_DTYPE)
    ev["addr"] = (word.astype(np.uint64) << np.uint64(40)) | (x[n:] & np.uint64((1 << 40) - 1))
    ev["ts"] = np.arange(n, dtype=np.uint64)
    return ev


@pytest.fixture
def rt():
    from paper_2512_12615_amd import gxbpf as G
    r = G.Runtime(0)
    yield r
    r.close()


@pytest.mark.parametrize("jit", [False, True], ids=["interpreted", "compiled"])
@pytest.mark.parametrize("hot", [1, 2, 4, 8, 0])
@pytest.mark.parametrize("addend", ["one", "lane"])
def test_add64_by_hot_words(rt, jit, hot, addend):
    print(f"aggregate add64 hot={hot} addend={addend} jit={jit}", flush=True)
    pol = _program("add", 8, addend)
    for n, seed in [(64, 1), (1000, 2), (100003, 3)]:
        ev = _events(n, hot, seed + hot)
        g = gpu_run(rt, pol, ev, jit=jit)
        assert_same(g, oracle_run(pol, ev), f"n={n}")
        assert g.stats["vm_errors"] == 0


@pytest.mark.parametrize("jit", [False, True], ids=["interpreted", "compiled"])
@pytest.mark.parametrize("op", ["add", "or", "and", "xor"])
@pytest.mark.parametrize("width", [4, 8])
def test_ops_and_widths_on_shared_words(rt, jit, op, width):
    print(f"aggregate {op} width={width} jit={jit}", flush=True)
    for addend in ("one", "lane"):
        pol = _program(op, width, addend)
        for hot in (1, 3):
            ev = _events(20011, hot, 50 + hot)
            # words the run touches start all ones (an AND on zero shows nothing)
            words = np.unique(((ev["addr"] >> np.uint64(40)) % np.uint64(WORDS)).astype(np.uint32))
            init = [(0, int(k).to_bytes(4, "little"), b"\xff" * width) for k in words]
            g = gpu_run(rt, pol, ev, init, jit=jit)
            assert_same(g, oracle_run(pol, ev, init), f"{addend} hot={hot}")
