"""Plain models of the two application kernels that carry device hooks:
the instrumented vector add's access records and the block scheduler's
work-unit results, written from their definitions (not from the kernels)."""

import numpy as np

from paper_2512_12615_amd import workloads as W

LCG_A = 6364136223846793005  # Knuth's MMIX linear congruential generator
LCG_C = 1442695040888963407
MASK = (1 << 64) - 1


def vadd_records(n: int, stride: int) -> np.ndarray:
    """The memory-access record of iteration i < n: the load of a[j] with
    j = (i stride) mod n, {addr = 8 j, stream = i // 64 (its 64-iteration
    tile), ts = i}, in iteration order."""
    i = np.arange(n, dtype=np.uint64)
    ev = np.zeros(n, W.MEM_DTYPE)
    assert n <= 2**32 and stride < n  # i stride < 2^64: exact in uint64
    ev["addr"] = np.uint64(8) * ((i * np.uint64(stride)) % np.uint64(n))
    ev["stream"] = (i // 64).astype(np.uint32)
    ev["ts"] = i
    return ev


def _affine_power(k: int):
    """(A^k, C (A^(k-1) + ... + 1)) mod 2^64: k steps of x -> A x + C as one
    affine map, by repeated squaring."""
    ra, rc = 1, 0          # the identity map
    ba, bc = LCG_A, LCG_C  # one step
    while k:
        if k & 1:
            ra, rc = (ba * ra) & MASK, (ba * rc + bc) & MASK
        ba, bc = (ba * ba) & MASK, (ba * bc + bc) & MASK
        k >>= 1
    return ra, rc


def lcg_results(cost: np.ndarray) -> np.ndarray:
    """out[64 u + l] after cost[u] generator steps from 64 u + l."""
    out = np.zeros(64 * len(cost), np.uint64)
    lanes = np.arange(64, dtype=np.uint64)
    with np.errstate(over="ignore"):
        for u, k in enumerate(cost):
            a, c = _affine_power(int(k))
            x0 = np.uint64(64 * u) + lanes
            out[64 * u:64 * u + 64] = x0 * np.uint64(a) + np.uint64(c)
    return out
