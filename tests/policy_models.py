"""Direct Python models of the three policies (no eBPF), used to pin the
oracle: access counter and latency histogram have closed forms; the stride
prefetcher is modelled per event with a dict of per-(stream, region tag)
state, exactly as the policy is described in prose."""

import math

import numpy as np


def access_counter(ev):
    region = (ev["addr"] >> np.uint64(21)).astype(np.int64)
    hist = np.bincount(region, minlength=4096).astype(np.uint64)
    rc = (region & 1).astype(np.uint32)
    return hist, rc


def floor_log2(lat):
    out = np.zeros(len(lat), dtype=np.int64)
    nz = lat > 0
    # exact: bit_length - 1 computed with integer arithmetic
    out[nz] = np.array([int(x).bit_length() - 1 for x in lat[nz].tolist()], dtype=np.int64)
    return out


def latency_hist(ev, T, kernels=4096):
    b = floor_log2(ev["lat"])
    k = ev["kernel_id"].astype(np.int64)
    hist = np.bincount(k * 64 + b, minlength=kernels * 64).astype(np.uint64).reshape(kernels, 64)
    sel = ev["lat"] > np.uint64(T)
    recs = sorted(zip(k[sel].tolist(), b[sel].tolist(), ev["lat"][sel].tolist()))
    records = [(kk, bb, ll, int(T), 0) for kk, bb, ll in recs]
    return hist, b.astype(np.uint32), records


def stride_prefetch(ev):
    """Returns (rc, state dict key -> (last_addr, stride, conf), records)."""
    state = {}
    rc = np.zeros(len(ev), dtype=np.uint32)
    records = []
    M = (1 << 64) - 1
    for i, (a, s, ts) in enumerate(zip(ev["addr"].tolist(), ev["stream"].tolist(), ev["ts"].tolist())):
        pg, rg = a >> 12, a >> 21
        key = (s << 32) | (rg & 31)
        if key not in state:
            state[key] = [a, 0, 0]
            continue
        v = state[key]
        if (v[0] >> 21) != rg:
            state[key] = [a, 0, 0]
            continue
        d = pg - (v[0] >> 12)
        v[0] = a
        if d == 0:
            continue
        if d == v[1]:
            v[2] = (v[2] + 1) & 0xFFFFFFFF
        else:
            v[1], v[2] = d, 0
        conf = v[2]
        if conf >= 2 and (conf & 7) == 2 and 1 <= abs(d) <= 16:
            n = 0
            for k in range(1, 9):
                p = pg + k * d
                if p < 0 or p >= (1 << 18) or (p >> 9) != (pg >> 9):
                    break
                n = k
            if n > 0:
                records.append((s, n, ((pg + d) << 12) & M, (d << 12) & M, ts))
                rc[i] = n
    return rc, {k: (v[0], v[1] & M, v[2]) for k, v in state.items()}, records


def percentile_threshold(lat):
    k = math.ceil(0.99 * len(lat)) - 1
    return int(np.sort(lat)[k])


def wave_tiles(ev):
    """Per tile of 64 consecutive records: (lo, hi, n, stream of the first
    record), by plain Python loops."""
    out = []
    addr = ev["addr"].tolist()
    stream = ev["stream"].tolist()
    for b in range(0, len(ev), 64):
        a = addr[b:b + 64]
        out.append((min(a), max(a), len(a), stream[b]))
    return out


def wave_monitor(ev):
    """The warp-leader monitor as described in prose: per tile, coalesced
    tiles (hi - lo < 4096) add n to coal[(lo >> 21) & 4095], others add 1 to
    scat[...] and, spanning more than 4 GiB, emit (lo, hi, n | stream << 32);
    every record of the tile gets the tile's page span."""
    coal = np.zeros(4096, np.uint64)
    scat = np.zeros(4096, np.uint64)
    ring, rc = [], np.zeros(len(ev), np.uint32)
    for t, (lo, hi, n, s0) in enumerate(wave_tiles(ev)):
        reg = (lo >> 21) & 4095
        if hi - lo < 4096:
            coal[reg] += np.uint64(n)
        else:
            scat[reg] += np.uint64(1)
            if (hi - lo) >> 32:
                ring.append(int(lo).to_bytes(8, "little") + int(hi).to_bytes(8, "little") +
                            ((s0 << 32) | n).to_bytes(8, "little"))
        rc[t * 64:t * 64 + n] = ((hi >> 12) - (lo >> 12) + 1) & 0xffffffff
    return coal, scat, sorted(ring), rc
