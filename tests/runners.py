"""Run a policy through the oracle and normalise the result for comparison:
return codes, map contents (array values in index order; hash contents as a
sorted key -> value list), ring records as a sorted multiset of payloads."""

from dataclasses import dataclass, field

import numpy as np

from paper_2512_12615_amd import workloads as W


@dataclass
class Result:
    rc: np.ndarray
    maps: list = field(default_factory=list)   # per map: bytes (array), list[(k, v)] (hash), None (ring)
    rings: list = field(default_factory=list)  # per map: sorted list of payloads (ring) else None
    stats: dict = field(default_factory=dict)


def normalise_hash(keys, vals):
    return sorted((bytes(k), bytes(v)) for k, v in zip(keys, vals))


def oracle_run(policy, events, init=None, order=0, seed=0, tracking=True):
    """``init``: list of (map_index, key bytes, value bytes) applied before the run."""
    from oracle import oracle as O
    o = O.Oracle()
    o.set_tracking(tracking)
    for m in policy.maps:
        r = o.create_map(m.type, m.key_size, m.value_size, m.max_entries, m.flags)
        assert r >= 0
    for mi, k, v in init or []:
        assert o.update(mi, k, v) == 0
    rc = o.run(policy.code, policy.hook, events, order=order, seed=seed)
    res = Result(rc=rc, stats=o.stats())
    for i, m in enumerate(policy.maps):
        if m.type == W.MAP_RINGBUF:
            res.maps.append(None)
            res.rings.append(sorted(o.drain(i)))
        else:
            keys, vals = o.dump(i)
            res.maps.append(vals.tobytes() if m.type == W.MAP_ARRAY else normalise_hash(keys, vals))
            res.rings.append(None)
    return res


def assert_same(a: Result, b: Result, what=""):
    assert np.array_equal(a.rc, b.rc), f"{what}: return codes differ at {np.nonzero(a.rc != b.rc)[0][:8]}"
    assert len(a.maps) == len(b.maps)
    for i, (x, y) in enumerate(zip(a.maps, b.maps)):
        assert x == y, f"{what}: map {i} differs"
    for i, (x, y) in enumerate(zip(a.rings, b.rings)):
        assert x == y, f"{what}: ring {i} differs ({None if x is None else len(x)} vs {None if y is None else len(y)} records)"
