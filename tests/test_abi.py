"""The C-ABI library: it loads, exports every symbol include/gxbpf.h declares,
and its verifier (which needs no device) agrees with the oracle's checker on
the reject and accept corpora."""

import ctypes
import os
import re

import pytest

from test_oracle_checker import RAW_REJECTS, REJECTS, chk

from paper_2512_12615_amd import asm
from paper_2512_12615_amd import gxbpf as G
from paper_2512_12615_amd import workloads as W
from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "gxbpf.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int64_t|int|void)\s+(gx_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(G.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), s
    assert set(G.EXPORTS) <= set(syms)


def _shapes(maps):
    return [tuple(m) for m in maps]


@pytest.mark.parametrize("name", sorted(REJECTS))
def test_runtime_verifier_rejects_corpus(name):
    text, maps = REJECTS[name]
    names = ["m", "n", "r"][:len(maps)]
    ok, log, _ = G.verify(asm.assemble(text, names), W.HOOK_MEM_ACCESS, _shapes(maps))
    assert not ok, f"{name} accepted by the runtime verifier"
    assert log


@pytest.mark.parametrize("name", sorted(RAW_REJECTS))
def test_runtime_verifier_rejects_raw(name):
    ok, log, _ = G.verify(RAW_REJECTS[name], W.HOOK_MEM_ACCESS, [])
    assert not ok


def _both(pol):
    shapes = [(m.type, m.key_size, m.value_size, m.max_entries, m.flags) for m in pol.maps]
    ok, log, info = G.verify(pol.code, pol.hook, shapes)
    r = O.check(pol.code, pol.hook, shapes)
    return ok, log, info, r


def test_verifiers_agree_on_policies():
    for pol in [W.access_counter_policy(), W.stride_prefetch_policy(), W.latency_hist_policy()]:
        ok, log, info, r = _both(pol)
        assert ok and r.ok, (pol.name, log, r.log)
        assert info.stack_bytes == r.stack_bytes
        assert info.max_insns == r.max_insns
        assert info.max_calls == r.max_calls
        assert info.max_ring_bytes == r.max_ring_bytes
        assert (info.mode == G.MODE_EVENT_PARALLEL) == r.event_parallel


def test_verifiers_agree_on_generated_corpus():
    """Same verdict, stack size and mode on 200 generated programs.  The
    dynamic bounds (instructions, helper calls) may differ a little because
    the two value domains prune different infeasible branches; both must be
    upper bounds of what the oracle retires (checked on a sample)."""
    import numpy as np
    for i in range(200):
        pol = W.gen_program(W.subseed(1003, 100 + i))
        ok, log, info, r = _both(pol)
        assert ok == r.ok, (i, log, r.log)
        assert ok, (i, log)
        assert info.stack_bytes == r.stack_bytes
        assert (info.mode == G.MODE_EVENT_PARALLEL) == r.event_parallel
        assert abs(int(info.max_insns) - int(r.max_insns)) <= max(16, r.max_insns // 5), i
        assert abs(int(info.max_calls) - int(r.max_calls)) <= max(2, r.max_calls // 5), i
        if i < 16:
            ev = W.gen_mem_uniform(150, 40 + i)
            o = O.Oracle()
            for m in pol.maps:
                o.create_map(m.type, m.key_size, m.value_size, m.max_entries, m.flags)
            for e in range(len(ev)):
                o.reset_stats()
                o.run(pol.code, pol.hook, ev[e:e + 1])
                st = o.stats()
                assert st["insns"] <= min(info.max_insns, r.max_insns), (i, e)
                assert st["helper_calls"] <= min(info.max_calls, r.max_calls), (i, e)


def test_verifiers_agree_on_small_programs():
    """Verdict agreement over the brute-force alphabet of the checker tests."""
    from test_oracle_checker import _alphabet
    import itertools
    a = _alphabet()
    n = agree = 0
    for p in itertools.product(a, repeat=2):
        code = asm.assemble("\n".join(p))
        ok, _, _ = G.verify(code, W.HOOK_MEM_ACCESS, [])
        r = O.check(code, W.HOOK_MEM_ACCESS, [])
        n += 1
        agree += ok == r.ok
    assert agree == n


def test_verify_reports_facts():
    ok, log, info = G.verify(asm.assemble("mov64 r0, 0\nmov64 r6, 0\nl: add64 r0, 2\nadd64 r6, 1\njlt r6, 10, l\nexit"),
                             W.HOOK_MEM_ACCESS, [])
    assert ok and info.max_insns == 33 and info.mode == G.MODE_EVENT_PARALLEL
    code = asm.assemble("mov64 r0, 0\nexit") * 2049
    ok, log, _ = G.verify(code, W.HOOK_MEM_ACCESS, [])
    assert not ok
