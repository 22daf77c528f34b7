"""The JIT's source generation and gfx950 compilation, on the CPU: every
policy and a corpus of generated programs must compile; the generated code
names every helper the program calls and has one label per jump target."""

import re

import pytest

from paper_2512_12615_amd import workloads as W


def _shapes(pol):
    return [(m.type, m.key_size, m.value_size, m.max_entries, m.flags) for m in pol.maps]


@pytest.fixture(scope="module")
def G():
    from paper_2512_12615_amd import gxbpf
    return gxbpf


@pytest.mark.parametrize("name", ["access_counter", "stride_prefetch", "latency_hist"])
def test_policies_compile(G, name):
    pol = getattr(W, f"{name}_policy")()
    src = G.jit_source(pol.code, pol.hook, _shapes(pol), compile=True)
    assert "gx_j_event_parallel" in src and "gx_j_stream_seq" in src


@pytest.mark.parametrize("i", range(6))
def test_generated_programs_compile(G, i):
    pol = W.gen_program(W.subseed(1003, 100 + i))
    G.jit_source(pol.code, pol.hook, _shapes(pol), compile=True)


def test_source_structure(G):
    pol = W.stride_prefetch_policy()
    src = G.jit_source(pol.code, pol.hook, _shapes(pol))
    assert src.count("hash_lookup(") == 1 and src.count("hash_update(") == 1
    assert src.count("ring_output(") == 1
    labels = set(re.findall(r"^L(\d+):;", src, re.M))
    gotos = set(re.findall(r"goto L(\d+);", src))
    assert labels == gotos


def test_rejected_program_reports_reason(G):
    code = W.Policy("loop", W.HOOK_MEM_ACCESS, "l:\n mov64 r0, 0\n ja l\n exit", []).code
    with pytest.raises(G.GxError) as e:
        G.jit_source(code, W.HOOK_MEM_ACCESS, [])
    assert e.value.errno == 13
