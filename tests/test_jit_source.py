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
    # only the kernel of the program's mode
    if name == "stride_prefetch":
        assert "gx_j_stream_seq" in src and "gx_j_event_parallel" not in src
    else:
        assert "gx_j_event_parallel" in src and "gx_j_stream_seq" not in src


@pytest.mark.parametrize("i", range(6))
def test_generated_programs_compile(G, i):
    pol = W.gen_program(W.subseed(1003, 100 + i))
    G.jit_source(pol.code, pol.hook, _shapes(pol), compile=True)


def test_source_structure(G):
    pol = W.stride_prefetch_policy()
    src = G.jit_source(pol.code, pol.hook, _shapes(pol))
    # the lookup is emitted twice: through the LDS memo table (one queue per
    # wave) and through the per-lane register memo (several queues per wave);
    # its key lies in a frame word (private frame), so it is passed by value
    assert src.count("hash_lookup_k(") == 2 and src.count("hash_update(") == 1
    assert "saddr(stk, (uint32_t)" not in src  # no stack access left in LDS
    # the ring record lies in the frame too: its words go to the helper by value
    assert src.count("ring_output_words(") == 1 and "ring_output_chunked(" not in src
    labels = set(re.findall(r"^L(\d+):;", src, re.M))
    gotos = set(re.findall(r"goto L(\d+);", src))
    assert labels == gotos


def test_rejected_program_reports_reason(G):
    code = W.Policy("loop", W.HOOK_MEM_ACCESS, "l:\n mov64 r0, 0\n ja l\n exit", []).code
    with pytest.raises(G.GxError) as e:
        G.jit_source(code, W.HOOK_MEM_ACCESS, [])
    assert e.value.errno == 13


BIG_STACK_SHARED = """
    ldxdw r6, [r1+0]
    stdw [r10-512], 0
    stxdw [r10-8], r6
    mov64 r1, r6
    and64 r1, 4095
    stxw [r10-16], r1
    lddw r1, map:sh
    mov64 r2, r10
    add64 r2, -16
    call map_lookup_elem
    jeq r0, 0, out
    mov64 r1, 1
    aadd64 [r0+0], r1
out:
    ldxdw r0, [r10-512]
    exit
"""


@pytest.mark.parametrize("entries", [4096, 1 << 16])
def test_largest_frame_with_accumulators_compiles(G, entries):
    """A 512-byte frame (the largest) plus a shared map's LDS accumulator
    (whole-map mirror or tagged cache) stays within the LDS of a block."""
    pol = W.Policy("big", W.HOOK_MEM_ACCESS, BIG_STACK_SHARED, [W.MapSpec("sh", W.MAP_ARRAY, 4, 8, entries, W.F_SHARED)])
    src = G.jit_source(pol.code, pol.hook, _shapes(pol), compile=True)
    assert "g_acc0" in src or "g_tag0" in src or "if (PRIV)" not in src


UNALIGNED_RECORD = """
    ldxdw r6, [r1+0]
    stxdw [r10-16], r6
    stxdw [r10-8], r6
    lddw r1, map:ring
    mov64 r2, r10
    add64 r2, -12
    mov64 r3, 12
    mov64 r4, 0
    call ringbuf_output
    mov64 r0, 0
    exit
"""


def test_frames_and_cache_layout(G):
    """An event-parallel program whose stack never leaves its private frame
    keeps no LDS frames (the latency histogram: its ring record goes to the
    helper by value; the 512-byte frame above: its key goes by value), and
    its histogram's cache takes 8-bit tags (word index / sets < 255, four
    tags per 32-bit word); a record the helper must read from the stack (not
    word-aligned) keeps the LDS frames, and a map too large for 8-bit tags
    keeps 32-bit ones."""
    pol = W.latency_hist_policy()
    src = G.jit_source(pol.code, pol.hook, _shapes(pol))
    assert "#define GX_LDS_BYTES 16\n" in src
    body = src[src.index("uint64_t r10"):]
    assert "cache_add_narrow<true>(" in src and not re.search(r"\bstk\b", body[:body.index("\n};\n")])
    sets = int(re.search(r"g_tag0\[(\d+)\]", src).group(1))
    assert int(re.search(r"g_val0\[(\d+)\]", src).group(1)) == 4 * sets and sets % 2 == 1
    assert 4096 * 64 // sets < 255
    big = W.Policy("big", W.HOOK_MEM_ACCESS, BIG_STACK_SHARED, [W.MapSpec("sh", W.MAP_ARRAY, 4, 8, 1 << 21, W.F_SHARED)])
    src = G.jit_source(big.code, big.hook, _shapes(big), compile=True)
    assert "#define GX_LDS_BYTES 16\n" in src
    sets = int(re.search(r"g_val0\[(\d+)\]", src).group(1)) // 4
    assert (1 << 21) // sets >= 255 and "cache_add_narrow<false>(" in src
    assert int(re.search(r"g_tag0\[(\d+)\]", src).group(1)) == 4 * sets
    una = W.Policy("una", W.HOOK_MEM_ACCESS, UNALIGNED_RECORD, [W.MapSpec("ring", W.MAP_RINGBUF, 0, 0, 1 << 16, 0)])
    src = G.jit_source(una.code, una.hook, _shapes(una), compile=True)
    assert "#define GX_LDS_BYTES 16\n" not in src and "ring_output_chunked(" in src


def test_source_holds_no_map_addresses(G):
    """Map addresses come from the run's map table, so the text carries only
    shapes: program instances with same-shaped maps share one module."""
    for pol in (W.stride_prefetch_policy(), W.latency_hist_policy(), W.gen_program(W.subseed(1003, 101))):
        src = G.jit_source(pol.code, pol.hook, _shapes(pol))
        assert "0x1000000" not in src and "0x2000000" not in src  # the stand-in descriptor/data addresses
        assert "A.maptab" in src


def test_program_set_compiles(G):
    """A set of programs of both modes compiles into one module with one
    persistent kernel that switches on the program's slot."""
    pols = [W.access_counter_policy(), W.stride_prefetch_policy(), W.latency_hist_policy()] + \
        [W.gen_program(W.subseed(1003, 100 + i)) for i in range(3)]
    src = G.jit_set_source([(p.code, p.hook, _shapes(p)) for p in pols], compile=True)
    assert src.count("gx_j_set(") == 1
    for k in range(len(pols)):
        assert f"namespace p{k} " in src and f"case {k}u:" in src


def test_map_value_windows(G):
    """The stride policy's value reads come from the window loaded after its
    one lookup; in the alias programs every read after a store through
    another pointer, an atomic or an update goes to memory."""
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    import jit_window_programs as P
    pol = W.stride_prefetch_policy()
    src = G.jit_source(pol.code, pol.hook, _shapes(pol))
    assert src.count("if (r0) { w0_0 = ") == 2  # both memo forms
    # no value load through a pointer is left: every LDX reads the window
    assert "r1 = uni<UNI>((uint64_t)(*(const GX_GLOBAL" not in src
    assert src.count("(w0_0 >> 0)") == 1 and src.count("(w0_1 >> 0)") == 1 and src.count("(w0_2 >> 0)") == 1
    for name in P.PROGRAMS:
        p = P.policy(name)
        s = G.jit_source(p.code, p.hook, _shapes(p), compile=True)
        body = s[s.index("uint64_t r10"):]
        lines = body.splitlines()
        if name == "alias":
            # after the store through the second pointer, reads of the first go to memory
            i = next(k for k, l in enumerate(lines) if "w1_0 = (uint64_t)" in l)
            assert all(" >> " not in l for l in lines[i:])
        if name in ("atomic", "update"):
            i = next(k for k, l in enumerate(lines) if "atomic_global(" in l or "array_update(" in l)
            assert all(" >> " not in l for l in lines[i:])


def test_lookup_memo(G):
    """The stride policy's one lookup site keeps its key, value address and
    window across events; the insert (an update of the map) clears every
    memo entry, and the entry of the key held in registers is written back
    to the LDS table when the registers move on to another key.  In the
    memo test program the delete and the in-place update clear it too, and
    the second lookup site is a memo of its own."""
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    import jit_window_programs as P
    pol = W.stride_prefetch_policy()
    src = G.jit_source(pol.code, pol.hook, _shapes(pol))
    assert "__shared__ __attribute__((aligned(16))) uint64_t g_memo0[384];" in src  # 64 entries x 6 words
    assert src.count("gen0++") == 1
    i_gen, i_upd = src.index("gen0++"), src.index("hash_update(")
    assert i_gen < i_upd and "hash_lookup(" not in src[i_gen:i_upd]
    for j in range(3):
        assert f"g_memo0[cur0 * 6u + {3 + j}u] = w0_{j};" in src
    p = P.policy("memo")
    s = G.jit_source(p.code, p.hook, _shapes(p), compile=True)
    # the first site's table takes 3 KiB of the 4 KiB budget: the second
    # site keeps one entry in registers
    assert "g_memo0[" in s and "g_memo1[" not in s and "mk1 = mk;" in s
    for call in ("hash_delete(", "hash_update("):
        head = s[:s.index(call)]
        assert head.rstrip().splitlines()[-1].strip().startswith("mv0 = false; gen0++;") or "gen0++" in head[-400:]
    # an event-parallel program has no memo (its lanes take other streams' events)
    hist = W.latency_hist_policy()
    assert "g_memo" not in G.jit_source(hist.code, hist.hook, _shapes(hist))
