"""Pins for the oracle's bounds/termination checker.

* A reject corpus: one program per rule class (unbounded loops, out-of-bounds
  or uninitialised accesses, missing null checks, pointer leaks, shared-map
  misuse, budgets, malformed encodings).  Each must be rejected.
* An accept corpus: the three policy programs and generated programs.
* Soundness by brute force: every accepted program over a small instruction
  alphabet runs in the oracle without a dynamic fault and retires no more
  instructions than the checker's bound.
"""

import itertools

import numpy as np
import pytest

from paper_2512_12615_amd import asm
from paper_2512_12615_amd import workloads as W
from oracle import oracle as O

ARR8 = (W.MAP_ARRAY, 4, 8, 16, 0)
SHARED = (W.MAP_ARRAY, 4, 8, 16, W.F_SHARED)
RO = (W.MAP_ARRAY, 4, 8, 16, W.F_READ_ONLY)
HASH = (W.MAP_HASH, 8, 16, 64, 0)
RING = (W.MAP_RINGBUF, 0, 0, 4096, 0)

LOOKUP_M0 = """
    stw [r10-4], 0
    lddw r1, map:m
    mov64 r2, r10
    add64 r2, -4
    call map_lookup_elem
"""


def chk(text, maps=(), hook=W.HOOK_MEM_ACCESS, names=None, raw=None):
    names = names or ["m", "n", "r"][:len(maps)]
    code = raw if raw is not None else asm.assemble(text, names)
    return O.check(code, hook, list(maps))


REJECTS = {
    "ja_self": ("l: ja l", ()),
    "loop_data_counter": ("ldxdw r2, [r1+0]\nl: add64 r2, 1\njlt r2, 10, l\nmov64 r0, 0\nexit", ()),
    "loop_no_update": ("mov64 r2, 0\nl: mov64 r3, 1\njeq r3, 1, l\nmov64 r0, 0\nexit", ()),
    "loop_ja_backedge": ("mov64 r2, 0\nl: add64 r2, 1\njgt r2, 5, out\nja l\nout: mov64 r0, 0\nexit", ()),
    "loop_counter_written_in_body": ("mov64 r6, 0\nl: mov64 r6, 1\nadd64 r6, 1\njlt r6, 4, l\nmov64 r0, 0\nexit", ()),
    "loop_counter_clobbered_by_call": ("mov64 r2, 0\nl:" + LOOKUP_M0 + "mov64 r2, 0\nadd64 r2, 1\njlt r2, 3, l\nmov64 r0, 0\nexit", (ARR8,)),
    "loop_too_many_trips": ("mov64 r6, 0\nl: add64 r6, 1\njlt r6, 100000, l\nmov64 r0, 0\nexit", ()),
    "loop_jump_into_body": ("mov64 r6, 0\nja mid\nl: mov64 r0, 0\nmid: mov64 r0, 1\nadd64 r6, 1\njlt r6, 3, l\nexit", ()),
    "loop_skips_update": ("mov64 r6, 0\nmov64 r0, 0\nl: jeq r0, 0, be\nadd64 r6, 1\nbe: jlt r6, 3, l\nexit", ()),
    "insn_budget": ("mov64 r6, 0\nl: add64 r6, 1\njlt r6, 40000, l\nmov64 r0, 0\nexit", ()),
    "call_budget": ("mov64 r6, 0\nl:" + LOOKUP_M0 + "add64 r6, 1\njlt r6, 65, l\nmov64 r0, 0\nexit", (ARR8,)),
    "stack_oob": ("mov64 r0, 0\nstdw [r10-520], 1\nexit", ()),
    "stack_positive": ("mov64 r0, 0\nstdw [r10+0], 1\nexit", ()),
    "stack_uninit_read": ("ldxdw r0, [r10-8]\nexit", ()),
    "stack_misaligned": ("stdw [r10-8], 1\nldxdw r0, [r10-4]\nexit", ()),
    "stack_partial_init": ("stw [r10-8], 1\nldxdw r0, [r10-8]\nexit", ()),
    "map_value_oob": (LOOKUP_M0 + "jeq r0, 0, o\nldxdw r0, [r0+8]\no: mov64 r0, 0\nexit", (ARR8,)),
    "no_null_check": (LOOKUP_M0 + "ldxdw r0, [r0+0]\nexit", (ARR8,)),
    "variable_offset_unbounded": ("ldxdw r6, [r1+0]\n" + LOOKUP_M0 + "jeq r0, 0, o\nadd64 r0, r6\nldxb r0, [r0+0]\no: mov64 r0, 0\nexit", (ARR8,)),
    "variable_offset_misaligned": ("ldxdw r6, [r1+0]\nand64 r6, 3\n" + LOOKUP_M0 + "jeq r0, 0, o\nadd64 r0, r6\nldxw r0, [r0+0]\no: mov64 r0, 0\nexit", (ARR8,)),
    "uninit_register": ("mov64 r0, r2\nexit", ()),
    "uninit_r0_at_exit": ("exit", ()),
    "pointer_in_r0": ("mov64 r0, r10\nexit", ()),
    "write_r10": ("mov64 r10, 0\nmov64 r0, 0\nexit", ()),
    "write_ctx": ("stdw [r1+0], 1\nmov64 r0, 0\nexit", ()),
    "ctx_bad_size": ("ldxw r0, [r1+0]\nexit", ()),
    "ctx_bad_offset": ("ldxdw r0, [r1+4]\nexit", ()),
    "ctx_out_of_record": ("ldxdw r0, [r1+24]\nexit", ()),
    "ctx_arithmetic": ("add64 r1, 8\nldxw r0, [r1+0]\nexit", ()),
    "jump_out_of_range": ("mov64 r0, 0\nja +5\nexit", ()),
    "jump_into_lddw": ("mov64 r0, 0\nja +1\nlddw r1, 5\nexit", ()),
    "fall_off_end": ("mov64 r0, 0", ()),
    "conditional_falls_off": ("mov64 r0, 0\njeq r0, 0, -2", ()),
    "unreachable": ("mov64 r0, 0\nexit\nmov64 r0, 1\nexit", ()),
    "div_by_const_zero": ("mov64 r0, 1\ndiv64 r0, 0\nexit", ()),
    "mod_by_const_zero": ("mov64 r0, 1\nmod32 r0, 0\nexit", ()),
    "shift_const_64": ("mov64 r0, 1\nlsh64 r0, 64\nexit", ()),
    "shift_const_32": ("mov64 r0, 1\nrsh32 r0, 32\nexit", ()),
    "helper_scalar_map": ("mov64 r1, 0\nmov64 r2, r10\ncall map_lookup_elem\nmov64 r0, 0\nexit", ()),
    "helper_key_uninit": ("lddw r1, map:m\nmov64 r2, r10\nadd64 r2, -4\ncall map_lookup_elem\nmov64 r0, 0\nexit", (ARR8,)),
    "helper_unknown": ("call 6\nmov64 r0, 0\nexit", ()),
    "ring_size_variable": ("ldxdw r3, [r1+0]\nstdw [r10-8], 0\nlddw r1, map:m\nmov64 r2, r10\nadd64 r2, -8\nmov64 r4, 0\ncall ringbuf_output\nmov64 r0, 0\nexit", (RING,)),
    "ring_size_too_big": ("stdw [r10-8], 0\nlddw r1, map:m\nmov64 r2, r10\nadd64 r2, -8\nmov64 r3, 5000\nmov64 r4, 0\ncall ringbuf_output\nmov64 r0, 0\nexit", (RING,)),
    "ring_data_beyond_stack": ("stdw [r10-8], 0\nlddw r1, map:m\nmov64 r2, r10\nadd64 r2, -8\nmov64 r3, 16\nmov64 r4, 0\ncall ringbuf_output\nmov64 r0, 0\nexit", (RING,)),
    "store_pointer": (LOOKUP_M0 + "jeq r0, 0, o\nstxdw [r0+0], r10\no: mov64 r0, 0\nexit", (ARR8,)),
    "spill_pointer": ("stxdw [r10-8], r1\nmov64 r0, 0\nexit", ()),
    "pointer_compare": ("mov64 r0, 0\njgt r10, 5, +0\nexit", ()),
    "shared_plain_store": (LOOKUP_M0 + "jeq r0, 0, o\nstdw [r0+0], 1\no: mov64 r0, 0\nexit", (SHARED,)),
    "shared_plain_load": (LOOKUP_M0 + "jeq r0, 0, o\nldxdw r0, [r0+0]\no: mov64 r0, 0\nexit", (SHARED,)),
    "shared_fetch_add": (LOOKUP_M0 + "jeq r0, 0, o\nmov64 r1, 1\nafadd64 [r0+0], r1\no: mov64 r0, 0\nexit", (SHARED,)),
    "shared_xchg": (LOOKUP_M0 + "jeq r0, 0, o\nmov64 r1, 1\naxchg64 [r0+0], r1\no: mov64 r0, 0\nexit", (SHARED,)),
    "shared_cmpxchg": (LOOKUP_M0 + "jeq r0, 0, o\nmov64 r1, 1\nmov64 r9, r0\nmov64 r0, 0\nacmpxchg64 [r9+0], r1\no: mov64 r0, 0\nexit", (SHARED,)),
    "shared_update": ("stw [r10-4], 0\nstdw [r10-16], 0\nlddw r1, map:m\nmov64 r2, r10\nadd64 r2, -4\nmov64 r3, r10\nadd64 r3, -16\nmov64 r4, 0\ncall map_update_elem\nmov64 r0, 0\nexit", (SHARED,)),
    "shared_mixed_ops": (LOOKUP_M0 + "jeq r0, 0, o\nmov64 r1, 1\naadd64 [r0+0], r1\naor64 [r0+0], r1\no: mov64 r0, 0\nexit", (SHARED,)),
    "shared_mixed_widths": (LOOKUP_M0 + "jeq r0, 0, o\nmov64 r1, 1\naadd64 [r0+0], r1\naadd32 [r0+0], r1\no: mov64 r0, 0\nexit", (SHARED,)),
    "readonly_store": (LOOKUP_M0 + "jeq r0, 0, o\nstdw [r0+0], 1\no: mov64 r0, 0\nexit", (RO,)),
    "readonly_atomic": (LOOKUP_M0 + "jeq r0, 0, o\nmov64 r1, 1\naadd64 [r0+0], r1\no: mov64 r0, 0\nexit", (RO,)),
    "hash_pointer_after_update": ("stdw [r10-8], 1\nstdw [r10-24], 0\nstdw [r10-16], 0\nlddw r1, map:m\nmov64 r2, r10\nadd64 r2, -8\ncall map_lookup_elem\njeq r0, 0, o\nmov64 r6, r0\nlddw r1, map:m\nmov64 r2, r10\nadd64 r2, -8\nmov64 r3, r10\nadd64 r3, -24\nmov64 r4, 0\ncall map_update_elem\nldxdw r0, [r6+0]\nexit\no: mov64 r0, 0\nexit", (HASH,)),
    "lookup_on_ring": ("stw [r10-4], 0\nlddw r1, map:m\nmov64 r2, r10\nadd64 r2, -4\ncall map_lookup_elem\nmov64 r0, 0\nexit", (RING,)),
    "map32_move_leak": ("mov32 r0, r10\nexit", ()),
}

RAW_REJECTS = {
    "unknown_opcode": bytes.fromhex("ff00000000000000") + asm.assemble("exit"),
    "alu_k_src_set": asm.encode(0x07, 1, 2, 0, 1) + asm.assemble("mov64 r0, 0\nexit"),
    "alu_x_imm_set": asm.assemble("mov64 r1, 0") + asm.encode(0x0F, 1, 1, 0, 7) + asm.assemble("mov64 r0, 0\nexit"),
    "bad_end_width": asm.assemble("mov64 r0, 0") + asm.encode(0xD4, 0, 0, 0, 8) + asm.assemble("exit"),
    "exit_fields": asm.assemble("mov64 r0, 0") + asm.encode(0x95, 0, 0, 0, 1),
    "lddw_src_2": asm.encode(0x18, 1, 2, 0, 0) + asm.encode(0) + asm.assemble("mov64 r0, 0\nexit"),
    "lddw_truncated": asm.assemble("mov64 r0, 0\nexit") + asm.encode(0x18, 1, 0, 0, 0),
    "bad_register": asm.encode(0xB7, 11, 0, 0, 0) + asm.assemble("exit"),
    "ldx_abs_mode": asm.encode(0x20, 0, 0, 0, 0) + asm.assemble("exit"),
    "movsx_k_form": asm.encode(0xB7, 0, 0, 8, 1) + asm.assemble("exit"),
    "too_long": asm.assemble("mov64 r0, 0\n" * 4096 + "exit"),
    "empty": b"",
}


@pytest.mark.parametrize("name", sorted(REJECTS))
def test_reject_corpus(name):
    text, maps = REJECTS[name]
    r = chk(text, maps)
    assert not r.ok, f"{name} accepted"


@pytest.mark.parametrize("name", sorted(RAW_REJECTS))
def test_reject_raw(name):
    r = O.check(RAW_REJECTS[name], W.HOOK_MEM_ACCESS, [])
    assert not r.ok, f"{name} accepted"


def test_accept_bounded_loop_facts():
    r = chk("mov64 r0, 0\nmov64 r6, 0\nl: add64 r0, 2\nadd64 r6, 1\njlt r6, 10, l\nexit")
    assert r.ok, r.log
    assert r.max_insns == 2 + 3 * 10 + 1
    assert r.stack_bytes == 0 and r.event_parallel


def test_accept_variable_offset_in_bounds():
    text = ("ldxdw r6, [r1+0]\nand64 r6, 1\nlsh64 r6, 3\n" + LOOKUP_M0 +
            "jeq r0, 0, o\nadd64 r0, r6\nldxdw r0, [r0+0]\nexit\no: mov64 r0, 0\nexit")
    r = chk(text, ((W.MAP_ARRAY, 4, 16, 4, 0),))
    assert r.ok, r.log
    assert not r.event_parallel  # owned array => stream-sequential


def test_policies_accepted_with_facts():
    facts = {}
    for pol in [W.access_counter_policy(), W.stride_prefetch_policy(), W.latency_hist_policy()]:
        shapes = [(m.type, m.key_size, m.value_size, m.max_entries, m.flags) for m in pol.maps]
        r = O.check(pol.code, pol.hook, shapes)
        assert r.ok, (pol.name, r.log)
        facts[pol.name] = r
    assert facts["access_counter"].event_parallel
    assert facts["latency_hist"].event_parallel
    assert not facts["stride_prefetch"].event_parallel
    assert facts["stride_prefetch"].max_ring_bytes == 40
    assert facts["latency_hist"].max_ring_bytes == 40
    assert facts["access_counter"].max_calls == 1


def test_generated_programs_accepted():
    for seed in range(48):
        pol = W.gen_program(W.subseed(1003, 100 + seed))
        shapes = [(m.type, m.key_size, m.value_size, m.max_entries, m.flags) for m in pol.maps]
        r = O.check(pol.code, pol.hook, shapes)
        assert r.ok, (seed, r.log, pol.text)
        assert 16 <= len(pol.code) // 8 <= 600


# -------------------------------------------------------------------------
# soundness by brute force

ALPHABET = ["mov64 r0, 0", "mov64 r0, 1", "add64 r0, 1", "sub64 r0, 1", "mov64 r1, 0",
            "ldxdw r0, [r1+0]", "stdw [r10-8], 1", "ldxdw r0, [r10-8]", "exit",
            "mov64 r6, 0", "add64 r6, 1"]
JUMPS = ["ja {k}", "jeq r0, 0, {k}", "jlt r0, 2, {k}", "jgt r0, 1, {k}", "jlt r6, 3, {k}"]
OFFS = [-3, -2, -1, 0, 1, 2, 3]


def _alphabet():
    out = list(ALPHABET)
    for j in JUMPS:
        for k in OFFS:
            out.append(j.format(k=f"{k:+d}"))
    return out


def _sound(progs):
    ev = np.zeros(4, dtype=W.MEM_DTYPE)
    ev["addr"] = [0, 1, 2, 0xFFFFFFFFFFFFFFFF]
    accepted = 0
    for p in progs:
        code = asm.assemble("\n".join(p))
        r = O.check(code, W.HOOK_MEM_ACCESS, [])
        if not r.ok:
            continue
        accepted += 1
        o = O.Oracle()
        o.run(code, W.HOOK_MEM_ACCESS, ev)
        st = o.stats()
        assert st["faults"] == 0, (p, st["fault_msg"])
        assert st["insns"] <= 4 * r.max_insns, (p, st["insns"], r.max_insns)
    return accepted


def test_soundness_all_programs_up_to_3():
    a = _alphabet()
    progs = [p for n in (1, 2, 3) for p in itertools.product(a, repeat=n)]
    assert _sound(progs) > 20


# every program of four instructions over a core alphabet: the loads and
# stores, a counter and its counted-loop jumps back, forward jumps over one
# or two instructions, an unconditional loop and the exit
CORE4 = ["mov64 r0, 0", "add64 r0, 1", "mov64 r1, 0", "ldxdw r0, [r1+0]", "stdw [r10-8], 1",
         "ldxdw r0, [r10-8]", "exit", "mov64 r6, 0", "add64 r6, 1", "ja -1", "ja +1",
         "jeq r0, 0, +1", "jgt r0, 1, +2", "jeq r0, 0, -2", "jlt r6, 3, -2", "jlt r6, 3, -3"]


def test_soundness_all_programs_of_4_over_a_core_alphabet():
    progs = list(itertools.product(CORE4, repeat=4))
    assert len(progs) == 16 ** 4
    assert _sound(progs) > 100


def test_soundness_framed_programs():
    """Three enumerated instructions between an initialising prefix and an
    exit, so that loops and branches over initialised registers are covered."""
    a = _alphabet()
    rng = np.random.default_rng(7)
    pre, post = ("mov64 r0, 0", "mov64 r6, 0"), ("exit",)
    progs = [pre + tuple(a[i] for i in rng.integers(0, len(a), 3)) + post for _ in range(40000)]
    loops = [p for p in progs if any(x.startswith("jlt r6, 3, -") for x in p)]
    assert _sound(progs) > 1000
    assert _sound(loops) > 10
