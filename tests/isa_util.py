"""Shared helpers for the oracle tests: tiny harness programs around one
instruction, and table readers for the golden fixtures."""

import os

import numpy as np

from paper_2512_12615_amd import asm
from paper_2512_12615_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            rows.append([c.strip() for c in line.split("|")])
    return rows


def one_event():
    ev = np.zeros(1, dtype=W.MEM_DTYPE)
    return ev


def alu_program(mnem, form, a, b):
    """Compute ``mnem`` on r6 = a (and r7 = b or the imm b); store r6 into an
    8-byte array map at index 0."""
    if form == "X":
        op = f"{mnem} r6, r7"
    elif form == "K":
        op = f"{mnem} r6, {b}"
    else:
        op = f"{mnem} r6"
    text = f"""
        lddw r6, {a & 0xFFFFFFFFFFFFFFFF}
        lddw r7, {b & 0xFFFFFFFFFFFFFFFF}
        {op}
        stw [r10-4], 0
        lddw r1, map:out
        mov64 r2, r10
        add64 r2, -4
        call map_lookup_elem
        jeq r0, 0, done
        stxdw [r0+0], r6
    done:
        mov64 r0, 0
        exit
    """
    return asm.assemble(text, ["out"])


def jmp_program(mnem, form, a, b):
    rhs = "r7" if form == "X" else str(b)
    text = f"""
        lddw r6, {a & 0xFFFFFFFFFFFFFFFF}
        lddw r7, {b & 0xFFFFFFFFFFFFFFFF}
        mov64 r0, 0
        {mnem} r6, {rhs}, taken
        exit
    taken:
        mov64 r0, 1
        exit
    """
    return asm.assemble(text)


def run_alu(mnem, form, a, b):
    from oracle import oracle as O
    o = O.Oracle()
    o.create_map(W.MAP_ARRAY, 4, 8, 1, 0)
    o.run(alu_program(mnem, form, a, b), W.HOOK_MEM_ACCESS, one_event())
    st = o.stats()
    assert st["faults"] == 0, st
    return int(o.dump(0)[1].view("<u8")[0, 0])


def run_jmp(mnem, form, a, b):
    from oracle import oracle as O
    o = O.Oracle()
    rc = o.run(jmp_program(mnem, form, a, b), W.HOOK_MEM_ACCESS, one_event())
    assert o.stats()["faults"] == 0
    return int(rc[0])


def pair_program(op_line, hi):
    """Per-event op on r6 = record.addr and r7 = record.ts; returns the low
    (hi=False) or high (hi=True) 32 bits of the result as rc."""
    text = f"""
        ldxdw r6, [r1+0]
        ldxdw r7, [r1+16]
        {op_line}
        {"rsh64 r6, 32" if hi else ""}
        mov64 r0, r6
        exit
    """
    return asm.assemble(text)


def run_pairs(op_line, a, b):
    """64-bit results of ``op_line`` over operand arrays a, b (uint64)."""
    from oracle import oracle as O
    ev = np.zeros(len(a), dtype=W.MEM_DTYPE)
    ev["addr"] = a
    ev["ts"] = b
    o = O.Oracle()
    lo = o.run(pair_program(op_line, False), W.HOOK_MEM_ACCESS, ev)
    hi = o.run(pair_program(op_line, True), W.HOOK_MEM_ACCESS, ev)
    assert o.stats()["faults"] == 0
    return lo.astype(np.uint64) | (hi.astype(np.uint64) << np.uint64(32))


def edge_operands(n, seed):
    """Operands mixing edge values with random ones."""
    edges = np.array([0, 1, 2, 3, 7, 31, 32, 33, 63, 64, 65, 0x7F, 0x80, 0xFF, 0x7FFF, 0x8000,
                      0x7FFFFFFF, 0x80000000, 0xFFFFFFFF, 0x100000000, 0x7FFFFFFFFFFFFFFF,
                      0x8000000000000000, 0xFFFFFFFFFFFFFFFF, 0xFFFFFFFFFFFFFFFE,
                      0xFFFFFFFF80000000, 0x123456789ABCDEF0], dtype=np.uint64)
    x = W.splitmix(seed, n)
    pick = (x % np.uint64(3)) == 0
    idx = (W.splitmix(seed + 1, n) % np.uint64(len(edges))).astype(np.int64)
    rnd = W.splitmix(seed + 2, n)
    small = W.splitmix(seed + 3, n) % np.uint64(100)
    out = np.where(pick, edges[idx], np.where((x % np.uint64(3)) == 1, small, rnd))
    return out.astype(np.uint64)
