"""Pins for the oracle's instruction semantics.

1. Hand-worked edge tables (tests/golden/alu_edge.txt, jmp_edge.txt) derived
   from the eBPF instruction-set standard.
2. Per-opcode cross-checks over thousands of edge-heavy operand pairs against
   what numpy's fixed-width integer arithmetic or Python's exact integers
   define for the same operation (wrapping add/sub/mul, masked shifts,
   unsigned division, two's-complement comparisons, byte swaps, sign
   extension), plus identities for signed division (q*b + r == a, |r| < |b|,
   r has the sign of a).
3. Memory forms: sign/zero extension of loads, store truncation, byte order,
   and every atomic operation on literal values.
"""

import numpy as np
import pytest

from isa_util import edge_operands, read_table, run_alu, run_jmp, run_pairs

from paper_2512_12615_amd import asm
from paper_2512_12615_amd import workloads as W

M64 = (1 << 64) - 1
M32 = (1 << 32) - 1


@pytest.mark.parametrize("row", read_table("alu_edge.txt"), ids=lambda r: f"{r[0]}-{r[2]}-{r[3]}")
def test_alu_edge_table(row):
    mnem, form, a, b, expected = row[0], row[1], int(row[2], 0), int(row[3], 0), int(row[4], 0)
    assert run_alu(mnem, form, a, b) == expected


@pytest.mark.parametrize("row", read_table("jmp_edge.txt"), ids=lambda r: f"{r[0]}-{r[2]}-{r[3]}")
def test_jmp_edge_table(row):
    mnem, form, a, b, taken = row[0], row[1], int(row[2], 0), int(row[3], 0), int(row[4], 0)
    assert run_jmp(mnem, form, a, b) == taken


N = 3000


@pytest.fixture(scope="module")
def ops():
    a = edge_operands(N, 11)
    b = edge_operands(N, 23)
    return a, b


def _s64(x):
    return x.view(np.int64)


def test_wrapping_ops_match_numpy(ops):
    a, b = ops
    with np.errstate(over="ignore"):
        assert np.array_equal(run_pairs("add64 r6, r7", a, b), a + b)
        assert np.array_equal(run_pairs("sub64 r6, r7", a, b), a - b)
        assert np.array_equal(run_pairs("mul64 r6, r7", a, b), a * b)
        assert np.array_equal(run_pairs("and64 r6, r7", a, b), a & b)
        assert np.array_equal(run_pairs("or64 r6, r7", a, b), a | b)
        assert np.array_equal(run_pairs("xor64 r6, r7", a, b), a ^ b)
        a32, b32 = a.astype(np.uint32), b.astype(np.uint32)
        for op, ref in [("add32", a32 + b32), ("sub32", a32 - b32), ("mul32", a32 * b32),
                        ("xor32", a32 ^ b32), ("and32", a32 & b32), ("or32", a32 | b32)]:
            assert np.array_equal(run_pairs(f"{op} r6, r7", a, b), ref.astype(np.uint64)), op


def test_shifts_are_masked(ops):
    a, b = ops
    k64 = b & np.uint64(63)
    k32 = (b & np.uint64(31)).astype(np.uint32)
    assert np.array_equal(run_pairs("lsh64 r6, r7", a, b), a << k64)
    assert np.array_equal(run_pairs("rsh64 r6, r7", a, b), a >> k64)
    assert np.array_equal(run_pairs("arsh64 r6, r7", a, b), (_s64(a) >> k64.astype(np.int64)).view(np.uint64))
    a32 = a.astype(np.uint32)
    assert np.array_equal(run_pairs("lsh32 r6, r7", a, b), (a32 << k32).astype(np.uint64))
    assert np.array_equal(run_pairs("rsh32 r6, r7", a, b), (a32 >> k32).astype(np.uint64))
    ar = (a32.view(np.int32) >> k32.astype(np.int32)).view(np.uint32).astype(np.uint64)
    assert np.array_equal(run_pairs("arsh32 r6, r7", a, b), ar)


def test_unsigned_division(ops):
    a, b = ops
    nz = np.where(b == 0, np.uint64(1), b)
    assert np.array_equal(run_pairs("div64 r6, r7", a, b), np.where(b == 0, np.uint64(0), a // nz))
    assert np.array_equal(run_pairs("mod64 r6, r7", a, b), np.where(b == 0, a, a % nz))
    a32, b32 = a.astype(np.uint32), b.astype(np.uint32)
    nz32 = np.where(b32 == 0, np.uint32(1), b32)
    assert np.array_equal(run_pairs("div32 r6, r7", a, b),
                          np.where(b32 == 0, 0, a32 // nz32).astype(np.uint64))
    assert np.array_equal(run_pairs("mod32 r6, r7", a, b),
                          np.where(b32 == 0, a32, a32 % nz32).astype(np.uint64))


@pytest.mark.parametrize("width", [64, 32])
def test_signed_division_identities(ops, width):
    a, b = ops
    q = run_pairs(f"sdiv{width} r6, r7", a, b)
    r = run_pairs(f"smod{width} r6, r7", a, b)
    mask = M64 if width == 64 else M32
    half = 1 << (width - 1)

    def sg(v):
        v &= mask
        return v - (1 << width) if v >= half else v

    for ai, bi, qi, ri in zip(a.tolist(), b.tolist(), q.tolist(), r.tolist()):
        if width == 32:
            assert qi >> 32 == 0 and ri >> 32 == 0  # zero-extended results
        sa, sb, sq, sr = sg(ai), sg(bi), sg(qi), sg(ri)
        if sb == 0:
            assert sq == 0 and sr == sa
        elif sa == -half and sb == -1:
            assert sq == -half and sr == 0
        else:
            assert sq * sb + sr == sa
            assert abs(sr) < abs(sb)
            assert sr == 0 or (sr < 0) == (sa < 0)
            # truncation toward zero
            assert sq == int(abs(sa) // abs(sb)) * (1 if (sa < 0) == (sb < 0) else -1)


def test_moves_and_extension(ops):
    a, b = ops
    assert np.array_equal(run_pairs("mov64 r6, r7", a, b), b)
    assert np.array_equal(run_pairs("mov32 r6, r7", a, b), b & np.uint64(M32))
    for bits, t in [(8, np.int8), (16, np.int16), (32, np.int32)]:
        want = b.astype(t).astype(np.int64).view(np.uint64)
        assert np.array_equal(run_pairs(f"movsx{bits}_64 r6, r7", a, b), want)
    for bits, t in [(8, np.int8), (16, np.int16)]:
        want = b.astype(t).astype(np.int32).view(np.uint32).astype(np.uint64)
        assert np.array_equal(run_pairs(f"movsx{bits}_32 r6, r7", a, b), want)
    assert np.array_equal(run_pairs("neg64 r6", a, b), (np.uint64(0) - a))
    assert np.array_equal(run_pairs("neg32 r6", a, b), (np.uint32(0) - a.astype(np.uint32)).astype(np.uint64))


def test_byte_swaps(ops):
    a, _ = ops
    assert np.array_equal(run_pairs("bswap64 r6", a, a), a.byteswap())
    assert np.array_equal(run_pairs("be64 r6", a, a), a.byteswap())
    assert np.array_equal(run_pairs("be32 r6", a, a), a.astype(np.uint32).byteswap().astype(np.uint64))
    assert np.array_equal(run_pairs("bswap16 r6", a, a), a.astype(np.uint16).byteswap().astype(np.uint64))
    assert np.array_equal(run_pairs("le16 r6", a, a), a & np.uint64(0xFFFF))
    assert np.array_equal(run_pairs("le32 r6", a, a), a & np.uint64(M32))
    assert np.array_equal(run_pairs("le64 r6", a, a), a)


JMPS = ["jeq", "jne", "jgt", "jge", "jlt", "jle", "jsgt", "jsge", "jslt", "jsle", "jset"]


def _ref_jump(op, a, b):
    sa, sb = a.view(np.int64), b.view(np.int64)
    return {
        "jeq": a == b, "jne": a != b, "jgt": a > b, "jge": a >= b, "jlt": a < b, "jle": a <= b,
        "jsgt": sa > sb, "jsge": sa >= sb, "jslt": sa < sb, "jsle": sa <= sb, "jset": (a & b) != 0,
    }[op]


@pytest.mark.parametrize("op", JMPS)
def test_jumps_match_twos_complement(ops, op):
    a, b = ops
    for suffix, aa, bb in [("", a, b), ("32", a.astype(np.uint32), b.astype(np.uint32))]:
        text = f"""
            ldxdw r6, [r1+0]
            ldxdw r7, [r1+16]
            mov64 r0, 1
            {op}{suffix} r6, r7, out
            mov64 r0, 0
        out:
            exit
        """
        ev = np.zeros(len(a), dtype=W.MEM_DTYPE)
        ev["addr"], ev["ts"] = a, b
        from oracle import oracle as O
        rc = O.Oracle().run(asm.assemble(text), W.HOOK_MEM_ACCESS, ev)
        if suffix:
            signed = op.startswith("js") and op != "jset"
            widen = (lambda v: v.view(np.int32).astype(np.int64).view(np.uint64)) if signed else \
                (lambda v: v.astype(np.uint64))
            ref = _ref_jump(op, widen(aa), widen(bb))
        else:
            ref = _ref_jump(op, aa, bb)
        assert np.array_equal(rc.astype(bool), ref), op + suffix


def _mem_program(body):
    return asm.assemble(f"""
        stw [r10-4], 0
        lddw r1, map:m
        mov64 r2, r10
        add64 r2, -4
        call map_lookup_elem
        jeq r0, 0, out
        mov64 r9, r0
        {body}
    out:
        exit
    """, ["m"])


def _run_mem(body, init: bytes, vsz=16):
    from oracle import oracle as O
    o = O.Oracle()
    o.create_map(W.MAP_ARRAY, 4, vsz, 1, 0)
    o.update(0, b"\0\0\0\0", init.ljust(vsz, b"\0"))
    ev = np.zeros(1, dtype=W.MEM_DTYPE)
    rc = o.run(_mem_program(body), W.HOOK_MEM_ACCESS, ev)
    assert o.stats()["faults"] == 0, o.stats()
    return int(rc[0]), o.dump(0)[1][0].tobytes()


# (body, initial value bytes, expected rc, expected value bytes or None)
MEM_CASES = [
    ("ldxb r0, [r9+0]", b"\x80", 0x80, None),                        # zero-extending byte load
    ("ldxsb r0, [r9+0]\nrsh64 r0, 32", b"\x80", 0xFFFFFFFF, None),   # sign-extended to 64 bits
    ("ldxsh r0, [r9+0]", b"\x00\x80", 0xFFFF8000, None),
    ("ldxsw r0, [r9+0]\nrsh64 r0, 32", b"\x00\x00\x00\x80", 0xFFFFFFFF, None),
    ("ldxw r0, [r9+0]\nrsh64 r0, 32", b"\xff\xff\xff\xff", 0, None),  # zero-extended
    ("ldxh r0, [r9+2]", b"\x11\x22\x33\x44", 0x4433, None),          # little endian
    ("stw [r9+0], 0x11223344\nldxb r0, [r9+0]", b"", 0x44, b"\x44\x33\x22\x11"),
    ("stb [r9+1], 0x1ff\nmov64 r0, 0", b"", 0, b"\x00\xff"),          # store truncates
    ("stdw [r9+8], -1\nldxw r0, [r9+12]", b"", 0xFFFFFFFF, b"\0" * 8 + b"\xff" * 8),  # imm sign-extends
    ("mov64 r1, 3\naadd64 [r9+0], r1\nmov64 r0, r1", b"\x05", 3, b"\x08"),
    ("mov64 r1, 3\nafadd64 [r9+0], r1\nmov64 r0, r1", b"\x05", 5, b"\x08"),   # fetch returns old
    ("mov64 r1, 1\naadd32 [r9+0], r1\nmov64 r0, 0", b"\xff\xff\xff\xff\x07", 0, b"\0\0\0\0\x07"),  # W wraps alone
    ("lddw r1, 0x100000001\nafadd32 [r9+0], r1\nrsh64 r1, 32\nmov64 r0, r1", b"\x05", 0, b"\x06"),
    ("mov64 r1, 0x0c\naor64 [r9+0], r1\nmov64 r0, 0", b"\x03", 0, b"\x0f"),
    ("mov64 r1, 0x06\nafand64 [r9+0], r1\nmov64 r0, r1", b"\x0c", 0x0c, b"\x04"),
    ("mov64 r1, 0x06\nafxor64 [r9+0], r1\nmov64 r0, r1", b"\x0c", 0x0c, b"\x0a"),
    ("mov64 r1, 9\naxchg64 [r9+0], r1\nmov64 r0, r1", b"\x05", 5, b"\x09"),
    ("mov64 r0, 5\nmov64 r1, 9\nacmpxchg64 [r9+0], r1", b"\x05", 5, b"\x09"),   # equal: swap
    ("mov64 r0, 4\nmov64 r1, 9\nacmpxchg64 [r9+0], r1", b"\x05", 5, b"\x05"),   # not equal: keep
    ("lddw r0, 0x700000005\nmov64 r1, 9\nacmpxchg32 [r9+0], r1", b"\x05", 5, b"\x09"),  # low 32 compared
]


@pytest.mark.parametrize("case", MEM_CASES, ids=[c[0].replace("\n", ";") for c in MEM_CASES])
def test_memory_forms(case):
    body, init, want_rc, want_val = case
    rc, val = _run_mem(body, init)
    assert rc == want_rc
    if want_val is not None:
        assert val[:len(want_val)] == want_val


def test_lddw_counts_as_one_instruction():
    from oracle import oracle as O
    o = O.Oracle()
    o.run(asm.assemble("lddw r0, 0x1122334455667788\nexit"), W.HOOK_MEM_ACCESS, np.zeros(3, W.MEM_DTYPE))
    assert o.stats()["insns"] == 6


def test_return_code_is_low_32_bits():
    from oracle import oracle as O
    rc = O.Oracle().run(asm.assemble("lddw r0, 0xaabbccdd11223344\nexit"), W.HOOK_MEM_ACCESS,
                        np.zeros(1, W.MEM_DTYPE))
    assert int(rc[0]) == 0x11223344
