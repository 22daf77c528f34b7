"""eBPF text assembler and disassembler for policy programs.

Policy authors of the paper's system build bytecode with clang/libbpf (paper
section 4.2, "User-space Control Plane"); no BPF compiler backend is available
here, so programs are written in this small assembly language instead.  The
encoding is the standard eBPF one: 8-byte little-endian instructions
``opcode:u8 | dst:4 | src:4 | off:s16 | imm:s32``; ``lddw`` takes two slots.

This module only encodes instructions.  It holds none of the instruction
semantics: the CPU oracle and the GPU runtime each decode the bytes on their
own.

Syntax (one instruction per line, ``;`` or ``#`` starts a comment)::

    label:
    add64 r1, r2          ; ALU64 X form      add32 r1, 5  ; ALU32 K form
    sub mul div sdiv or and lsh rsh mod smod xor mov arsh  (+ 64 / 32)
    movsx8_64 r1, r2      ; MOVSX (also movsx16_64, movsx32_64, movsx8_32, movsx16_32)
    neg64 r1 | neg32 r1
    le16 r1 | le32 | le64 | be16 | be32 | be64 | bswap16 | bswap32 | bswap64
    ja label              ; ja32 label uses the imm field (JMP32|JA)
    jeq r1, r2, label     ; jeq jgt jge jset jne jsgt jsge jlt jle jslt jsle
    jeq32 r1, 7, label    ; JMP32 forms
    call map_lookup_elem  ; or call <number>
    exit
    ldxdw r0, [r1+8]      ; ldxb ldxh ldxw ldxdw, sign-extending ldxsb ldxsh ldxsw
    stdw [r10-8], 5       ; stb sth stw stdw
    stxw [r10-4], r2      ; stxb stxh stxw stxdw
    aadd64 [r0+0], r1     ; atomics: aadd aor aand axor (no fetch),
                          ; afadd afor afand afxor axchg acmpxchg  (+ 32 / 64)
    lddw r1, 0x1122334455667788
    lddw r1, map:name     ; src=5: index of ``name`` in the program's map table
    lddw r1, mapfd:3      ; src=1: runtime map fd 3
    .raw 0x07 1 0 0 5     ; opcode dst src off imm, emitted verbatim
"""

from __future__ import annotations

import re
import struct

# instruction classes
LD, LDX, ST, STX, ALU, JMP, JMP32, ALU64 = range(8)
K_SRC, X_SRC = 0x00, 0x08
SZ = {"w": 0x00, "h": 0x08, "b": 0x10, "dw": 0x18}
MODE_IMM, MODE_MEM, MODE_MEMSX, MODE_ATOMIC = 0x00, 0x60, 0x80, 0xC0

ALU_OPS = {
    "add": (0x00, 0), "sub": (0x10, 0), "mul": (0x20, 0), "div": (0x30, 0),
    "sdiv": (0x30, 1), "or": (0x40, 0), "and": (0x50, 0), "lsh": (0x60, 0),
    "rsh": (0x70, 0), "mod": (0x90, 0), "smod": (0x90, 1), "xor": (0xA0, 0),
    "mov": (0xB0, 0), "arsh": (0xC0, 0),
}
JMP_OPS = {
    "jeq": 0x10, "jgt": 0x20, "jge": 0x30, "jset": 0x40, "jne": 0x50,
    "jsgt": 0x60, "jsge": 0x70, "jlt": 0xA0, "jle": 0xB0, "jslt": 0xC0,
    "jsle": 0xD0,
}
ATOMIC_OPS = {
    "aadd": 0x00, "aor": 0x40, "aand": 0x50, "axor": 0xA0,
    "afadd": 0x01, "afor": 0x41, "afand": 0x51, "afxor": 0xA1,
    "axchg": 0xE1, "acmpxchg": 0xF1,
}
HELPERS = {
    "map_lookup_elem": 1, "map_update_elem": 2, "map_delete_elem": 3,
    "ringbuf_output": 130,
}
PSEUDO_MAP_FD = 1
PSEUDO_MAP_IDX = 5


class AsmError(ValueError):
    pass


def encode(op: int, dst: int = 0, src: int = 0, off: int = 0, imm: int = 0) -> bytes:
    """Pack one 8-byte instruction slot."""
    if not (0 <= op <= 0xFF and 0 <= dst <= 15 and 0 <= src <= 15):
        raise AsmError(f"field out of range: op={op} dst={dst} src={src}")
    if not -(1 << 15) <= off < (1 << 15):
        raise AsmError(f"offset out of range: {off}")
    if not -(1 << 31) <= imm < (1 << 32):
        raise AsmError(f"imm out of range: {imm}")
    if imm >= (1 << 31):
        imm -= 1 << 32
    return struct.pack("<BBhi", op, (src << 4) | dst, off, imm)


_REG = re.compile(r"^r(\d+)$")
_MEM = re.compile(r"^\[\s*r(\d+)\s*(?:([+-])\s*(\w+))?\s*\]$")


def _int(tok: str) -> int:
    try:
        return int(tok, 0)
    except ValueError as exc:
        raise AsmError(f"bad integer {tok!r}") from exc


def _reg(tok: str) -> int:
    m = _REG.match(tok)
    if not m or int(m.group(1)) > 10:
        raise AsmError(f"bad register {tok!r}")
    return int(m.group(1))


def _mem(tok: str) -> tuple[int, int]:
    m = _MEM.match(tok.replace(" ", ""))
    if not m:
        raise AsmError(f"bad memory operand {tok!r}")
    reg = int(m.group(1))
    off = 0
    if m.group(2):
        off = _int(m.group(3))
        if m.group(2) == "-":
            off = -off
    return reg, off


def _split_operands(rest: str) -> list[str]:
    out, depth, cur = [], 0, ""
    for ch in rest:
        if ch == "[":
            depth += 1
        elif ch == "]":
            depth -= 1
        if ch == "," and depth == 0:
            out.append(cur.strip())
            cur = ""
        else:
            cur += ch
    if cur.strip():
        out.append(cur.strip())
    return out


def _is_reg(tok: str) -> bool:
    return bool(_REG.match(tok))


def assemble(text: str, maps=None) -> bytes:
    """Assemble ``text`` into bytecode.

    ``maps`` names the program's map table (a list of names, or a dict
    name -> index); ``lddw rX, map:name`` refers to an entry of that table.
    """
    if maps is None:
        maps = {}
    if not isinstance(maps, dict):
        maps = {name: i for i, name in enumerate(maps)}

    # pass 1: strip, collect labels with slot positions
    lines = []
    labels: dict[str, int] = {}
    slot = 0
    for lineno, raw in enumerate(text.splitlines(), 1):
        line = re.split(r"[;#]", raw, maxsplit=1)[0].strip()
        while line:
            m = re.match(r"^([A-Za-z_.][\w.]*)\s*:(.*)$", line)
            if not m or m.group(1).startswith("."):
                break
            if m.group(1) in labels:
                raise AsmError(f"line {lineno}: duplicate label {m.group(1)}")
            labels[m.group(1)] = slot
            line = m.group(2).strip()
        if not line:
            continue
        mnem = line.split(None, 1)[0].lower()
        lines.append((lineno, slot, line))
        slot += 2 if mnem == "lddw" else 1

    out = bytearray()
    for lineno, pc, line in lines:
        try:
            out += _assemble_one(line, pc, labels, maps)
        except AsmError as exc:
            raise AsmError(f"line {lineno}: {exc}: {line!r}") from None
    return bytes(out)


def _target(tok: str, pc: int, labels) -> int:
    if tok in labels:
        return labels[tok] - (pc + 1)
    if re.match(r"^[+-]?\d+$", tok):
        return int(tok)  # raw relative offset
    raise AsmError(f"unknown label {tok!r}")


def _assemble_one(line: str, pc: int, labels, maps) -> bytes:
    parts = line.split(None, 1)
    mnem = parts[0].lower()
    ops = _split_operands(parts[1]) if len(parts) > 1 else []

    if mnem == ".raw":
        vals = [_int(t) for t in (parts[1].replace(",", " ").split() if len(parts) > 1 else [])]
        if len(vals) != 5:
            raise AsmError(".raw takes opcode dst src off imm")
        return encode(*vals)

    if mnem == "exit":
        return encode(JMP | 0x90)
    if mnem == "call":
        if len(ops) != 1:
            raise AsmError("call takes one operand")
        hid = HELPERS.get(ops[0])
        if hid is None:
            hid = _int(ops[0])
        return encode(JMP | 0x80, imm=hid)
    if mnem == "ja":
        return encode(JMP | 0x00, off=_target(ops[0], pc, labels))
    if mnem == "ja32":
        return encode(JMP32 | 0x00, imm=_target(ops[0], pc, labels))

    m = re.match(r"^(j[a-z]+?)(32)?$", mnem)
    if m and m.group(1) in JMP_OPS:
        cls = JMP32 if m.group(2) else JMP
        if len(ops) != 3:
            raise AsmError("conditional jump takes dst, src|imm, label")
        dst = _reg(ops[0])
        off = _target(ops[2], pc, labels)
        if _is_reg(ops[1]):
            return encode(cls | JMP_OPS[m.group(1)] | X_SRC, dst, _reg(ops[1]), off)
        return encode(cls | JMP_OPS[m.group(1)] | K_SRC, dst, 0, off, _int(ops[1]))

    m = re.match(r"^neg(64|32)$", mnem)
    if m:
        cls = ALU64 if m.group(1) == "64" else ALU
        return encode(cls | 0x80, _reg(ops[0]))

    m = re.match(r"^(le|be|bswap)(16|32|64)$", mnem)
    if m:
        kind, width = m.group(1), int(m.group(2))
        if kind == "le":
            op = ALU | 0xD0 | K_SRC
        elif kind == "be":
            op = ALU | 0xD0 | X_SRC
        else:
            op = ALU64 | 0xD0 | K_SRC
        return encode(op, _reg(ops[0]), imm=width)

    m = re.match(r"^movsx(8|16|32)_(64|32)$", mnem)
    if m:
        cls = ALU64 if m.group(2) == "64" else ALU
        return encode(cls | 0xB0 | X_SRC, _reg(ops[0]), _reg(ops[1]), int(m.group(1)))

    m = re.match(r"^([a-z]+?)(64|32)$", mnem)
    if m and m.group(1) in ALU_OPS:
        code, off = ALU_OPS[m.group(1)]
        cls = ALU64 if m.group(2) == "64" else ALU
        if len(ops) != 2:
            raise AsmError("ALU op takes dst, src|imm")
        dst = _reg(ops[0])
        if _is_reg(ops[1]):
            return encode(cls | code | X_SRC, dst, _reg(ops[1]), off)
        return encode(cls | code | K_SRC, dst, 0, off, _int(ops[1]))

    m = re.match(r"^ldx(s?)(b|h|w|dw)$", mnem)
    if m:
        mode = MODE_MEMSX if m.group(1) else MODE_MEM
        dst = _reg(ops[0])
        src, off = _mem(ops[1])
        return encode(LDX | mode | SZ[m.group(2)], dst, src, off)

    m = re.match(r"^st(b|h|w|dw)$", mnem)
    if m:
        dst, off = _mem(ops[0])
        return encode(ST | MODE_MEM | SZ[m.group(1)], dst, 0, off, _int(ops[1]))

    m = re.match(r"^stx(b|h|w|dw)$", mnem)
    if m:
        dst, off = _mem(ops[0])
        return encode(STX | MODE_MEM | SZ[m.group(1)], dst, _reg(ops[1]), off)

    m = re.match(r"^([a-z]+?)(32|64)$", mnem)
    if m and m.group(1) in ATOMIC_OPS:
        size = SZ["w"] if m.group(2) == "32" else SZ["dw"]
        dst, off = _mem(ops[0])
        return encode(STX | MODE_ATOMIC | size, dst, _reg(ops[1]), off, ATOMIC_OPS[m.group(1)])

    if mnem == "lddw":
        dst = _reg(ops[0])
        tok = ops[1]
        if tok.startswith("map:"):
            name = tok[4:]
            if name not in maps:
                raise AsmError(f"unknown map {name!r}")
            src, val = PSEUDO_MAP_IDX, maps[name]
        elif tok.startswith("mapfd:"):
            src, val = PSEUDO_MAP_FD, _int(tok[6:])
        else:
            src, val = 0, _int(tok) & 0xFFFFFFFFFFFFFFFF
        lo, hi = val & 0xFFFFFFFF, val >> 32
        return encode(LD | MODE_IMM | SZ["dw"], dst, src, 0, lo) + encode(0, 0, 0, 0, hi)

    raise AsmError(f"unknown mnemonic {mnem!r}")


# ----------------------------------------------------------------------------
# disassembler (debug aid)

_ALU_NAMES = {v: k for k, v in ALU_OPS.items()}
_JMP_NAMES = {v: k for k, v in JMP_OPS.items()}
_ATOMIC_NAMES = {v: k for k, v in ATOMIC_OPS.items()}
_SZ_NAMES = {v: k for k, v in SZ.items()}


def disassemble(code: bytes) -> str:
    out = []
    n = len(code) // 8
    pc = 0
    while pc < n:
        op, regs, off, imm = struct.unpack_from("<BBhi", code, pc * 8)
        dst, src = regs & 15, regs >> 4
        cls = op & 7
        text = f".raw {op:#04x} {dst} {src} {off} {imm}"
        if cls in (ALU, ALU64):
            w = "64" if cls == ALU64 else "32"
            code_ = op & 0xF0
            x = op & X_SRC
            if code_ == 0x80:
                text = f"neg{w} r{dst}"
            elif code_ == 0xD0:
                kind = "bswap" if cls == ALU64 else ("be" if x else "le")
                text = f"{kind}{imm} r{dst}"
            elif code_ == 0xB0 and off in (8, 16, 32) and x:
                text = f"movsx{off}_{w} r{dst}, r{src}"
            elif (code_, off if code_ in (0x30, 0x90) else 0) in _ALU_NAMES:
                name = _ALU_NAMES[(code_, off if code_ in (0x30, 0x90) else 0)]
                text = f"{name}{w} r{dst}, " + (f"r{src}" if x else f"{imm}")
        elif cls in (JMP, JMP32):
            code_ = op & 0xF0
            sfx = "32" if cls == JMP32 else ""
            if code_ == 0x90:
                text = "exit"
            elif code_ == 0x80:
                text = f"call {imm}"
            elif code_ == 0x00:
                text = f"ja{sfx} {imm if cls == JMP32 else off:+d}"
            elif code_ in _JMP_NAMES:
                rhs = f"r{src}" if op & X_SRC else f"{imm}"
                text = f"{_JMP_NAMES[code_]}{sfx} r{dst}, {rhs}, {off:+d}"
        elif cls == LDX:
            mode, sz = op & 0xE0, op & 0x18
            s = "s" if mode == MODE_MEMSX else ""
            text = f"ldx{s}{_SZ_NAMES[sz]} r{dst}, [r{src}{off:+d}]"
        elif cls == ST:
            text = f"st{_SZ_NAMES[op & 0x18]} [r{dst}{off:+d}], {imm}"
        elif cls == STX:
            if op & 0xE0 == MODE_ATOMIC:
                w = "64" if op & 0x18 == 0x18 else "32"
                text = f"{_ATOMIC_NAMES.get(imm & 0xFF, '?')}{w} [r{dst}{off:+d}], r{src}"
            else:
                text = f"stx{_SZ_NAMES[op & 0x18]} [r{dst}{off:+d}], r{src}"
        elif cls == LD and op == 0x18 and pc + 1 < n:
            hi = struct.unpack_from("<i", code, (pc + 1) * 8 + 4)[0]
            val = (imm & 0xFFFFFFFF) | ((hi & 0xFFFFFFFF) << 32)
            if src == PSEUDO_MAP_IDX:
                text = f"lddw r{dst}, map#{imm}"
            elif src == PSEUDO_MAP_FD:
                text = f"lddw r{dst}, mapfd:{imm}"
            else:
                text = f"lddw r{dst}, {val:#x}"
            out.append(f"{pc:4d}: {text}")
            pc += 2
            continue
        out.append(f"{pc:4d}: {text}")
        pc += 1
    return "\n".join(out)
