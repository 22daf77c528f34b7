"""Assembler pins: hand-written standard encodings (tests/golden/encodings.txt)."""

import pytest

from isa_util import read_table

from paper_2512_12615_amd import asm


@pytest.mark.parametrize("row", read_table("encodings.txt"), ids=lambda r: r[0])
def test_encoding(row):
    text, hexbytes = row
    # single instruction; relative jump offsets are written as raw numbers
    got = asm.assemble(text).hex(" ")
    assert got == hexbytes


def test_labels_count_lddw_as_two_slots():
    code = asm.assemble("ja end\nlddw r1, 5\nend:\nexit")
    assert code[:8].hex(" ") == "05 00 02 00 00 00 00 00"


def test_map_names_resolve_to_table_index():
    code = asm.assemble("lddw r1, map:b\nexit", ["a", "b"])
    assert code[1] == 0x51 and code[4] == 1  # src = 5 (map index), imm = 1


def test_disassemble_roundtrip():
    text = "add64 r1, r2\njeq r1, 0, +1\nexit\nlddw r3, 0x1122334455667788\nexit"
    code = asm.assemble(text)
    again = asm.assemble("\n".join(l.split(": ", 1)[1] for l in asm.disassemble(code).splitlines()))
    assert again == code


def test_errors():
    for bad in ["add64 r11, 1", "foo r1", "jeq r1, 0, nowhere", "ldxdw r1, r2"]:
        with pytest.raises(asm.AsmError):
            asm.assemble(bad)
