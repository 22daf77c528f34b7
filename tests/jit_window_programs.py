"""Programs that reach one map value through several pointers, for the map
value windows and lookup memos of compiled programs: every read after a
store, update, delete or atomic through another path, in this event or an
earlier one, must see memory's current value.  Keys are per stream
(stream << 32, or stream << 32 | page & 7), so runs are deterministic."""

from paper_2512_12615_amd import workloads as W

KEY = """
    ldxdw r6, [r1+0]
    ldxw r7, [r1+8]
    mov64 r2, r7
    lsh64 r2, 32
    mov64 r3, r6
    rsh64 r3, 12
    and64 r3, 7
    or64 r2, r3
    stxdw [r10-8], r2
"""

LOOKUP = """
    lddw r1, map:m
    mov64 r2, r10
    add64 r2, -8
    call map_lookup_elem
"""

INSERT = """
    jne r0, 0, have
    stxdw [r10-32], r6
    stdw [r10-24], 1
    stdw [r10-16], 0
    lddw r1, map:m
    mov64 r2, r10
    add64 r2, -8
    mov64 r3, r10
    add64 r3, -32
    mov64 r4, 0
    call map_update_elem
    mov64 r0, 0
    exit
have:
"""

# two pointers to one value: a store through the second, reads through the first
ALIAS = KEY + LOOKUP + INSERT + """
    mov64 r8, r0
""" + LOOKUP + """
    jeq r0, 0, out
    ldxdw r3, [r8+0]
    add64 r3, 3
    stxdw [r0+0], r3
    ldxdw r4, [r8+0]
    ldxdw r5, [r8+8]
    add64 r5, r4
    stxdw [r8+8], r5
    ldxw r2, [r0+12]
    add32 r2, 1
    stxw [r8+12], r2
    ldxdw r0, [r0+8]
    exit
out:
    mov64 r0, 0
    exit
"""

# an array map: an update of the same index, then a read through the
# pointer taken before it (array values stay in place)
UPDATE = """
    ldxdw r6, [r1+0]
    ldxw r7, [r1+8]
    and64 r7, 127
    lsh64 r7, 3
    mov64 r3, r6
    rsh64 r3, 12
    and64 r3, 7
    or64 r7, r3
    stxw [r10-4], r7
    lddw r1, map:a
    mov64 r2, r10
    add64 r2, -4
    call map_lookup_elem
    jeq r0, 0, out
    mov64 r8, r0
    ldxdw r3, [r8+8]
    add64 r3, r6
    stxdw [r10-32], r3
    stdw [r10-24], 5
    stdw [r10-16], 9
    lddw r1, map:a
    mov64 r2, r10
    add64 r2, -4
    mov64 r3, r10
    add64 r3, -32
    mov64 r4, 0
    call map_update_elem
    ldxdw r0, [r8+0]
    ldxdw r1, [r8+8]
    add64 r0, r1
    ldxdw r2, [r8+16]
    add64 r2, 1
    stxdw [r8+16], r2
    exit
out:
    mov64 r0, 0
    exit
"""

# an atomic add on the value, then reads; a pointer with an offset and a
# partial store
ATOMIC = KEY + LOOKUP + INSERT + """
    mov64 r8, r0
    ldxdw r3, [r8+8]
    mov64 r1, 7
    aadd64 [r8+8], r1
    ldxdw r4, [r8+8]
    mov64 r9, r8
    add64 r9, 8
    stxh [r9+2], r4
    ldxdw r5, [r9+0]
    ldxw r2, [r9+8]
    add64 r5, r2
    add64 r5, r3
    stxdw [r9+8], r5
    mov64 r0, r5
    exit
"""

# pointers to the values of two keys of one stream: a store through the
# second, a read through the first, then a delete of the second key and a
# fresh lookup of the first
DELETE = KEY + LOOKUP + INSERT + """
    mov64 r8, r0
    ldxdw r3, [r8+0]
    add64 r3, 1
    stxdw [r8+0], r3
    ldxdw r2, [r10-8]
    xor64 r2, 1
    stxdw [r10-16], r2
    lddw r1, map:m
    mov64 r2, r10
    add64 r2, -16
    call map_lookup_elem
    jeq r0, 0, nosecond
    ldxdw r4, [r0+0]
    add64 r4, 2
    stxdw [r0+0], r4
    ldxdw r5, [r8+0]
    jlt r5, 6, nosecond
    lddw r1, map:m
    mov64 r2, r10
    add64 r2, -16
    call map_delete_elem
nosecond:
    lddw r1, map:m
    mov64 r2, r10
    add64 r2, -8
    call map_lookup_elem
    jeq r0, 0, gone
    ldxdw r0, [r0+0]
    exit
gone:
    mov64 r0, 1
    exit
"""

# a lookup inside a bounded loop beside a pointer taken before it: the
# loop's stores through either pointer, reads through both
LOOP = KEY + LOOKUP + INSERT + """
    mov64 r8, r0
    mov64 r9, 1
loop:
    ldxdw r2, [r10-8]
    xor64 r2, r9
    stxdw [r10-16], r2
    lddw r1, map:m
    mov64 r2, r10
    add64 r2, -16
    call map_lookup_elem
    jeq r0, 0, skip
    ldxdw r3, [r8+0]
    ldxdw r4, [r0+8]
    add64 r4, r3
    stxdw [r0+8], r4
    ldxdw r5, [r8+8]
    add64 r5, r9
    stxdw [r8+8], r5
    ldxdw r4, [r0+8]
    stxdw [r8+16], r4
skip:
    add64 r9, 1
    jlt r9, 5, loop
    ldxdw r0, [r8+16]
    ldxdw r1, [r8+8]
    add64 r0, r1
    exit
"""

# one key per stream, so a compiled lookup finds the key of the stream's
# previous event on almost every event (the lookup memo): counts through the
# window; when page & 15 == 5 the key is deleted (the stream's next event
# inserts it again), when page & 3 == 0 it is rewritten in place by an update
# and read back through a second lookup
KEY1 = """
    ldxdw r6, [r1+0]
    ldxw r7, [r1+8]
    mov64 r2, r7
    lsh64 r2, 32
    stxdw [r10-8], r2
"""

MEMO = KEY1 + LOOKUP + INSERT + """
    mov64 r8, r0
    ldxdw r7, [r8+0]
    add64 r7, 1
    stxdw [r8+0], r7
    ldxdw r4, [r8+8]
    xor64 r4, r6
    stxdw [r8+8], r4
    mov64 r9, r6
    rsh64 r9, 12
    and64 r9, 15
    jne r9, 5, keep
    lddw r1, map:m
    mov64 r2, r10
    add64 r2, -8
    call map_delete_elem
    mov64 r0, r7
    exit
keep:
    and64 r9, 3
    jne r9, 0, done
    lsh64 r7, 1
    stxdw [r10-32], r7
    stxdw [r10-24], r4
    stdw [r10-16], 9
    lddw r1, map:m
    mov64 r2, r10
    add64 r2, -8
    mov64 r3, r10
    add64 r3, -32
    mov64 r4, 0
    call map_update_elem
done:
""" + LOOKUP + """
    jeq r0, 0, none
    ldxdw r1, [r0+0]
    ldxdw r2, [r0+16]
    add64 r1, r2
    ldxdw r2, [r0+8]
    xor64 r1, r2
    mov64 r0, r1
    exit
none:
    mov64 r0, 7
    exit
"""

# one key per stream through two lookup sites of the same key: stores
# through the second site's pointer while the first one's value is kept
# across events (every such store must drop the first site's memo)
MEMO_TWO = KEY1 + LOOKUP + INSERT + """
    mov64 r8, r0
    ldxdw r7, [r8+0]
    add64 r7, 1
    stxdw [r8+0], r7
    ldxdw r2, [r10-8]
    stxdw [r10-16], r2
    mov64 r9, r6
    rsh64 r9, 12
    and64 r9, 1
    jeq r9, 0, same
    lddw r1, map:m
    mov64 r2, r10
    add64 r2, -16
    call map_lookup_elem
    jeq r0, 0, same
    ldxdw r4, [r0+16]
    add64 r4, r7
    stxdw [r0+16], r4
    ldxdw r5, [r0+0]
    add64 r5, 5
    stxdw [r0+0], r5
same:
    ldxdw r0, [r8+0]
    ldxdw r1, [r8+16]
    add64 r0, r1
    exit
"""

PROGRAMS = {"alias": ALIAS, "update": UPDATE, "atomic": ATOMIC, "delete": DELETE, "loop": LOOP, "memo": MEMO,
            "memo_two": MEMO_TWO}


def policy(name: str) -> W.Policy:
    if name == "update":
        maps = [W.MapSpec("a", W.MAP_ARRAY, 4, 24, 1024, 0)]
    else:
        maps = [W.MapSpec("m", W.MAP_HASH, 8, 24, 4096, 0)]
    return W.Policy("win_" + name, W.HOOK_MEM_ACCESS, PROGRAMS[name], maps)
