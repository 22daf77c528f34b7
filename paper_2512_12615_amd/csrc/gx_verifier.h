// Load-time verifier of the runtime (independent of the test oracle's checker).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace gx {

struct MapShape {
  uint32_t type, key_size, value_size, max_entries, flags;
};

// Pointer kinds recorded per instruction for the pre-decoder.
enum : int8_t { KIND_NONE = -1, KIND_STACK = 0, KIND_MAPVAL = 1, KIND_CTX = 2 };

struct Insn {
  uint8_t op, dst, src;
  int16_t off;
  int32_t imm;
};

struct Verdict {
  bool ok = false;
  std::string log;
  uint32_t stack_bytes = 0;
  uint64_t max_insns = 0, max_calls = 0, max_ring = 0;
  bool event_parallel = true;
  // per instruction facts (indexed by slot)
  std::vector<int8_t> mem_kind;   // base pointer kind of LDX/ST/STX/atomics
  std::vector<int> call_map;      // map-table index used by a helper call
  std::vector<int8_t> arg2_kind;  // r2 pointer kind at a helper call
  std::vector<int8_t> arg3_kind;  // r3 pointer kind at a helper call (update)
  std::vector<uint32_t> ring_size;  // constant ringbuf_output size
  std::vector<int> ld_map;        // lddw map reference: map-table index
  std::vector<int> mem_map;       // map of a map-value memory access
};

std::vector<Insn> decode_insns(const uint64_t* raw, uint32_t n);

// ``table`` maps program map indices to shapes; ``fds`` are the runtime fds of
// the same entries (used for src=1 references).
Verdict verify(const std::vector<Insn>& prog, int hook, const std::vector<MapShape>& table,
               const std::vector<int>& fds);

// Record layout of a hook: size, stream-key field, readable fields.
bool hook_layout(int hook, uint32_t* record_size, uint32_t* stream_off, uint32_t* stream_size);

}  // namespace gx
