// CPU oracle for the device-side eBPF runtime: test infrastructure only.
//
// A plain, slow, sequential eBPF interpreter with its own maps and ring
// buffer, plus an independent bounds/termination checker.  It defines the
// result the GPU runtime must reproduce bit for bit: per-event return codes,
// final map contents and the ring-record multiset, with events executed one
// at a time in index order (the per-stream-sequential, commutative-across-
// streams contract).  Only the tests, the smoke check and the benchmark's CPU
// baseline use it; it shares no code with the GPU runtime.
//
// Paper anchors: program types and hooks (section 4.3), verified policy code
// with bounded loops and memory safety (section 4.4, "SIMT-aware
// Verification"), maps as shared key-value state (section 4.4, "Hierarchical
// Cross-layer Maps").  Instruction semantics follow the eBPF instruction-set
// standard (RFC 9669); the paper names only a "restricted eBPF subset".
#pragma once
#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

namespace gxo {

enum : int { MAP_HASH = 1, MAP_ARRAY = 2, MAP_RINGBUF = 27 };
enum : uint32_t { F_SHARED = 1, F_READ_ONLY = 2 };
// HOOK_WAVE_MEM: the warp-leader hook (section 4.4, warp-level execution):
// one invocation per tile of 64 consecutive memory-access records, whose
// context is the tile's aggregate (see hook_info).
// HOOK_SIMT_MEM: one invocation per memory-access record, whose context is
// the record followed by its tile's aggregate; the aggregate's fields are
// warp-uniform, the record's lane-varying, and the checker holds the program
// to warp-uniform control flow, map keys and side effects (section 4.4,
// "SIMT-aware Verification").
// HOOK_SCHED: the device block scheduler's steal decision (section 4.3.2,
// should_try_steal): one invocation per decision of a persistent worker,
// whose context is the worker's state at that point (see hook_info); a
// non-zero return code means "take one more work unit from another
// worker's range".
enum : int { HOOK_MEM_ACCESS = 1, HOOK_KERNEL_TIMING = 2, HOOK_WAVE_MEM = 3, HOOK_SIMT_MEM = 4, HOOK_SCHED = 5 };
enum : int { H_LOOKUP = 1, H_UPDATE = 2, H_DELETE = 3, H_RINGBUF_OUTPUT = 130 };
enum : int64_t { E_NOENT = 2, E_2BIG = 7, E_AGAIN = 11, E_EXIST = 17, E_INVAL = 22 };

constexpr int STACK_BYTES = 512;
constexpr int MAX_INSNS = 4096;

struct Insn {
  uint8_t op, dst, src;
  int16_t off;
  int32_t imm;
};

// Decode 8-byte little-endian slots.
std::vector<Insn> decode(const uint8_t* code, uint32_t n_slots);

// Hook record layout: size and readable fields (offset, size).
struct HookInfo {
  uint32_t record_size;
  uint32_t stream_off, stream_size;  // stream key field
  std::vector<std::pair<uint32_t, uint32_t>> fields;
  uint32_t uniform_off = ~0u;  // ctx bytes from here on are warp-uniform (SIMT hook)
};
bool hook_info(int hook, HookInfo* out);

using Bytes = std::vector<uint8_t>;

struct Map {
  int type = 0;
  uint32_t key_size = 0, value_size = 0, max_entries = 0, flags = 0;
  // ARRAY: max_entries * value_size bytes.
  Bytes array;
  // HASH: key bytes -> value storage.  Values live in shared_ptrs so that a
  // pointer taken by a lookup stays valid until the invocation exits.
  std::map<Bytes, std::shared_ptr<Bytes>> hash;
  // RINGBUF: committed, undrained records and the bytes they occupy.
  std::vector<Bytes> records;
  uint64_t ring_used = 0;
  // ownership tracking (D-3): slot -> first stream to touch it, written flag
  std::map<Bytes, std::pair<uint64_t, bool>> owner;
  std::map<Bytes, bool> multi;  // slot touched by more than one stream
  int shared_op = -1;            // shared maps: the one (atomic op, size) they take
};

struct Stats {
  uint64_t insns = 0;        // retired eBPF instructions (lddw counts once)
  uint64_t helper_calls = 0;
  uint64_t drops = 0;        // ringbuf_output without space
  uint64_t e2big = 0;        // hash insert into a full map
  uint64_t violations = 0;   // written slots touched by two streams
  uint64_t faults = 0;       // dynamic safety violations (checker soundness)
  std::string fault_msg;
};

struct Program {
  std::vector<Insn> insns;
  int hook = 0;
  std::vector<int> map_table;  // map references: pseudo idx -> oracle map id
};

class Oracle {
 public:
  int create_map(int type, uint32_t ksz, uint32_t vsz, uint32_t max, uint32_t flags);
  int map_update(int id, const uint8_t* key, const uint8_t* val, uint64_t flags);
  int map_lookup(int id, const uint8_t* key, uint8_t* val_out);
  int map_delete(int id, const uint8_t* key);
  // Copies out live (key, value) pairs in key order; returns the count.
  int64_t map_dump(int id, uint8_t* keys, uint8_t* vals, uint64_t cap);
  // Copies out ring records as {u32 len, u32 flags=0, payload padded to 8}.
  int64_t ring_drain(int id, uint8_t* buf, uint64_t cap, uint64_t* n_records);

  // Run ``prog`` over ``n`` events.  order: 0 = index order (the definition);
  // 1 = streams interleaved round-robin in descending key order; 2 = a seeded
  // random permutation (only valid for event-parallel programs); 3 = streams
  // one after another in descending key order.  rc_out may be null.
  int run(const Program& prog, const uint8_t* events, uint64_t n, int order, uint64_t seed,
          uint32_t* rc_out);

  std::vector<Map> maps;
  Stats stats;
  bool track_ownership = true;
};

// Checker verdict and facts.
struct CheckResult {
  bool ok = false;
  std::string log;
  uint32_t stack_bytes = 0;
  uint64_t max_insns = 0;      // longest path, loop bodies times trip counts
  uint64_t max_calls = 0;
  uint64_t max_ring_bytes = 0;
  bool event_parallel = false;
};

struct MapShape {
  int type;
  uint32_t key_size, value_size, max_entries, flags;
};

CheckResult check(const std::vector<Insn>& insns, int hook, const std::vector<MapShape>& maps,
                  const std::vector<int>& map_table);

}  // namespace gxo
