// Internal layouts shared by the host runtime and the device VM.
#pragma once
#include <stdint.h>

namespace gx {

// ---------------------------------------------------------------------------
// eBPF encoding constants (the standard encoding; the runtime decodes on its
// own, independently of any other component).
constexpr int kMaxInsns = 4096;
constexpr int kStackMax = 512;
// LDS an interpreted event-parallel block may take for its stack frames and
// the mirror of one shared map, and the largest mirrored value area
constexpr uint32_t kAccLdsMax = 128u << 10;
constexpr uint32_t kAccMirrorMax = 32u << 10;
constexpr uint64_t kMaxDynInsns = 65536;
constexpr uint64_t kMaxCalls = 64;
constexpr uint64_t kMaxRingBytes = 4096;

enum : int { MAP_HASH = 1, MAP_ARRAY = 2, MAP_RINGBUF = 27 };
// F_HOST: a read-only map kept in host memory (the cold tier), read by the
// device through its mapped address.
enum : uint32_t { F_SHARED = 1, F_READ_ONLY = 2, F_HOST = 4 };
// HOOK_WAVE_MEM: the warp-leader hook (section 4.4, warp-level execution):
// one invocation per wave tile of 64 memory-access records, with the tile's
// aggregate as context {u64 lo, u64 hi, u32 n, u32 stream of the first}.
// HOOK_SIMT_MEM: one invocation per memory-access record (one lane each),
// whose context is the record {u64 addr, u32 stream, u32 pad, u64 ts}
// followed by its wave tile's aggregate as above at byte 24; the verifier
// holds the program to warp-uniform control flow, keys and side effects.
// HOOK_SCHED: the device block scheduler's steal decision (section 4.3.2's
// should_try_steal), one invocation per decision of a persistent worker on
// {u32 worker, u32 done, u64 elapsed_ns, u64 steal_ns, u32 stolen, u32 left}.
enum : int { HOOK_MEM_ACCESS = 1, HOOK_KERNEL_TIMING = 2, HOOK_WAVE_MEM = 3, HOOK_SIMT_MEM = 4, HOOK_SCHED = 5 };
enum : int64_t { E_NOENT = 2, E_2BIG = 7, E_AGAIN = 11, E_EXIST = 17, E_INVAL = 22 };

// ---------------------------------------------------------------------------
// Pre-decoded micro-op: 16 bytes, fetched by the wave through the scalar
// cache with one uniform pc.
struct __attribute__((aligned(16))) Uop {
  uint32_t w0;   // h | dst << 8 | src << 12 | a8 << 16 | K << 24
  int32_t aux;   // jump target / memory offset / byte offset in ctx
  uint64_t imm;  // operand constant, lddw value, map descriptor pointer
};

inline constexpr uint32_t uop_w0(int h, int dst, int src, int a8, bool k) {
  return (uint32_t)h | ((uint32_t)dst << 8) | ((uint32_t)src << 12) | ((uint32_t)a8 << 16) |
         ((uint32_t)k << 24);
}

// Handler numbers.  ALU handlers take a = r[dst], b = K ? imm : r[src].
enum Handler : int {
  // 64-bit ALU
  H_ADD64 = 0, H_SUB64, H_MUL64, H_DIV64, H_SDIV64, H_OR64, H_AND64, H_LSH64, H_RSH64,
  H_NEG64, H_MOD64, H_SMOD64, H_XOR64, H_MOV64, H_ARSH64, H_MOVSX64, H_BSWAP,
  // 32-bit ALU (result zero-extended)
  H_ADD32, H_SUB32, H_MUL32, H_DIV32, H_SDIV32, H_OR32, H_AND32, H_LSH32, H_RSH32,
  H_NEG32, H_MOD32, H_SMOD32, H_XOR32, H_MOV32, H_ARSH32, H_MOVSX32, H_TRUNC,
  // jumps: aux = absolute target
  H_JA, H_JEQ, H_JGT, H_JGE, H_JSET, H_JNE, H_JSGT, H_JSGE, H_JLT, H_JLE, H_JSLT, H_JSLE,
  H_JEQ32, H_JGT32, H_JGE32, H_JSET32, H_JNE32, H_JSGT32, H_JSGE32, H_JLT32, H_JLE32,
  H_JSLT32, H_JSLE32,
  // memory: aux = offset; a8 = size code (0:1 1:2 2:4 3:8) | 4 if sign-extending
  H_LDX_CTX, H_LDX_STACK, H_LDX_MAP, H_ST_STACK, H_ST_MAP, H_STX_STACK, H_STX_MAP,
  // atomics: a8 = size code; imm = atomic op (ADD 0x00, OR 0x40, AND 0x50,
  // XOR 0xa0, |1 fetch, XCHG 0xe1, CMPXCHG 0xf1)
  H_ATOMIC_STACK, H_ATOMIC_MAP,
  H_LDIMM,
  // helpers: imm = map descriptor (device pointer)
  H_LOOKUP_ARRAY, H_LOOKUP_HASH, H_UPDATE_ARRAY, H_UPDATE_HASH, H_DELETE_HASH, H_RET_EINVAL,
  H_RINGBUF_OUTPUT,  // a8 unused; aux = size; src = data pointer kind (0 stack, 1 map value)
  H_EXIT,
  H_COUNT
};

// Pointer-argument kinds for helpers, encoded in aux bits or src field.
enum : int { PK_STACK = 0, PK_MAPVAL = 1 };

// ---------------------------------------------------------------------------
// Device map descriptor (64 B, in device memory).
struct __attribute__((aligned(64))) MapDev {
  uint32_t type, key_size, value_size, max_entries;
  uint32_t flags;
  uint32_t vstride;     // value stride (value_size rounded up to 8)
  uint32_t slot_mask;   // hash: slots - 1; ring: data bytes - 1
  uint32_t sstride;     // hash: slot header stride (8 + key bytes rounded to 8)
  uint8_t* data;        // array / hash: values; ring: data area
  uint8_t* slots;       // hash: slot headers {u32 state; u32 pad; key bytes}
  uint64_t* ctrl;       // hash: [0] live, [1] e2big; ring: [0] head, [1] tail, [2] drops,
                        // [3] ~(start of the first overflowing reservation) or 0,
                        // [kRingUnknown], [kRingCount...]: see below
  uint64_t pad;
};

// Ring counts of discard bytes and records: kRingCountSlots pairs from word
// kRingCount on (a block adds its totals to pair blockIdx mod the slot
// count, so that blocks rarely add to one address), apart from the head's
// cache line; ctrl[kRingUnknown] = 1 marks them incomplete.  Control area
// bytes per map.
constexpr uint32_t kRingUnknown = 16, kRingCount = 32, kRingCountSlots = 64;
constexpr uint32_t kCtrlBytes = 2048;

// Ring record header word: {u32 len, u32 flags}; a header of 0 marks space
// that is reserved but not yet written.  Padding that closes a chunk of
// reserved space is a record with the discard flag, which the drain skips.
constexpr uint32_t RING_DISCARD = 1;

// Hash slot states.
enum : uint32_t { SLOT_EMPTY = 0, SLOT_BUSY = 1, SLOT_LIVE = 2, SLOT_TOMB = 3 };

// Kernel arguments of one program run.
struct RunArgs {
  const Uop* uops;
  const uint8_t* events;
  uint32_t* rc;            // nullable
  uint64_t n_events;
  uint32_t record_size;
  uint32_t stack_bytes;    // frame bytes per lane (multiple of 8)
  uint32_t stream_off, stream_size;
  uint64_t step_limit;     // wave-level micro-op budget (runaway guard)
  // stream-sequential mode: queue q owns order[qstart[q] .. qstart[q+1])
  const uint32_t* order;
  const uint32_t* qstart;  // n_queues + 1 entries
  uint32_t n_queues;
  uint32_t checked;        // 1: bounds-check map-value accesses against guards
  uint32_t epoch;          // launch counter (tombstones of this launch stay unclaimed)
  uint32_t pad2;
  uint64_t* err;           // device error counter
  const uint64_t* guards;  // per slot {lo, hi} of the map data a map-value access may touch
  const uint8_t* sorted;   // stream-sequential: the records in queue order, kSortedStride apart
  const uint64_t* maptab;  // device addresses of the program's map descriptors, in its map-table order
  uint8_t* spill;          // compiled event-parallel runs: LDS cache spill area (null: caches flush directly)
  uint32_t leader;         // 1: warp-leader hook (one invocation per wave tile)
  uint32_t pad3;
  // interpreted event-parallel runs: a shared array map whose atomics the
  // block sums in an LDS mirror (value area [acc_lo, acc_hi); mirror at LDS
  // byte acc_lds; operation acc_op at width 2^acc_sc bytes); acc_hi == acc_lo
  // when none
  uint64_t acc_lo, acc_hi;
  uint32_t acc_lds, acc_op, acc_sc;
  uint32_t simt;           // 1: SIMT hook (each lane's context carries its tile's aggregate)
};

// Stride of the queue-ordered record copy (the largest record).
constexpr uint32_t kSortedStride = 24;

// The instrumented vector add (a hook inside an application kernel):
// c[j] = a[j] + b[j] for j = (i stride) mod n, iterations i < n.
struct AppArgs {
  const double* a;
  const double* b;
  double* c;
  uint64_t n;       // 1 <= n <= 2^32
  uint64_t stride;  // < n, coprime to n
  uint64_t mu;      // floor((2^64 - 1) / n), for reductions mod n
};

// The device block scheduler: persistent workers over imbalanced work units.
struct SchedArgs {
  const uint32_t* cost;  // per unit: iterations of the unit's work
  uint64_t* out;         // per unit: 64 results
  uint32_t* next;        // per worker: units of its range claimed so far (zeroed by the host)
  uint64_t* log;         // per decision: its 32-byte context record (nullable)
  uint32_t* log_rc;      // per decision: the program's return code
  uint32_t* log_n;       // decisions made (zeroed by the host; may exceed log_cap)
  uint32_t n_units, workers, log_cap, pad;
  uint64_t tick_num, tick_den;  // wall-clock ticks to ns: ticks * num / den
};

// Batched form: one entry per run in a persistent launch.
struct BatchDev {
  RunArgs A;
  uint32_t mode;       // 0 event-parallel, 1 stream-sequential
  uint32_t lanes;
  uint32_t qstride;
  uint32_t qend_last;  // position after the run's last queue in order[]
  uint32_t slot;       // compiled program sets: the program's index in its set
  uint32_t pad;
};

// Stable-partition job of one stream-sequential run.
struct PartJob {
  const uint8_t* events;
  uint64_t n_events;
  uint32_t record_size, stream_off;
  uint32_t lbits, tile;
  uint32_t nt, pad;
  uint64_t cbase;  // offset of this run's counts matrix (L x nt, queue-major)
};

}  // namespace gx

namespace gx {

#if defined(__HIPCC__)
#define GX_HD __host__ __device__
#else
#define GX_HD
#endif

// Hash of a key given as zero-padded 8-byte little-endian words.  Not
// observable by programs (maps compare by (key, value) sets).
GX_HD inline uint64_t hash_step(uint64_t h, uint64_t w) {
  h ^= w;
  h *= 0x9E3779B97F4A7C15ull;
  return h ^ (h >> 32);
}
GX_HD inline uint64_t hash_final(uint64_t h) {
  h ^= h >> 29;
  h *= 0xBF58476D1CE4E5B9ull;
  return h ^ (h >> 32);
}

}  // namespace gx
