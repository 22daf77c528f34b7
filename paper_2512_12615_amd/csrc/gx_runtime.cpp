// Host runtime behind the C ABI of include/gxbpf.h: runtime object, maps in
// device memory, program loading (verify + pre-decode), batch launch,
// ring-buffer drain and statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "gx_internal.h"
#include "gx_jit.h"
#include "gx_verifier.h"
#include "gxbpf.h"

namespace gx {
hipError_t vm_init();
hipError_t launch_event_parallel(const RunArgs& A, hipStream_t s);
hipError_t launch_event_parallel_acc(RunArgs A, uint32_t n_cu, hipStream_t s);
hipError_t launch_stream_seq(const RunArgs& A, uint32_t lanes, uint32_t qstride, hipStream_t s);
hipError_t launch_partition(const RunArgs& A, uint32_t lbits, uint32_t tile, uint32_t nt, uint32_t* counts,
                            uint32_t* sums, uint32_t* order, uint8_t* sorted, hipStream_t s);
hipError_t launch_map_op(const MapDev* m, int op, const uint8_t* key, const uint8_t* val, uint64_t flags,
                         int64_t* ret, uint8_t* val_out, uint32_t epoch, hipStream_t s);
hipError_t launch_partition_jobs(const PartJob* d_jobs, const uint2* d_tiles, uint32_t n_tiles, uint32_t max_lbits,
                                 uint64_t total_counts, uint32_t* counts, uint32_t* sums, uint32_t* order,
                                 uint8_t* sorted, hipStream_t s);
hipError_t launch_batched(const BatchDev* d_batches, const uint2* d_items, uint32_t n_items, uint32_t* d_next,
                          uint32_t waves, uint32_t stack_max, hipStream_t s);
hipError_t launch_zero(uint32_t* p, uint32_t n, hipStream_t s);
hipError_t launch_app_vadd(const RunArgs& A, const AppArgs& P, hipStream_t s);
hipError_t launch_app_vadd_acc(RunArgs A, const AppArgs& P, uint32_t n_cu, hipStream_t s);
hipError_t launch_app_plain(const AppArgs& P, uint32_t n_cu, hipStream_t s);
hipError_t launch_sched(const RunArgs& A, const SchedArgs& S, hipStream_t s);
hipError_t launch_sched_plain(const SchedArgs& S, hipStream_t s);
hipError_t scratch_region(int dev, uint8_t** ptr, uint64_t* bytes);
}  // namespace gx

using namespace gx;

namespace {

// Blocks of a compiled event-parallel launch: enough for every CU to hold
// several (256 CUs), each looping over tiles beyond that.
constexpr uint64_t kJitMaxBlocks = 2048;
// Program sets one phase launches at most (each takes one of the runtime's
// item counters; the interpreter takes counter 0 of 16)
constexpr size_t kMaxSetsPerPhase = 15;
// Programs one compiled set holds at most
constexpr uint32_t kMaxSetPrograms = 64;
// Block scheduler: workers of one launch at most
constexpr uint32_t kMaxWorkers = 1u << 16;

struct MapObj {
  bool live = false;
  MapDev h{};              // host copy of the descriptor
  MapDev* d_desc = nullptr;
  size_t data_bytes = 0, slot_bytes = 0;
  uint8_t* h_pin = nullptr;  // ring: pinned staging for drains
  size_t pin_cap = 0;
  // ring: a drain started by gx_drain_ringbuf_start, whose copy and the
  // ring's new control words are queued on the runtime's copy stream and
  // done at drain_ev; launches that write the ring wait for that event
  hipEvent_t drain_ev = nullptr;
  bool drain_pending = false;
  uint64_t* ctrl_pin = nullptr;  // pinned source of the new control words
  uint64_t pend_bytes = 0, pend_kept = 0, pend_recs = 0;
  bool pend_counted = false;  // the drain's bytes are already in the runtime's counters
  // host tier (F_HOST): the pinned host allocations behind h.data / h.slots
  uint8_t* host_data = nullptr;
  uint8_t* host_slots = nullptr;
};

// Host snapshots of device maps (gx_snapshot_*): pinned copies taken by a
// daemon thread between runs on one stream; the latest complete copy is
// published under the lock.
struct SnapMap {
  int fd = -1;
  size_t data_bytes = 0, slot_bytes = 0;
  uint8_t* pin[2] = {nullptr, nullptr};  // copy target / published copy
  uint64_t version = 0;
};
struct SnapDaemon {
  std::thread th;
  std::mutex mu;               // the published copies and versions
  std::mutex take_mu;          // one snapshot at a time (daemon or flush)
  std::condition_variable cv;
  bool stop = false;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  uint64_t interval_us = 0;
  std::vector<SnapMap> maps;
};

struct ProgObj {
  bool live = false;
  int hook = 0;
  uint32_t record_size = 0, stream_off = 0, stream_size = 0;
  Verdict v;
  uint32_t n_insns = 0;
  Uop* d_uops = nullptr;
  uint64_t* d_guards = nullptr;
  std::vector<int> fds;
  std::vector<Uop> uops;  // host copy (source of the compiled form)
  uint64_t* d_maptab = nullptr;  // device addresses of its map descriptors (map-table order)
  // compiled form (gx_jit_program): module and its kernels (event-parallel;
  // stream-sequential with any lanes per wave, and with one queue per wave
  // run on wave-uniform values)
  hipModule_t jmod = nullptr;
  hipFunction_t jf_ep = nullptr, jf_seq = nullptr, jf_uni = nullptr, jf_red = nullptr;
  uint64_t jacc_words = 0;  // LDS accumulator words each block flushes
  uint64_t jspill = 0;      // LDS cache spill bytes per block (0: caches flush directly)
  uint32_t jred_blocks = 0; // blocks of its reduce kernel
  // compiled kernel with the program at a hook inside an application kernel
  // (the instrumented vector add, or the block scheduler's workers for
  // HOOK_SCHED programs) and that module's reduce kernel
  hipFunction_t jf_app = nullptr, jf_app_red = nullptr;
  // launch shape chosen by gx_autotune (0: default)
  uint32_t tuned_lanes = 0, tuned_qbits = 0, tuned_blocks = 0;
  // interpreted event-parallel runs: the shared array map summed in an LDS
  // mirror (value area [acc_lo, acc_hi), operation, width code); none if equal
  uint64_t acc_lo = 0, acc_hi = 0;
  uint32_t acc_op = 0, acc_sc = 0;
  // member of a compiled program set: its set and its slot there (-1: none)
  int set_id = -1;
  uint32_t set_slot = 0;
};

// Launch shape of one run.
struct Knobs {
  uint32_t lanes;   // stream-sequential: queues (lanes) per wave
  uint32_t qbits;   // stream-sequential: log2 of the queue count
  uint32_t blocks;  // compiled event-parallel: blocks (0: sized from the run)
};


uint64_t next_pow2(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

int env_int(const char* name, int dflt) {
  const char* s = std::getenv(name);
  return s && *s ? std::atoi(s) : dflt;
}

// Default queues per wave: a compiled program runs one queue per wave (its
// lanes' paths would otherwise serialize under divergence: measured 1.9x
// faster than 64 on the stride-prefetch workload); the interpreter fills the
// wave (its dispatch costs the same for one lane or 64).
uint32_t default_lanes(const ProgObj* p) {
  return (uint32_t)std::min(64, std::max(1, env_int("GX_SEQ_LANES", p->jmod ? 1 : 64)));
}

Knobs knobs_of(const ProgObj* p) {
  Knobs k;
  k.lanes = p->tuned_lanes ? p->tuned_lanes : default_lanes(p);
  k.qbits = p->tuned_qbits ? p->tuned_qbits : (uint32_t)std::min(16, std::max(6, env_int("GX_QUEUE_BITS", 12)));
  k.blocks = p->tuned_blocks ? p->tuned_blocks : (uint32_t)std::min(65536, std::max(0, env_int("GX_JIT_BLOCKS", 0)));
  return k;
}

// Execution resources of runs: the stream-sequential workspace, the batched
// form's side streams, table staging and work counters.  The runtime has one
// set; a captured graph owns another, swapped in while it is captured.
constexpr int kExecSide = 4;
struct Stage {
  uint8_t* h = nullptr;  // pinned host copy of a phase's tables
  uint8_t* d = nullptr;  // device tables
  size_t cap = 0;
  hipEvent_t ev = nullptr;  // after the tables' copy
  bool used = false;
};
struct Exec {
  // batched form: compiled runs of a phase run side by side on these
  hipStream_t side[kExecSide] = {};
  hipEvent_t fork_ev = nullptr, join_ev[kExecSide] = {};
  // staging of batched tables: a ring of slots, so a phase never waits for
  // the previous phase's table copy (a capture takes a fresh slot per phase)
  std::vector<Stage> stage;
  uint32_t stage_next = 0;
  // stream-sequential workspace
  uint32_t* d_counts = nullptr;
  uint32_t* d_sums = nullptr;
  uint32_t* d_order = nullptr;
  uint8_t* d_sorted = nullptr;  // records in queue order (kSortedStride apart)
  size_t counts_cap = 0, sums_cap = 0, order_cap = 0, sorted_cap = 0;
  hipEvent_t ws_event = nullptr;
  bool ws_used = false;
  uint32_t* d_next = nullptr;  // work counters of persistent launches (16)
  uint32_t* d_wnext = nullptr;  // block scheduler: per-worker unit counters and the log count
  size_t wnext_cap = 0;
  // LDS cache spill areas of compiled event-parallel runs (one per run of a
  // phase), free again once the reduce kernels that read them are done
  uint8_t* d_spill = nullptr;
  size_t spill_cap = 0;
  hipEvent_t spill_ev = nullptr;
  bool spill_used = false;
  bool capturing = false;      // launches are being captured into a graph
  bool per_phase = false;      // staging: slot i for the i-th phase (graphs)
  size_t stage_cursor = 0;
};

constexpr int kStageRing = 4;

int exec_init(Exec& x) {
  if (hipEventCreateWithFlags(&x.ws_event, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&x.fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&x.spill_ev, hipEventDisableTiming) != hipSuccess ||
      hipMalloc((void**)&x.d_next, 64) != hipSuccess)
    return -ENOMEM;
  for (int i = 0; i < kExecSide; i++)
    if (hipStreamCreateWithFlags(&x.side[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&x.join_ev[i], hipEventDisableTiming) != hipSuccess)
      return -ENOMEM;
  return 0;
}

void exec_free(Exec& x) {
  for (int i = 0; i < kExecSide; i++) {
    if (x.side[i]) (void)hipStreamDestroy(x.side[i]);
    if (x.join_ev[i]) (void)hipEventDestroy(x.join_ev[i]);
  }
  if (x.fork_ev) (void)hipEventDestroy(x.fork_ev);
  for (auto& st : x.stage) {
    if (st.h) (void)hipHostFree(st.h);
    if (st.d) (void)hipFree(st.d);
    if (st.ev) (void)hipEventDestroy(st.ev);
  }
  if (x.ws_event) (void)hipEventDestroy(x.ws_event);
  if (x.spill_ev) (void)hipEventDestroy(x.spill_ev);
  for (void* p : {(void*)x.d_counts, (void*)x.d_sums, (void*)x.d_order, (void*)x.d_sorted, (void*)x.d_next,
                  (void*)x.d_spill, (void*)x.d_wnext})
    if (p) (void)hipFree(p);
  x = Exec{};
}

}  // namespace

struct gx_rt {
  int dev = 0;
  hipStream_t internal = nullptr;
  hipStream_t copy = nullptr;  // started drains (created on first use)
  // compiled modules by generated source (instances of one program with
  // same-shaped maps share one); guarded for concurrent gx_jit_program calls
  struct JitMod {
    hipModule_t mod = nullptr;
    hipFunction_t fe = nullptr, fs = nullptr, fu = nullptr, fr = nullptr;
    JitInfo info;
  };
  std::map<std::string, JitMod> jit_cache;
  std::mutex jit_mu;
  // compiled program sets (gx_jit_program_set): persistent kernel per set
  struct JitSet {
    hipFunction_t f = nullptr;
    uint32_t blocks_per_cu = 0;  // resident one-wave blocks per CU (occupancy)
  };
  uint32_t n_cu = 256;  // compute units of the device
  uint32_t wall_khz = 100000;  // frequency of the device's constant wall clock (s_memrealtime)
  std::vector<JitSet> sets;
  static constexpr int kSide = kExecSide;
  // execution resources per launch stream: runs on different streams share
  // no workspace, staging, side streams or spill area, so they overlap; a
  // graph being built uses its own set (cap_ex)
  std::vector<std::pair<hipStream_t, Exec*>> execs;
  Exec* cap_ex = nullptr;
  std::vector<MapObj> maps;
  std::vector<ProgObj> progs;
  uint64_t* d_err = nullptr;
  uint8_t* d_stage = nullptr;  // control-plane staging (keys, values, results)
  // gx_run_batch_noalloc: this device's scratch array (device address) and
  // the event its latest run recorded
  uint8_t* d_scratch = nullptr;
  uint64_t scratch_bytes = 0;
  hipEvent_t noalloc_ev = nullptr;
  bool noalloc_used = false;
  // host snapshot daemon; runs are issued under enq_mu while it runs, so
  // that its copies land between runs
  SnapDaemon* snap = nullptr;
  std::mutex enq_mu;
  std::vector<std::pair<hipStream_t, hipEvent_t>> stream_events;
  gx_stats stats{};
  uint32_t epoch = 0;  // launch counter for hash tombstone reuse
  uint32_t batch_per_cu = 0;  // waves per CU of the batched interpreter launch (gx_autotune_batches; 0: default)
  // measurement: event pairs bracketing VM kernels
  bool profile = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pending, prof_free;
};

namespace {

std::pair<hipEvent_t, hipEvent_t> prof_pair(gx_rt* rt) {
  if (!rt->prof_free.empty()) {
    auto p = rt->prof_free.back();
    rt->prof_free.pop_back();
    return p;
  }
  std::pair<hipEvent_t, hipEvent_t> p{nullptr, nullptr};
  (void)hipEventCreate(&p.first);
  (void)hipEventCreate(&p.second);
  return p;
}

int to_errno(hipError_t e) { return e == hipErrorOutOfMemory ? -ENOMEM : -EIO; }

struct DevGuard {
  int prev = 0;
  explicit DevGuard(int dev) {
    (void)hipGetDevice(&prev);
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DevGuard() {
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != prev) (void)hipSetDevice(prev);
  }
};

MapObj* get_map(gx_rt* rt, int fd) {
  if (!rt || fd < 0 || fd >= (int)rt->maps.size() || !rt->maps[fd].live) return nullptr;
  return &rt->maps[fd];
}

ProgObj* get_prog(gx_rt* rt, int fd) {
  if (!rt || fd < 0 || fd >= (int)rt->progs.size() || !rt->progs[fd].live) return nullptr;
  return &rt->progs[fd];
}

void free_map(MapObj& m) {
  if (m.host_data) (void)hipHostFree(m.host_data);
  else if (m.h.data) (void)hipFree(m.h.data);
  if (m.host_slots) (void)hipHostFree(m.host_slots);
  else if (m.h.slots) (void)hipFree(m.h.slots);
  if (m.h.ctrl) (void)hipFree(m.h.ctrl);
  if (m.d_desc) (void)hipFree(m.d_desc);
  if (m.drain_ev) {
    (void)hipEventSynchronize(m.drain_ev);  // a started drain still copying
    (void)hipEventDestroy(m.drain_ev);
  }
  if (m.h_pin) (void)hipHostFree(m.h_pin);
  if (m.ctrl_pin) (void)hipHostFree(m.ctrl_pin);
  m = MapObj{};
}

// Launches on stream s that may write the program's rings wait for the
// copies of those rings' started drains (the copies read the ring's
// committed range and then move its tail).
void wait_drains(gx_rt* rt, const ProgObj* p, hipStream_t s) {
  for (int fd : p->fds) {
    const MapObj& m = rt->maps[fd];
    if (m.drain_pending && m.drain_ev) (void)hipStreamWaitEvent(s, m.drain_ev, 0);
  }
}

// Entry points without that stream ordering wait on the host for every
// started drain's copy before they launch.
int drain_barrier(gx_rt* rt) {
  for (const MapObj& m : rt->maps)
    if (m.drain_pending && m.drain_ev && hipEventSynchronize(m.drain_ev) != hipSuccess) return -EIO;
  return 0;
}

void note_stream(gx_rt* rt, hipStream_t s) {
  for (auto& se : rt->stream_events)
    if (se.first == s) {
      (void)hipEventRecord(se.second, s);
      return;
    }
  hipEvent_t e;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return;
  (void)hipEventRecord(e, s);
  rt->stream_events.push_back({s, e});
}

// Execution resources of runs launched on stream s (created on first use).
Exec* exec_for(gx_rt* rt, hipStream_t s) {
  if (rt->cap_ex) return rt->cap_ex;
  for (auto& e : rt->execs)
    if (e.first == s) return e.second;
  Exec* x = new (std::nothrow) Exec();
  if (!x) return nullptr;
  if (exec_init(*x)) {
    exec_free(*x);
    delete x;
    return nullptr;
  }
  rt->execs.push_back({s, x});
  return x;
}

int wait_all(gx_rt* rt) {
  for (auto& se : rt->stream_events)
    if (hipEventSynchronize(se.second) != hipSuccess) return -EIO;
  if (rt->noalloc_used && hipEventSynchronize(rt->noalloc_ev) != hipSuccess) return -EIO;
  if (hipStreamSynchronize(rt->internal) != hipSuccess) return -EIO;
  return 0;
}

// ---------------------------------------------------------------------------
// pre-decoder: one 16-byte micro-op per slot

const int kSizeCode[4] = {2, 1, 0, 3};  // eBPF size bits W, H, B, DW -> log2 bytes

int alu_handler(int o, int16_t off, bool x, bool w64) {
  int base;
  switch (o) {
    case 0x00: base = H_ADD64; break;
    case 0x10: base = H_SUB64; break;
    case 0x20: base = H_MUL64; break;
    case 0x30: base = off ? H_SDIV64 : H_DIV64; break;
    case 0x40: base = H_OR64; break;
    case 0x50: base = H_AND64; break;
    case 0x60: base = H_LSH64; break;
    case 0x70: base = H_RSH64; break;
    case 0x80: base = H_NEG64; break;
    case 0x90: base = off ? H_SMOD64 : H_MOD64; break;
    case 0xa0: base = H_XOR64; break;
    case 0xb0: base = (x && off) ? H_MOVSX64 : H_MOV64; break;
    case 0xc0: base = H_ARSH64; break;
    default: return -1;
  }
  return w64 ? base : base + (H_ADD32 - H_ADD64);
}

int jmp_handler(int o, bool w32) {
  static const int t64[16] = {H_JA, H_JEQ, H_JGT, H_JGE, H_JSET, H_JNE, H_JSGT, H_JSGE,
                              -1,   -1,    H_JLT, H_JLE, H_JSLT, H_JSLE, -1,   -1};
  static const int t32[16] = {H_JA, H_JEQ32, H_JGT32, H_JGE32, H_JSET32, H_JNE32, H_JSGT32, H_JSGE32,
                              -1,   -1,      H_JLT32, H_JLE32, H_JSLT32, H_JSLE32, -1,      -1};
  return (w32 ? t32 : t64)[o >> 4];
}

struct MapRef {
  uint32_t type;
  uint64_t desc;  // device address of the map descriptor
};

std::vector<Uop> predecode(const std::vector<Insn>& P, const Verdict& V, const std::vector<MapRef>& tab) {
  std::vector<Uop> U(P.size());
  for (auto& u : U) u = Uop{uop_w0(H_EXIT, 0, 0, 0, true), 0, 0};
  for (size_t pc = 0; pc < P.size(); pc++) {
    const Insn& in = P[pc];
    int c = in.op & 7, o = in.op & 0xf0;
    bool x = in.op & 8;
    Uop u{0, 0, 0};
    if (c == 4 || c == 7) {
      bool w64 = c == 7;
      if (o == 0xd0) {
        int h = (w64 || x) ? H_BSWAP : H_TRUNC;
        u = Uop{uop_w0(h, in.dst, 0, in.imm, true), 0, 0};
      } else {
        int h = alu_handler(o, in.off, x, w64);
        int a8 = (o == 0xb0 && x) ? in.off : 0;
        uint64_t k = x ? 0 : (w64 ? (uint64_t)(int64_t)in.imm : (uint64_t)(uint32_t)in.imm);
        u = Uop{uop_w0(h, in.dst, x ? in.src : 0, a8, !x), 0, k};
      }
    } else if (c == 5 || c == 6) {
      bool w32 = c == 6;
      if (o == 0x90) {
        u = Uop{uop_w0(H_EXIT, 0, 0, 0, true), 0, 0};
      } else if (o == 0x80) {
        int mi = V.call_map[pc];
        if (mi < 0) continue;  // unreachable
        const MapRef& m = tab[mi];
        int a2 = V.arg2_kind[pc] < 0 ? 0 : V.arg2_kind[pc];
        int a3 = V.arg3_kind[pc] < 0 ? 0 : V.arg3_kind[pc];
        int h = H_EXIT, aux = 0;
        bool arr = m.type == MAP_ARRAY;
        switch (in.imm) {
          case 1: h = arr ? H_LOOKUP_ARRAY : H_LOOKUP_HASH; break;
          case 2: h = arr ? H_UPDATE_ARRAY : H_UPDATE_HASH; break;
          case 3: h = arr ? H_RET_EINVAL : H_DELETE_HASH; break;
          case 130: h = H_RINGBUF_OUTPUT; aux = (int)V.ring_size[pc]; break;
        }
        u = Uop{uop_w0(h, 0, 0, a2 | (a3 << 1), true), aux, m.desc};
      } else {
        int t = (int)pc + 1 + ((w32 && o == 0) ? in.imm : in.off);
        int h = jmp_handler(o, w32);
        uint64_t k = x ? 0 : (w32 ? (uint64_t)(uint32_t)in.imm : (uint64_t)(int64_t)in.imm);
        u = Uop{uop_w0(h, in.dst, x ? in.src : 0, 0, !x), t, k};
      }
    } else if (c == 1) {
      int sc = kSizeCode[(in.op >> 3) & 3];
      int sxf = (in.op & 0xe0) == 0x80 ? 4 : 0;
      int k = V.mem_kind[pc];
      int h = k == KIND_CTX ? H_LDX_CTX : k == KIND_STACK ? H_LDX_STACK : H_LDX_MAP;
      u = Uop{uop_w0(h, in.dst, in.src, sc | sxf, false), in.off, 0};
    } else if (c == 2) {
      int sc = kSizeCode[(in.op >> 3) & 3];
      int h = V.mem_kind[pc] == KIND_STACK ? H_ST_STACK : H_ST_MAP;
      u = Uop{uop_w0(h, in.dst, 0, sc, true), in.off, (uint64_t)(int64_t)in.imm};
    } else if (c == 3) {
      int sc = kSizeCode[(in.op >> 3) & 3];
      bool stack = V.mem_kind[pc] == KIND_STACK;
      if ((in.op & 0xe0) == 0xc0)
        u = Uop{uop_w0(stack ? H_ATOMIC_STACK : H_ATOMIC_MAP, in.dst, in.src, sc, false), in.off,
                (uint64_t)(uint32_t)in.imm};
      else
        u = Uop{uop_w0(stack ? H_STX_STACK : H_STX_MAP, in.dst, in.src, sc, false), in.off, 0};
    } else if (c == 0 && in.op == 0x18) {
      uint64_t val;
      if (in.src == 0) {
        val = (uint64_t)(uint32_t)in.imm | ((uint64_t)(uint32_t)P[pc + 1].imm << 32);
      } else {
        int mi = V.ld_map[pc];
        val = mi >= 0 ? tab[mi].desc : 0;
      }
      u = Uop{uop_w0(H_LDIMM, in.dst, 0, 0, true), 0, val};
      U[pc] = u;
      pc++;  // the second slot is never executed
      continue;
    } else {
      continue;
    }
    U[pc] = u;
  }
  return U;
}

// Events per partition tile (one wave each): at least 4096, and about 2048
// tiles for large runs, so that the partition's waves fill the device (its
// per-queue counts then take 2^qbits x tiles words).
uint64_t part_tile(uint64_t n_events) { return std::max<uint64_t>(4096, next_pow2((n_events + 2047) / 2048)); }

int ensure_ws(Exec& X, size_t counts, size_t sums, size_t order) {
  auto grow = [](uint32_t** p, size_t* cap, size_t need) -> int {
    if (*cap >= need) return 0;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    size_t n = std::max<size_t>(need, 1024);
    if (hipMalloc((void**)p, n * sizeof(uint32_t)) != hipSuccess) return -ENOMEM;
    *cap = n;
    return 0;
  };
  int r;
  if ((r = grow(&X.d_counts, &X.counts_cap, counts))) return r;
  if ((r = grow(&X.d_sums, &X.sums_cap, sums))) return r;
  if ((r = grow(&X.d_order, &X.order_cap, order))) return r;
  // the queue-ordered records: kSortedStride bytes per event (u32 units)
  if ((r = grow((uint32_t**)&X.d_sorted, &X.sorted_cap, order * (kSortedStride / 4)))) return r;
  return 0;
}

int ensure_spill(Exec& X, size_t bytes) {
  if (X.spill_cap >= bytes) return 0;
  if (X.d_spill) (void)hipFree(X.d_spill);
  X.d_spill = nullptr;
  X.spill_cap = 0;
  if (hipMalloc((void**)&X.d_spill, bytes) != hipSuccess) return -ENOMEM;
  X.spill_cap = bytes;
  return 0;
}

// Launch a program's compiled kernel over one run.  mode 0: event-parallel;
// mode 1: stream-sequential over queues [0, A.n_queues) of ``lanes`` per
// wave, counts with row stride ``qstride``, the run's last queue ending at
// ``qend_last`` in order[].
uint32_t jit_ep_blocks(const ProgObj* p, uint64_t n_events, uint32_t blocks_override) {
  const uint64_t tiles = (n_events + 63) / 64;
  const uint32_t nw = jit_waves(p->v.stack_bytes, true);
  uint64_t nb = std::min<uint64_t>((tiles + nw - 1) / nw, kJitMaxBlocks);
  // each block flushes its accumulators once: give every block at least
  // as many events as it flushes words (but keep one block per CU)
  if (p->jacc_words) nb = std::min(nb, std::max<uint64_t>(256, n_events / p->jacc_words));
  if (blocks_override) nb = blocks_override;
  return (uint32_t)std::max<uint64_t>(nb, 1);
}

// Spill bytes a compiled event-parallel run needs (0: none).
uint64_t jit_spill_bytes(const ProgObj* p, uint64_t n_events, uint32_t blocks_override) {
  if (!p->jf_ep || !p->jspill || !p->jf_red) return 0;
  return (uint64_t)jit_ep_blocks(p, n_events, blocks_override) * p->jspill;
}

// ``spill``: the run's spill area (jit_spill_bytes), or null to flush the
// caches directly.
hipError_t launch_jit(const ProgObj* p, RunArgs A, uint32_t mode, uint32_t lanes, uint32_t qstride,
                      uint32_t qend_last, uint32_t blocks_override, uint8_t* spill, hipStream_t s) {
  if (mode == 0) {
    uint32_t nb = jit_ep_blocks(p, A.n_events, blocks_override);
    A.spill = p->jspill && p->jf_red ? spill : nullptr;
    void* args[] = {&A};
    const uint32_t nw = jit_waves(p->v.stack_bytes, true);
    hipError_t e = hipModuleLaunchKernel(p->jf_ep, nb, 1, 1, 64 * nw, 1, 1, 0, s, args, nullptr);
    if (e != hipSuccess || !A.spill) return e;
    void* rargs[] = {&A, &nb};
    return hipModuleLaunchKernel(p->jf_red, p->jred_blocks, 1, 1, 256, 1, 1, 0, s, rargs, nullptr);
  }
  if (lanes == 1 && p->jf_uni) {
    void* args[] = {&A, &qstride, &qend_last};
    return hipModuleLaunchKernel(p->jf_uni, A.n_queues, 1, 1, 64, 1, 1, 0, s, args, nullptr);
  }
  void* args[] = {&A, &lanes, &qstride, &qend_last};
  return hipModuleLaunchKernel(p->jf_seq, (A.n_queues + lanes - 1) / lanes, 1, 1, 64, 1, 1, 0, s, args, nullptr);
}

// The interpreter's event-parallel launch: with the block-level LDS mirror
// when the program updates a small shared array map.
hipError_t launch_interp_ep(gx_rt* rt, const ProgObj* p, RunArgs A, hipStream_t s) {
  if (p->acc_hi <= p->acc_lo || !env_int("GX_INTERP_ACC", 1)) return launch_event_parallel(A, s);
  A.acc_lo = p->acc_lo;
  A.acc_hi = p->acc_hi;
  A.acc_op = p->acc_op;
  A.acc_sc = p->acc_sc;
  return launch_event_parallel_acc(A, rt->n_cu, s);
}

// One plain run of a program with launch shape k (validated arguments).
int run_one(gx_rt* rt, ProgObj* p, const void* d_events, uint64_t n_events, uint32_t* d_rc, hipStream_t s,
            const Knobs& k) {
  Exec* Xp = exec_for(rt, s);
  if (!Xp) return -ENOMEM;
  Exec& X = *Xp;
  RunArgs A{};
  A.uops = p->d_uops;
  A.events = (const uint8_t*)d_events;
  A.rc = d_rc;
  A.n_events = n_events;
  A.record_size = p->record_size;
  A.stack_bytes = p->v.stack_bytes;
  A.stream_off = p->stream_off;
  A.stream_size = p->stream_size;
  A.err = rt->d_err;
  A.guards = p->d_guards;
  A.maptab = p->d_maptab;
  A.leader = p->hook == HOOK_WAVE_MEM ? 1u : 0u;
  A.simt = p->hook == HOOK_SIMT_MEM ? 1u : 0u;
  A.checked = env_int("GX_CHECKED", 0) ? 1u : 0u;
  A.epoch = ++rt->epoch;
  uint64_t per_event = 64 * (p->v.max_insns + 1) + 64;
  hipError_t e;
  std::pair<hipEvent_t, hipEvent_t> pe{nullptr, nullptr};
  if (rt->profile) pe = prof_pair(rt);
  if (p->v.event_parallel) {
    A.step_limit = per_event;
    wait_drains(rt, p, s);
    if (pe.first) (void)hipEventRecord(pe.first, s);
    if (p->jf_ep) {
      const uint64_t need = jit_spill_bytes(p, n_events, k.blocks);
      uint8_t* sp = nullptr;
      if (need) {
        int r = ensure_spill(X, need);
        if (r) return r;
        if (X.spill_used) (void)hipStreamWaitEvent(s, X.spill_ev, 0);
        sp = X.d_spill;
      }
      e = launch_jit(p, A, 0, 0, 0, 0, k.blocks, sp, s);
      if (sp) {
        (void)hipEventRecord(X.spill_ev, s);
        X.spill_used = true;
        rt->stats.launches += 1;
      }
    } else {
      e = launch_interp_ep(rt, p, A, s);
    }
    if (pe.second) (void)hipEventRecord(pe.second, s);
    rt->stats.launches += 1;
  } else {
    const uint32_t lbits = k.qbits;
    const uint32_t L = 1u << lbits;
    uint64_t tile = part_tile(n_events);
    uint32_t nt = (uint32_t)((n_events + tile - 1) / tile);
    uint64_t m = (uint64_t)L * nt;
    int r = ensure_ws(X, m, (m + 4095) / 4096 + 1, n_events);
    if (r) return r;
    if (X.ws_used) (void)hipStreamWaitEvent(s, X.ws_event, 0);
    A.step_limit = per_event * n_events;
    // the one-queue compiled kernel gathers its records through order[], so
    // the partition writes only the indices
    const bool gather = p->jf_uni && k.lanes == 1;
    e = launch_partition(A, lbits, (uint32_t)tile, nt, X.d_counts, X.d_sums, X.d_order, gather ? nullptr : X.d_sorted,
                         s);
    if (e == hipSuccess) {
      A.order = X.d_order;
      A.sorted = gather ? nullptr : X.d_sorted;
      A.qstart = X.d_counts;
      A.n_queues = L;
      // the partition above may run while a started drain still copies
      wait_drains(rt, p, s);
      if (pe.first) (void)hipEventRecord(pe.first, s);
      if (p->jf_seq) {
        e = launch_jit(p, A, 1, k.lanes, nt, (uint32_t)n_events, 0, nullptr, s);
      } else {
        e = launch_stream_seq(A, k.lanes, nt, s);
      }
      if (pe.second) (void)hipEventRecord(pe.second, s);
    }
    (void)hipEventRecord(X.ws_event, s);
    X.ws_used = true;
    rt->stats.launches += 6;
  }
  if (pe.first) rt->prof_pending.push_back(pe);
  if (e != hipSuccess) return to_errno(e);
  rt->stats.events += n_events;
  note_stream(rt, s);
  return 0;
}

// A program verified and pre-decoded against stand-in map descriptors, for
// showing or compiling generated source without a device.
struct StandIn {
  Verdict v;
  std::vector<Uop> U;
  std::vector<std::pair<uint64_t, MapDev>> maps;
  std::string log;
  int hook = 0;
  JitProg prog() const {
    JitProg q{&U, v.stack_bytes, &maps, &v.mem_map, &v.ld_map, v.event_parallel, hook == HOOK_WAVE_MEM,
              hook == HOOK_SIMT_MEM};
    q.max_insns = v.max_insns;
    return q;
  }
};

int stand_in(const uint64_t* insns, uint32_t n_insns, uint32_t hook_type, const uint32_t* map_shapes, uint32_t n_maps,
             StandIn* out) {
  if (!insns && n_insns) return -EINVAL;
  if (n_insns > (uint32_t)kMaxInsns) return -E2BIG;
  uint32_t rs, so, ss;
  if (!hook_layout((int)hook_type, &rs, &so, &ss)) return -EINVAL;
  std::vector<MapShape> shapes(n_maps);
  std::vector<int> fds(n_maps);
  std::vector<MapRef> refs(n_maps);
  for (uint32_t i = 0; i < n_maps; i++) {
    shapes[i] = MapShape{map_shapes[5 * i], map_shapes[5 * i + 1], map_shapes[5 * i + 2], map_shapes[5 * i + 3],
                         map_shapes[5 * i + 4]};
    fds[i] = (int)i;
    refs[i] = MapRef{map_shapes[5 * i], 0x100000000ull + 64ull * i};  // stand-in descriptor addresses
  }
  for (uint32_t i = 0; i < n_maps; i++) {
    MapDev d{};
    d.type = shapes[i].type;
    d.key_size = shapes[i].key_size;
    d.value_size = shapes[i].value_size;
    d.max_entries = shapes[i].max_entries;
    d.flags = shapes[i].flags;
    d.vstride = (d.value_size + 7) & ~7u;
    d.slot_mask = d.type == MAP_RINGBUF ? d.max_entries - 1
                  : d.type == MAP_HASH  ? (uint32_t)next_pow2(std::max<uint64_t>(2ull * d.max_entries, 16)) - 1
                                        : 0;
    d.sstride = 8 + ((d.key_size + 7) & ~7u);
    out->maps.push_back({refs[i].desc, d});
  }
  std::vector<Insn> P = decode_insns(insns, n_insns);
  out->hook = (int)hook_type;
  out->v = verify(P, (int)hook_type, shapes, fds);
  if (!out->v.ok) {
    out->log = out->v.log;
    return -EACCES;
  }
  out->U = predecode(P, out->v, refs);
  return 0;
}

// Device copies of maps' state (values, hash slots, control words, ring
// data), taken and put back on a stream: runs made only to measure or to
// size something leave no trace.
struct MapSnapshot {
  struct Part {
    void* src;
    void* tmp;
    size_t bytes;
  };
  std::vector<Part> parts;
  int take(gx_rt* rt, const std::vector<int>& fds, hipStream_t s) {
    std::vector<int> seen;
    for (int fd : fds) {
      if (std::find(seen.begin(), seen.end(), fd) != seen.end()) continue;
      seen.push_back(fd);
      MapObj* m = get_map(rt, fd);
      if (!m) continue;
      for (auto pr : {std::make_pair((void*)m->h.data, m->data_bytes), std::make_pair((void*)m->h.slots, m->slot_bytes),
                      std::make_pair((void*)m->h.ctrl, (size_t)kCtrlBytes)}) {
        if (!pr.first || !pr.second) continue;
        Part pt{pr.first, nullptr, pr.second};
        if (hipMalloc(&pt.tmp, pt.bytes) != hipSuccess) return -ENOMEM;
        parts.push_back(pt);
        (void)hipMemcpyAsync(pt.tmp, pt.src, pt.bytes, hipMemcpyDeviceToDevice, s);
      }
    }
    return 0;
  }
  void restore(hipStream_t s) {
    for (auto& pt : parts) (void)hipMemcpyAsync(pt.src, pt.tmp, pt.bytes, hipMemcpyDeviceToDevice, s);
  }
  ~MapSnapshot() {
    for (auto& pt : parts)
      if (pt.tmp) (void)hipFree(pt.tmp);
  }
};

int jit_app_module(gx_rt* rt, ProgObj* p, int kind, hipModule_t* mod, hipFunction_t* f, hipFunction_t* fr,
                   JitInfo* info_out);

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

int gx_open(int hip_device, gx_rt** out) {
  if (!out) return -EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return -ENODEV;
  gx_rt* rt = new (std::nothrow) gx_rt();
  if (!rt) return -ENOMEM;
  rt->dev = hip_device;
  DevGuard g(hip_device);
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, hip_device) == hipSuccess && ncu > 0)
    rt->n_cu = (uint32_t)ncu;
  int wkhz = 0;
  if (hipDeviceGetAttribute(&wkhz, hipDeviceAttributeWallClockRate, hip_device) == hipSuccess && wkhz > 0)
    rt->wall_khz = (uint32_t)wkhz;
  if (hipStreamCreateWithFlags(&rt->internal, hipStreamNonBlocking) != hipSuccess ||
      hipMalloc((void**)&rt->d_err, 64) != hipSuccess || hipMalloc((void**)&rt->d_stage, 16384) != hipSuccess ||
      hipEventCreateWithFlags(&rt->noalloc_ev, hipEventDisableTiming) != hipSuccess ||
      scratch_region(hip_device, &rt->d_scratch, &rt->scratch_bytes) != hipSuccess || vm_init() != hipSuccess) {
    gx_close(rt);
    return -ENOMEM;
  }
  (void)hipMemset(rt->d_err, 0, 64);
  (void)hipDeviceSynchronize();
  *out = rt;
  return 0;
}

void gx_close(gx_rt* rt) {
  if (!rt) return;
  gx_snapshot_stop(rt);
  DevGuard g(rt->dev);
  (void)hipDeviceSynchronize();
  for (auto& m : rt->maps)
    if (m.live) free_map(m);
  for (auto& p : rt->progs) {
    if (p.d_uops) (void)hipFree(p.d_uops);
    if (p.d_guards) (void)hipFree(p.d_guards);
    if (p.d_maptab) (void)hipFree(p.d_maptab);
  }
  for (auto& jm : rt->jit_cache)
    if (jm.second.mod) (void)hipModuleUnload(jm.second.mod);
  for (auto& se : rt->stream_events) (void)hipEventDestroy(se.second);
  if (rt->noalloc_ev) (void)hipEventDestroy(rt->noalloc_ev);
  for (auto* v : {&rt->prof_pending, &rt->prof_free})
    for (auto& pe : *v) {
      (void)hipEventDestroy(pe.first);
      (void)hipEventDestroy(pe.second);
    }
  for (auto& e : rt->execs) {
    exec_free(*e.second);
    delete e.second;
  }
  for (void* p : {(void*)rt->d_err, (void*)rt->d_stage})
    if (p) (void)hipFree(p);
  if (rt->internal) (void)hipStreamDestroy(rt->internal);
  if (rt->copy) (void)hipStreamDestroy(rt->copy);
  delete rt;
}

int gx_create_map(gx_rt* rt, uint32_t type, uint32_t key_size, uint32_t value_size, uint32_t max_entries,
                  uint32_t flags) {
  if (!rt) return -EINVAL;
  if (flags & ~(uint32_t)(F_SHARED | F_READ_ONLY | F_HOST)) return -EINVAL;
  if ((flags & F_SHARED) && (flags & F_READ_ONLY)) return -EINVAL;
  if ((flags & F_HOST) && (!(flags & F_READ_ONLY) || (type != MAP_ARRAY && type != MAP_HASH))) return -EINVAL;
  MapObj m;
  m.h.type = type;
  m.h.key_size = key_size;
  m.h.value_size = value_size;
  m.h.max_entries = max_entries;
  m.h.flags = flags;
  m.h.vstride = (value_size + 7) & ~7u;
  if (type == MAP_ARRAY) {
    if (key_size != 4 || value_size == 0 || value_size > 4096 || max_entries == 0) return -EINVAL;
    m.data_bytes = (size_t)max_entries * m.h.vstride;
  } else if (type == MAP_HASH) {
    if (key_size == 0 || key_size > 64 || value_size == 0 || value_size > 4096 || max_entries == 0 ||
        max_entries > (1u << 28))
      return -EINVAL;
    uint64_t slots = next_pow2(std::max<uint64_t>(2ull * max_entries, 16));
    m.h.slot_mask = (uint32_t)(slots - 1);
    m.h.sstride = 8 + ((key_size + 7) & ~7u);
    m.slot_bytes = slots * m.h.sstride;
    m.data_bytes = slots * m.h.vstride;
  } else if (type == MAP_RINGBUF) {
    if (key_size || value_size || max_entries < 4096 || (max_entries & (max_entries - 1)) || flags) return -EINVAL;
    m.h.slot_mask = max_entries - 1;
    m.data_bytes = max_entries;
  } else {
    return -EINVAL;
  }
  DevGuard g(rt->dev);
  bool ok;
  if (flags & F_HOST) {
    // the cold tier: pinned host memory, mapped for the device's loads
    auto host = [&](size_t bytes, uint8_t** hp, uint8_t** dp) {
      if (hipHostMalloc((void**)hp, bytes, hipHostMallocMapped) != hipSuccess) return false;
      std::memset(*hp, 0, bytes);
      return hipHostGetDevicePointer((void**)dp, *hp, 0) == hipSuccess;
    };
    ok = host(m.data_bytes, &m.host_data, &m.h.data) && (!m.slot_bytes || host(m.slot_bytes, &m.host_slots, &m.h.slots));
  } else {
    ok = hipMalloc((void**)&m.h.data, m.data_bytes) == hipSuccess &&
         (!m.slot_bytes || hipMalloc((void**)&m.h.slots, m.slot_bytes) == hipSuccess);
  }
  ok = ok && hipMalloc((void**)&m.h.ctrl, kCtrlBytes) == hipSuccess &&
       hipMalloc((void**)&m.d_desc, sizeof(MapDev)) == hipSuccess;
  if (!ok) {
    free_map(m);
    return -ENOMEM;
  }
  ok = (m.host_data || hipMemsetAsync(m.h.data, 0, m.data_bytes, rt->internal) == hipSuccess) &&
       hipMemsetAsync(m.h.ctrl, 0, kCtrlBytes, rt->internal) == hipSuccess &&
       (!m.slot_bytes || m.host_slots || hipMemsetAsync(m.h.slots, 0, m.slot_bytes, rt->internal) == hipSuccess) &&
       hipMemcpyAsync(m.d_desc, &m.h, sizeof(MapDev), hipMemcpyHostToDevice, rt->internal) == hipSuccess &&
       hipStreamSynchronize(rt->internal) == hipSuccess;
  if (!ok) {
    free_map(m);
    return -EIO;
  }
  m.live = true;
  rt->maps.push_back(m);
  return (int)rt->maps.size() - 1;
}

static int map_op(gx_rt* rt, int fd, int op, const void* key, const void* val, uint64_t flags, void* val_out) {
  MapObj* m = get_map(rt, fd);
  if (!m || !key || m->h.type == MAP_RINGBUF) return -EINVAL;
  if (op == 1 && !val) return -EINVAL;
  if (op == 2 && m->h.type == MAP_ARRAY) return -EINVAL;
  DevGuard g(rt->dev);
  if (wait_all(rt)) return -EIO;
  uint32_t ks = m->h.key_size, vs = m->h.value_size;
  // staging layout: key @0 (<= 64 B), result @64, value in @128, value out @4224
  uint8_t* dk = rt->d_stage;
  int64_t* dret = (int64_t*)(rt->d_stage + 64);
  uint8_t* dv = rt->d_stage + 128;
  uint8_t* dout = rt->d_stage + 128 + 4096;
  int64_t ret = -EIO;
  bool ok = hipMemcpyAsync(dk, key, ks, hipMemcpyHostToDevice, rt->internal) == hipSuccess &&
            (op != 1 || hipMemcpyAsync(dv, val, vs, hipMemcpyHostToDevice, rt->internal) == hipSuccess) &&
            launch_map_op(m->d_desc, op, dk, dv, flags, dret, dout, ++rt->epoch, rt->internal) == hipSuccess &&
            hipMemcpyAsync(&ret, dret, 8, hipMemcpyDeviceToHost, rt->internal) == hipSuccess &&
            hipStreamSynchronize(rt->internal) == hipSuccess;
  if (!ok) return -EIO;
  if (op == 0 && ret == 0 && val_out)
    if (hipMemcpy(val_out, dout, vs, hipMemcpyDeviceToHost) != hipSuccess) return -EIO;
  return (int)ret;
}

int gx_map_update(gx_rt* rt, int map_fd, const void* key, const void* val, uint64_t flags) {
  return map_op(rt, map_fd, 1, key, val, flags, nullptr);
}
int gx_map_lookup(gx_rt* rt, int map_fd, const void* key, void* val_out) {
  return map_op(rt, map_fd, 0, key, nullptr, 0, val_out);
}
int gx_map_delete(gx_rt* rt, int map_fd, const void* key) {
  return map_op(rt, map_fd, 2, key, nullptr, 0, nullptr);
}

int64_t gx_map_dump(gx_rt* rt, int map_fd, void* keys, void* vals, uint64_t cap) {
  MapObj* m = get_map(rt, map_fd);
  if (!m || m->h.type == MAP_RINGBUF) return -EINVAL;
  DevGuard g(rt->dev);
  if (wait_all(rt)) return -EIO;
  const MapDev& d = m->h;
  if (d.type == MAP_ARRAY) {
    uint64_t n = d.max_entries;
    if ((keys || vals) && cap) {
      std::vector<uint8_t> buf(m->data_bytes);
      if (hipMemcpy(buf.data(), d.data, m->data_bytes, hipMemcpyDeviceToHost) != hipSuccess) return -EIO;
      for (uint64_t i = 0; i < n && i < cap; i++) {
        if (keys) std::memcpy((uint8_t*)keys + 4 * i, &i, 4);
        if (vals) std::memcpy((uint8_t*)vals + i * d.value_size, buf.data() + i * d.vstride, d.value_size);
      }
    }
    return (int64_t)n;
  }
  std::vector<uint8_t> slots(m->slot_bytes), data(m->data_bytes);
  if (hipMemcpy(slots.data(), d.slots, m->slot_bytes, hipMemcpyDeviceToHost) != hipSuccess) return -EIO;
  if ((vals && cap) && hipMemcpy(data.data(), d.data, m->data_bytes, hipMemcpyDeviceToHost) != hipSuccess)
    return -EIO;
  uint64_t n = 0;
  for (uint64_t i = 0; i <= d.slot_mask; i++) {
    const uint8_t* hdr = slots.data() + i * d.sstride;
    uint32_t st;
    std::memcpy(&st, hdr, 4);
    if ((st & 0xff) != SLOT_LIVE) continue;  // header: {u8 state, u24 epoch, u32 tag}
    if (n < cap) {
      if (keys) std::memcpy((uint8_t*)keys + n * d.key_size, hdr + 8, d.key_size);
      if (vals) std::memcpy((uint8_t*)vals + n * d.value_size, data.data() + i * d.vstride, d.value_size);
    }
    n++;
  }
  return (int64_t)n;
}

int gx_map_clear(gx_rt* rt, int map_fd) {
  MapObj* m = get_map(rt, map_fd);
  if (!m) return -EINVAL;
  DevGuard g(rt->dev);
  if (wait_all(rt)) return -EIO;
  if (m->host_data) std::memset(m->host_data, 0, m->data_bytes);
  if (m->host_slots) std::memset(m->host_slots, 0, m->slot_bytes);
  bool ok = (m->host_data || hipMemset(m->h.data, 0, m->data_bytes) == hipSuccess) &&
            hipMemset(m->h.ctrl, 0, kCtrlBytes) == hipSuccess &&
            (!m->slot_bytes || m->host_slots || hipMemset(m->h.slots, 0, m->slot_bytes) == hipSuccess) &&
            hipDeviceSynchronize() == hipSuccess;
  return ok ? 0 : -EIO;
}

static void fill_info(const Verdict& v, uint32_t hook, uint32_t n, gx_prog_info* out) {
  out->mode = v.event_parallel ? GX_MODE_EVENT_PARALLEL : GX_MODE_STREAM_SEQUENTIAL;
  out->hook = hook;
  out->n_insns = n;
  out->stack_bytes = v.stack_bytes;
  out->max_insns = v.max_insns;
  out->max_calls = v.max_calls;
  out->max_ring_bytes = v.max_ring;
}

static void write_log(char* log, uint32_t size, const std::string& s) {
  if (!log || !size) return;
  size_t n = std::min<size_t>(size - 1, s.size());
  std::memcpy(log, s.data(), n);
  log[n] = 0;
}

int gx_verify(const uint64_t* insns, uint32_t n_insns, uint32_t hook_type, const uint32_t* map_shapes,
              uint32_t n_maps, char* log, uint32_t log_size, gx_prog_info* info) {
  if (n_insns > (uint32_t)kMaxInsns) {
    write_log(log, log_size, "program has more than 4096 instructions");
    return -E2BIG;
  }
  if (!insns && n_insns) return -EINVAL;
  std::vector<MapShape> shapes(n_maps);
  std::vector<int> fds(n_maps);
  for (uint32_t i = 0; i < n_maps; i++) {
    shapes[i] = MapShape{map_shapes[5 * i], map_shapes[5 * i + 1], map_shapes[5 * i + 2], map_shapes[5 * i + 3],
                         map_shapes[5 * i + 4]};
    fds[i] = (int)i;
  }
  Verdict v = verify(decode_insns(insns, n_insns), (int)hook_type, shapes, fds);
  write_log(log, log_size, v.log);
  if (!v.ok) return -EACCES;
  if (info) fill_info(v, hook_type, n_insns, info);
  return 0;
}

int gx_load_program(gx_rt* rt, const uint64_t* insns, uint32_t n_insns, uint32_t hook_type, const int* map_fds,
                    uint32_t n_maps, char* log, uint32_t log_size) {
  if (!rt || (!insns && n_insns)) return -EINVAL;
  if (n_insns > (uint32_t)kMaxInsns) {
    write_log(log, log_size, "program has more than 4096 instructions");
    return -E2BIG;
  }
  uint32_t rs, so, ss;
  if (!hook_layout((int)hook_type, &rs, &so, &ss)) return -EINVAL;
  std::vector<MapShape> shapes;
  std::vector<int> fds;
  std::vector<MapObj*> tab;
  for (uint32_t i = 0; i < n_maps; i++) {
    MapObj* m = get_map(rt, map_fds[i]);
    if (!m) return -EINVAL;
    shapes.push_back(MapShape{m->h.type, m->h.key_size, m->h.value_size, m->h.max_entries, m->h.flags});
    fds.push_back(map_fds[i]);
    tab.push_back(m);
  }
  std::vector<Insn> P = decode_insns(insns, n_insns);
  Verdict v = verify(P, (int)hook_type, shapes, fds);
  write_log(log, log_size, v.log);
  if (!v.ok) return -EACCES;
  std::vector<MapRef> refs;
  for (MapObj* m : tab) refs.push_back(MapRef{m->h.type, (uint64_t)(uintptr_t)m->d_desc});
  std::vector<Uop> U = predecode(P, v, refs);
  std::vector<uint64_t> guards(2 * P.size(), 0);
  for (size_t pc = 0; pc < P.size(); pc++)
    if (v.mem_map[pc] >= 0) {
      MapObj* m = tab[v.mem_map[pc]];
      guards[2 * pc] = (uint64_t)(uintptr_t)m->h.data;
      guards[2 * pc + 1] = (uint64_t)(uintptr_t)m->h.data + m->data_bytes;
    }
  ProgObj p;
  // the first shared array map the program updates with atomics, if its
  // value area fits an LDS mirror (the verifier allows one operation at one
  // width per shared map)
  for (size_t pc = 0; pc < U.size() && pc < v.mem_map.size(); pc++) {
    if ((U[pc].w0 & 0xff) != H_ATOMIC_MAP || v.mem_map[pc] < 0) continue;
    const MapObj* m = tab[v.mem_map[pc]];
    if (m->h.type != MAP_ARRAY || !(m->h.flags & F_SHARED)) continue;
    const uint64_t area = (uint64_t)m->h.max_entries * m->h.vstride;
    if (area > kAccMirrorMax) continue;
    p.acc_lo = (uint64_t)(uintptr_t)m->h.data;
    p.acc_hi = p.acc_lo + area;
    p.acc_op = (uint32_t)U[pc].imm & 0xf0;
    p.acc_sc = (U[pc].w0 >> 16) & 3;
    break;
  }
  p.hook = (int)hook_type;
  p.record_size = rs;
  p.stream_off = so;
  p.stream_size = ss;
  p.n_insns = n_insns;
  p.fds = fds;
  DevGuard g(rt->dev);
  if (hipMalloc((void**)&p.d_uops, U.size() * sizeof(Uop)) != hipSuccess) return -ENOMEM;
  if (hipMalloc((void**)&p.d_guards, guards.size() * sizeof(uint64_t)) != hipSuccess) {
    (void)hipFree(p.d_uops);
    return -ENOMEM;
  }
  if (hipMemcpy(p.d_uops, U.data(), U.size() * sizeof(Uop), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p.d_guards, guards.data(), guards.size() * sizeof(uint64_t), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p.d_uops);
    (void)hipFree(p.d_guards);
    return -EIO;
  }
  std::vector<uint64_t> mt(std::max<size_t>(tab.size(), 1), 0);
  for (size_t i = 0; i < tab.size(); i++) mt[i] = (uint64_t)(uintptr_t)tab[i]->d_desc;
  if (hipMalloc((void**)&p.d_maptab, mt.size() * 8) != hipSuccess ||
      hipMemcpy(p.d_maptab, mt.data(), mt.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p.d_uops);
    (void)hipFree(p.d_guards);
    if (p.d_maptab) (void)hipFree(p.d_maptab);
    return -ENOMEM;
  }
  p.v = std::move(v);
  p.uops = std::move(U);
  p.live = true;
  rt->progs.push_back(std::move(p));
  return (int)rt->progs.size() - 1;
}

int gx_autotune(gx_rt* rt, int prog_fd, const void* d_events, uint64_t n_events, uint32_t record_size, uint32_t* d_rc,
                void* stream, gx_tune* out) {
  ProgObj* p = get_prog(rt, prog_fd);
  if (!p || record_size != p->record_size || p->hook == HOOK_SCHED || !d_events || n_events == 0) return -EINVAL;
  if (n_events >= (1ull << 32)) return -E2BIG;
  DevGuard g(rt->dev);
  if (drain_barrier(rt)) return -EIO;  // started drains finish copying first
  hipStream_t s = (hipStream_t)stream;
  // candidate shapes
  std::vector<Knobs> cand;
  const Knobs def = Knobs{default_lanes(p), (uint32_t)std::min(16, std::max(6, env_int("GX_QUEUE_BITS", 12))), 0};
  cand.push_back(def);
  if (p->v.event_parallel) {
    if (p->jf_ep)
      for (uint32_t b : {64u, 128u, 256u, 512u, 1024u, 2048u, 4096u, 8192u}) cand.push_back(Knobs{def.lanes, def.qbits, b});
  } else {
    for (uint32_t q : {10u, 12u, 14u})
      for (uint32_t l : {1u, 2u, 4u, 8u, 16u, 32u, 64u}) cand.push_back(Knobs{l, q, 0});
  }
  // the trials run the program for real: save every map's state and put it
  // back before each trial and at the end
  if (wait_all(rt)) return -EIO;
  MapSnapshot snap;
  if (snap.take(rt, p->fds, s)) return -ENOMEM;
  auto restore = [&]() { snap.restore(s); };
  const bool prof = rt->profile;
  const gx_stats st = rt->stats;
  rt->profile = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int r = 0;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) r = -ENOMEM;
  double best = 1e300, def_ms = 0;
  Knobs bestk = def;
  // one untimed run first (first-touch of workspaces and code)
  if (!r) {
    restore();
    r = run_one(rt, p, d_events, n_events, d_rc, s, def);
  }
  for (size_t c = 0; c < cand.size() && !r; c++) {
    restore();
    (void)hipEventRecord(e0, s);
    r = run_one(rt, p, d_events, n_events, d_rc, s, cand[c]);
    (void)hipEventRecord(e1, s);
    if (r) break;
    float ms = 0;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      r = -EIO;
      break;
    }
    if (c == 0) def_ms = ms;
    // another shape replaces the default only if clearly faster (3 %):
    // near-ties are timing noise, and the default keeps runs comparable
    if (c == 0 ? ms < best : ms < best && ms < 0.97 * def_ms) {
      best = ms;
      bestk = cand[c];
    }
  }
  restore();
  (void)hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  rt->profile = prof;
  rt->stats = st;
  if (r) return r;
  p->tuned_lanes = bestk.lanes;
  p->tuned_qbits = bestk.qbits;
  p->tuned_blocks = bestk.blocks;
  if (out) {
    out->lanes = bestk.lanes;
    out->qbits = bestk.qbits;
    out->blocks = bestk.blocks;
    out->trials = (uint32_t)cand.size();
    out->best_ms = best;
    out->default_ms = def_ms;
  }
  return 0;
}

int gx_jit_program(gx_rt* rt, int prog_fd, char* log, uint32_t log_size) {
  ProgObj* p = get_prog(rt, prog_fd);
  if (!p) return -EINVAL;
  if (p->jmod) return 0;
  std::vector<std::pair<uint64_t, MapDev>> maps;
  for (int fd : p->fds) {
    MapObj* m = get_map(rt, fd);
    if (!m) return -EINVAL;
    maps.push_back({(uint64_t)(uintptr_t)m->d_desc, m->h});
  }
  if (p->hook == HOOK_SCHED) {
    // the program's only kernel is the block scheduler's
    hipModule_t mod = nullptr;
    JitInfo ji;
    int r = jit_app_module(rt, p, 2, &mod, &p->jf_app, &p->jf_app_red, &ji);
    write_log(log, log_size, "");
    if (r) return r;
    p->jacc_words = ji.acc_words;
    p->jspill = p->jf_app_red ? ji.spill_block_bytes : 0;
    p->jred_blocks = ji.reduce_blocks;
    p->jmod = mod;
    return 0;
  }
  JitInfo info;
  JitProg jp{&p->uops, p->v.stack_bytes, &maps, &p->v.mem_map, &p->v.ld_map, p->v.event_parallel,
             p->hook == HOOK_WAVE_MEM, p->hook == HOOK_SIMT_MEM};
  jp.max_insns = p->v.max_insns;
  const std::string src = jit_source(jp, &info);
  auto adopt = [&](const gx_rt::JitMod& jm) {
    p->jf_ep = jm.fe;
    p->jf_seq = jm.fs;
    p->jf_uni = jm.fu;
    p->jf_red = jm.fr;
    p->jacc_words = jm.info.acc_words;
    p->jspill = jm.fr ? jm.info.spill_block_bytes : 0;
    p->jred_blocks = jm.info.reduce_blocks;
    p->jmod = jm.mod;
  };
  {
    std::lock_guard<std::mutex> lk(rt->jit_mu);
    auto it = rt->jit_cache.find(src);
    if (it != rt->jit_cache.end()) {
      adopt(it->second);
      write_log(log, log_size, "");
      return 0;
    }
  }
  std::vector<char> code;
  std::string lg;
  int r = jit_compile(src, &code, &lg);
  write_log(log, log_size, lg);
  if (r) return r;
  DevGuard g(rt->dev);
  gx_rt::JitMod jm;
  jm.info = info;
  if (hipModuleLoadData(&jm.mod, code.data()) != hipSuccess) return -EIO;
  if (p->v.event_parallel ? hipModuleGetFunction(&jm.fe, jm.mod, "gx_j_event_parallel") != hipSuccess ||
                                (info.spill_block_bytes &&
                                 hipModuleGetFunction(&jm.fr, jm.mod, "gx_j_reduce") != hipSuccess)
                          : (hipModuleGetFunction(&jm.fs, jm.mod, "gx_j_stream_seq") != hipSuccess ||
                             hipModuleGetFunction(&jm.fu, jm.mod, "gx_j_stream_uni") != hipSuccess)) {
    (void)hipModuleUnload(jm.mod);
    return -EIO;
  }
  std::lock_guard<std::mutex> lk(rt->jit_mu);
  auto ins = rt->jit_cache.emplace(src, jm);
  if (!ins.second) (void)hipModuleUnload(jm.mod);  // compiled concurrently by another call
  adopt(ins.first->second);
  return 0;
}

int gx_jit_program_set(gx_rt* rt, const int* prog_fds, uint32_t n, char* log, uint32_t log_size) {
  if (!rt || !prog_fds || n == 0 || n > kMaxSetPrograms) return -EINVAL;
  std::vector<ProgObj*> ps;
  std::vector<std::vector<std::pair<uint64_t, MapDev>>> maps(n);
  std::vector<JitProg> jp;
  for (uint32_t i = 0; i < n; i++) {
    ProgObj* p = get_prog(rt, prog_fds[i]);
    if (!p) return -EINVAL;
    for (ProgObj* q : ps)
      if (q == p) return -EINVAL;  // each program once
    ps.push_back(p);
    for (int fd : p->fds) {
      MapObj* m = get_map(rt, fd);
      if (!m) return -EINVAL;
      maps[i].push_back({(uint64_t)(uintptr_t)m->d_desc, m->h});
    }
  }
  // instances of one program with same-shaped maps share a slot (their
  // generated text is the same)
  std::vector<uint32_t> slot(n);
  std::map<std::string, uint32_t> uniq;
  for (uint32_t i = 0; i < n; i++) {
    const JitProg q{&ps[i]->uops, ps[i]->v.stack_bytes, &maps[i], &ps[i]->v.mem_map, &ps[i]->v.ld_map,
                    ps[i]->v.event_parallel, ps[i]->hook == HOOK_WAVE_MEM, ps[i]->hook == HOOK_SIMT_MEM};
    auto ins = uniq.emplace(jit_source(q), (uint32_t)jp.size());
    if (ins.second) jp.push_back(q);
    slot[i] = ins.first->second;
  }
  const std::string src = jit_set_source(jp);
  hipFunction_t f = nullptr;
  {
    std::lock_guard<std::mutex> lk(rt->jit_mu);
    auto it = rt->jit_cache.find(src);
    if (it != rt->jit_cache.end()) f = it->second.fs;
  }
  if (!f) {
    std::vector<char> code;
    std::string lg;
    int r = jit_compile(src, &code, &lg);
    write_log(log, log_size, lg);
    if (r) return r;
    DevGuard g(rt->dev);
    gx_rt::JitMod jm;
    if (hipModuleLoadData(&jm.mod, code.data()) != hipSuccess) return -EIO;
    if (hipModuleGetFunction(&jm.fs, jm.mod, "gx_j_set") != hipSuccess) {
      (void)hipModuleUnload(jm.mod);
      return -EIO;
    }
    std::lock_guard<std::mutex> lk(rt->jit_mu);
    auto ins = rt->jit_cache.emplace(src, jm);
    if (!ins.second) (void)hipModuleUnload(jm.mod);
    f = ins.first->second.fs;
  } else {
    write_log(log, log_size, "");
  }
  std::lock_guard<std::mutex> lk(rt->jit_mu);
  const int id = (int)rt->sets.size();
  int bpc = 0;
  if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, f, 64, 0) != hipSuccess) bpc = 0;
  rt->sets.push_back(gx_rt::JitSet{f, (uint32_t)std::max(bpc, 0)});
  for (uint32_t i = 0; i < n; i++) {
    ps[i]->set_id = id;
    ps[i]->set_slot = slot[i];
  }
  return id;
}

int64_t gx_jit_set_source(const uint64_t* insns, const uint32_t* n_insns, const uint32_t* hooks,
                          const uint32_t* map_shapes, const uint32_t* n_maps, uint32_t n_progs, int compile, char* out,
                          uint64_t cap) {
  if (!insns || !n_insns || !hooks || !n_maps || n_progs == 0 || n_progs > kMaxSetPrograms) return -EINVAL;
  std::vector<StandIn> sp(n_progs);
  std::vector<JitProg> jp;
  const uint64_t* ip = insns;
  const uint32_t* sh = map_shapes;
  for (uint32_t i = 0; i < n_progs; i++) {
    int r = stand_in(ip, n_insns[i], hooks[i], sh, n_maps[i], &sp[i]);
    if (r) {
      write_log(out, (uint32_t)std::min<uint64_t>(cap, 0xffffffffu), sp[i].log);
      return r;
    }
    ip += n_insns[i];
    sh += 5 * n_maps[i];
  }
  for (auto& x : sp) jp.push_back(x.prog());
  std::string src = jit_set_source(jp);
  if (compile) {
    std::vector<char> code;
    std::string lg;
    int r = jit_compile(src, &code, &lg);
    if (r) {
      write_log(out, (uint32_t)std::min<uint64_t>(cap, 0xffffffffu), lg);
      return r;
    }
  }
  if (out && cap) write_log(out, (uint32_t)std::min<uint64_t>(cap, 0xffffffffu), src);
  return (int64_t)src.size();
}

int64_t gx_jit_source(const uint64_t* insns, uint32_t n_insns, uint32_t hook_type, const uint32_t* map_shapes,
                      uint32_t n_maps, int compile, char* out, uint64_t cap) {
  StandIn si;
  int r = stand_in(insns, n_insns, hook_type, map_shapes, n_maps, &si);
  if (r) {
    if (r == -EACCES) write_log(out, (uint32_t)std::min<uint64_t>(cap, 0xffffffffu), si.log);
    return r;
  }
  JitProg jp = si.prog();
  jp.kernel = hook_type == HOOK_SCHED ? 2 : (compile & 2) ? 1 : 0;
  if (jp.kernel == 1 && (!jp.event_parallel || hook_type == HOOK_KERNEL_TIMING)) return -EINVAL;
  std::string src = jit_source(jp);
  if (compile & 1) {
    std::vector<char> code;
    std::string lg;
    r = jit_compile(src, &code, &lg);
    if (r) {
      write_log(out, (uint32_t)std::min<uint64_t>(cap, 0xffffffffu), lg);
      return r;
    }
  }
  if (out && cap) write_log(out, (uint32_t)std::min<uint64_t>(cap, 0xffffffffu), src);
  return (int64_t)src.size();
}

int gx_prog_info_get(gx_rt* rt, int prog_fd, gx_prog_info* out) {
  ProgObj* p = get_prog(rt, prog_fd);
  if (!p || !out) return -EINVAL;
  fill_info(p->v, (uint32_t)p->hook, p->n_insns, out);
  return 0;
}

int gx_run_batch(gx_rt* rt, int prog_fd, const void* d_events, uint64_t n_events, uint32_t record_size,
                 uint32_t* d_rc, void* stream) {
  ProgObj* p = get_prog(rt, prog_fd);
  if (!p) return -EINVAL;
  if (record_size != p->record_size || p->hook == HOOK_SCHED) return -EINVAL;
  if (n_events == 0) return 0;
  if (!d_events) return -EINVAL;
  if (n_events >= (1ull << 32)) return -E2BIG;
  DevGuard g(rt->dev);
  // a run's launches stay together between the snapshot daemon's copies
  std::unique_lock<std::mutex> lk(rt->enq_mu, std::defer_lock);
  if (rt->snap) lk.lock();
  return run_one(rt, p, d_events, n_events, d_rc, (hipStream_t)stream, knobs_of(p));
}

}  // extern "C"

namespace {

RunArgs make_args(gx_rt* rt, ProgObj* p, const void* d_events, uint64_t n_events, uint32_t* d_rc) {
  RunArgs A{};
  A.uops = p->d_uops;
  A.events = (const uint8_t*)d_events;
  A.rc = d_rc;
  A.n_events = n_events;
  A.record_size = p->record_size;
  A.stack_bytes = p->v.stack_bytes;
  A.stream_off = p->stream_off;
  A.stream_size = p->stream_size;
  A.err = rt->d_err;
  A.guards = p->d_guards;
  A.maptab = p->d_maptab;
  A.leader = p->hook == HOOK_WAVE_MEM ? 1u : 0u;
  A.simt = p->hook == HOOK_SIMT_MEM ? 1u : 0u;
  A.checked = env_int("GX_CHECKED", 0) ? 1u : 0u;
  A.epoch = ++rt->epoch;
  uint64_t per_event = 64 * (p->v.max_insns + 1) + 64;
  A.step_limit = p->v.event_parallel ? per_event : per_event * n_events;
  return A;
}

// ---------------------------------------------------------------------------
// Hooks inside application kernels: the instrumented vector add and the
// block scheduler's workers (section 5.3).

// The module of a compiled program whose kernel is gx_j_app_vadd (kind 1)
// or gx_j_sched (kind 2), built on first use and shared through the source
// cache; *fr: its reduce kernel (null: none).
int jit_app_module(gx_rt* rt, ProgObj* p, int kind, hipModule_t* mod, hipFunction_t* f, hipFunction_t* fr,
                   JitInfo* info_out) {
  std::vector<std::pair<uint64_t, MapDev>> maps;
  for (int fd : p->fds) {
    MapObj* m = get_map(rt, fd);
    if (!m) return -EINVAL;
    maps.push_back({(uint64_t)(uintptr_t)m->d_desc, m->h});
  }
  JitProg jp{&p->uops, p->v.stack_bytes, &maps, &p->v.mem_map, &p->v.ld_map, p->v.event_parallel,
             p->hook == HOOK_WAVE_MEM, p->hook == HOOK_SIMT_MEM};
  jp.kernel = kind;
  jp.max_insns = p->v.max_insns;
  JitInfo info;
  const std::string src = jit_source(jp, &info);
  auto adopt = [&](const gx_rt::JitMod& jm) {
    *mod = jm.mod;
    *f = jm.fe;
    *fr = jm.fr;
    *info_out = jm.info;
  };
  {
    std::lock_guard<std::mutex> lk(rt->jit_mu);
    auto it = rt->jit_cache.find(src);
    if (it != rt->jit_cache.end()) {
      adopt(it->second);
      return 0;
    }
  }
  std::vector<char> code;
  std::string lg;
  int r = jit_compile(src, &code, &lg);
  if (r) return r;
  DevGuard g(rt->dev);
  gx_rt::JitMod jm;
  jm.info = info;
  if (hipModuleLoadData(&jm.mod, code.data()) != hipSuccess) return -EIO;
  if (hipModuleGetFunction(&jm.fe, jm.mod, kind == 1 ? "gx_j_app_vadd" : "gx_j_sched") != hipSuccess ||
      (kind == 1 && info.spill_block_bytes && hipModuleGetFunction(&jm.fr, jm.mod, "gx_j_reduce") != hipSuccess)) {
    (void)hipModuleUnload(jm.mod);
    return -EIO;
  }
  std::lock_guard<std::mutex> lk(rt->jit_mu);
  auto ins = rt->jit_cache.emplace(src, jm);
  if (!ins.second) (void)hipModuleUnload(jm.mod);  // compiled concurrently by another call
  adopt(ins.first->second);
  return 0;
}

// Launch a program's compiled application kernel (nb blocks of ``nw``
// waves, RunArgs then ``x`` as arguments), then its reduce kernel when the
// program's LDS caches spill.
template <class X>
int launch_jit_app(gx_rt* rt, const ProgObj* p, RunArgs A, X x, uint32_t nb, uint32_t nw, hipStream_t s) {
  Exec* Xp = exec_for(rt, s);
  if (!Xp) return -ENOMEM;
  Exec& E = *Xp;
  uint8_t* sp = nullptr;
  if (p->jspill && p->jf_app_red) {
    int r = ensure_spill(E, (size_t)nb * p->jspill);
    if (r) return r;
    if (E.spill_used) (void)hipStreamWaitEvent(s, E.spill_ev, 0);
    sp = E.d_spill;
  }
  A.spill = sp;
  void* args[] = {&A, &x};
  hipError_t e = hipModuleLaunchKernel(p->jf_app, nb, 1, 1, 64 * nw, 1, 1, 0, s, args, nullptr);
  if (e == hipSuccess && sp) {
    void* rargs[] = {&A, &nb};
    e = hipModuleLaunchKernel(p->jf_app_red, p->jred_blocks, 1, 1, 256, 1, 1, 0, s, rargs, nullptr);
    (void)hipEventRecord(E.spill_ev, s);
    E.spill_used = true;
  }
  return e == hipSuccess ? 0 : to_errno(e);
}

uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// Layout of a stream-sequential run's workspace in one region: counts,
// sums, order, queue-ordered records, each 256-byte aligned.  Returns the
// bytes needed.
uint64_t seq_layout(uint64_t n_events, uint32_t lbits, uint64_t off[4]) {
  const uint64_t tile = part_tile(n_events);
  const uint64_t nt = (n_events + tile - 1) / tile;
  const uint64_t m = ((uint64_t)1 << lbits) * nt;
  const uint64_t sz[4] = {m * 4, ((m + 4095) / 4096 + 1) * 4, n_events * 4, n_events * kSortedStride};
  uint64_t at = 0;
  for (int i = 0; i < 4; i++) {
    off[i] = at;
    at += (sz[i] + 255) & ~255ull;
  }
  return at;
}

// One plain run that allocates nothing: the stream partition (and a
// compiled event-parallel run's cache spill, when it fits) use the device's
// scratch array instead of the runtime's workspace; no events, streams or
// staging are created.  Every call on the device shares the array, so
// calls that overlap on the device race.
int run_noalloc(gx_rt* rt, ProgObj* p, const void* d_events, uint64_t n_events, uint32_t* d_rc, hipStream_t s,
                const Knobs& k) {
  RunArgs A = make_args(rt, p, d_events, n_events, d_rc);
  hipError_t e;
  if (p->v.event_parallel) {
    if (p->jf_ep) {
      // a spill area beyond the array: the caches flush to the map directly
      const uint64_t need = jit_spill_bytes(p, n_events, k.blocks);
      uint8_t* sp = need && need <= rt->scratch_bytes ? rt->d_scratch : nullptr;
      e = launch_jit(p, A, 0, 0, 0, 0, k.blocks, sp, s);
      rt->stats.launches += sp ? 2 : 1;
    } else {
      e = launch_interp_ep(rt, p, A, s);
      rt->stats.launches += 1;
    }
  } else {
    uint64_t off[4];
    if (seq_layout(n_events, k.qbits, off) > rt->scratch_bytes) return -E2BIG;
    const uint64_t tile = part_tile(n_events);
    const uint32_t nt = (uint32_t)((n_events + tile - 1) / tile);
    uint32_t* counts = (uint32_t*)(rt->d_scratch + off[0]);
    uint32_t* sums = (uint32_t*)(rt->d_scratch + off[1]);
    uint32_t* order = (uint32_t*)(rt->d_scratch + off[2]);
    uint8_t* sorted = p->jf_uni && k.lanes == 1 ? nullptr : rt->d_scratch + off[3];
    e = launch_partition(A, k.qbits, (uint32_t)tile, nt, counts, sums, order, sorted, s);
    if (e == hipSuccess) {
      A.order = order;
      A.sorted = sorted;
      A.qstart = counts;
      A.n_queues = 1u << k.qbits;
      e = p->jf_seq ? launch_jit(p, A, 1, k.lanes, nt, (uint32_t)n_events, 0, nullptr, s)
                    : launch_stream_seq(A, k.lanes, nt, s);
    }
    rt->stats.launches += 6;
  }
  if (e != hipSuccess) return to_errno(e);
  // drains and map reads wait for this event
  if (hipEventRecord(rt->noalloc_ev, s) != hipSuccess) return -EIO;
  rt->noalloc_used = true;
  rt->stats.events += n_events;
  return 0;
}

bool shares_map(ProgObj* a, ProgObj* b, const std::vector<MapObj>& maps) {
  for (int x : a->fds)
    for (int y : b->fds)
      if (x == y && maps[x].h.type != MAP_RINGBUF) return true;
  return false;
}

// One phase: runs that share no map, so running them concurrently gives the
// result of running them in order.  One combined partition of the
// stream-sequential runs, then one persistent interpreter launch over the
// runs of interpreted programs and, side by side with it, one launch per
// run of a compiled program.
int run_phase(gx_rt* rt, const gx_batch* d, uint32_t n, hipStream_t s) {
  Exec* Xp = exec_for(rt, s);
  if (!Xp) return -ENOMEM;
  Exec& X = *Xp;
  std::vector<BatchDev> B;
  std::vector<PartJob> J;
  std::vector<uint2> tiles, items;
  std::vector<std::pair<uint64_t, uint32_t>> order_by_cost;  // (cost, batch)
  std::vector<const ProgObj*> bprog;  // program of each run
  uint64_t counts_total = 0, order_total = 0;
  uint32_t stack_max = 0, max_lbits = 0;
  for (uint32_t i = 0; i < n; i++) {
    if (d[i].n_events == 0) continue;
    ProgObj* p = get_prog(rt, d[i].prog_fd);
    const Knobs kn = knobs_of(p);
    const uint32_t lanes = kn.lanes, qbits = kn.qbits;
    RunArgs A = make_args(rt, p, d[i].d_events, d[i].n_events, d[i].d_rc);
    BatchDev bd{};
    stack_max = std::max(stack_max, p->v.stack_bytes);
    uint32_t nchunks;
    if (p->v.event_parallel) {
      bd.mode = 0;
      bd.lanes = 64;
      nchunks = (uint32_t)((d[i].n_events + 63) / 64);
    } else {
      uint32_t lbits = qbits;
      uint32_t L = 1u << lbits;
      uint64_t tile = part_tile(d[i].n_events);
      uint32_t nt = (uint32_t)((d[i].n_events + tile - 1) / tile);
      PartJob pj{A.events, A.n_events, A.record_size, A.stream_off, lbits, (uint32_t)tile, nt, 0, counts_total};
      for (uint32_t t = 0; t < nt; t++) tiles.push_back(make_uint2((uint32_t)J.size(), t));
      J.push_back(pj);
      max_lbits = std::max(max_lbits, lbits);
      A.qstart = nullptr;  // patched below once the workspace exists
      A.n_queues = L;
      bd.mode = 1;
      bd.lanes = lanes;
      bd.qstride = nt;
      bd.qend_last = (uint32_t)(order_total + d[i].n_events);
      bd.A.pad2 = 0;
      // remember where this run's counts start (patched into qstart)
      A.pad2 = (uint32_t)J.size();  // 1 + job index
      counts_total += (uint64_t)L * nt;
      order_total += d[i].n_events;
      nchunks = (L + lanes - 1) / lanes;
    }
    bd.A = A;
    uint64_t cost = (uint64_t)(p->v.max_insns + 1) * (p->v.event_parallel ? 64 : (d[i].n_events / 64 + 1));
    order_by_cost.push_back({cost, (uint32_t)B.size()});
    B.push_back(bd);
    bprog.push_back(p);
    (void)nchunks;
  }
  if (B.empty()) return 0;
  if (order_total >= (1ull << 32) || counts_total >= (1ull << 32)) return -E2BIG;
  int r = ensure_ws(X, counts_total + 1, (counts_total + 4095) / 4096 + 1, order_total + 1);
  if (r) return r;
  for (auto& bd : B)
    if (bd.mode == 1) {
      const PartJob& pj = J[bd.A.pad2 - 1];
      bd.A.qstart = X.d_counts + pj.cbase;
      bd.A.order = X.d_order;
      bd.A.sorted = X.d_sorted;
      bd.A.pad2 = 0;
    }
  // items, largest runs first
  std::stable_sort(order_by_cost.begin(), order_by_cost.end(),
                   [](const std::pair<uint64_t, uint32_t>& a, const std::pair<uint64_t, uint32_t>& b) {
                     return a.first > b.first;
                   });
  // runs of compiled programs get their own kernels (below); the rest are
  // work items of the persistent interpreter
  std::vector<uint32_t> jit_runs;
  std::map<int, std::vector<uint2>> set_items;  // set id -> its work items
  for (auto& oc : order_by_cost) {
    BatchDev& bd = B[oc.second];
    const ProgObj* bp = bprog[oc.second];
    if (bp->set_id >= 0 && (set_items.count(bp->set_id) || set_items.size() < kMaxSetsPerPhase)) {
      bd.slot = bp->set_slot;
      if (bd.mode == 1) bd.lanes = 1;  // a set runs each queue on wave-uniform values
      uint32_t nchunks = bd.mode == 0 ? (uint32_t)((bd.A.n_events + 63) / 64) : (bd.A.n_queues + bd.lanes - 1) / bd.lanes;
      auto& v = set_items[bp->set_id];
      for (uint32_t c = 0; c < nchunks; c++) v.push_back(make_uint2(oc.second, c));
      continue;
    }
    if (bp->jmod) {
      jit_runs.push_back(oc.second);
      continue;
    }
    uint32_t nchunks = bd.mode == 0 ? (uint32_t)((bd.A.n_events + 63) / 64) : (bd.A.n_queues + bd.lanes - 1) / bd.lanes;
    for (uint32_t c = 0; c < nchunks; c++) items.push_back(make_uint2(oc.second, c));
  }
  // spill areas of the compiled event-parallel runs with LDS caches: one
  // each, as they run side by side
  std::vector<uint64_t> spill_at(B.size(), UINT64_MAX);
  uint64_t spill_total = 0;
  for (uint32_t b : jit_runs)
    if (B[b].mode == 0) {
      const uint64_t need = jit_spill_bytes(bprog[b], B[b].A.n_events, knobs_of(bprog[b]).blocks);
      if (!need) continue;
      spill_at[b] = spill_total;
      spill_total += (need + 255) & ~255ull;
    }
  if (spill_total) {
    int rs = ensure_spill(X, spill_total);
    if (rs) return rs;
  }
  // pack the tables: batches | items | jobs | tiles (each 64-byte aligned)
  auto al = [](size_t x) { return (x + 63) & ~(size_t)63; };
  size_t ob = 0, oi = al(ob + B.size() * sizeof(BatchDev)), os_ = al(oi + items.size() * sizeof(uint2));
  std::vector<std::pair<int, size_t>> set_off;  // (set id, offset of its items)
  for (auto& si : set_items) {
    set_off.push_back({si.first, os_});
    os_ = al(os_ + si.second.size() * sizeof(uint2));
  }
  size_t oj = os_, ot = al(oj + J.size() * sizeof(PartJob)), total = al(ot + tiles.size() * sizeof(uint2));
  // a staging slot whose previous copy has long completed; a capture takes
  // a fresh slot per phase, which the graph then owns
  size_t k;
  if (X.per_phase) {
    k = X.stage_cursor++;
    if (k >= X.stage.size()) X.stage.emplace_back();
  } else {
    if (X.stage.size() < (size_t)kStageRing) X.stage.resize(kStageRing);
    k = X.stage_next++ % kStageRing;
  }
  Stage& st = X.stage[k];
  if (!st.ev && hipEventCreateWithFlags(&st.ev, hipEventDisableTiming) != hipSuccess) return -ENOMEM;
  if (st.used && hipEventSynchronize(st.ev) != hipSuccess) return -EIO;
  if (st.cap < total) {
    if (st.h) (void)hipHostFree(st.h);
    if (st.d) (void)hipFree(st.d);
    st.h = nullptr;
    st.d = nullptr;
    st.cap = 0;
    size_t cap = std::max<size_t>(total, 1 << 16);
    if (hipHostMalloc((void**)&st.h, cap, hipHostMallocDefault) != hipSuccess) return -ENOMEM;
    if (hipMalloc((void**)&st.d, cap) != hipSuccess) return -ENOMEM;
    st.cap = cap;
  }
  uint8_t* h_stage = st.h;
  uint8_t* d_tables = st.d;
  if (X.ws_used) (void)hipStreamWaitEvent(s, X.ws_event, 0);
  std::memcpy(h_stage + ob, B.data(), B.size() * sizeof(BatchDev));
  std::memcpy(h_stage + oi, items.data(), items.size() * sizeof(uint2));
  for (auto& so : set_off) {
    const auto& v = set_items[so.first];
    std::memcpy(h_stage + so.second, v.data(), v.size() * sizeof(uint2));
  }
  if (!J.empty()) std::memcpy(h_stage + oj, J.data(), J.size() * sizeof(PartJob));
  if (!tiles.empty()) std::memcpy(h_stage + ot, tiles.data(), tiles.size() * sizeof(uint2));
  if (hipMemcpyAsync(d_tables, h_stage, total, hipMemcpyHostToDevice, s) != hipSuccess) return -EIO;
  (void)hipEventRecord(st.ev, s);
  st.used = !X.per_phase;
  hipError_t e = hipSuccess;
  if (!J.empty())
    e = launch_partition_jobs((const PartJob*)(d_tables + oj), (const uint2*)(d_tables + ot), (uint32_t)tiles.size(),
                              max_lbits, counts_total, X.d_counts, X.d_sums, X.d_order, X.d_sorted, s);
  std::pair<hipEvent_t, hipEvent_t> pe{nullptr, nullptr};
  if (rt->profile) pe = prof_pair(rt);
  if (pe.first) (void)hipEventRecord(pe.first, s);
  // compiled runs: their own kernels, side by side on the side streams,
  // after the partition; joined back into s
  int used_side = 0;
  size_t x = 0;  // launches handed to side streams so far
  auto side = [&]() {
    hipStream_t ss = X.side[x % kExecSide];
    if ((int)x < kExecSide) {
      (void)hipStreamWaitEvent(ss, X.fork_ev, 0);
      used_side++;
    }
    x++;
    return ss;
  };
  if (spill_total && X.spill_used) (void)hipStreamWaitEvent(s, X.spill_ev, 0);
  if (e == hipSuccess && (!jit_runs.empty() || !set_off.empty())) (void)hipEventRecord(X.fork_ev, s);
  // program sets: one persistent launch each, with a counter of its own
  for (size_t k = 0; k < set_off.size() && e == hipSuccess; k++) {
    hipStream_t ss = side();
    const auto& v = set_items[set_off[k].first];
    const BatchDev* db = (const BatchDev*)(d_tables + ob);
    const uint2* di = (const uint2*)(d_tables + set_off[k].second);
    uint32_t ni = (uint32_t)v.size();
    uint32_t* next = X.d_next + 1 + k;
    // as many waves as the device holds at once: the items are chains of
    // dependent memory accesses, so throughput comes from concurrency
    const gx_rt::JitSet& js = rt->sets[set_off[k].first];
    uint32_t per_cu = js.blocks_per_cu ? js.blocks_per_cu : 8;
    per_cu = (uint32_t)std::min(32, std::max(1, env_int("GX_BATCH_WAVES_PER_CU", (int)per_cu)));
    uint32_t waves = (uint32_t)std::min<size_t>(v.size(), (size_t)rt->n_cu * per_cu);
    e = launch_zero(next, 1, ss);
    void* args[] = {&db, &di, &ni, &next};
    if (e == hipSuccess)
      e = hipModuleLaunchKernel(rt->sets[set_off[k].first].f, waves, 1, 1, 64, 1, 1, 0, ss, args, nullptr);
  }
  for (size_t y = 0; y < jit_runs.size() && e == hipSuccess; y++) {
    const uint32_t b = jit_runs[y];
    e = launch_jit(bprog[b], B[b].A, B[b].mode, B[b].lanes, B[b].qstride, B[b].qend_last, knobs_of(bprog[b]).blocks,
                   spill_at[b] != UINT64_MAX ? X.d_spill + spill_at[b] : nullptr, side());
  }
  if (e == hipSuccess && !items.empty()) {
    uint32_t per_cu = rt->batch_per_cu ? rt->batch_per_cu
                                       : (uint32_t)std::min(32, std::max(1, env_int("GX_BATCH_WAVES_PER_CU", 8)));
    uint32_t waves = (uint32_t)std::min<size_t>(items.size(), 256 * per_cu);
    e = launch_batched((const BatchDev*)(d_tables + ob), (const uint2*)(d_tables + oi), (uint32_t)items.size(),
                       X.d_next, waves, stack_max, s);
  }
  for (int x = 0; x < used_side; x++) {
    (void)hipEventRecord(X.join_ev[x], X.side[x]);
    (void)hipStreamWaitEvent(s, X.join_ev[x], 0);
  }
  if (pe.second) (void)hipEventRecord(pe.second, s);
  if (pe.first) rt->prof_pending.push_back(pe);
  (void)hipEventRecord(X.ws_event, s);
  X.ws_used = true;
  if (spill_total) {
    (void)hipEventRecord(X.spill_ev, s);
    X.spill_used = true;
  }
  if (e != hipSuccess) return to_errno(e);
  if (X.capturing) return 0;  // a graph's launches are counted when it is launched
  size_t reduces = 0;
  for (uint64_t at : spill_at) reduces += at != UINT64_MAX;
  rt->stats.launches += (J.empty() ? 0 : 5) + (items.empty() ? 0 : 2) + jit_runs.size() + reduces + 2 * set_off.size();
  for (auto& bd : B) rt->stats.events += bd.A.n_events;
  note_stream(rt, s);
  return 0;
}

// The phases of a batch, one after another on s (validated descriptors).
int run_batches_impl(gx_rt* rt, const gx_batch* descs, uint32_t n, hipStream_t s) {
  // split into phases of runs that share no map (their order then cannot
  // matter); phases run one after another on the stream
  uint32_t a = 0;
  while (a < n) {
    uint32_t b = a + 1;
    while (b < n) {
      bool clash = false;
      for (uint32_t k = a; k < b && !clash; k++)
        clash = shares_map(get_prog(rt, descs[k].prog_fd), get_prog(rt, descs[b].prog_fd), rt->maps);
      if (clash) break;
      b++;
    }
    int r = run_phase(rt, descs + a, b - a, s);
    if (r) return r;
    a = b;
  }
  return 0;
}

int check_batches(gx_rt* rt, const gx_batch* descs, uint32_t n) {
  if (!rt || (!descs && n)) return -EINVAL;
  for (uint32_t i = 0; i < n; i++) {
    ProgObj* p = get_prog(rt, descs[i].prog_fd);
    if (!p || descs[i].record_size != p->record_size || p->hook == HOOK_SCHED ||
        (descs[i].n_events && !descs[i].d_events))
      return -EINVAL;
    if (descs[i].n_events >= (1ull << 32)) return -E2BIG;
  }
  return 0;
}

}  // namespace

extern "C" {

int gx_run_batches(gx_rt* rt, const gx_batch* descs, uint32_t n, void* stream) {
  int r = check_batches(rt, descs, n);
  if (r) return r;
  DevGuard g(rt->dev);
  if (drain_barrier(rt)) return -EIO;  // started drains finish copying first
  std::unique_lock<std::mutex> lk(rt->enq_mu, std::defer_lock);
  if (rt->snap) lk.lock();
  return run_batches_impl(rt, descs, n, (hipStream_t)stream);
}

int gx_run_batch_noalloc(gx_rt* rt, int prog_fd, const void* d_events, uint64_t n_events, uint32_t record_size,
                         uint32_t* d_rc, void* stream) {
  ProgObj* p = get_prog(rt, prog_fd);
  if (!p) return -EINVAL;
  if (record_size != p->record_size || p->hook == HOOK_SCHED) return -EINVAL;
  if (n_events == 0) return 0;
  if (!d_events) return -EINVAL;
  if (n_events >= (1ull << 32)) return -E2BIG;
  DevGuard g(rt->dev);
  if (drain_barrier(rt)) return -EIO;  // started drains finish copying first
  std::unique_lock<std::mutex> lk(rt->enq_mu, std::defer_lock);
  if (rt->snap) lk.lock();
  return run_noalloc(rt, p, d_events, n_events, d_rc, (hipStream_t)stream, knobs_of(p));
}

int gx_autotune_batches(gx_rt* rt, const gx_batch* descs, uint32_t n, void* stream, gx_tune* out) {
  int r = check_batches(rt, descs, n);
  if (r) return r;
  if (!n) return -EINVAL;
  DevGuard g(rt->dev);
  if (drain_barrier(rt)) return -EIO;  // started drains finish copying first
  hipStream_t s = (hipStream_t)stream;
  const uint32_t def = (uint32_t)std::min(32, std::max(1, env_int("GX_BATCH_WAVES_PER_CU", 8)));
  std::vector<uint32_t> cand{def};
  for (uint32_t w : {2u, 4u, 8u, 16u, 32u})
    if (w != def) cand.push_back(w);
  std::vector<int> fds;
  for (uint32_t i = 0; i < n; i++)
    for (int fd : get_prog(rt, descs[i].prog_fd)->fds) fds.push_back(fd);
  if (wait_all(rt)) return -EIO;
  MapSnapshot snap;
  if (snap.take(rt, fds, s)) return -ENOMEM;
  const bool prof = rt->profile;
  const gx_stats st = rt->stats;
  const uint32_t saved = rt->batch_per_cu;
  rt->profile = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) r = -ENOMEM;
  double best = 1e300, def_ms = 0;
  uint32_t bestw = def;
  if (!r) {  // one untimed run first
    snap.restore(s);
    rt->batch_per_cu = def;
    r = run_batches_impl(rt, descs, n, s);
  }
  for (size_t c = 0; c < cand.size() && !r; c++) {
    snap.restore(s);
    rt->batch_per_cu = cand[c];
    (void)hipEventRecord(e0, s);
    r = run_batches_impl(rt, descs, n, s);
    (void)hipEventRecord(e1, s);
    if (r) break;
    float ms = 0;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      r = -EIO;
      break;
    }
    if (c == 0) def_ms = ms;
    if (c == 0 ? ms < best : ms < best && ms < 0.97 * def_ms) {
      best = ms;
      bestw = cand[c];
    }
  }
  snap.restore(s);
  (void)hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  rt->profile = prof;
  rt->stats = st;
  rt->batch_per_cu = r ? saved : bestw;
  if (r) return r;
  if (out) {
    out->lanes = 0;
    out->qbits = 0;
    out->blocks = bestw;
    out->trials = (uint32_t)cand.size();
    out->best_ms = best;
    out->default_ms = def_ms;
  }
  return 0;
}

struct gx_graph {
  gx_rt* rt = nullptr;
  Exec ex;  // the graph's own workspace, staging and side streams
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t events = 0;
  uint32_t phases = 0;
};

int gx_graph_create(gx_rt* rt, const gx_batch* descs, uint32_t n, gx_graph** out) {
  if (!out) return -EINVAL;
  *out = nullptr;
  int r = check_batches(rt, descs, n);
  if (r) return r;
  DevGuard g(rt->dev);
  gx_graph* G = new (std::nothrow) gx_graph();
  if (!G) return -ENOMEM;
  G->rt = rt;
  auto fail = [&](int code) {
    if (G->exec) (void)hipGraphExecDestroy(G->exec);
    if (G->graph) (void)hipGraphDestroy(G->graph);
    if (G->cs) (void)hipStreamDestroy(G->cs);
    exec_free(G->ex);
    delete G;
    return code;
  };
  if (exec_init(G->ex) || hipStreamCreateWithFlags(&G->cs, hipStreamNonBlocking) != hipSuccess) return fail(-ENOMEM);
  for (uint32_t i = 0; i < n; i++) G->events += descs[i].n_events;
  // the batch runs once for real to size the graph's workspace and tables
  // (nothing may be allocated while capturing); the maps it touches are
  // saved first and put back after
  std::vector<int> fds;
  for (uint32_t i = 0; i < n; i++)
    for (int fd : get_prog(rt, descs[i].prog_fd)->fds) fds.push_back(fd);
  if (wait_all(rt)) return fail(-EIO);
  MapSnapshot snap;
  if (snap.take(rt, fds, G->cs)) return fail(-ENOMEM);
  const bool prof = rt->profile;
  const gx_stats st = rt->stats;
  rt->profile = false;
  rt->cap_ex = &G->ex;
  G->ex.per_phase = true;
  G->ex.stage_cursor = 0;
  r = run_batches_impl(rt, descs, n, G->cs);
  if (!r) {
    snap.restore(G->cs);
    if (hipStreamSynchronize(G->cs) != hipSuccess) r = -EIO;
  }
  if (!r) {
    G->ex.capturing = true;
    // events recorded outside the capture may not be waited on inside it
    G->ex.ws_used = false;
    G->ex.spill_used = false;
    G->ex.stage_cursor = 0;
    if (hipStreamBeginCapture(G->cs, hipStreamCaptureModeRelaxed) != hipSuccess) {
      r = -EIO;
    } else {
      r = run_batches_impl(rt, descs, n, G->cs);
      if (hipStreamEndCapture(G->cs, &G->graph) != hipSuccess && !r) r = -EIO;
    }
    G->ex.capturing = false;
    G->phases = (uint32_t)G->ex.stage_cursor;
  }
  rt->cap_ex = nullptr;
  rt->profile = prof;
  rt->stats = st;
  if (r) return fail(r);
  if (hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0) != hipSuccess) return fail(-EIO);
  *out = G;
  return 0;
}

int gx_graph_launch(gx_graph* G, void* stream) {
  if (!G) return -EINVAL;
  gx_rt* rt = G->rt;
  DevGuard g(rt->dev);
  if (drain_barrier(rt)) return -EIO;  // started drains finish copying first
  hipStream_t s = (hipStream_t)stream;
  std::unique_lock<std::mutex> lk(rt->enq_mu, std::defer_lock);
  if (rt->snap) lk.lock();
  if (hipGraphLaunch(G->exec, s) != hipSuccess) return -EIO;
  rt->stats.launches += 1;
  rt->stats.events += G->events;
  note_stream(rt, s);
  return 0;
}

void gx_graph_destroy(gx_graph* G) {
  if (!G) return;
  DevGuard g(G->rt->dev);
  (void)hipDeviceSynchronize();
  if (G->exec) (void)hipGraphExecDestroy(G->exec);
  if (G->graph) (void)hipGraphDestroy(G->graph);
  if (G->cs) (void)hipStreamDestroy(G->cs);
  exec_free(G->ex);
  delete G;
}

int64_t gx_drain_ringbuf(gx_rt* rt, int ring_fd, void* host_buf, uint64_t buf_bytes, uint64_t* n_records) {
  MapObj* m = get_map(rt, ring_fd);
  if (!m || m->h.type != MAP_RINGBUF || (!host_buf && buf_bytes)) return -EINVAL;
  if (m->drain_pending) return -EBUSY;  // a started drain is not finished
  DevGuard g(rt->dev);
  if (wait_all(rt)) return -EIO;
  uint64_t ctrl[kRingCount + 2 * kRingCountSlots];
  if (hipMemcpy(ctrl, m->h.ctrl, sizeof ctrl, hipMemcpyDeviceToHost) != hipSuccess) return -EIO;
  uint64_t head = ctrl[0], tail = ctrl[1], cap = (uint64_t)m->h.slot_mask + 1;
  // a reservation that overflowed ended the committed data at its start
  const bool cut = ctrl[3] != 0;
  if (cut && ~ctrl[3] < head) head = ~ctrl[3];
  if (n_records) *n_records = 0;
  // Every byte of [tail, head) has been written: reservations are
  // contiguous and every one is filled (records, or a discard record over a
  // chunk's unused rest) before its launch ends, and no launch is running.
  const uint64_t avail = head - tail;
  uint64_t pos = 0, out = 0, nrec = 0;
  if (avail) {
    if (m->pin_cap < avail) {
      if (m->h_pin) (void)hipHostFree(m->h_pin);
      m->h_pin = nullptr;
      m->pin_cap = 0;
      if (hipHostMalloc((void**)&m->h_pin, avail, hipHostMallocDefault) != hipSuccess) return -ENOMEM;
      m->pin_cap = avail;
    }
    uint8_t* buf = m->h_pin;
    const uint64_t t0 = tail & (cap - 1);
    const uint64_t first = std::min(avail, cap - t0);
    if (hipMemcpy(buf, m->h.data + t0, first, hipMemcpyDeviceToHost) != hipSuccess) return -EIO;
    if (first < avail && hipMemcpy(buf + first, m->h.data, avail - first, hipMemcpyDeviceToHost) != hipSuccess)
      return -EIO;
    // records between discards are copied as one run
    uint64_t run = 0;  // start of the current run of kept records
    auto flush = [&](uint64_t end) {
      if (end > run) std::memcpy((uint8_t*)host_buf + out, buf + run, end - run);
      out += end - run;
    };
    while (pos + 8 <= avail) {
      uint32_t len, flags;
      std::memcpy(&len, buf + pos, 4);
      std::memcpy(&flags, buf + pos + 4, 4);
      if (len == 0 && flags == 0) break;  // not written (cannot happen after a completed launch)
      const uint64_t need = 8 + ((len + 7ull) & ~7ull);
      if (pos + need > avail) break;
      if (flags & RING_DISCARD) {
        flush(pos);
        run = pos + need;
      } else {
        if (out + (pos - run) + need > buf_bytes) break;
        nrec++;
      }
      pos += need;
    }
    flush(pos);
  }
  if (pos || cut) {
    // publish the new tail (and, after an overflow, the cut-back head); the
    // device's counts of discards and records cover what remains only when
    // nothing remains
    uint64_t nc[kRingCount + 2 * kRingCountSlots] = {head, tail + pos, ctrl[2], 0};
    nc[kRingUnknown] = pos == avail ? 0 : 1;
    if (hipMemcpy(m->h.ctrl, nc, sizeof nc, hipMemcpyHostToDevice) != hipSuccess) return -EIO;
  }
  rt->stats.bytes_drained += out;
  if (n_records) *n_records = nrec;
  return (int64_t)out;
}

int64_t gx_drain_ringbuf_view(gx_rt* rt, int ring_fd, const void** view, uint64_t* view_bytes,
                              uint64_t* n_records) {
  MapObj* m = get_map(rt, ring_fd);
  if (!m || m->h.type != MAP_RINGBUF || !view || !view_bytes) return -EINVAL;
  if (m->drain_pending) return -EBUSY;  // a started drain is not finished
  DevGuard g(rt->dev);
  if (wait_all(rt)) return -EIO;
  uint64_t ctrl[kRingCount + 2 * kRingCountSlots];
  if (hipMemcpy(ctrl, m->h.ctrl, sizeof ctrl, hipMemcpyDeviceToHost) != hipSuccess) return -EIO;
  uint64_t head = ctrl[0], tail = ctrl[1], cap = (uint64_t)m->h.slot_mask + 1;
  const bool cut = ctrl[3] != 0;
  if (cut && ~ctrl[3] < head) head = ~ctrl[3];
  *view = nullptr;
  *view_bytes = 0;
  if (n_records) *n_records = 0;
  const uint64_t avail = head - tail;
  uint64_t pos = 0, kept = 0, nrec = 0;
  if (avail) {
    if (m->pin_cap < avail) {
      if (m->h_pin) (void)hipHostFree(m->h_pin);
      m->h_pin = nullptr;
      m->pin_cap = 0;
      if (hipHostMalloc((void**)&m->h_pin, avail, hipHostMallocDefault) != hipSuccess) return -ENOMEM;
      m->pin_cap = avail;
    }
    uint8_t* buf = m->h_pin;
    const uint64_t t0 = tail & (cap - 1);
    const uint64_t first = std::min(avail, cap - t0);
    if (hipMemcpy(buf, m->h.data + t0, first, hipMemcpyDeviceToHost) != hipSuccess) return -EIO;
    if (first < avail && hipMemcpy(buf + first, m->h.data, avail - first, hipMemcpyDeviceToHost) != hipSuccess)
      return -EIO;
    uint64_t disc = 0, recs = 0;
    for (uint32_t k = 0; k < kRingCountSlots; k++) {
      disc += ctrl[kRingCount + 2 * k];
      recs += ctrl[kRingCount + 2 * k + 1];
    }
    if (!cut && !ctrl[kRingUnknown] && disc <= avail) {
      // every byte of the range is a record or a discard record (no launch
      // is running), and the device counted both: no walk over the range
      pos = avail;
      kept = avail - disc;
      nrec = recs;
    } else {
      while (pos + 8 <= avail) {
        uint32_t len, flags;
        std::memcpy(&len, buf + pos, 4);
        std::memcpy(&flags, buf + pos + 4, 4);
        if (len == 0 && flags == 0) break;
        const uint64_t need = 8 + ((len + 7ull) & ~7ull);
        if (pos + need > avail) break;
        if (!(flags & RING_DISCARD)) {
          kept += need;
          nrec++;
        }
        pos += need;
      }
    }
    *view = buf;
    *view_bytes = pos;
  }
  if (pos || cut) {
    uint64_t nc[kRingCount + 2 * kRingCountSlots] = {head, tail + pos, ctrl[2], 0};
    nc[kRingUnknown] = pos == avail ? 0 : 1;
    if (hipMemcpy(m->h.ctrl, nc, sizeof nc, hipMemcpyHostToDevice) != hipSuccess) return -EIO;
  }
  rt->stats.bytes_drained += kept;
  if (n_records) *n_records = nrec;
  return (int64_t)kept;
}

int gx_drain_ringbuf_start(gx_rt* rt, int ring_fd) {
  MapObj* m = get_map(rt, ring_fd);
  if (!m || m->h.type != MAP_RINGBUF) return -EINVAL;
  if (m->drain_pending) return -EBUSY;
  DevGuard g(rt->dev);
  if (wait_all(rt)) return -EIO;
  uint64_t ctrl[kRingCount + 2 * kRingCountSlots];
  if (hipMemcpy(ctrl, m->h.ctrl, sizeof ctrl, hipMemcpyDeviceToHost) != hipSuccess) return -EIO;
  const uint64_t head = ctrl[0], tail = ctrl[1], cap = (uint64_t)m->h.slot_mask + 1, avail = head - tail;
  uint64_t disc = 0, recs = 0;
  for (uint32_t k = 0; k < kRingCountSlots; k++) {
    disc += ctrl[kRingCount + 2 * k];
    recs += ctrl[kRingCount + 2 * k + 1];
  }
  if (ctrl[3] != 0 || ctrl[kRingUnknown] || disc > avail || avail == 0) {
    // a range the host must walk, a head to cut back, or nothing: drained
    // here and now, as gx_drain_ringbuf_view does
    const void* v = nullptr;
    uint64_t vb = 0, n = 0;
    const int64_t kept = gx_drain_ringbuf_view(rt, ring_fd, &v, &vb, &n);
    if (kept < 0) return (int)kept;
    m->pend_bytes = vb;
    m->pend_kept = (uint64_t)kept;
    m->pend_recs = n;
    m->pend_counted = true;
    m->drain_pending = true;
    return 0;
  }
  if (!rt->copy && hipStreamCreateWithFlags(&rt->copy, hipStreamNonBlocking) != hipSuccess) {
    rt->copy = nullptr;
    return -EIO;
  }
  if (!m->drain_ev && hipEventCreateWithFlags(&m->drain_ev, hipEventDisableTiming) != hipSuccess) {
    m->drain_ev = nullptr;
    return -EIO;
  }
  if (!m->ctrl_pin && hipHostMalloc((void**)&m->ctrl_pin, sizeof ctrl, hipHostMallocDefault) != hipSuccess) {
    m->ctrl_pin = nullptr;
    return -ENOMEM;
  }
  if (m->pin_cap < avail) {
    if (m->h_pin) (void)hipHostFree(m->h_pin);
    m->h_pin = nullptr;
    m->pin_cap = 0;
    if (hipHostMalloc((void**)&m->h_pin, avail, hipHostMallocDefault) != hipSuccess) return -ENOMEM;
    m->pin_cap = avail;
  }
  // the committed range, then the ring's new control words (tail moved
  // past the range, the device's counts cleared), in order on the copy
  // stream
  const uint64_t t0 = tail & (cap - 1), first = std::min(avail, cap - t0);
  std::memset(m->ctrl_pin, 0, sizeof ctrl);
  m->ctrl_pin[0] = head;
  m->ctrl_pin[1] = tail + avail;
  m->ctrl_pin[2] = ctrl[2];
  if (hipMemcpyAsync(m->h_pin, m->h.data + t0, first, hipMemcpyDeviceToHost, rt->copy) != hipSuccess ||
      (first < avail && hipMemcpyAsync(m->h_pin + first, m->h.data, avail - first, hipMemcpyDeviceToHost,
                                       rt->copy) != hipSuccess) ||
      hipMemcpyAsync(m->h.ctrl, m->ctrl_pin, sizeof ctrl, hipMemcpyHostToDevice, rt->copy) != hipSuccess ||
      hipEventRecord(m->drain_ev, rt->copy) != hipSuccess)
    return -EIO;
  m->pend_bytes = avail;
  m->pend_kept = avail - disc;
  m->pend_recs = recs;
  m->pend_counted = false;
  m->drain_pending = true;
  return 0;
}

int64_t gx_drain_ringbuf_finish(gx_rt* rt, int ring_fd, const void** view, uint64_t* view_bytes,
                                uint64_t* n_records) {
  MapObj* m = get_map(rt, ring_fd);
  if (!m || m->h.type != MAP_RINGBUF || !view || !view_bytes || !m->drain_pending) return -EINVAL;
  DevGuard g(rt->dev);
  if (m->drain_ev && hipEventSynchronize(m->drain_ev) != hipSuccess) return -EIO;
  m->drain_pending = false;
  *view = m->pend_bytes ? m->h_pin : nullptr;
  *view_bytes = m->pend_bytes;
  if (n_records) *n_records = m->pend_recs;
  if (!m->pend_counted) rt->stats.bytes_drained += m->pend_kept;
  return (int64_t)m->pend_kept;
}

}  // extern "C"

namespace {

// One snapshot of every map of the daemon: copies issued on its stream
// between two runs (the enqueue lock keeps runs whole), waited for, then
// published.  Returns 0 or -EIO.
int snap_take(gx_rt* rt, SnapDaemon* d) {
  std::lock_guard<std::mutex> one(d->take_mu);
  {
    std::lock_guard<std::mutex> lk(rt->enq_mu);
    for (SnapMap& sm : d->maps) {
      const MapObj& m = rt->maps[sm.fd];
      if (hipMemcpyAsync(sm.pin[0], m.h.data, sm.data_bytes, hipMemcpyDeviceToHost, d->stream) != hipSuccess ||
          (sm.slot_bytes && hipMemcpyAsync(sm.pin[0] + sm.data_bytes, m.h.slots, sm.slot_bytes, hipMemcpyDeviceToHost,
                                           d->stream) != hipSuccess))
        return -EIO;
    }
    if (hipEventRecord(d->ev, d->stream) != hipSuccess) return -EIO;
  }
  if (hipEventSynchronize(d->ev) != hipSuccess) return -EIO;
  std::lock_guard<std::mutex> lk(d->mu);
  for (SnapMap& sm : d->maps) {
    std::swap(sm.pin[0], sm.pin[1]);
    sm.version++;
  }
  return 0;
}

void snap_free(SnapDaemon* d) {
  for (SnapMap& sm : d->maps)
    for (uint8_t* p : sm.pin)
      if (p) (void)hipHostFree(p);
  if (d->ev) (void)hipEventDestroy(d->ev);
  delete d;
}

}  // namespace

extern "C" {

int gx_snapshot_start(gx_rt* rt, const int* map_fds, uint32_t n, uint64_t interval_us, void* stream) {
  if (!rt || (!map_fds && n)) return -EINVAL;
  if (rt->snap) return -EBUSY;
  DevGuard g(rt->dev);
  SnapDaemon* d = new (std::nothrow) SnapDaemon();
  if (!d) return -ENOMEM;
  d->stream = (hipStream_t)stream;
  d->interval_us = std::max<uint64_t>(interval_us, 100);
  for (uint32_t i = 0; i < n; i++) {
    const MapObj* m = get_map(rt, map_fds[i]);
    if (!m || m->h.type == MAP_RINGBUF) {
      snap_free(d);
      return -EINVAL;
    }
    SnapMap sm;
    sm.fd = map_fds[i];
    sm.data_bytes = m->data_bytes;
    sm.slot_bytes = m->slot_bytes;
    d->maps.push_back(sm);
    for (uint8_t*& p : d->maps.back().pin)
      if (hipHostMalloc((void**)&p, sm.data_bytes + sm.slot_bytes, hipHostMallocDefault) != hipSuccess) {
        snap_free(d);
        return -ENOMEM;
      }
  }
  if (hipEventCreateWithFlags(&d->ev, hipEventDisableTiming) != hipSuccess) {
    snap_free(d);
    return -ENOMEM;
  }
  rt->snap = d;
  const int dev = rt->dev;
  d->th = std::thread([rt, d, dev]() {
    (void)hipSetDevice(dev);
    std::unique_lock<std::mutex> lk(d->mu);
    while (!d->stop) {
      d->cv.wait_for(lk, std::chrono::microseconds(d->interval_us), [d] { return d->stop; });
      if (d->stop) break;
      lk.unlock();
      (void)snap_take(rt, d);
      lk.lock();
    }
  });
  return 0;
}

int64_t gx_snapshot_read(gx_rt* rt, int map_fd, void* keys, void* vals, uint64_t cap, uint64_t* version) {
  if (!rt) return -EINVAL;
  SnapDaemon* d = rt->snap;
  if (!d) return -ENOENT;
  const MapObj* m = get_map(rt, map_fd);
  if (!m) return -EINVAL;
  std::lock_guard<std::mutex> lk(d->mu);
  for (const SnapMap& sm : d->maps) {
    if (sm.fd != map_fd) continue;
    if (version) *version = sm.version;
    const MapDev& h = m->h;
    const uint8_t* data = sm.pin[1];
    if (h.type == MAP_ARRAY) {
      for (uint64_t i = 0; i < h.max_entries && i < cap; i++) {
        if (keys) std::memcpy((uint8_t*)keys + 4 * i, &i, 4);
        if (vals) std::memcpy((uint8_t*)vals + i * h.value_size, data + i * h.vstride, h.value_size);
      }
      return h.max_entries;
    }
    const uint8_t* slots = data + sm.data_bytes;
    uint64_t cnt = 0;
    for (uint64_t i = 0; i <= h.slot_mask; i++) {
      const uint8_t* hdr = slots + i * h.sstride;
      uint32_t st;
      std::memcpy(&st, hdr, 4);
      if ((st & 0xff) != SLOT_LIVE) continue;
      if (cnt < cap) {
        if (keys) std::memcpy((uint8_t*)keys + cnt * h.key_size, hdr + 8, h.key_size);
        if (vals) std::memcpy((uint8_t*)vals + cnt * h.value_size, data + i * h.vstride, h.value_size);
      }
      cnt++;
    }
    return (int64_t)cnt;
  }
  return -ENOENT;
}

int gx_snapshot_flush(gx_rt* rt) {
  if (!rt || !rt->snap) return -ENOENT;
  DevGuard g(rt->dev);
  return snap_take(rt, rt->snap);
}

void gx_snapshot_stop(gx_rt* rt) {
  if (!rt || !rt->snap) return;
  SnapDaemon* d = rt->snap;
  {
    std::lock_guard<std::mutex> lk(d->mu);
    d->stop = true;
  }
  d->cv.notify_all();
  if (d->th.joinable()) d->th.join();
  DevGuard g(rt->dev);
  (void)hipStreamSynchronize(d->stream);
  rt->snap = nullptr;
  snap_free(d);
}

int gx_run_app_vadd(gx_rt* rt, int prog_fd, const double* d_a, const double* d_b, double* d_c, uint64_t n,
                    uint64_t stride, uint32_t* d_rc, void* stream) {
  if (!rt || !d_a || !d_b || !d_c || n == 0 || n > (1ull << 32) || stride >= n || gcd64(stride, n) != 1)
    return -EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const AppArgs P{d_a, d_b, d_c, n, stride, ~0ull / n};
  DevGuard g(rt->dev);
  if (drain_barrier(rt)) return -EIO;  // started drains finish copying first
  if (prog_fd < 0) {
    hipError_t e = launch_app_plain(P, rt->n_cu, s);
    return e == hipSuccess ? 0 : to_errno(e);
  }
  ProgObj* p = get_prog(rt, prog_fd);
  if (!p || !p->v.event_parallel ||
      (p->hook != HOOK_MEM_ACCESS && p->hook != HOOK_WAVE_MEM && p->hook != HOOK_SIMT_MEM))
    return -EINVAL;
  std::unique_lock<std::mutex> lk(rt->enq_mu, std::defer_lock);
  if (rt->snap) lk.lock();
  RunArgs A = make_args(rt, p, nullptr, n, d_rc);
  int r = 0;
  if (p->jf_ep) {
    if (!p->jf_app) {
      hipModule_t mod = nullptr;
      JitInfo ji;
      r = jit_app_module(rt, p, 1, &mod, &p->jf_app, &p->jf_app_red, &ji);
      if (r) return r;
    }
    r = launch_jit_app(rt, p, A, P, jit_ep_blocks(p, n, 0), jit_waves(p->v.stack_bytes, true), s);
  } else if (p->acc_hi > p->acc_lo && env_int("GX_INTERP_ACC", 1)) {
    // the interpreter's LDS mirror of a small shared array map
    A.acc_lo = p->acc_lo;
    A.acc_hi = p->acc_hi;
    A.acc_op = p->acc_op;
    A.acc_sc = p->acc_sc;
    hipError_t e = launch_app_vadd_acc(A, P, rt->n_cu, s);
    r = e == hipSuccess ? 0 : to_errno(e);
  } else {
    hipError_t e = launch_app_vadd(A, P, s);
    r = e == hipSuccess ? 0 : to_errno(e);
  }
  if (r) return r;
  rt->stats.launches += 1;
  rt->stats.events += n;
  note_stream(rt, s);
  return 0;
}

int gx_run_sched(gx_rt* rt, int prog_fd, const uint32_t* d_cost, uint32_t n_units, uint32_t workers,
                 uint64_t* d_out, uint64_t* d_log, uint32_t* d_log_rc, uint32_t log_cap, uint32_t* d_log_n,
                 void* stream) {
  if (!rt || !d_cost || !d_out || n_units == 0 || workers == 0 || workers > kMaxWorkers ||
      (log_cap && (!d_log || !d_log_rc)))
    return -EINVAL;
  ProgObj* p = nullptr;
  if (prog_fd >= 0) {
    p = get_prog(rt, prog_fd);
    if (!p || p->hook != HOOK_SCHED || !p->v.event_parallel) return -EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  DevGuard g(rt->dev);
  if (drain_barrier(rt)) return -EIO;  // started drains finish copying first
  std::unique_lock<std::mutex> lk(rt->enq_mu, std::defer_lock);
  if (rt->snap) lk.lock();
  Exec* Xp = exec_for(rt, s);
  if (!Xp) return -ENOMEM;
  Exec& E = *Xp;
  // per-worker counters, then the runtime's own log count
  if (E.wnext_cap < (size_t)workers + 1) {
    if (E.d_wnext) (void)hipFree(E.d_wnext);
    E.d_wnext = nullptr;
    E.wnext_cap = 0;
    if (hipMalloc((void**)&E.d_wnext, ((size_t)workers + 1) * 4) != hipSuccess) return -ENOMEM;
    E.wnext_cap = (size_t)workers + 1;
  }
  hipError_t e = launch_zero(E.d_wnext, workers + 1, s);
  if (e == hipSuccess && d_log_n) e = launch_zero(d_log_n, 1, s);
  if (e != hipSuccess) return to_errno(e);
  SchedArgs S{};
  S.cost = d_cost;
  S.out = d_out;
  S.next = E.d_wnext;
  S.log = log_cap ? d_log : nullptr;
  S.log_rc = d_log_rc;
  S.log_n = d_log_n ? d_log_n : E.d_wnext + workers;
  S.n_units = n_units;
  S.workers = workers;
  S.log_cap = log_cap;
  S.tick_num = 1000000;  // kHz ticks to ns
  S.tick_den = rt->wall_khz;
  int r = 0;
  if (!p) {
    e = launch_sched_plain(S, s);
    r = e == hipSuccess ? 0 : to_errno(e);
  } else {
    RunArgs A = make_args(rt, p, nullptr, 0, nullptr);
    if (p->jf_app) {
      r = launch_jit_app(rt, p, A, S, workers, 1, s);
    } else {
      e = launch_sched(A, S, s);
      r = e == hipSuccess ? 0 : to_errno(e);
    }
  }
  if (r) return r;
  rt->stats.launches += 1;
  note_stream(rt, s);
  return 0;
}

int gx_ringbuf_pos(gx_rt* rt, int ring_fd, uint64_t* head, uint64_t* tail) {
  MapObj* m = get_map(rt, ring_fd);
  if (!m || m->h.type != MAP_RINGBUF || !head || !tail) return -EINVAL;
  DevGuard g(rt->dev);
  if (drain_barrier(rt)) return -EIO;  // started drains finish copying first
  if (wait_all(rt)) return -EIO;
  uint64_t ctrl[4];
  if (hipMemcpy(ctrl, m->h.ctrl, sizeof ctrl, hipMemcpyDeviceToHost) != hipSuccess) return -EIO;
  // an overflowed reservation's start, once a drain has cut the head back
  *head = ctrl[3] != 0 && ~ctrl[3] < ctrl[0] ? ~ctrl[3] : ctrl[0];
  *tail = ctrl[1];
  return 0;
}

int gx_profile_enable(gx_rt* rt, int on) {
  if (!rt) return -EINVAL;
  rt->profile = on != 0;
  return 0;
}

int gx_profile_read(gx_rt* rt, double* vm_ms, uint64_t* vm_launches) {
  if (!rt) return -EINVAL;
  DevGuard g(rt->dev);
  double total = 0;
  uint64_t n = 0;
  for (auto& pe : rt->prof_pending) {
    float ms = 0;
    if (hipEventSynchronize(pe.second) != hipSuccess || hipEventElapsedTime(&ms, pe.first, pe.second) != hipSuccess)
      return -EIO;
    total += ms;
    n++;
    rt->prof_free.push_back(pe);
  }
  rt->prof_pending.clear();
  if (vm_ms) *vm_ms = total;
  if (vm_launches) *vm_launches = n;
  return 0;
}

int gx_stats_get(gx_rt* rt, gx_stats* out) {
  if (!rt || !out) return -EINVAL;
  DevGuard g(rt->dev);
  if (wait_all(rt)) return -EIO;
  gx_stats s = rt->stats;
  s.ring_drops = s.hash_e2big = 0;
  for (auto& m : rt->maps) {
    if (!m.live) continue;
    uint64_t c[3] = {0, 0, 0};
    if (hipMemcpy(c, m.h.ctrl, 24, hipMemcpyDeviceToHost) != hipSuccess) return -EIO;
    if (m.h.type == MAP_RINGBUF) s.ring_drops += c[2];
    if (m.h.type == MAP_HASH) s.hash_e2big += c[1];
  }
  uint64_t err = 0;
  if (hipMemcpy(&err, rt->d_err, 8, hipMemcpyDeviceToHost) != hipSuccess) return -EIO;
  s.vm_errors = err;
  *out = s;
  return 0;
}

}  // extern "C"
