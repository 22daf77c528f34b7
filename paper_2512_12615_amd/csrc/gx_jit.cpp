// Compilation of verified programs to native gfx950 code.
//
// The paper lowers verified bytecode through LLVM to the GPU's own ISA and
// inlines the helpers and map accesses (sections 5.1 and 5.3, section 4.4
// "Warp-level Execution Optimizations").  Here the pre-decoded micro-ops of
// a verified program are written out as HIP source, one statement per
// instruction with a label at every jump target, and compiled at load time
// with hipRTC for gfx950.  eBPF registers become 64-bit locals, so the
// compiler keeps them in VGPRs, folds constant stack offsets into LDS
// addresses and lets the hardware's EXEC mask handle divergent branches;
// helper calls go straight to the same device helpers the interpreter uses,
// with each map's shape as constants.  Verification has
// already bounded every loop, so the generated code carries no step counter.
#include "gx_jit.h"

#include <hip/hiprtc.h>

#include <algorithm>
#include <cctype>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

namespace gx {

namespace {

std::string lit(uint64_t v) {
  char b[40];
  std::snprintf(b, sizeof b, "0x%llxull", (unsigned long long)v);
  return b;
}

std::string reg(uint32_t i) { return "r" + std::to_string(i); }

const char* kTy[4] = {"uint8_t", "uint16_t", "uint32_t", "uint64_t"};
const char* kSTy[3] = {"int8_t", "int16_t", "int32_t"};

// value of size code sc, sign-extended when sx
std::string extend(const std::string& v, int sc, bool sx) {
  if (!sx || sc == 3) return "(uint64_t)(" + v + ")";
  return std::string("(uint64_t)(int64_t)(") + kSTy[sc] + ")(" + v + ")";
}

// How the event-parallel kernel accumulates one shared map's atomics.
struct Acc {
  int kind = 0;        // 0 none, 1 whole-map mirror in LDS, 2 tagged LDS cache
  uint32_t op = 0;     // ADD 0x00, OR 0x40, AND 0x50, XOR 0xa0
  int sc = -1;         // operand width: 2 (u32) or 3 (u64); -1 if the map takes no atomics
  uint32_t words = 0;  // mirror: words of the value area; cache: slots (4 per set)
  bool narrow = false; // cache of 64-bit sums kept as 32-bit partial sums
  bool tag8 = false;   // cache with 8-bit tags (word index / sets + 1, four per 32-bit word)
  std::string word_type() const { return sc == 3 ? "uint64_t" : "uint32_t"; }
  std::string slot_type() const { return sc == 3 && !narrow ? "uint64_t" : "uint32_t"; }
};

// LDS a workgroup may take (gfx950: 160 KiB per CU), of which the
// accumulators get what stacks and ring slots leave; caches are capped at
// kCacheMax each (every slot in use costs one device atomic, or one spilled
// slot, at the flush; the latency histogram measured 562 -> 537 us per 2^26
// events when the cap went from 80 to 112 KiB, and slower below 64 KiB).
constexpr uint64_t kLdsMax = 150 << 10;
constexpr uint64_t kCacheMax = 112 << 10;
constexpr uint64_t kCacheSlotsPerSet = 4;  // the device cache's ways
constexpr uint64_t kReduceMax = 8192;      // words of a reduce block's LDS sums
constexpr uint32_t kCombSlots = 4;         // shared-map words a one-lane run combines in registers
constexpr uint32_t kMemoEntries = 64;      // LDS lookup-memo entries per site (one queue per wave)
constexpr uint32_t kMemoLds = 4096;        // LDS bytes of a program's memo tables (the rest keep one entry)
// Shared-map updates of event-parallel kernels may be aggregated per wave
// by distinct word before the LDS accumulator (GX_AGG_LDS=1).  Off by
// default: measured on the access counter (2^20 events, 16.2 -> 21.2 us)
// and the latency histogram (2^26 events, 581 -> 641 us), the grouping
// costs more than the LDS atomics it saves.
bool agg_lds() {
  const char* v = std::getenv("GX_AGG_LDS");
  return v && *v && std::atoi(v) != 0;
}

// The checked mode's bounds checks of map-value accesses (GX_CHECKED, read
// again by every run) are compiled in only when it is on at compile time:
// otherwise each access would test the run's flag on the event chain.
std::string guards_define() {
  const char* v = std::getenv("GX_CHECKED");
  return std::string("#define GX_GUARDS ") + (v && *v && std::atoi(v) != 0 ? "1" : "0") + "\n";
}

// Cap on each cache in KiB from the environment (tuning experiments).
int env_int_jit(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v && *v ? std::atoi(v) : dflt;
}

// Maps of a program as the generated code sees them.
struct JMaps {
  const std::vector<std::pair<uint64_t, MapDev>>& m;
  const std::vector<int>& mem_map;  // map of each map-value access (by slot)
  const std::vector<int>& ld_map;   // map of each lddw map reference (by slot)
  std::vector<int> ring;  // ring index per map (-1 if not a ring)
  int n_rings = 0;
  std::vector<Acc> acc;   // per map
  bool simt = false;      // SIMT hook: a wave's shared-map updates hit one word, combined first
  std::vector<std::pair<int, int>> comb;  // per map: {op, width} of its register combiner, op -1 if none
  JMaps(const std::vector<std::pair<uint64_t, MapDev>>& maps, const std::vector<int>& mm, const std::vector<int>& lm)
      : m(maps), mem_map(mm), ld_map(lm) {
    for (auto& e : maps) ring.push_back(e.second.type == MAP_RINGBUF ? n_rings++ : -1);
    acc.resize(maps.size());
  }
  // plan the LDS accumulators of the shared maps the program updates
  void plan(const std::vector<Uop>& U, uint64_t lds_used) {
    for (uint32_t pc = 0; pc < U.size() && pc < mem_map.size(); pc++) {
      if ((U[pc].w0 & 0xff) != H_ATOMIC_MAP || mem_map[pc] < 0 || mem_map[pc] >= (int)m.size()) continue;
      const MapDev& d = m[mem_map[pc]].second;
      if (!(d.flags & F_SHARED) || d.type != MAP_ARRAY) continue;
      Acc& a = acc[mem_map[pc]];
      a.op = (uint32_t)U[pc].imm & 0xf0;
      a.sc = (int)((U[pc].w0 >> 16) & 3);
    }
    uint64_t left = kLdsMax > lds_used ? kLdsMax - lds_used : 0;
    // small maps are mirrored whole; the others share what is left as caches
    int n_cache = 0;
    for (size_t k = 0; k < m.size(); k++) {
      Acc& a = acc[k];
      if (a.sc < 2) continue;
      const uint64_t area = (uint64_t)m[k].second.max_entries * m[k].second.vstride;
      if (area <= left && area <= (32u << 10)) {
        a.kind = 1;
        a.words = (uint32_t)(area / (a.sc == 3 ? 8 : 4));
        left -= area;
      } else {
        n_cache++;
      }
    }
    const uint64_t cap = std::min<uint64_t>(kCacheMax, (uint64_t)std::max(16, env_int_jit("GX_ACC_KIB", 1 << 20)) << 10);
    const uint64_t share = n_cache ? std::min<uint64_t>(left / n_cache, cap) : 0;
    for (size_t k = 0; k < m.size(); k++) {
      Acc& a = acc[k];
      if (a.sc < 2 || a.kind) continue;
      a.narrow = a.op == 0x00 && a.sc == 3;
      const uint64_t val_bytes = a.slot_type() == "uint64_t" ? 8 : 4;
      // an odd set count (the device maps keys to sets modulo it)
      auto odd = [](uint64_t n) { return n - (n % 2 == 0 && n > 0); };
      // 8-bit tags when every word's quotient by the set count fits (the
      // tags then take a quarter of the LDS); 32-bit tags otherwise
      const uint64_t map_words = (uint64_t)m[k].second.max_entries * m[k].second.vstride / (a.sc == 3 ? 8 : 4);
      uint64_t sets = odd(share / (kCacheSlotsPerSet * (val_bytes + 1)));
      a.tag8 = sets >= 64 && (map_words + sets - 1) / sets <= 254;
      if (!a.tag8) sets = odd(share / (kCacheSlotsPerSet * (val_bytes + 4)));
      if (sets >= 64) {
        a.kind = 2;
        a.words = (uint32_t)(sets * kCacheSlotsPerSet);
      }
    }
  }
  int index(uint64_t desc) const {
    for (size_t k = 0; k < m.size(); k++)
      if (m[k].first == desc) return (int)k;
    return -1;
  }
  uint64_t ring_cap(int k) const { return (uint64_t)m[k].second.slot_mask + 1; }
};

// Map-value windows: a lookup of a map whose values this program's lane
// alone writes (not shared, not read-only; at most 64 bytes) loads the whole
// value into locals right after the call, one parallel burst of loads, and
// later reads through that pointer take the locals instead of waiting for
// one memory round trip each.  Stores through the pointer still go to
// memory and also update the locals.  A forward data-flow pass over the
// micro-ops finds, for every access, whether its base register holds the
// pointer of the lookup site's latest run (copies and constant offsets
// followed) with no store through another pointer, atomic, update or delete
// on that map in between; only those accesses use a window.  Anything else
// reads memory as before, which the stores keep current.
struct Windows {
  struct W {
    uint32_t pc;
    int map;
    uint32_t words;
    bool used;
  };
  std::vector<W> win;
  std::vector<int> site;     // window of each lookup site, by slot (-1 none)
  std::vector<int> acc;      // window of each map access, by slot (-1 none)
  std::vector<int32_t> off;  // its byte offset in the value
  std::vector<char> memo;    // per window: its key, pointer and words kept across events
  std::vector<char> table;   // per memo: an LDS table when one queue runs per wave
  std::vector<uint64_t> inval;  // per slot: memo windows a slot's write may make stale
  // per memo table: written back (window stores stay in the table until the
  // entry is evicted, the memo is cleared or the run ends) instead of
  // written through; for a map with one memo site, in the one-queue kernel
  std::vector<char> wb;
  std::vector<uint64_t> sync;  // per slot: written-back tables a slot's read of map memory must flush first
};

Windows plan_windows(const std::vector<Uop>& U, const JMaps& J) {
  Windows R;
  const uint32_t n = (uint32_t)U.size();
  R.site.assign(n, -1);
  R.acc.assign(n, -1);
  R.off.assign(n, 0);
  for (uint32_t pc = 0; pc < n; pc++) {
    const uint32_t h = U[pc].w0 & 0xff;
    if (h == H_LDIMM) {
      pc++;
      continue;
    }
    if (h != H_LOOKUP_HASH && h != H_LOOKUP_ARRAY) continue;
    const int k = J.index(U[pc].imm);
    if (k < 0 || R.win.size() >= 64) continue;
    const MapDev& md = J.m[k].second;
    if ((md.flags & (F_SHARED | F_READ_ONLY)) || md.value_size == 0 || md.value_size > 64) continue;
    R.site[pc] = (int)R.win.size();
    R.win.push_back({pc, k, (md.value_size + 7) / 8, false});
  }
  if (R.win.empty()) return R;
  struct St {
    bool reached = false;
    int w[11];
    int64_t d[11];
    uint64_t valid = 0;
  };
  std::vector<St> in(n);
  // the access [o, o + size) of window w fits in one of its words
  auto fits = [&](int w, int64_t o, uint32_t size) {
    return o >= 0 && o + size <= 8ull * R.win[w].words && (uint64_t)(o & 7) + size <= 8;
  };
  auto kill_map = [&](St& s, int k) {
    for (size_t i = 0; i < R.win.size(); i++)
      if (k < 0 || R.win[i].map == k) s.valid &= ~(1ull << i);
  };
  auto holds = [&](const St& s, uint32_t r) { return r < 11 && s.w[r] >= 0 && ((s.valid >> s.w[r]) & 1); };
  // transfer: state after slot pc; successors into succ
  auto step = [&](uint32_t pc, St s, std::vector<uint32_t>& succ, bool mark) {
    const Uop& u = U[pc];
    const uint32_t h = u.w0 & 0xff, d = (u.w0 >> 8) & 15, src = (u.w0 >> 12) & 15, a8 = (u.w0 >> 16) & 0xff;
    const bool K = (u.w0 >> 24) & 1;
    const uint32_t size = 1u << (a8 & 3);
    uint32_t next = pc + 1;
    auto set_reg = [&](uint32_t r, int w, int64_t dd) {
      if (r < 11) {
        s.w[r] = w;
        s.d[r] = dd;
      }
    };
    if (h <= H_TRUNC) {
      if (h == H_MOV64 && !K && src < 11)
        set_reg(d, s.w[src], s.d[src]);
      else if ((h == H_ADD64 || h == H_SUB64) && K && d < 11 && s.w[d] >= 0)
        s.d[d] += h == H_ADD64 ? (int64_t)u.imm : -(int64_t)u.imm;
      else
        set_reg(d, -1, 0);
      succ.push_back(next);
    } else if (h >= H_JA && h <= H_JSLE32) {
      if (h != H_JA) succ.push_back(next);
      succ.push_back((uint32_t)u.aux);
    } else {
      switch (h) {
        case H_LDX_MAP:
          if (mark && holds(s, src) && fits(s.w[src], s.d[src] + u.aux, size)) {
            R.acc[pc] = s.w[src];
            R.off[pc] = (int32_t)(s.d[src] + u.aux);
            R.win[s.w[src]].used = true;
          }
          set_reg(d, -1, 0);
          succ.push_back(next);
          break;
        case H_LDX_CTX:
        case H_LDX_STACK:
          set_reg(d, -1, 0);
          succ.push_back(next);
          break;
        case H_ST_STACK:
        case H_STX_STACK:
          succ.push_back(next);
          break;
        case H_ST_MAP:
        case H_STX_MAP: {
          const int k = pc < J.mem_map.size() ? J.mem_map[pc] : -1;
          if (holds(s, d) && fits(s.w[d], s.d[d] + u.aux, size)) {
            // a store through the window: the locals follow it; any other
            // pointer into the map may alias it
            const int w = s.w[d];
            if (mark) {
              R.acc[pc] = w;
              R.off[pc] = (int32_t)(s.d[d] + u.aux);
            }
            kill_map(s, R.win[w].map);
            s.valid |= 1ull << w;
          } else {
            kill_map(s, k);
          }
          succ.push_back(next);
          break;
        }
        case H_ATOMIC_STACK:
        case H_ATOMIC_MAP:
          if (h == H_ATOMIC_MAP) kill_map(s, pc < J.mem_map.size() ? J.mem_map[pc] : -1);
          if ((uint32_t)u.imm == 0xf1)
            set_reg(0, -1, 0);
          else if (u.imm & 1)
            set_reg(src, -1, 0);
          succ.push_back(next);
          break;
        case H_LDIMM:
          set_reg(d, -1, 0);
          succ.push_back(pc + 2);
          break;
        case H_LOOKUP_ARRAY:
        case H_LOOKUP_HASH:
        case H_UPDATE_ARRAY:
        case H_UPDATE_HASH:
        case H_DELETE_HASH:
        case H_RET_EINVAL:
        case H_RINGBUF_OUTPUT: {
          for (uint32_t r = 0; r <= 5; r++) set_reg(r, -1, 0);
          if (h == H_UPDATE_ARRAY || h == H_UPDATE_HASH || h == H_DELETE_HASH) kill_map(s, J.index(u.imm));
          const int w = R.site[pc];
          if (w >= 0) {
            for (uint32_t r = 0; r < 11; r++)
              if (s.w[r] == w) set_reg(r, -1, 0);
            set_reg(0, w, 0);
            s.valid |= 1ull << w;
          }
          succ.push_back(next);
          break;
        }
        default:  // exit
          break;
      }
    }
    return s;
  };
  St entry;
  entry.reached = true;
  for (int r = 0; r < 11; r++) {
    entry.w[r] = -1;
    entry.d[r] = 0;
  }
  in[0] = entry;
  std::vector<uint32_t> work{0};
  std::vector<char> queued(n, 0);
  queued[0] = 1;
  while (!work.empty()) {
    const uint32_t pc = work.back();
    work.pop_back();
    queued[pc] = 0;
    std::vector<uint32_t> succ;
    const St out = step(pc, in[pc], succ, false);
    for (uint32_t t : succ) {
      if (t >= n) continue;
      St& dst = in[t];
      bool changed = false;
      if (!dst.reached) {
        dst = out;
        changed = true;
      } else {
        for (int r = 0; r < 11; r++)
          if (dst.w[r] >= 0 && (dst.w[r] != out.w[r] || dst.d[r] != out.d[r])) {
            dst.w[r] = -1;
            changed = true;
          }
        const uint64_t v = dst.valid & out.valid;
        if (v != dst.valid) {
          dst.valid = v;
          changed = true;
        }
      }
      if (changed && !queued[t]) {
        queued[t] = 1;
        work.push_back(t);
      }
    }
  }
  for (uint32_t pc = 0; pc < n; pc++) {
    if (!in[pc].reached) continue;
    std::vector<uint32_t> succ;
    (void)step(pc, in[pc], succ, true);
  }
  return R;
}

// Private frames: when every stack access and every stack argument of a
// helper call has a base register whose offset from the frame pointer r10
// is known (r10 itself, or r10 moved and shifted by constants), the frame's
// 8-byte words become locals of the generated code (registers: scalar ones
// in the wave-uniform kernel), and the accesses become shifts and masks of
// those locals.  The LDS frame stays as the place helpers read their stack
// arguments from: the words a helper reads are stored there right before
// the call (helpers only read the stack).  A forward data-flow pass over the
// micro-ops finds each access's byte in the frame; any unknown base leaves
// the program on the LDS frame.
struct Frame {
  bool priv = false;
  std::vector<int32_t> at;   // per slot: frame byte of the stack access, or of the helper's r2 argument
  std::vector<int32_t> at3;  // per slot: frame byte of an update's r3 (value) argument
};

Frame plan_frame(const std::vector<Uop>& U, uint32_t stack_bytes) {
  Frame F;
  const uint32_t n = (uint32_t)U.size();
  F.at.assign(n, -1);
  F.at3.assign(n, -1);
  if (!stack_bytes || stack_bytes > 512) return F;
  struct St {
    bool reached = false;
    bool k[11];
    int64_t d[11];
  };
  std::vector<St> in(n);
  bool ok = true;
  auto step = [&](uint32_t pc, St s, std::vector<uint32_t>& succ, bool mark) {
    const Uop& u = U[pc];
    const uint32_t h = u.w0 & 0xff, d = (u.w0 >> 8) & 15, src = (u.w0 >> 12) & 15, a8 = (u.w0 >> 16) & 0xff;
    const bool K = (u.w0 >> 24) & 1;
    auto kill = [&](uint32_t r) {
      if (r < 10) s.k[r] = false;
    };
    // frame byte of base register r plus offset o (-1 if unknown or outside)
    auto byte = [&](uint32_t r, int64_t o) -> int32_t {
      if (r > 10 || !s.k[r]) return -1;
      const int64_t b = (int64_t)stack_bytes + s.d[r] + o;
      return b >= 0 && b < (int64_t)stack_bytes ? (int32_t)b : -1;
    };
    auto need = [&](std::vector<int32_t>& v, uint32_t r, int64_t o) {
      const int32_t b = byte(r, o);
      if (b < 0) ok = false;
      if (mark) v[pc] = b;
    };
    uint32_t next = pc + 1;
    if (h <= H_TRUNC) {
      if (h == H_MOV64 && !K && src <= 10 && d < 10) {
        s.k[d] = s.k[src];
        s.d[d] = s.d[src];
      } else if ((h == H_ADD64 || h == H_SUB64) && K && d < 10 && s.k[d]) {
        s.d[d] += h == H_ADD64 ? (int64_t)u.imm : -(int64_t)u.imm;
      } else {
        kill(d);
      }
      succ.push_back(next);
      return s;
    }
    if (h >= H_JA && h <= H_JSLE32) {
      if (h != H_JA) succ.push_back(next);
      succ.push_back((uint32_t)u.aux);
      return s;
    }
    switch (h) {
      case H_LDX_STACK:
        need(F.at, src, u.aux);
        kill(d);
        break;
      case H_ST_STACK:
      case H_STX_STACK:
        need(F.at, d, u.aux);
        break;
      case H_ATOMIC_STACK:
        need(F.at, d, u.aux);
        if ((uint32_t)u.imm == 0xf1) kill(0);
        else if (u.imm & 1) kill(src);
        break;
      case H_ATOMIC_MAP:
        if ((uint32_t)u.imm == 0xf1) kill(0);
        else if (u.imm & 1) kill(src);
        break;
      case H_LDIMM:
        kill(d);
        next = pc + 2;
        break;
      case H_LOOKUP_ARRAY:
      case H_LOOKUP_HASH:
      case H_DELETE_HASH:
      case H_RINGBUF_OUTPUT:
        if ((a8 & 1) == PK_STACK) need(F.at, 2, 0);
        for (uint32_t r = 0; r <= 5; r++) kill(r);
        break;
      case H_RET_EINVAL:
        for (uint32_t r = 0; r <= 5; r++) kill(r);
        break;
      case H_UPDATE_ARRAY:
      case H_UPDATE_HASH:
        if ((a8 & 1) == PK_STACK) need(F.at, 2, 0);
        if (((a8 >> 1) & 1) == PK_STACK) need(F.at3, 3, 0);
        for (uint32_t r = 0; r <= 5; r++) kill(r);
        break;
      case H_EXIT:
        return s;
      default:
        if (h == H_LDX_CTX || h == H_LDX_MAP) kill(d);
        break;
    }
    succ.push_back(next);
    return s;
  };
  St entry;
  entry.reached = true;
  for (int r = 0; r < 11; r++) {
    entry.k[r] = r == 10;
    entry.d[r] = 0;
  }
  if (n) in[0] = entry;
  std::vector<uint32_t> work;
  if (n) work.push_back(0);
  std::vector<char> queued(n, 0);
  if (n) queued[0] = 1;
  while (!work.empty()) {
    const uint32_t pc = work.back();
    work.pop_back();
    queued[pc] = 0;
    std::vector<uint32_t> succ;
    const St out = step(pc, in[pc], succ, false);
    for (uint32_t t : succ) {
      if (t >= n) continue;
      St& dst = in[t];
      bool changed = false;
      if (!dst.reached) {
        dst = out;
        changed = true;
      } else {
        for (int r = 0; r < 10; r++)
          if (dst.k[r] && (!out.k[r] || dst.d[r] != out.d[r])) {
            dst.k[r] = false;
            changed = true;
          }
      }
      if (changed && !queued[t]) {
        queued[t] = 1;
        work.push_back(t);
      }
    }
  }
  for (uint32_t pc = 0; pc < n; pc++) {
    if (!in[pc].reached) continue;
    std::vector<uint32_t> succ;
    (void)step(pc, in[pc], succ, true);
  }
  F.priv = ok && std::getenv("GX_LDS_FRAME") == nullptr;
  return F;
}

// Statements storing the frame words that bytes [b, b + len) of the frame
// occupy into the LDS frame (before a helper reads them there).
std::string frame_spill(int32_t b, uint32_t len) {
  std::string o;
  for (uint32_t w = (uint32_t)b / 8; w < ((uint32_t)b + len + 7) / 8; w++)
    o += "*(uint64_t*)saddr(stk, " + std::to_string(8 * w) + "u) = f" + std::to_string(w) + "; ";
  return o;
}

// Expression for the first min(8, len) bytes at frame byte b, when they lie
// in one frame word; "" otherwise.
std::string frame_bytes(int32_t b, uint32_t len) {
  const uint32_t n = len < 8 ? len : 8;
  if ((uint32_t)b % 8 + n > 8) return "";
  const std::string w = "f" + std::to_string(b / 8);
  const uint32_t sh = 8 * ((uint32_t)b % 8);
  std::string e = sh ? "(" + w + " >> " + std::to_string(sh) + ")" : w;
  if (n < 8) e = "(" + e + " & " + lit((1ull << (8 * n)) - 1) + ")";
  return e;
}

// Lookup memos: a hash lookup site whose window belongs to a map of keys of
// at most 8 bytes keeps, across the events of a run, the last key it found,
// the value's address and the window's words.  When the next event looks up
// the same key, the probe and the window load are skipped.  This holds for
// the same reason as the windows themselves: a key's values are written by
// the one lane that owns the key (its stream's events run in order on that
// lane), a live slot never moves (deletes leave tombstones), and every write
// of this program that may reach the value without going through the window
// - a store or atomic through another pointer, an update or delete of the
// map - clears the memo first.  With one queue per wave (lane 0 runs it)
// the memo is a table of kMemoEntries entries in LDS, indexed by the key's
// two 32-bit halves xor-ed: {key, value address, generation, window
// words}; an entry counts only while its generation is the site's current
// one, so clearing the memo is one increment.  Tables go to a program's
// sites while they fit kMemoLds; with several queues per wave, and at the
// other sites, each lane keeps one entry in registers.
void plan_memo(const std::vector<Uop>& U, const JMaps& J, Windows& R, bool event_parallel, bool tables) {
  R.memo.assign(R.win.size(), 0);
  R.table.assign(R.win.size(), 0);
  R.inval.assign(U.size(), 0);
  R.wb.assign(R.win.size(), 0);
  R.sync.assign(U.size(), 0);
  if (event_parallel) return;  // lanes run different streams' events in turn
  bool any = false;
  uint32_t lds = 0;
  for (size_t w = 0; w < R.win.size(); w++) {
    const MapDev& md = J.m[R.win[w].map].second;
    if ((U[R.win[w].pc].w0 & 0xff) == H_LOOKUP_HASH && md.type == MAP_HASH && md.key_size <= 8 && md.sstride == 16) {
      R.memo[w] = any = 1;
      // tables while they fit the budget: LDS taken from the one-wave
      // blocks would cost the kernel resident waves
      const uint32_t bytes = kMemoEntries * 8 * (3 + R.win[w].words);
      if (tables && lds + bytes <= kMemoLds) {
        R.table[w] = 1;
        lds += bytes;
      }
    }
  }
  if (!any) return;
  for (uint32_t pc = 0; pc < U.size(); pc++) {
    const uint32_t h = U[pc].w0 & 0xff;
    if (h == H_LDIMM) {
      pc++;
      continue;
    }
    int k;  // map whose values the slot may write (-1: any)
    if (h == H_ST_MAP || h == H_STX_MAP || h == H_ATOMIC_MAP)
      k = pc < J.mem_map.size() ? J.mem_map[pc] : -1;
    else if (h == H_UPDATE_ARRAY || h == H_UPDATE_HASH || h == H_DELETE_HASH)
      k = J.index(U[pc].imm);
    else
      continue;
    for (size_t w = 0; w < R.win.size(); w++) {
      if (!R.memo[w] || (k >= 0 && R.win[w].map != k)) continue;
      if ((h == H_ST_MAP || h == H_STX_MAP) && R.acc[pc] == (int)w) continue;  // through the window
      R.inval[pc] |= 1ull << w;
    }
  }
  // write-back tables: the only memo site of their map; every other read of
  // map memory that may reach its values - a load not through the window, a
  // helper reading a map-value argument - writes the table back first
  for (size_t w = 0; w < R.win.size(); w++) {
    if (!R.table[w]) continue;
    int sites = 0;
    for (size_t x = 0; x < R.win.size(); x++) sites += R.memo[x] && R.win[x].map == R.win[w].map;
    R.wb[w] = sites == 1 && std::getenv("GX_WRITE_THROUGH") == nullptr;
  }
  for (uint32_t pc = 0; pc < U.size(); pc++) {
    const uint32_t h = U[pc].w0 & 0xff, a8 = (U[pc].w0 >> 16) & 0xff;
    if (h == H_LDIMM) {
      pc++;
      continue;
    }
    for (size_t w = 0; w < R.win.size(); w++) {
      if (!R.wb[w]) continue;
      if (h == H_LDX_MAP) {
        const int k = pc < J.mem_map.size() ? J.mem_map[pc] : -1;
        if ((k < 0 || k == R.win[w].map) && R.acc[pc] != (int)w) R.sync[pc] |= 1ull << w;
      } else if (h >= H_LOOKUP_ARRAY && h <= H_RINGBUF_OUTPUT && ((a8 & 1) == PK_MAPVAL || ((a8 >> 1) & 1) == PK_MAPVAL)) {
        R.sync[pc] |= 1ull << w;
      }
    }
  }
}

std::string map_name(const JMaps& J, uint64_t desc) {
  int k = J.index(desc);
  return k >= 0 ? "&M" + std::to_string(k) : "(const MapDev*)" + lit(desc);
}

// The descriptor of map k: its shape as constants (sizes, masks and strides
// fold into the code), its addresses from the run's map table (the program
// instance's maps), so instances of one program with maps of one shape share
// a compiled module.  The loads are from constant memory and become scalar.
std::string map_fn(size_t k, const MapDev& m) {
  char b[800];
  std::snprintf(b, sizeof b,
                "__device__ __forceinline__ MapDev gx_map%zu(const RunArgs& A) {\n"
                "  typedef const __attribute__((address_space(4))) uint64_t cu64;\n"
                "  const cu64* d = (const cu64*)(((const cu64*)A.maptab)[%zu]);\n"
                "  return MapDev{%uu, %uu, %uu, %uu, %uu, %uu, %uu, %uu, (uint8_t*)d[4], (uint8_t*)d[5], "
                "(uint64_t*)d[6], 0ull};\n}\n",
                k, k, m.type, m.key_size, m.value_size, m.max_entries, m.flags, m.vstride, m.slot_mask, m.sstride);
  return b;
}

void emit_uop(std::string& o, const Uop& u, uint32_t pc, const JMaps& J, const Windows& Wn, const Frame& Fr) {
  const uint32_t h = u.w0 & 0xff, d = (u.w0 >> 8) & 15, s = (u.w0 >> 12) & 15, a8 = (u.w0 >> 16) & 0xff;
  const bool K = (u.w0 >> 24) & 1;
  const std::string D = reg(d), S = reg(s);
  const std::string B = K ? lit(u.imm) : S;
  const std::string xa = "(uint32_t)" + D, xb = "(uint32_t)" + B;
  const int sc = a8 & 3;
  const bool sxf = (a8 & 4) != 0;
  const std::string off = std::to_string(u.aux);
  const std::string tgt = "goto L" + std::to_string((uint32_t)u.aux) + ";";
  const std::string M = map_name(J, u.imm);
  auto set = [&](const std::string& e) { o += "  " + D + " = " + e + ";\n"; };
  auto set32 = [&](const std::string& e) { o += "  " + D + " = (uint64_t)(uint32_t)(" + e + ");\n"; };
  auto jmp = [&](const std::string& c) { o += "  if (" + c + ") " + tgt + "\n"; };
  auto guarded = [&](const std::string& addr, uint32_t size, const std::string& body) {
    o += "  { const uint64_t ad = " + addr + ";\n    if (!GX_GUARDS || !A.checked || guard_ok(A, " + std::to_string(pc) + "u, ad, " +
         std::to_string(size) + "u)) { " + body + " } }\n";
  };
  const std::string sgn_a = "(int64_t)" + D, sgn_b = "(int64_t)" + B;
  // window word holding this access, and the access's bit shift in it
  const int wa = pc < Wn.acc.size() ? Wn.acc[pc] : -1;
  const std::string wword =
      wa >= 0 ? "w" + std::to_string(wa) + "_" + std::to_string(Wn.off[pc] / 8) : std::string();
  const std::string wsh = wa >= 0 ? std::to_string(8 * (Wn.off[pc] % 8)) : std::string();
  // after a lookup with a window: the value's words, loaded together
  auto window_load = [&]() {
    const int w = pc < Wn.site.size() ? Wn.site[pc] : -1;
    if (w < 0 || !Wn.win[w].used) return;
    o += "  if (r0) {";
    for (uint32_t j = 0; j < Wn.win[w].words; j++)
      o += " w" + std::to_string(w) + "_" + std::to_string(j) + " = uni<UNI>(*(const GX_GLOBAL uint64_t*)(r0 + " +
           std::to_string(8 * j) + "ull));";
    o += " }\n";
  };
  const std::string sa32 = "(int32_t)" + xa, sb32 = "(int32_t)" + xb;
  // private frame: the frame word and bit shift of this slot's stack access
  const int32_t fb = Fr.priv && pc < Fr.at.size() ? Fr.at[pc] : -1;
  const std::string fw = fb >= 0 ? "f" + std::to_string(fb / 8) : std::string();
  const std::string fsh = fb >= 0 ? std::to_string(8 * (fb % 8)) : std::string();
  // a helper's stack arguments stored to the LDS frame first (key at r2 of
  // klen bytes, an update's value at r3 of vlen bytes)
  const int hk = J.index(u.imm);
  const uint32_t klen = hk >= 0 ? J.m[hk].second.key_size : 0, vlen = hk >= 0 ? J.m[hk].second.value_size : 0;
  auto spill_args = [&](uint32_t len2, uint32_t len3) {
    std::string t;
    if (Fr.priv && (a8 & 1) == PK_STACK && pc < Fr.at.size() && Fr.at[pc] >= 0) t += frame_spill(Fr.at[pc], len2);
    if (Fr.priv && len3 && ((a8 >> 1) & 1) == PK_STACK && pc < Fr.at3.size() && Fr.at3[pc] >= 0)
      t += frame_spill(Fr.at3[pc], len3);
    return t;
  };
  // the helper's r2 key as a value, when it is a frame word's bytes
  const std::string kval = Fr.priv && (a8 & 1) == PK_STACK && fb >= 0 ? frame_bytes(fb, klen) : std::string();
  // a write that may reach a memo's value other than through its window
  // (a written-back table is written back first), or a read of map memory
  // that a written-back table may hold newer words of
  if (pc < Wn.inval.size() && Wn.inval[pc])
    for (size_t w = 0; w < Wn.win.size(); w++)
      if ((Wn.inval[pc] >> w) & 1)
        o += std::string(Wn.wb[w] ? "  if (UNI) memo_flush" + std::to_string(w) + "();\n" : "") + "  mv" +
             std::to_string(w) + " = false; gen" + std::to_string(w) + "++;\n";
  if (pc < Wn.sync.size() && Wn.sync[pc])
    for (size_t w = 0; w < Wn.win.size(); w++)
      if ((Wn.sync[pc] >> w) & 1) o += "  if (UNI) memo_flush" + std::to_string(w) + "();\n";
  switch (h) {
    case H_ADD64: set(D + " + " + B); break;
    case H_SUB64: set(D + " - " + B); break;
    case H_MUL64: set(D + " * " + B); break;
    case H_DIV64: set(B + " ? " + D + " / " + B + " : 0ull"); break;
    case H_SDIV64:
      set("!" + B + " ? 0ull : (" + sgn_a + " == INT64_MIN && " + sgn_b + " == -1) ? " + D + " : (uint64_t)(" + sgn_a +
          " / " + sgn_b + ")");
      break;
    case H_OR64: set(D + " | " + B); break;
    case H_AND64: set(D + " & " + B); break;
    case H_LSH64: set(D + " << (" + B + " & 63)"); break;
    case H_RSH64: set(D + " >> (" + B + " & 63)"); break;
    case H_NEG64: set("0ull - " + D); break;
    case H_MOD64: set(B + " ? " + D + " % " + B + " : " + D); break;
    case H_SMOD64:
      set("!" + B + " ? " + D + " : (" + sgn_b + " == -1) ? 0ull : (uint64_t)(" + sgn_a + " % " + sgn_b + ")");
      break;
    case H_XOR64: set(D + " ^ " + B); break;
    case H_MOV64: set(B); break;
    case H_ARSH64: set("(uint64_t)(" + sgn_a + " >> (" + B + " & 63))"); break;
    case H_MOVSX64: set(extend(B, a8 == 8 ? 0 : a8 == 16 ? 1 : 2, true)); break;
    case H_BSWAP:
      if (a8 == 16) set("(uint64_t)__builtin_bswap16((uint16_t)" + D + ")");
      else if (a8 == 32) set("(uint64_t)__builtin_bswap32((uint32_t)" + D + ")");
      else set("__builtin_bswap64(" + D + ")");
      break;
    case H_TRUNC:
      if (a8 == 16) set(D + " & 0xffffull");
      else if (a8 == 32) set(D + " & 0xffffffffull");
      break;
    case H_ADD32: set32(xa + " + " + xb); break;
    case H_SUB32: set32(xa + " - " + xb); break;
    case H_MUL32: set32(xa + " * " + xb); break;
    case H_DIV32: set32(xb + " ? " + xa + " / " + xb + " : 0u"); break;
    case H_SDIV32:
      set32("!" + xb + " ? 0u : (" + sa32 + " == INT32_MIN && " + sb32 + " == -1) ? " + xa + " : (uint32_t)(" +
            sa32 + " / " + sb32 + ")");
      break;
    case H_OR32: set32(xa + " | " + xb); break;
    case H_AND32: set32(xa + " & " + xb); break;
    case H_LSH32: set32(xa + " << (" + xb + " & 31)"); break;
    case H_RSH32: set32(xa + " >> (" + xb + " & 31)"); break;
    case H_NEG32: set32("0u - " + xa); break;
    case H_MOD32: set32(xb + " ? " + xa + " % " + xb + " : " + xa); break;
    case H_SMOD32:
      set32("!" + xb + " ? " + xa + " : (" + sb32 + " == -1) ? 0u : (uint32_t)(" + sa32 + " % " + sb32 + ")");
      break;
    case H_XOR32: set32(xa + " ^ " + xb); break;
    case H_MOV32: set32(xb); break;
    case H_ARSH32: set32("(uint32_t)(" + sa32 + " >> (" + xb + " & 31))"); break;
    case H_MOVSX32: set32(extend(B, a8 == 8 ? 0 : 1, true)); break;
    case H_JA: o += "  " + tgt + "\n"; break;
    case H_JEQ: jmp(D + " == " + B); break;
    case H_JGT: jmp(D + " > " + B); break;
    case H_JGE: jmp(D + " >= " + B); break;
    case H_JSET: jmp("(" + D + " & " + B + ") != 0"); break;
    case H_JNE: jmp(D + " != " + B); break;
    case H_JSGT: jmp(sgn_a + " > " + sgn_b); break;
    case H_JSGE: jmp(sgn_a + " >= " + sgn_b); break;
    case H_JLT: jmp(D + " < " + B); break;
    case H_JLE: jmp(D + " <= " + B); break;
    case H_JSLT: jmp(sgn_a + " < " + sgn_b); break;
    case H_JSLE: jmp(sgn_a + " <= " + sgn_b); break;
    case H_JEQ32: jmp(xa + " == " + xb); break;
    case H_JGT32: jmp(xa + " > " + xb); break;
    case H_JGE32: jmp(xa + " >= " + xb); break;
    case H_JSET32: jmp("(" + xa + " & " + xb + ") != 0u"); break;
    case H_JNE32: jmp(xa + " != " + xb); break;
    case H_JSGT32: jmp(sa32 + " > " + sb32); break;
    case H_JSGE32: jmp(sa32 + " >= " + sb32); break;
    case H_JLT32: jmp(xa + " < " + xb); break;
    case H_JLE32: jmp(xa + " <= " + xb); break;
    case H_JSLT32: jmp(sa32 + " < " + sb32); break;
    case H_JSLE32: jmp(sa32 + " <= " + sb32); break;
    case H_LDX_CTX: {
      const uint32_t wi = (uint32_t)u.aux >> 3, sh = 8 * ((uint32_t)u.aux & 7);
      // words 3..5: the tile's aggregate (SIMT hook), wave-uniform
      std::string w = wi < 3 ? "(c" + std::to_string(wi) + " >> " + std::to_string(sh) + ")"
                             : "(uni<true>(g.c" + std::to_string(wi - 3) + ") >> " + std::to_string(sh) + ")";
      set(extend(std::string("(") + kTy[sc] + ")" + w, sc, sxf));
      break;
    }
    case H_LDX_STACK:
      if (fb >= 0)
        set(extend(std::string("(") + kTy[sc] + ")(" + fw + " >> " + fsh + ")", sc, sxf));
      else
        set("uni<UNI>(" + extend(std::string("*(const ") + kTy[sc] + "*)saddr(stk, (uint32_t)" + S + " + " + off + ")", sc, sxf) + ")");
      break;
    case H_LDX_MAP: {
      const int mk = pc < J.mem_map.size() ? J.mem_map[pc] : -1;
      const bool ro = mk >= 0 && mk < (int)J.m.size() && (J.m[mk].second.flags & F_READ_ONLY);
      if (ro) {
        // read-only map: constant for the launch, so when the wave reads one
        // address it is read with a scalar load, which does not wait behind
        // the wave's outstanding vector loads (they complete in order)
        guarded(S + " + (uint64_t)(int64_t)" + off, 1u << sc,
                D + " = " + extend(std::string("load_uniform<") + kTy[sc] + ">(ad)", sc, sxf) + ";");
      } else if (wa >= 0) {
        set(extend(std::string("(") + kTy[sc] + ")(" + wword + " >> " + wsh + ")", sc, sxf));
      } else {
        guarded(S + " + (uint64_t)(int64_t)" + off, 1u << sc,
                D + " = uni<UNI>(" + extend(std::string("*(const GX_GLOBAL ") + kTy[sc] + "*)ad", sc, sxf) + ");");
      }
      break;
    }
    case H_ST_STACK:
    case H_STX_STACK: {
      const std::string val = std::string("(") + kTy[sc] + ")" + (h == H_ST_STACK ? lit(u.imm) : S);
      if (fb >= 0)
        o += sc == 3 ? "  " + fw + " = (uint64_t)" + val + ";\n"
                     : "  " + fw + " = (" + fw + " & ~((uint64_t)(" + kTy[sc] + ")~0ull << " + fsh + ")) | ((uint64_t)" +
                           val + " << " + fsh + ");\n";
      else
        o += std::string("  *(") + kTy[sc] + "*)saddr(stk, (uint32_t)" + D + " + " + off + ") = " + val + ";\n";
      break;
    }
    case H_ST_MAP:
    case H_STX_MAP: {
      const std::string val = std::string("(") + kTy[sc] + ")" + (h == H_ST_MAP ? lit(u.imm) : S);
      std::string body = std::string("*(GX_GLOBAL ") + kTy[sc] + "*)ad = " + val + ";";
      if (wa >= 0) {
        const std::string local = sc == 3 ? " " + wword + " = (uint64_t)" + val + ";"
                                          : " " + wword + " = (" + wword + " & ~((uint64_t)(" + kTy[sc] +
                                                ")~0ull << " + wsh + ")) | ((uint64_t)" + val + " << " + wsh + ");";
        // a written-back table: the window's words are the value's newest
        body = Wn.wb[wa] ? "if (UNI) {" + local + " dy" + std::to_string(wa) + " = true; } else { " + body + local + " }"
                         : body + local;
      }
      guarded(D + " + (uint64_t)(int64_t)" + off, 1u << sc, body);
      break;
    }
    case H_ATOMIC_STACK:
    case H_ATOMIC_MAP: {
      const uint32_t op = (uint32_t)u.imm;
      std::string call = h == H_ATOMIC_STACK
                             ? "atomic_stack(saddr(stk, (uint32_t)" + D + " + " + off + "), " + S + ", " +
                                   std::to_string(op) + "u, " + std::to_string(sc) + ", r0)"
                             : "atomic_global(ad, " + S + ", " + std::to_string(op) + "u, " + std::to_string(sc) +
                                   ", r0)";
      std::string wb = op == 0xf1 ? "r0 = t;" : (op & 1) ? S + " = t;" : "(void)t;";
      const int mk = pc < J.mem_map.size() ? J.mem_map[pc] : -1;
      const Acc* ac = (h == H_ATOMIC_MAP && mk >= 0 && mk < (int)J.acc.size() && J.acc[mk].kind) ? &J.acc[mk] : nullptr;
      if (h == H_ATOMIC_STACK && fb >= 0) {
        o += "  { const uint64_t t = frame_rmw(" + fw + ", " + fsh + "u, " + S + ", " + std::to_string(op) + "u, " +
             std::to_string(sc) + ", r0); " + wb + " }\n";
      } else if (h == H_ATOMIC_STACK) {
        o += "  { const uint64_t t = uni<UNI>(" + call + "); " + wb + " }\n";
      } else if (ac) {
        // shared map: summed in LDS by the event-parallel kernel
        const std::string T = ac->word_type(), K = std::to_string(mk);
        const std::string ops = std::to_string(ac->op) + "u";
        const std::string sets = std::to_string(ac->words / kCacheSlotsPerSet) + "u";
        const std::string tg = ac->tag8 ? "true" : "false";
        // the update of word a_ by x_ in the block's LDS accumulator
        const std::string lds =
            ac->kind == 1 ? "lds_rmw<" + T + ">(&g_acc" + K + "[(a_ - (uint64_t)(uintptr_t)M" + K + ".data) >> " +
                                std::to_string(ac->sc) + "], (" + T + ")x_, " + ops + ");"
            : ac->narrow ? "cache_add_narrow<" + tg + ">(g_tag" + K + ", g_val" + K + ", " + sets + ", M" + K +
                               ".data, a_, x_, nmax);"
                         : "cache_rmw<" + T + ", " + tg + ">(g_tag" + K + ", g_val" + K + ", " + sets + ", M" + K +
                               ".data, a_, (" + T + ")x_, " + ops + ");";
        // lanes of the wave that update one word are combined first (one
        // LDS atomic per distinct word instead of one per lane)
        const std::string fn = "auto acc_ = [&](uint64_t a_, uint64_t x_) { " + lds + " }; ";
        const std::string priv = agg_lds() || J.simt ? fn + "if (wave_aggregate(ad, (uint64_t)" + S + ", " + ops + ", acc_)) acc_(ad, (uint64_t)" + S + ");"
                                         : fn + "acc_(ad, (uint64_t)" + S + ");";
        const std::string cmb = mk >= 0 && mk < (int)J.comb.size() && J.comb[mk].first >= 0
                                    ? "if (UNI) { comb" + std::to_string(mk) + "(ad, (uint64_t)" + S + "); } else "
                                    : std::string();
        guarded(D + " + (uint64_t)(int64_t)" + off, 1u << sc,
                "if (PRIV) { " + priv + " } else " + cmb + "{ const uint64_t t = uni<UNI>(" + call + "); " + wb + " }");
      } else if (h == H_ATOMIC_MAP && mk >= 0 && mk < (int)J.comb.size() && J.comb[mk].first >= 0) {
        guarded(D + " + (uint64_t)(int64_t)" + off, 1u << sc,
                "if (UNI && !PRIV) { comb" + std::to_string(mk) + "(ad, (uint64_t)" + S + "); } else { const uint64_t t = uni<UNI>(" +
                    call + "); " + wb + " }");
      } else {
        guarded(D + " + (uint64_t)(int64_t)" + off, 1u << sc, "const uint64_t t = uni<UNI>(" + call + "); " + wb);
      }
      break;
    }
    case H_LDIMM:
      // a map reference only reaches helper calls, which name the map by
      // index; the handle's value is left out so that the source holds no
      // address of this instance's maps
      if (pc < J.ld_map.size() && J.ld_map[pc] >= 0)
        set(std::to_string(J.ld_map[pc]) + "ull /* map */");
      else
        set(lit(u.imm));
      break;
    case H_LOOKUP_ARRAY:
      if (!kval.empty())
        o += "  r0 = uni<UNI>(array_lookup_idx(" + M + ", (uint32_t)" + kval + "));\n";
      else
        o += "  " + spill_args(4, 0) + "r0 = uni<UNI>(array_lookup(" + M + ", " + std::to_string(a8 & 1) + ", r2, stk));\n";
      window_load();
      break;
    case H_LOOKUP_HASH: {
      const int w = pc < Wn.site.size() ? Wn.site[pc] : -1;
      const bool kv = !kval.empty() && klen <= 8 && hk >= 0 && J.m[hk].second.sstride == 16;
      const std::string call =
          kv ? "r0 = uni<UNI>(hash_lookup_k(" + M + ", " + kval + ", A.epoch));"
             : spill_args(klen, 0) + "r0 = uni<UNI>(hash_lookup(" + M + ", " + std::to_string(a8 & 1) + ", r2, stk, A.epoch));";
      if (w >= 0 && Wn.memo[w]) {
        const std::string W = std::to_string(w);
        const int km = J.index(u.imm);
        const uint32_t nw = Wn.win[w].words;
        const std::string S = std::to_string(3 + nw);
        if (!kval.empty())
          o += "  { const uint64_t mk = uni<UNI>(" + kval + ");\n";
        else
          o += "  { " + spill_args(klen, 0) + "const uint64_t mk = uni<UNI>(gx::chunk(" + std::to_string(a8 & 1) +
               ", r2, 0, " + std::to_string(J.m[km].second.key_size) + "u, stk));\n";
        // one queue per wave: the last key's entry in registers, in front of
        // the LDS table; the table entry of a key is written back when the
        // registers move on to another key (window stores touch registers only)
        if (Wn.table[w]) {
          const bool used = Wn.win[w].used;
          o += "    if (UNI) {\n      if (mv" + W + " && mk == mk" + W + ") {\n        r0 = mp" + W + ";\n      } else {\n";
          const bool wbk = Wn.wb[w];
          if (used) {
            o += "        if (mv" + W + ") {";
            for (uint32_t j = 0; j < nw; j++)
              o += " g_memo" + W + "[cur" + W + " * " + S + "u + " + std::to_string(3 + j) + "u] = w" + W + "_" +
                   std::to_string(j) + ";";
            if (wbk)
              o += " g_memo" + W + "[cur" + W + " * " + S + "u + 2u] = gen" + W + " | ((uint64_t)dy" + W + " << 63); dm" +
                   W + " = dy" + W + " ? dm" + W + " | (1ull << cur" + W + ") : dm" + W + " & ~(1ull << cur" + W + ");";
            o += " }\n";
          }
          o += "        const uint32_t me = ((uint32_t)mk ^ (uint32_t)(mk >> 32)) & " + std::to_string(kMemoEntries - 1) +
               "u;\n        uint64_t* ent = &g_memo" + W + "[me * " + S + "u];\n        cur" + W + " = me;\n";
          // the whole entry in one burst of LDS reads, then the checks
          const uint32_t rd = used ? 3 + nw : 3;
          o += "        uint64_t ev[" + std::to_string(rd) + "];\n        for (uint32_t i = 0; i < " + std::to_string(rd) +
               "u; i++) ev[i] = uni<UNI>(ent[i]);\n";
          const std::string g2 = wbk ? "(ev[2] & kMemoGen)" : "ev[2]";
          o += "        if (" + g2 + " == gen" + W + " && ev[0] == mk) {\n          r0 = ev[1];";
          for (uint32_t j = 0; j < nw && used; j++)
            o += " w" + W + "_" + std::to_string(j) + " = ev[" + std::to_string(3 + j) + "];";
          if (wbk) o += " dy" + W + " = (ev[2] >> 63) != 0;";
          o += "\n        } else {\n";
          if (wbk) {
            // the entry's current key, if its words are newer than memory
            o += "        if ((ev[2] & kMemoGen) == gen" + W + " && (ev[2] >> 63)) {";
            for (uint32_t j = 0; j < nw; j++)
              o += " *(GX_GLOBAL uint64_t*)(ev[1] + " + std::to_string(8 * j) + "ull) = ev[" + std::to_string(3 + j) + "];";
            o += " }\n        dy" + W + " = false; dm" + W + " &= ~(1ull << me);\n";
          }
          o += "        " + call + "\n      ";
          window_load();
          o += "          ent[0] = mk; ent[1] = r0; ent[2] = r0 ? gen" + W + " : 0;";
          for (uint32_t j = 0; j < nw && used; j++)
            o += " ent[" + std::to_string(3 + j) + "] = w" + W + "_" + std::to_string(j) + ";";
          o += "\n        }\n        mk" + W + " = mk; mp" + W + " = r0; mv" + W + " = r0 != 0;\n      }\n    } else {\n";
        }
        // several queues per wave, or no table: one entry per lane, in registers
        o += "    if (mv" + W + " && mk == mk" + W + ") {\n      r0 = mp" + W + ";\n    } else {\n    " + call + "\n  ";
        window_load();
        o += "    mk" + W + " = mk; mp" + W + " = r0; mv" + W + " = r0 != 0;\n    }\n" +
             std::string(Wn.table[w] ? "    }\n" : "") + "  }\n";
      } else {
        o += "  " + call + "\n";
        window_load();
      }
      break;
    }
    case H_UPDATE_ARRAY:
      o += "  " + spill_args(4, vlen) + "r0 = uni<UNI>((uint64_t)array_update(" + M + ", " + std::to_string(a8 & 1) +
           ", r2, " + std::to_string((a8 >> 1) & 1) + ", r3, r4, stk));\n";
      break;
    case H_UPDATE_HASH:
      o += "  " + spill_args(klen, vlen) + "r0 = uni<UNI>((uint64_t)hash_update(" + M + ", " + std::to_string(a8 & 1) +
           ", r2, " + std::to_string((a8 >> 1) & 1) + ", r3, r4, stk, A.epoch));\n";
      break;
    case H_DELETE_HASH:
      o += "  " + spill_args(klen, 0) + "r0 = uni<UNI>((uint64_t)hash_delete(" + M + ", " + std::to_string(a8 & 1) +
           ", r2, stk, A.epoch));\n";
      break;
    case H_RET_EINVAL: o += "  r0 = (uint64_t)-22ll;\n"; break;
    case H_RINGBUF_OUTPUT: {
      const int k = J.index(u.imm);
      const uint32_t size = (uint32_t)u.aux;
      // a record in the private frame, word-aligned, of at most 64 bytes:
      // its words go to the helper by value (no stack memory is read)
      if (k >= 0 && J.ring[k] >= 0 && Fr.priv && (a8 & 1) == PK_STACK && fb >= 0 && fb % 8 == 0 && size <= 64) {
        o += "  { RecVal rv_{};";
        for (uint32_t j = 0; j < (size + 7) / 8; j++)
          o += " rv_.w[" + std::to_string(j) + "] = f" + std::to_string(fb / 8 + j) + ";";
        o += "\n    r0 = uni<UNI>(ring_output_words(" + M + ", wave * GX_NRINGS + " + std::to_string(J.ring[k]) + "u, " +
             std::to_string(J.ring[k]) + "u, chunk[" + std::to_string(J.ring[k]) + "], bchunk[" +
             std::to_string(J.ring[k]) + "], rv_, " + std::to_string(size) + "u, r4)); }\n";
        break;
      }
      o += "  " + spill_args((uint32_t)u.aux, 0) + "\n";
      if (k >= 0 && J.ring[k] >= 0)
        o += "  r0 = uni<UNI>(ring_output_chunked(" + M + ", wave * GX_NRINGS + " + std::to_string(J.ring[k]) + "u, " +
             std::to_string(J.ring[k]) + "u, chunk[" + std::to_string(J.ring[k]) + "], bchunk[" +
             std::to_string(J.ring[k]) + "], " + std::to_string(a8 & 1) + ", r2, " + std::to_string((uint32_t)u.aux) +
             "u, r4, stk));\n";
      else
        o += "  r0 = uni<UNI>(ring_output(" + M + ", " + std::to_string(a8 & 1) + ", r2, " +
             std::to_string((uint32_t)u.aux) + "u, r4, true, stk));\n";
      break;
    }
    case H_EXIT:
    default: o += "  return (uint32_t)r0;\n"; break;
  }
}

bool is_jump(uint32_t h) { return h >= H_JA && h <= H_JSLE32; }

}  // namespace

uint32_t jit_waves(uint32_t stack_bytes, bool event_parallel) {
  if (!event_parallel) return 1;
  uint32_t w = kJitMaxWaves;
  while (w > 1 && (uint64_t)w * 64 * stack_bytes > (64u << 10)) w /= 2;
  return w;
}

namespace {

// One program's part of a source, in namespace gx::<ns>: map descriptor
// functions, LDS accumulators (when ``allow_acc``) and struct Prog<PRIV>
// with begin / end / run.  ``lds_used``: LDS the kernel already takes.
std::string emit_prog(const JitProg& P, const std::string& ns, bool allow_acc, uint64_t lds_used,
                      JitInfo* info) {
  const std::vector<Uop>& U = *P.U;
  const auto& maps = *P.maps;
  JMaps J(maps, *P.mem_map, *P.ld_map);
  J.simt = P.simt;
  std::vector<char> target(U.size() + 1, 0);
  for (const Uop& u : U)
    if (is_jump(u.w0 & 0xff) && (uint32_t)u.aux < target.size()) target[(uint32_t)u.aux] = 1;
  if (allow_acc) J.plan(U, lds_used);
  // spill layout of the caches, per launch of nb blocks: cache k's tags
  // [sets][nb][4] (u32), then its slots [sets][nb][4]; cache k starts at
  // nb * spill_off[k].  Every cache needs a reduce LDS array of
  // ceil(map words / sets) words, at most kReduceMax.
  std::vector<uint64_t> spill_off(maps.size(), 0);
  uint64_t spill_block = 0;
  uint32_t red_blocks = 0;
  bool spill = allow_acc;
  for (size_t k = 0; k < maps.size(); k++) {
    const Acc& a = J.acc[k];
    if (a.kind != 2) continue;
    const uint64_t sets = a.words / kCacheSlotsPerSet;
    const uint64_t words = (uint64_t)maps[k].second.max_entries * maps[k].second.vstride / (a.sc == 3 ? 8 : 4);
    if ((words + sets - 1) / sets > kReduceMax) spill = false;
    spill_off[k] = spill_block;
    spill_block += (a.tag8 ? sets : a.words) * 4 + (uint64_t)a.words * (a.slot_type() == "uint64_t" ? 8 : 4);
    red_blocks += (uint32_t)sets;
  }
  if (!spill) spill_block = red_blocks = 0;
  if (info) {
    info->acc_words = 0;
    for (const Acc& a : J.acc)
      if (a.kind) info->acc_words += a.words;
    info->spill_block_bytes = spill_block;
    info->reduce_blocks = red_blocks;
  }
  std::string o = "namespace gx {\nnamespace " + ns + " {\n\n";
  for (size_t k = 0; k < maps.size(); k++) o += map_fn(k, maps[k].second);
  bool any_acc = false;
  for (size_t k = 0; k < maps.size(); k++) {
    const Acc& a = J.acc[k];
    if (!a.kind) continue;
    any_acc = true;
    const std::string T = a.word_type(), K = std::to_string(k), N = std::to_string(a.words);
    if (a.kind == 1)
      o += "__shared__ " + T + " g_acc" + K + "[" + N + "];\n";
    else
      o += "__shared__ __attribute__((aligned(16))) uint32_t g_tag" + K + "[" +
           std::to_string(a.tag8 ? a.words / kCacheSlotsPerSet : a.words) + "];\n__shared__ " + a.slot_type() +
           " g_val" + K + "[" + N + "];\n";
  }
  Windows Wn = plan_windows(U, J);
  const Frame Fr = plan_frame(U, P.stack_bytes);
  // shared maps' atomics in one-lane (UNI) runs: combined per wave in a few
  // registers (map -> {op, width}; -1: none)
  std::vector<std::pair<int, int>> comb(maps.size(), {-1, 0});
  for (uint32_t pc = 0; pc < U.size(); pc++) {
    if ((U[pc].w0 & 0xff) == H_LDIMM) {
      pc++;
      continue;
    }
    if ((U[pc].w0 & 0xff) != H_ATOMIC_MAP) continue;
    const int mk = pc < J.mem_map.size() ? J.mem_map[pc] : -1;
    const uint32_t op = (uint32_t)U[pc].imm;
    if (mk < 0 || mk >= (int)maps.size() || !(maps[mk].second.flags & F_SHARED) || (op & 1)) continue;
    comb[mk] = {(int)(op & 0xf0), (int)((U[pc].w0 >> 16) & 3)};
  }
  J.comb = comb;
  // a program set's kernel would hold every member's tables at once: there
  // each lane keeps one entry in registers
  plan_memo(U, J, Wn, P.event_parallel, allow_acc);
  for (size_t w = 0; w < Wn.win.size(); w++)
    if (Wn.table[w])
      o += "__shared__ __attribute__((aligned(16))) uint64_t g_memo" + std::to_string(w) + "[" +
           std::to_string(kMemoEntries * (3 + Wn.win[w].words)) + "];\n";
  // PRIV: the event-parallel kernel sums shared-map atomics in LDS
  // UNI: run by one lane with wave-uniform values (one queue per wave)
  o += "\ntemplate <bool PRIV, bool UNI = false>\nstruct Prog {\n  uint32_t wave;  // wave index in the block: selects its ring chunks\n"
       "  uint64_t chunk[GX_NRINGS];  // bytes of ring space a wave takes at once, per ring\n"
       "  uint64_t bchunk[GX_NRINGS];  // bytes of ring space the block reserves at once, per ring\n";
  // the maps' descriptors, read from the map table once per run (they stay
  // in scalar registers instead of being reloaded for every event)
  for (size_t k = 0; k < maps.size(); k++) o += "  MapDev m" + std::to_string(k) + ";\n";
  // narrow caches: updates per invocation (every site once without loops,
  // else the verifier's instruction bound) and the addend bound it gives
  uint64_t narrow_sites = 0;
  bool loops = false;
  for (uint32_t pc = 0; pc < U.size(); pc++) {
    const uint32_t h = U[pc].w0 & 0xff;
    if (h == H_LDIMM) {
      pc++;
      continue;
    }
    if (is_jump(h) && (uint32_t)U[pc].aux <= pc) loops = true;
    const int mk = pc < J.mem_map.size() ? J.mem_map[pc] : -1;
    if (h == H_ATOMIC_MAP && mk >= 0 && mk < (int)J.acc.size() && J.acc[mk].kind == 2 && J.acc[mk].narrow)
      narrow_sites++;
  }
  const uint64_t per_inv = loops ? std::max<uint64_t>(P.max_insns, 1) : std::max<uint64_t>(narrow_sites, 1);
  if (narrow_sites) o += "  uint32_t nmax = 0;  // largest addend the narrow caches sum in LDS\n";
  // combiners: a one-lane run's updates of a shared map word gather in
  // registers (kCombSlots words, replaced round robin) and reach the map as
  // one device atomic per word when replaced or at the end; only atomics
  // touch a shared map's values, so nothing in the run can see the delay
  for (size_t k = 0; k < maps.size(); k++) {
    if (comb[k].first < 0) continue;
    const std::string K = std::to_string(k), OP = std::to_string(comb[k].first) + "u",
                      SC = std::to_string(comb[k].second);
    for (uint32_t j = 0; j < kCombSlots; j++)
      o += "  uint64_t ca" + K + "_" + std::to_string(j) + " = 0, cv" + K + "_" + std::to_string(j) + " = 0;\n";
    o += "  uint32_t cr" + K + " = 0;\n";
    o += "  __device__ __forceinline__ void comb" + K + "(uint64_t a, uint64_t x) {\n";
    for (uint32_t j = 0; j < kCombSlots; j++) {
      const std::string J2 = K + "_" + std::to_string(j);
      o += "    if (a == ca" + J2 + ") { cv" + J2 + " = agg_apply(cv" + J2 + ", x, " + OP + "); return; }\n";
    }
    o += "    switch (cr" + K + ") {\n";
    for (uint32_t j = 0; j < kCombSlots; j++) {
      const std::string J2 = K + "_" + std::to_string(j);
      o += "      case " + std::to_string(j) + "u: if (ca" + J2 + ") (void)atomic_global(ca" + J2 + ", cv" + J2 + ", " + OP +
           ", " + SC + ", 0); ca" + J2 + " = a; cv" + J2 + " = x; break;\n";
    }
    o += "    }\n    cr" + K + " = (cr" + K + " + 1u) % " + std::to_string(kCombSlots) + "u;\n  }\n";
  }
  // lookup memos: last key found, its value's address, the window's words;
  // with one queue per wave, the LDS table's generation and current entry
  for (size_t w = 0; w < Wn.win.size(); w++) {
    if (!Wn.memo[w]) continue;
    const std::string W = std::to_string(w);
    o += "  uint64_t mk" + W + " = 0, mp" + W + " = 0, gen" + W + " = 1;\n  bool mv" + W + " = false;\n  uint32_t cur" +
         W + " = 0;\n";
    if (Wn.wb[w])
      o += "  bool dy" + W + " = false;  // the registers' window is newer than memory\n  uint64_t dm" + W +
           " = 0;  // table slots whose words are newer than memory\n";
    for (uint32_t j = 0; j < Wn.win[w].words; j++) o += "  uint64_t w" + W + "_" + std::to_string(j) + " = 0;\n";
  }
  o += "\n";
  // write-back tables: write every entry whose words are newer than memory
  // back to the map (one lane, in the middle of a run, visiting only the
  // slots the dirty mask names; end() does it with one lane per entry)
  for (size_t w = 0; w < Wn.win.size(); w++) {
    if (!Wn.wb[w]) continue;
    const std::string W = std::to_string(w), S = std::to_string(3 + Wn.win[w].words);
    o += "  __device__ __forceinline__ void memo_flush" + W + "() {\n    if (mv" + W + ") {";
    for (uint32_t j = 0; j < Wn.win[w].words; j++)
      o += " g_memo" + W + "[cur" + W + " * " + S + "u + " + std::to_string(3 + j) + "u] = w" + W + "_" + std::to_string(j) + ";";
    o += " g_memo" + W + "[cur" + W + " * " + S + "u + 2u] = gen" + W + " | ((uint64_t)dy" + W + " << 63); dm" + W +
         " = dy" + W + " ? dm" + W + " | (1ull << cur" + W + ") : dm" + W + " & ~(1ull << cur" + W + "); }\n    dy" + W +
         " = false;\n    for (uint64_t d = dm" + W + "; d; d &= d - 1) memo_writeback" + W +
         "((uint32_t)__builtin_ctzll(d));\n    dm" + W + " = 0;\n  }\n";
    o += "  __device__ __forceinline__ void memo_writeback" + W + "(uint32_t e) {\n    uint64_t* ent = &g_memo" + W +
         "[e * " + S + "u];\n    const uint64_t g = ent[2];\n    if ((g & kMemoGen) == gen" + W +
         " && (g >> 63)) {\n";
    for (uint32_t j = 0; j < Wn.win[w].words; j++)
      o += "      *(GX_GLOBAL uint64_t*)(ent[1] + " + std::to_string(8 * j) + "ull) = ent[" + std::to_string(3 + j) + "];\n";
    o += "      ent[2] = g & kMemoGen;\n    }\n  }\n";
  }
  // begin / end: open and close the wave's and the block's ring chunks and
  // the block's accumulators (wave 0 sets up the block's part; the barrier
  // makes it visible to the other waves).
  o += "  __device__ __forceinline__ void begin(const RunArgs& A) {\n    (void)A;\n";
  o += "    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64u);\n    (void)waves;\n";
  for (size_t k = 0; k < maps.size(); k++) o += "    m" + std::to_string(k) + " = gx_map" + std::to_string(k) + "(A);\n";
  for (size_t k = 0; k < maps.size(); k++)
    if (J.ring[k] >= 0)
      o += "    chunk[" + std::to_string(J.ring[k]) + "] = ring_chunk_bytes(" + std::to_string(J.ring_cap((int)k)) +
           "ull, waves);\n    bchunk[" + std::to_string(J.ring[k]) + "] = ring_block_bytes(" +
           std::to_string(J.ring_cap((int)k)) + "ull, gridDim.x);\n";
  for (int r = 0; r < J.n_rings; r++)
    o += "    ring_chunk_init(wave * GX_NRINGS + " + std::to_string(r) + "u);\n    if (wave == 0) ring_block_init(" +
         std::to_string(r) + "u);\n";
  if (J.n_rings) o += "    __syncthreads();\n";
  for (size_t w = 0; w < Wn.win.size(); w++)
    if (Wn.table[w])
      o += "    if (UNI) g_memo" + std::to_string(w) + "[lane_id() * " + std::to_string(3 + Wn.win[w].words) +
           "u + 2u] = 0;  // no entry is current\n";
  if (any_acc) {
    o += "    if (PRIV) {\n";
    for (size_t k = 0; k < maps.size(); k++) {
      const Acc& a = J.acc[k];
      const std::string T = a.sc == 3 ? "uint64_t" : "uint32_t", K = std::to_string(k);
      if (a.kind == 1)
        o += "      mirror_init<" + T + ">(g_acc" + K + ", " + std::to_string(a.words) + "u, " + std::to_string(a.op) +
             "u);\n";
      else if (a.kind == 2)
        o += "      cache_init<" + a.slot_type() + ", " + (a.tag8 ? "true" : "false") + ">(g_tag" + K + ", g_val" + K + ", " +
             std::to_string(a.words / kCacheSlotsPerSet) + "u, " + std::to_string(a.op) + "u);\n";
    }
    if (narrow_sites) o += "      nmax = narrow_vmax(A.n_events, " + std::to_string(per_inv) + "ull);\n";
    o += "      __syncthreads();\n    }\n";
  }
  o += "  }\n  __device__ __forceinline__ void end(const RunArgs& A) {\n    (void)A;\n";
  for (size_t k = 0; k < maps.size(); k++) {
    if (comb[k].first < 0) continue;
    const std::string K = std::to_string(k);
    o += "    if (UNI && !PRIV) {\n";
    for (uint32_t j = 0; j < kCombSlots; j++) {
      const std::string J2 = K + "_" + std::to_string(j);
      o += "      { const uint64_t a = rfl64(ca" + J2 + "), x = rfl64(cv" + J2 + "); if (a && lane_id() == 0) (void)atomic_global(a, x, " +
           std::to_string(comb[k].first) + "u, " + std::to_string(comb[k].second) + ", 0); ca" + J2 + " = 0; }\n";
    }
    o += "    }\n";
  }
  // the one-queue kernel's written-back tables: the registers' entry into
  // its table slot, then each lane writes back one slot
  for (size_t w = 0; w < Wn.win.size(); w++) {
    if (!Wn.wb[w]) continue;
    const std::string W = std::to_string(w), S = std::to_string(3 + Wn.win[w].words);
    o += "    if (UNI) {\n      if (mv" + W + ") {";
    for (uint32_t j = 0; j < Wn.win[w].words; j++)
      o += " g_memo" + W + "[cur" + W + " * " + S + "u + " + std::to_string(3 + j) + "u] = w" + W + "_" + std::to_string(j) + ";";
    o += " g_memo" + W + "[cur" + W + " * " + S + "u + 2u] = gen" + W + " | ((uint64_t)dy" + W + " << 63); }\n      memo_writeback" +
         W + "(lane_id());\n    }\n";
  }
  for (size_t k = 0; k < maps.size(); k++)
    if (J.ring[k] >= 0)
      o += "    ring_chunk_close(&m" + std::to_string(k) + ", wave * GX_NRINGS + " + std::to_string(J.ring[k]) + "u);\n";
  if (J.n_rings) {
    o += "    __syncthreads();\n";
    for (size_t k = 0; k < maps.size(); k++)
      if (J.ring[k] >= 0)
        o += "    if (wave == 0) ring_block_close(&m" + std::to_string(k) + ", " + std::to_string(J.ring[k]) + "u);\n";
  }
  if (any_acc) {
    o += "    if (PRIV) {\n      __syncthreads();\n";
    for (size_t k = 0; k < maps.size(); k++) {
      const Acc& a = J.acc[k];
      const std::string T = a.sc == 3 ? "uint64_t" : "uint32_t", K = std::to_string(k);
      const std::string tg = a.tag8 ? "true" : "false";
      if (a.kind == 1)
        o += "      mirror_flush<" + T + ">(g_acc" + K + ", " + std::to_string(a.words) + "u, " + std::to_string(a.op) +
             "u, m" + K + ".data);\n";
      else if (a.kind == 2 && spill_block)
        o += "      if (A.spill) cache_spill<" + a.slot_type() + ", " + tg + ">(g_tag" + K + ", g_val" + K + ", " +
             std::to_string(a.words / kCacheSlotsPerSet) + "u, A.spill + (uint64_t)gridDim.x * " +
             std::to_string(spill_off[k]) + "ull, blockIdx.x, gridDim.x);\n      else cache_flush<" + T + ", " +
             a.slot_type() + ", " + tg + ">(g_tag" + K + ", g_val" + K + ", " + std::to_string(a.words / kCacheSlotsPerSet) +
             "u, " + std::to_string(a.op) + "u, m" + K + ".data);\n";
      else if (a.kind == 2)
        o += "      cache_flush<" + T + ", " + a.slot_type() + ", " + tg + ">(g_tag" + K + ", g_val" + K + ", " +
             std::to_string(a.words / kCacheSlotsPerSet) + "u, " + std::to_string(a.op) + "u, m" + K + ".data);\n";
    }
    o += "    }\n";
  }
  o += "  }\n\n";
  // after lane 0 ran a block of events with the other lanes idle: its memo
  // state, read from lane 0, so that the compiler keeps it wave-uniform
  o += "  __device__ __forceinline__ void uniformize() {\n";
  for (size_t k = 0; k < maps.size(); k++) {
    if (comb[k].first < 0) continue;
    const std::string K = std::to_string(k);
    for (uint32_t j = 0; j < kCombSlots; j++) {
      const std::string J2 = K + "_" + std::to_string(j);
      o += "    ca" + J2 + " = rfl64(ca" + J2 + ");\n    cv" + J2 + " = rfl64(cv" + J2 + ");\n";
    }
    o += "    cr" + K + " = __builtin_amdgcn_readfirstlane(cr" + K + ");\n";
  }
  for (size_t w = 0; w < Wn.win.size(); w++) {
    if (!Wn.memo[w]) continue;
    const std::string W = std::to_string(w);
    o += "    mk" + W + " = rfl64(mk" + W + ");\n    mp" + W + " = rfl64(mp" + W + ");\n    gen" + W + " = rfl64(gen" +
         W + ");\n    mv" + W + " = __builtin_amdgcn_readfirstlane((int)mv" + W + ") != 0;\n    cur" + W +
         " = __builtin_amdgcn_readfirstlane(cur" + W + ");\n";
    if (Wn.wb[w])
      o += "    dy" + W + " = __builtin_amdgcn_readfirstlane((int)dy" + W + ") != 0;\n    dm" + W + " = rfl64(dm" + W + ");\n";
    for (uint32_t j = 0; j < Wn.win[w].words; j++) {
      const std::string nm = "w" + W + "_" + std::to_string(j);
      o += "    " + nm + " = rfl64(" + nm + ");\n";
    }
  }
  o += "  }\n\n";
  o += "  __device__ __forceinline__ uint32_t run(const RunArgs& A, bool live, uint64_t c0, uint64_t c1, uint64_t c2, "
       "const Ctx& g, const Stk stk, uint64_t& steps) {\n  (void)g;\n";
  o += "  (void)c0; (void)c1; (void)c2; (void)steps;\n  if (!live) return 0;\n";
  o += "  if (UNI) { c0 = rfl64(c0); c1 = rfl64(c1); c2 = rfl64(c2); }\n";
  o += "  uint64_t r0 = 0, r1 = 0, r2 = 0, r3 = 0, r4 = 0, r5 = 0, r6 = 0, r7 = 0, r8 = 0, r9 = 0;\n";
  o += "  uint64_t r10 = " + std::to_string(P.stack_bytes) + "ull;\n";
  for (size_t k = 0; k < maps.size(); k++)
    o += "  const MapDev& M" + std::to_string(k) + " = m" + std::to_string(k) + ";\n";
  o += "  (void)r1; (void)r3; (void)r4; (void)r5; (void)r6; (void)r7; (void)r8; (void)r9; (void)r10;\n";
  for (size_t w = 0; w < Wn.win.size(); w++)
    for (uint32_t j = 0; j < Wn.win[w].words && !Wn.memo[w]; j++) {
      const std::string nm = "w" + std::to_string(w) + "_" + std::to_string(j);
      o += "  uint64_t " + nm + " = 0; (void)" + nm + ";\n";
    }
  if (Fr.priv) {
    o += "  uint64_t";
    for (uint32_t w = 0; w < P.stack_bytes / 8; w++) o += std::string(w ? "," : "") + " f" + std::to_string(w) + " = 0";
    o += ";  // the frame's words (private frame)\n";
  }
  for (uint32_t pc = 0; pc < U.size(); pc++) {
    if (target[pc]) o += "L" + std::to_string(pc) + ":;\n";
    emit_uop(o, U[pc], pc, J, Wn, Fr);
    if ((U[pc].w0 & 0xff) == H_LDIMM) pc++;  // second slot of lddw
  }
  o += "  return (uint32_t)r0;\n  }\n};\n\n";
  if (spill_block) {
    // one block of gx_j_reduce per cache set
    o += "__device__ __forceinline__ void reduce(const RunArgs& A, uint32_t nb) {\n  uint32_t b = blockIdx.x;\n";
    for (size_t k = 0; k < maps.size(); k++) {
      const Acc& a = J.acc[k];
      if (a.kind != 2) continue;
      const uint64_t sets = a.words / kCacheSlotsPerSet;
      const uint64_t words = (uint64_t)maps[k].second.max_entries * maps[k].second.vstride / (a.sc == 3 ? 8 : 4);
      const std::string S = std::to_string(sets) + "u", K = std::to_string(k);
      o += "  if (b < " + S + ") {\n    cache_reduce<" + a.word_type() + ", " + a.slot_type() + ", " +
           std::to_string((words + sets - 1) / sets) + "u, " + (a.tag8 ? "true" : "false") +
           ">(A.spill + (uint64_t)nb * " + std::to_string(spill_off[k]) +
           "ull, " + S + ", b, nb, " + std::to_string(a.op) + "u, gx_map" + K + "(A).data, " + std::to_string(words) +
           "u);\n    return;\n  }\n  b -= " + S + ";\n";
    }
    o += "}\n\n";
  }
  o += "}  // namespace " + ns + "\n}  // namespace gx\n\n";
  return o;
}

// The event-parallel kernel's tile loop: records of GX_EP_AHEAD tiles (1 to
// 7, default 4) loaded ahead of the running one, or none (0).  Latency
// histogram, 2^26 events: 420 / 382 / 368 / 363 / 361 / 363 us for 1, 2, 3,
// 4, 5 and 7 tiles ahead (each depth is one more inlined copy of the
// program).
std::string ahead_loop() {
  const int a = std::min(7, std::max(0, env_int_jit("GX_EP_AHEAD", 4)));
  return a ? "event_loop_ahead<" + std::to_string(a) + ">" : std::string("event_loop");
}

// Whether generated code uses the LDS frames: any mention of stk besides
// the parameter declarations ("const Stk stk").
bool reads_stack(const std::string& body) {
  size_t uses = 0, decls = 0;
  for (size_t at = body.find("stk"); at != std::string::npos; at = body.find("stk", at + 3)) {
    const bool word = (at == 0 || !(std::isalnum((unsigned char)body[at - 1]) || body[at - 1] == '_')) &&
                      (at + 3 >= body.size() || !(std::isalnum((unsigned char)body[at + 3]) || body[at + 3] == '_'));
    if (!word) continue;
    uses++;
    if (at >= 10 && body.compare(at - 10, 10, "const Stk ") == 0) decls++;
  }
  return uses > decls;
}

int ring_count(const JitProg& P) {
  int n = 0;
  for (auto& m : *P.maps) n += m.second.type == MAP_RINGBUF;
  return n;
}

}  // namespace

std::string jit_source(const JitProg& P, JitInfo* info) {
  // the block scheduler's workers: one wave per block, no LDS accumulators
  // (decisions are rare; their map updates go to the map directly)
  const bool sched = P.kernel == 2;
  const uint32_t nw = sched ? 1u : jit_waves(P.stack_bytes, P.event_parallel);
  uint32_t lds = P.stack_bytes ? nw * 64u * P.stack_bytes : 16u;
  const int nr = std::max(ring_count(P), 1);
  const uint64_t ring_lds = (uint64_t)sizeof(uint64_t) * 3 * nw * nr;  // the waves' ring chunks
  JitInfo ji;
  std::string body = emit_prog(P, "p0", !sched, sched ? 0 : lds + ring_lds, &ji);
  // An event-parallel program whose stack lives wholly in its private frame
  // (no access and no helper argument reads stack memory: the generated
  // code never touches stk) needs no LDS frames, and its accumulators take
  // that LDS instead.
  if (P.event_parallel && !sched && P.stack_bytes && !reads_stack(body)) {
    lds = 16u;
    body = emit_prog(P, "p0", true, lds + ring_lds, &ji);
  }
  std::string o;
  o += "#define GX_LDS_BYTES " + std::to_string(lds) + "\n";
  o += guards_define();
  o += "#define GX_NRINGS " + std::to_string(nr) + "u\n";
  o += "#define GX_RING_SLOTS " + std::to_string(nw * nr) + "\n";
  o += "#include \"gx_dev.h\"\n\n";
  o += body;
  if (info) *info = ji;
  const std::string W = std::to_string(nw), T = std::to_string(64 * nw);
  const std::string head = "  const uint32_t wave = threadIdx.x >> 6;\n"
                           "  gx::Stk stk{wave * 64u * " + std::to_string(P.stack_bytes) +
                           "u, gx::lane_id() * 8u, blockIdx.x * " + T + "u + threadIdx.x};\n"
                           "  gx::p0::Prog<true" + std::string(P.leader ? ", true" : "") + "> P{wave};\n  P.begin(A);\n";
  const std::string reduce =
      ji.spill_block_bytes ? std::string("extern \"C\" __global__ void __launch_bounds__(256) gx_j_reduce(gx::RunArgs A, "
                                         "uint32_t nb) {\n  gx::p0::reduce(A, nb);\n}\n\n")
                           : std::string();
  if (P.event_parallel && P.kernel == 1)
    o += "extern \"C\" __global__ void __launch_bounds__(" + T + ") gx_j_app_vadd(gx::RunArgs A, gx::AppArgs Pa) {\n" +
         head + "  gx::app_vadd_loop<true>(P, A, Pa, (uint64_t)blockIdx.x * " + W + "u + wave, (uint64_t)gridDim.x * " +
         W + "u, stk);\n  P.end(A);\n}\n\n" + reduce;
  else if (P.event_parallel && sched)
    o += "extern \"C\" __global__ void __launch_bounds__(64) gx_j_sched(gx::RunArgs A, gx::SchedArgs S) {\n"
         "  gx::Stk stk{0, gx::lane_id() * 8u, blockIdx.x * 64u + threadIdx.x};\n"
         "  gx::p0::Prog<false> P{0u};\n  P.begin(A);\n"
         "  gx::sched_worker<true>(P, A, S, blockIdx.x, stk);\n  P.end(A);\n}\n\n";
  else if (P.event_parallel)
    o += "extern \"C\" __global__ void __launch_bounds__(" + T + ") gx_j_event_parallel(gx::RunArgs A) {\n" + head +
         "  gx::" + ahead_loop() + "(P, A, (uint64_t)blockIdx.x * " + W + "u + wave, (uint64_t)gridDim.x * " + W +
         "u, stk);\n"
         "  P.end(A);\n}\n\n" + reduce;
  else
    o += "extern \"C\" __global__ void __launch_bounds__(64) gx_j_stream_seq(gx::RunArgs A, uint32_t lanes, "
       "uint32_t qstride, uint32_t qend_last) {\n  gx::Stk stk{0, gx::lane_id() * 8u, blockIdx.x * 64u + threadIdx.x};\n"
       "  gx::p0::Prog<false> P{0u};\n  P.begin(A);\n  uint64_t steps = 0;\n"
       "  gx::stream_wave(P, A, blockIdx.x * lanes, lanes, qstride, qend_last, stk, steps);\n"
       "  P.end(A);\n}\n\n"
       "extern \"C\" __global__ void __launch_bounds__(64) gx_j_stream_uni(gx::RunArgs A, uint32_t qstride, "
       "uint32_t qend_last) {\n  gx::Stk stk{0, 0u, blockIdx.x * 64u + threadIdx.x};\n"
       "  gx::p0::Prog<false, true> P{0u};\n  P.begin(A);\n  uint64_t steps = 0;\n"
       "  gx::stream_uni<true>(P, A, blockIdx.x, qstride, qend_last, stk, steps);\n"
       "  P.end(A);\n}\n";
  return o;
}

std::string jit_set_source(const std::vector<JitProg>& progs) {
  uint32_t stack = 8;
  int nr = 1;
  for (auto& P : progs) {
    stack = std::max(stack, P.stack_bytes);
    nr = std::max(nr, ring_count(P));
  }
  std::string o;
  o += "#define GX_LDS_BYTES " + std::to_string(64u * stack) + "\n";
  o += guards_define();
  o += "#define GX_NRINGS " + std::to_string(nr) + "u\n";
  o += "#define GX_RING_SLOTS " + std::to_string(nr) + "\n";
  o += "#include \"gx_dev.h\"\n\n";
  for (size_t k = 0; k < progs.size(); k++) o += emit_prog(progs[k], "p" + std::to_string(k), false, 0, nullptr);
  o += "extern \"C\" __global__ void __launch_bounds__(64) gx_j_set(const gx::BatchDev* B, const uint2* items, "
       "uint32_t n_items, uint32_t* next) {\n"
       "  gx::Stk stk{0, gx::lane_id() * 8u, blockIdx.x * 64u + threadIdx.x};\n"
       "  gx::Stk stku{0, 0u, blockIdx.x * 64u + threadIdx.x};\n  (void)stku;\n"
       "  gx::batched_items(B, items, n_items, next, [&](const gx::BatchDev& bd, uint32_t chunk) {\n"
       "    uint64_t steps = 0;\n    switch (bd.slot) {\n";
  for (size_t k = 0; k < progs.size(); k++) {
    const std::string K = std::to_string(k);
    const bool ep = progs[k].event_parallel;
    o += "      case " + K + "u: {\n        gx::p" + K + "::Prog<false" + (ep && !progs[k].leader ? "" : ", true") +
         "> P{0u};\n        P.begin(bd.A);\n";
    if (ep)
      o += "        gx::event_tile(P, bd.A, (uint64_t)chunk * 64u, stk, steps);\n";
    else
      o += "        gx::stream_uni<false>(P, bd.A, chunk, bd.qstride, bd.qend_last, stku, steps);\n";
    o += "        P.end(bd.A);\n        break;\n      }\n";
  }
  o += "      default: break;\n    }\n  });\n}\n";
  return o;
}

int jit_compile(const std::string& src, std::vector<char>* code, std::string* log) {
  hiprtcProgram prog;
  const char* hdrs[2] = {kJitHdrDev, kJitHdrInternal};
  const char* names[2] = {"gx_dev.h", "gx_internal.h"};
  if (hiprtcCreateProgram(&prog, src.c_str(), "gx_prog.hip", 2, hdrs, names) != HIPRTC_SUCCESS) {
    if (log) *log = "hiprtcCreateProgram failed";
    return -EIO;
  }
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops", "-Wno-unused-label"};
  hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
  size_t n = 0;
  if (log && hiprtcGetProgramLogSize(prog, &n) == HIPRTC_SUCCESS && n > 1) {
    log->assign(n, '\0');
    (void)hiprtcGetProgramLog(prog, &(*log)[0]);
    log->resize(n - 1);
  }
  if (r != HIPRTC_SUCCESS) {
    (void)hiprtcDestroyProgram(&prog);
    return -EIO;
  }
  size_t cs = 0;
  if (hiprtcGetCodeSize(prog, &cs) != HIPRTC_SUCCESS || cs == 0) {
    (void)hiprtcDestroyProgram(&prog);
    return -EIO;
  }
  code->assign(cs, 0);
  r = hiprtcGetCode(prog, code->data());
  (void)hiprtcDestroyProgram(&prog);
  return r == HIPRTC_SUCCESS ? 0 : -EIO;
}

}  // namespace gx
