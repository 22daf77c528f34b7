// Load-time verifier (paper section 4.4, "SIMT-aware Verification", and
// section 5.3: bounded loops, memory safety, type correctness, per-hook
// resource budgets, no global synchronisation, commutative-only updates of
// shared state).
//
// Structure: decode -> encoding rules -> CFG (targets, reachability, no
// fall-through past the end) -> counted-loop recognition -> abstract
// interpretation in program order with loops unrolled trip by trip.
// Value domain: tracked bits (value/mask pairs) combined with an unsigned
// interval.  Facts for the pre-decoder are recorded per instruction and must
// agree on every path that reaches the instruction.
#include "gx_verifier.h"

#include <algorithm>
#include <cstring>
#include <map>
#include <sstream>

#include "gx_internal.h"

namespace gx {

std::vector<Insn> decode_insns(const uint64_t* raw, uint32_t n) {
  std::vector<Insn> v(n);
  for (uint32_t i = 0; i < n; i++) {
    uint64_t w = raw[i];
    v[i].op = (uint8_t)(w & 0xff);
    v[i].dst = (uint8_t)((w >> 8) & 0xf);
    v[i].src = (uint8_t)((w >> 12) & 0xf);
    v[i].off = (int16_t)(uint16_t)((w >> 16) & 0xffff);
    v[i].imm = (int32_t)(uint32_t)(w >> 32);
  }
  return v;
}

bool hook_layout(int hook, uint32_t* record_size, uint32_t* stream_off, uint32_t* stream_size) {
  if (hook == HOOK_MEM_ACCESS) {
    *record_size = 24;
    *stream_off = 8;
    *stream_size = 4;
    return true;
  }
  if (hook == HOOK_KERNEL_TIMING) {
    *record_size = 16;
    *stream_off = 0;
    *stream_size = 4;
    return true;
  }
  if (hook == HOOK_WAVE_MEM || hook == HOOK_SIMT_MEM) {  // input records as HOOK_MEM_ACCESS
    *record_size = 24;
    *stream_off = 8;
    *stream_size = 4;
    return true;
  }
  if (hook == HOOK_SCHED) {  // the worker is the stream
    *record_size = 32;
    *stream_off = 0;
    *stream_size = 4;
    return true;
  }
  return false;
}

namespace {

// readable ctx fields per hook: (offset, size)
bool ctx_field(int hook, int64_t off, int size) {
  if (hook == HOOK_MEM_ACCESS)
    return (off == 0 && size == 8) || (off == 8 && size == 4) || (off == 16 && size == 8);
  if (hook == HOOK_KERNEL_TIMING) return (off == 0 && size == 4) || (off == 8 && size == 8);
  if (hook == HOOK_WAVE_MEM)
    return (off == 0 && size == 8) || (off == 8 && size == 8) || (off == 16 && size == 4) || (off == 20 && size == 4);
  if (hook == HOOK_SIMT_MEM)  // the record's fields, then the tile aggregate's at 24
    return ctx_field(HOOK_MEM_ACCESS, off, size) || (off >= 24 && ctx_field(HOOK_WAVE_MEM, off - 24, size));
  if (hook == HOOK_SCHED)
    return ((off == 0 || off == 4 || off == 24 || off == 28) && size == 4) || ((off == 8 || off == 16) && size == 8);
  return false;
}

// SIMT hook: ctx bytes from this offset on are warp-uniform (the tile's
// aggregate); the record's own fields before it vary by lane.
constexpr int64_t kSimtUniformFrom = 24;

// ---------------------------------------------------------------------------
// tracked-bits domain: bit i is known iff mask bit i is 0, then equals v bit i.
struct Bits {
  uint64_t v, m;
};
constexpr Bits kUnknownBits{0, ~0ull};
Bits bconst(uint64_t x) { return Bits{x, 0}; }
Bits badd(Bits a, Bits b) {
  uint64_t sm = a.m + b.m, sv = a.v + b.v, sigma = sm + sv, chi = sigma ^ sv, mu = chi | a.m | b.m;
  return Bits{sv & ~mu, mu};
}
Bits bsub(Bits a, Bits b) {
  uint64_t dv = a.v - b.v, alpha = dv + a.m, beta = dv - b.m, chi = alpha ^ beta, mu = chi | a.m | b.m;
  return Bits{dv & ~mu, mu};
}
Bits band(Bits a, Bits b) {
  uint64_t alpha = a.v | a.m, beta = b.v | b.m, v = a.v & b.v;
  return Bits{v, alpha & beta & ~v};
}
Bits bor(Bits a, Bits b) {
  uint64_t v = a.v | b.v, mu = a.m | b.m;
  return Bits{v, mu & ~v};
}
Bits bxor(Bits a, Bits b) {
  uint64_t v = a.v ^ b.v, mu = a.m | b.m;
  return Bits{v & ~mu, mu};
}
Bits bunion(Bits a, Bits b) {
  uint64_t mu = a.m | b.m | (a.v ^ b.v);
  return Bits{a.v & ~mu, mu};
}
Bits btrunc32(Bits a) { return Bits{a.v & 0xffffffffull, a.m & 0xffffffffull}; }

enum Ty : uint8_t { T_NONE, T_SCALAR, T_CTX, T_STACK, T_MAPVAL, T_MAPVAL_NULL, T_MAP, T_CONFLICT };

struct Val {
  Ty t = T_NONE;
  Bits b = kUnknownBits;     // scalar value / pointer offset bits
  uint64_t lo = 0, hi = ~0ull;  // unsigned range (scalar) / offset range as signed (pointers)
  int map = -1;
  bool lanes = false;        // differs between the lanes of a wave (SIMT hook)
};

Val scal(Bits b, uint64_t lo, uint64_t hi) {
  Val v;
  v.t = T_SCALAR;
  // tighten both ways
  lo = std::max(lo, b.v);
  hi = std::min(hi, b.v | b.m);
  if (lo == hi) b = bconst(lo);
  v.b = b;
  v.lo = lo;
  v.hi = hi;
  return v;
}
Val sconst(uint64_t x) { return scal(bconst(x), x, x); }
Val sany() { return scal(kUnknownBits, 0, ~0ull); }
Val s32any() { return scal(Bits{0, 0xffffffffull}, 0, 0xffffffffull); }
bool is_const(const Val& v) { return v.t == T_SCALAR && v.lo == v.hi; }

Val vjoin(const Val& a, const Val& b) {
  if (a.t == T_NONE || b.t == T_NONE) return Val{};
  if (a.t == T_CONFLICT || b.t == T_CONFLICT) return Val{T_CONFLICT};
  Ty t = a.t;
  if (a.t != b.t) {
    bool ptrs = (a.t == T_MAPVAL || a.t == T_MAPVAL_NULL) && (b.t == T_MAPVAL || b.t == T_MAPVAL_NULL);
    if (!ptrs) return Val{T_CONFLICT};
    t = T_MAPVAL_NULL;
  }
  if (t != T_SCALAR && a.map != b.map) return Val{T_CONFLICT};
  Val r;
  r.t = t;
  r.map = a.map;
  r.b = bunion(a.b, b.b);
  r.lanes = a.lanes || b.lanes;
  if (t == T_SCALAR) {
    r.lo = std::min(a.lo, b.lo);
    r.hi = std::max(a.hi, b.hi);
  } else {
    r.lo = (uint64_t)std::min((int64_t)a.lo, (int64_t)b.lo);
    r.hi = (uint64_t)std::max((int64_t)a.hi, (int64_t)b.hi);
  }
  return r;
}

struct State {
  bool live = false;
  Val r[11];
  uint64_t init[kStackMax / 64];   // stack byte initialised bits (byte i of the 512-byte frame)
  uint64_t lanes[kStackMax / 64];  // stack byte holds a lane-varying value (SIMT hook)
  uint64_t steps = 0, calls = 0, ring = 0;
};

void sjoin(State& d, const State& s) {
  if (!s.live) return;
  if (!d.live) {
    d = s;
    return;
  }
  for (int i = 0; i < 11; i++) d.r[i] = vjoin(d.r[i], s.r[i]);
  for (int i = 0; i < kStackMax / 64; i++) d.init[i] &= s.init[i];
  for (int i = 0; i < kStackMax / 64; i++) d.lanes[i] |= s.lanes[i];
  d.steps = std::max(d.steps, s.steps);
  d.calls = std::max(d.calls, s.calls);
  d.ring = std::max(d.ring, s.ring);
}

bool init_all(const State& s, int64_t o, int64_t n) {
  for (int64_t i = o; i < o + n; i++)
    if (!((s.init[i >> 6] >> (i & 63)) & 1)) return false;
  return true;
}
void init_set(State& s, int64_t o, int64_t n) {
  for (int64_t i = o; i < o + n; i++) s.init[i >> 6] |= 1ull << (i & 63);
}
bool lanes_any(const State& s, int64_t o, int64_t n) {
  for (int64_t i = o; i < o + n; i++)
    if ((s.lanes[i >> 6] >> (i & 63)) & 1) return true;
  return false;
}
void lanes_set(State& s, int64_t o, int64_t n, bool v) {
  for (int64_t i = o; i < o + n; i++) {
    if (v) s.lanes[i >> 6] |= 1ull << (i & 63);
    else s.lanes[i >> 6] &= ~(1ull << (i & 63));
  }
}

struct Fail {
  std::string msg;
};

uint64_t umax_bits(uint64_t x) {
  for (int s = 1; s < 64; s <<= 1) x |= x >> s;
  return x;
}

// Concrete ALU for constant operands (the runtime's own definition).
uint64_t eval_alu(bool w64, int op, int16_t off, bool x, int32_t imm, uint64_t a, uint64_t b) {
  if (!w64) {
    uint32_t p = (uint32_t)a, q = (uint32_t)b;
    int32_t sp = (int32_t)p, sq = (int32_t)q;
    switch (op) {
      case 0x00: return (uint32_t)(p + q);
      case 0x10: return (uint32_t)(p - q);
      case 0x20: return (uint32_t)(p * q);
      case 0x30:
        if (!q) return 0;
        if (!off) return p / q;
        return (sp == INT32_MIN && sq == -1) ? p : (uint32_t)(sp / sq);
      case 0x40: return p | q;
      case 0x50: return p & q;
      case 0x60: return (uint32_t)(p << (q & 31));
      case 0x70: return p >> (q & 31);
      case 0x80: return (uint32_t)(0u - p);
      case 0x90:
        if (!q) return p;
        if (!off) return p % q;
        return sq == -1 ? 0 : (uint32_t)(sp % sq);
      case 0xa0: return p ^ q;
      case 0xb0:
        if (x && off == 8) return (uint32_t)(int32_t)(int8_t)q;
        if (x && off == 16) return (uint32_t)(int32_t)(int16_t)q;
        return q;
      case 0xc0: return (uint32_t)(sp >> (q & 31));
      case 0xd0: {
        if (!x) return imm == 64 ? a : a & ((1ull << imm) - 1);
        uint64_t r = 0;
        for (int i = 0; i < imm / 8; i++) r = (r << 8) | ((a >> (8 * i)) & 0xff);
        return r;
      }
    }
    return 0;
  }
  int64_t sa = (int64_t)a, sb = (int64_t)b;
  switch (op) {
    case 0x00: return a + b;
    case 0x10: return a - b;
    case 0x20: return a * b;
    case 0x30:
      if (!b) return 0;
      if (!off) return a / b;
      return (sa == INT64_MIN && sb == -1) ? a : (uint64_t)(sa / sb);
    case 0x40: return a | b;
    case 0x50: return a & b;
    case 0x60: return a << (b & 63);
    case 0x70: return a >> (b & 63);
    case 0x80: return 0 - a;
    case 0x90:
      if (!b) return a;
      if (!off) return a % b;
      return sb == -1 ? 0 : (uint64_t)(sa % sb);
    case 0xa0: return a ^ b;
    case 0xb0:
      if (x && off == 8) return (uint64_t)(int64_t)(int8_t)b;
      if (x && off == 16) return (uint64_t)(int64_t)(int16_t)b;
      if (x && off == 32) return (uint64_t)(int64_t)(int32_t)b;
      return b;
    case 0xc0: return (uint64_t)(sa >> (b & 63));
    case 0xd0: {
      uint64_t r = 0;
      for (int i = 0; i < imm / 8; i++) r = (r << 8) | ((a >> (8 * i)) & 0xff);
      return r;
    }
  }
  return 0;
}

class Verifier {
 public:
  Verifier(const std::vector<Insn>& p, int hook, const std::vector<MapShape>& t, const std::vector<int>& fds)
      : P(p), N((int)p.size()), hook_(hook), simt_(hook == HOOK_SIMT_MEM), maps_(t), fds_(fds) {}

  Verdict run() {
    Verdict& V = out_;
    try {
      uint32_t rs, so, ss;
      if (!hook_layout(hook_, &rs, &so, &ss)) throw Fail{"unknown hook type"};
      if (N == 0) throw Fail{"empty program"};
      if (N > kMaxInsns) throw Fail{"program has more than 4096 instructions"};
      V.mem_kind.assign(N, KIND_NONE);
      V.call_map.assign(N, -1);
      V.arg2_kind.assign(N, KIND_NONE);
      V.arg3_kind.assign(N, KIND_NONE);
      V.ring_size.assign(N, 0);
      V.ld_map.assign(N, -1);
      V.mem_map.assign(N, -1);
      used_.assign(maps_.size(), 0);
      shared_op_.assign(maps_.size(), -1);
      seen_.assign(N, 0);
      encodings();
      cfg();
      loops();
      State s;
      s.live = true;
      s.r[1].t = T_CTX;
      s.r[1].b = bconst(0);
      s.r[1].lo = s.r[1].hi = 0;
      s.r[10].t = T_STACK;
      s.r[10].b = bconst(kStackMax);
      s.r[10].lo = s.r[10].hi = kStackMax;
      std::memset(s.init, 0, sizeof s.init);
      std::memset(s.lanes, 0, sizeof s.lanes);
      std::map<int, State> exits;
      walk(0, N - 1, s, exits, nullptr);
      if (!exits.empty()) fail(exits.begin()->first, "control leaves the program");
      V.ok = true;
      V.log = "ok";
      V.stack_bytes = (uint32_t)((kStackMax - low_stack_ + 7) & ~7);
      V.event_parallel = true;
      for (size_t i = 0; i < maps_.size(); i++)
        if (used_[i] && maps_[i].type != MAP_RINGBUF && !(maps_[i].flags & (F_SHARED | F_READ_ONLY)))
          V.event_parallel = false;
      if (hook_ == HOOK_WAVE_MEM && !V.event_parallel)
        fail(0, "a warp-leader hook runs once per wave: its maps must be shared, read-only or ring buffers");
      if (hook_ == HOOK_SCHED && !V.event_parallel)
        fail(0, "a scheduling hook runs in all workers at once: its maps must be shared, read-only or ring buffers");
      if (simt_ && !V.event_parallel)
        fail(0, "the lanes of a SIMT hook run one wave's events at once: its maps must be shared, read-only or ring buffers");
    } catch (const Fail& f) {
      Verdict bad;
      bad.ok = false;
      bad.log = f.msg;
      out_ = bad;
    }
    return out_;
  }

 private:
  const std::vector<Insn>& P;
  const int N;
  const int hook_;
  // SIMT hook (section 4.4, "SIMT-aware Verification"): values are tracked
  // as warp-uniform or lane-varying; branches, map keys, ring records and
  // their flags, and map-update addresses must be uniform
  const bool simt_;
  const std::vector<MapShape>& maps_;
  const std::vector<int>& fds_;
  Verdict out_;
  std::vector<char> second_, used_, seen_;
  std::vector<int> back_of_head_;  // loop head -> back-edge slot
  std::vector<int> shared_op_;     // shared map -> its single (atomic op, size)
  int low_stack_ = kStackMax;

  [[noreturn]] void fail(int pc, const std::string& m) {
    std::ostringstream os;
    os << "slot " << pc << ": " << m;
    throw Fail{os.str()};
  }

  static int cls(const Insn& i) { return i.op & 7; }
  static int opc(const Insn& i) { return i.op & 0xf0; }
  static bool xsrc(const Insn& i) { return (i.op & 8) != 0; }
  bool is_lddw(int pc) const { return P[pc].op == 0x18; }
  bool is_branch(const Insn& i) const {
    return (cls(i) == 5 || cls(i) == 6) && opc(i) != 0x80 && opc(i) != 0x90;
  }
  int target(int pc) const {
    const Insn& i = P[pc];
    int d = (cls(i) == 6 && opc(i) == 0) ? i.imm : i.off;
    return pc + 1 + d;
  }
  bool falls(const Insn& i) const {
    if (cls(i) == 5 || cls(i) == 6) return opc(i) != 0x90 && opc(i) != 0x00;
    return true;
  }

  // ---------------- encoding rules ----------------
  void encodings() {
    second_.assign(N, 0);
    for (int pc = 0; pc < N; pc++) {
      if (second_[pc]) continue;
      const Insn& i = P[pc];
      if (i.dst > 10 || i.src > 10) fail(pc, "invalid register");
      int c = cls(i), o = opc(i);
      bool x = xsrc(i);
      if (c == 4 || c == 7) {
        bool w64 = c == 7;
        if (o >= 0xe0) fail(pc, "invalid ALU opcode");
        if (i.dst == 10) fail(pc, "r10 is read-only");
        if (o == 0x80) {
          if (x || i.src || i.off || i.imm) fail(pc, "invalid NEG encoding");
        } else if (o == 0xd0) {
          if (i.src || i.off || !(i.imm == 16 || i.imm == 32 || i.imm == 64)) fail(pc, "invalid byte-swap encoding");
          if (w64 && x) fail(pc, "invalid BSWAP encoding");
        } else {
          if (x ? i.imm != 0 : i.src != 0) fail(pc, "reserved field not zero");
          bool off_ok = i.off == 0 || ((o == 0x30 || o == 0x90) && i.off == 1) ||
                        (o == 0xb0 && x && (i.off == 8 || i.off == 16 || (w64 && i.off == 32)));
          if (!off_ok) fail(pc, "reserved offset not zero");
          if (!x && (o == 0x30 || o == 0x90) && i.imm == 0) fail(pc, "division by zero constant");
          if (!x && (o == 0x60 || o == 0x70 || o == 0xc0) && (i.imm < 0 || i.imm >= (w64 ? 64 : 32)))
            fail(pc, "shift by a constant out of range");
        }
      } else if (c == 5 || c == 6) {
        if (o >= 0xe0) fail(pc, "invalid jump opcode");
        if (o == 0x80) {
          if (c == 6 || x || i.src || i.dst || i.off) fail(pc, "invalid CALL encoding (only helper calls)");
        } else if (o == 0x90) {
          if (c == 6 || x || i.src || i.dst || i.off || i.imm) fail(pc, "invalid EXIT encoding");
        } else if (o == 0x00) {
          if (x || i.src || i.dst || (c == 6 ? i.off : i.imm)) fail(pc, "invalid JA encoding");
        } else if (x ? i.imm != 0 : i.src != 0) {
          fail(pc, "reserved field not zero");
        }
      } else if (c == 1) {
        int mode = i.op & 0xe0;
        if (mode != 0x60 && mode != 0x80) fail(pc, "unsupported load mode");
        if (mode == 0x80 && (i.op & 0x18) == 0x18) fail(pc, "invalid sign-extending load size");
        if (i.imm) fail(pc, "reserved field not zero");
        if (i.dst == 10) fail(pc, "r10 is read-only");
      } else if (c == 2) {
        if ((i.op & 0xe0) != 0x60 || i.src) fail(pc, "invalid ST encoding");
      } else if (c == 3) {
        int mode = i.op & 0xe0;
        if (mode == 0x60) {
          if (i.imm) fail(pc, "reserved field not zero");
        } else if (mode == 0xc0) {
          int sz = i.op & 0x18;
          if (sz != 0 && sz != 0x18) fail(pc, "atomics are 32 or 64 bit");
          static const int ok[] = {0x00, 0x40, 0x50, 0xa0, 0x01, 0x41, 0x51, 0xa1, 0xe1, 0xf1};
          if (std::find(std::begin(ok), std::end(ok), i.imm) == std::end(ok)) fail(pc, "invalid atomic operation");
        } else {
          fail(pc, "unsupported store mode");
        }
      } else {  // class 0
        if (i.op != 0x18) fail(pc, "unsupported LD instruction");
        if (pc + 1 >= N) fail(pc, "lddw needs two slots");
        if (i.off) fail(pc, "reserved field not zero");
        if (i.src != 0 && i.src != 1 && i.src != 5) fail(pc, "unsupported lddw form");
        if (i.dst == 10) fail(pc, "r10 is read-only");
        const Insn& j = P[pc + 1];
        if (j.op || j.dst || j.src || j.off) fail(pc + 1, "invalid second lddw slot");
        if (i.src && j.imm) fail(pc + 1, "map reference with upper bits");
        second_[pc + 1] = 1;
      }
    }
  }

  // ---------------- control flow ----------------
  void cfg() {
    std::vector<char> reach(N, 0);
    std::vector<int> stack{0};
    reach[0] = 1;
    while (!stack.empty()) {
      int pc = stack.back();
      stack.pop_back();
      const Insn& i = P[pc];
      int nx = pc + (is_lddw(pc) ? 2 : 1);
      auto push = [&](int t) {
        if (!reach[t]) {
          reach[t] = 1;
          stack.push_back(t);
        }
      };
      if (is_branch(i)) {
        int t = target(pc);
        if (t < 0 || t >= N) fail(pc, "jump target out of range");
        if (second_[t]) fail(pc, "jump into the second slot of lddw");
        push(t);
      }
      if (falls(i)) {
        if (nx >= N) fail(pc, "execution falls off the end");
        push(nx);
      }
    }
    for (int pc = 0; pc < N; pc++)
      if (!second_[pc] && !reach[pc]) fail(pc, "unreachable instruction");
  }

  bool writes(const Insn& i, int r) const {
    switch (cls(i)) {
      case 0: case 1: case 4: case 7: return i.dst == r;
      case 5: return opc(i) == 0x80 && r <= 5;
      case 3:
        if ((i.op & 0xe0) == 0xc0) {
          if (i.imm == 0xf1) return r == 0;
          if (i.imm & 1) return i.src == r;
        }
        return false;
    }
    return false;
  }

  void loops() {
    back_of_head_.assign(N, -1);
    std::vector<std::pair<int, int>> L;
    for (int j = 0; j < N; j++) {
      if (second_[j] || !is_branch(P[j])) continue;
      int h = target(j);
      if (h > j) continue;
      const Insn& be = P[j];
      if (cls(be) != 5 || opc(be) == 0x00 || xsrc(be))
        fail(j, "back-edge is not a counted-loop compare of a counter against a constant");
      int c = be.dst;
      if (j == h) fail(j, "loop without a counter update");
      const Insn& inc = P[j - 1];
      if (second_[j - 1] || !(inc.op == 0x07 || inc.op == 0x17) || inc.dst != c || inc.imm == 0)
        fail(j, "the back-edge must directly follow the counter update (add/sub of a constant)");
      if (back_of_head_[h] >= 0) fail(j, "a loop head with two back-edges");
      for (int p = h; p < j - 1; p++)
        if (!second_[p] && writes(P[p], c)) fail(p, "loop counter written in the loop body");
      back_of_head_[h] = j;
      L.push_back({h, j});
    }
    for (size_t a = 0; a < L.size(); a++)
      for (size_t b = 0; b < L.size(); b++) {
        if (a == b) continue;
        bool apart = L[a].second < L[b].first || L[b].second < L[a].first;
        bool inner = L[a].first <= L[b].first && L[b].second <= L[a].second;
        bool outer = L[b].first <= L[a].first && L[a].second <= L[b].second;
        if (!apart && !inner && !outer) fail(L[a].first, "loops overlap without nesting");
      }
    for (int p = 0; p < N; p++) {
      if (second_[p] || !is_branch(P[p])) continue;
      int t = target(p);
      for (auto& l : L) {
        bool in = p >= l.first && p <= l.second;
        if (!in && t > l.first && t <= l.second) fail(p, "jump into a loop body");
        if (in && p != l.second && t == l.second) fail(p, "jump bypasses the loop counter update");
      }
    }
  }

  // ---------------- facts ----------------
  void fact(std::vector<int8_t>& f, int pc, int8_t k, const char* what) {
    if (f[pc] == KIND_NONE) f[pc] = k;
    else if (f[pc] != k) fail(pc, std::string(what) + " has different pointer kinds on different paths");
  }
  void fact_map(std::vector<int>& f, int pc, int m) {
    if (f[pc] < 0) f[pc] = m;
    else if (f[pc] != m) fail(pc, "map differs between paths");
  }

  const Val& use(const State& s, int pc, int r) {
    const Val& v = s.r[r];
    if (v.t == T_NONE) fail(pc, "r" + std::to_string(r) + " is not initialised");
    if (v.t == T_CONFLICT) fail(pc, "r" + std::to_string(r) + " has no single type here");
    return v;
  }

  // Memory access through ``base``; mode: 0 load, 1 store, 2 commutative
  // atomic, 3 atomic that reads.  ``in_lanes``: the stored value varies by
  // lane.  Returns whether the value read varies by lane.
  bool access(State& s, int pc, const Val& base, int64_t off, int size, int mode, bool in_lanes = false) {
    switch (base.t) {
      case T_CTX:
        if (mode != 0) fail(pc, "ctx is read-only");
        if (base.lo != 0 || base.hi != 0 || !ctx_field(hook_, off, size)) fail(pc, "invalid ctx field access");
        fact(out_.mem_kind, pc, KIND_CTX, "memory access");
        return simt_ && off < kSimtUniformFrom;
      case T_STACK: {
        if (base.lo != base.hi) fail(pc, "stack access with a variable offset");
        int64_t o = (int64_t)base.lo + off;
        if (o < 0 || o + size > kStackMax) fail(pc, "stack access out of bounds");
        if (o & (size - 1)) fail(pc, "misaligned stack access");
        if (mode != 1 && !init_all(s, o, size)) fail(pc, "stack read before write");
        const bool was = mode != 1 && lanes_any(s, o, size);
        if (mode != 0) {
          init_set(s, o, size);
          lanes_set(s, o, size, in_lanes || was);
        }
        low_stack_ = std::min<int>(low_stack_, (int)o);
        fact(out_.mem_kind, pc, KIND_STACK, "memory access");
        return was;
      }
      case T_MAPVAL: {
        const MapShape& m = maps_[base.map];
        int64_t lo = (int64_t)base.lo + off, hi = (int64_t)base.hi + off;
        if (lo < 0 || hi + size > (int64_t)m.value_size) fail(pc, "map value access out of bounds");
        uint64_t al = (uint64_t)size - 1;
        if (((base.b.v + (uint64_t)off) & al) || (base.b.m & al)) fail(pc, "map value access may be misaligned");
        if (simt_ && mode != 0 && base.lanes) fail(pc, "SIMT hook: a map update at a lane-varying address");
        if (simt_ && mode == 3) fail(pc, "SIMT hook: an atomic that reads a map value is not warp-uniform");
        if ((m.flags & F_READ_ONLY) && mode != 0) fail(pc, "write to a read-only map");
        if ((m.flags & F_SHARED) && mode != 2) fail(pc, "shared maps take only commutative atomics");
        if (m.flags & F_SHARED) {
          // different operations (or widths) on one slot do not commute
          int op = (P[pc].imm & 0xff) | (size << 8);
          if (shared_op_[base.map] < 0) shared_op_[base.map] = op;
          if (shared_op_[base.map] != op) fail(pc, "a shared map must take one atomic operation at one width");
        }
        fact(out_.mem_kind, pc, KIND_MAPVAL, "memory access");
        fact_map(out_.mem_map, pc, base.map);
        return base.lanes;
      }
      case T_MAPVAL_NULL:
        fail(pc, "map value used before its null check");
      default:
        fail(pc, "memory access through a non-pointer");
    }
  }

  // A helper's memory argument; ``uniform``: what it is, when the SIMT hook
  // needs it warp-uniform (nullptr: no such need).
  void mem_arg(State& s, int pc, int reg, uint64_t n, std::vector<int8_t>& kinds, const char* uniform = nullptr) {
    const Val& v = use(s, pc, reg);
    if (simt_ && uniform && v.lanes) fail(pc, std::string("SIMT hook: ") + uniform + " through a lane-varying pointer");
    if (v.t == T_STACK) {
      if (v.lo != v.hi) fail(pc, "helper stack argument with a variable offset");
      int64_t o = (int64_t)v.lo;
      if (o < 0 || o + (int64_t)n > kStackMax) fail(pc, "helper stack argument out of bounds");
      if (!init_all(s, o, (int64_t)n)) fail(pc, "helper reads uninitialised stack");
      if (simt_ && uniform && lanes_any(s, o, (int64_t)n)) fail(pc, std::string("SIMT hook: lane-varying ") + uniform);
      low_stack_ = std::min<int>(low_stack_, (int)o);
      fact(kinds, pc, KIND_STACK, "helper argument");
      return;
    }
    if (v.t == T_MAPVAL) {
      const MapShape& m = maps_[v.map];
      if ((int64_t)v.lo < 0 || (int64_t)v.hi + (int64_t)n > (int64_t)m.value_size)
        fail(pc, "helper map-value argument out of bounds");
      if (m.flags & F_SHARED) fail(pc, "shared map values cannot be helper inputs");
      fact(kinds, pc, KIND_MAPVAL, "helper argument");
      return;
    }
    fail(pc, "helper memory argument must be a stack or map-value pointer");
  }

  int map_arg(const State& s, int pc) {
    const Val& v = use(s, pc, 1);
    if (v.t != T_MAP) fail(pc, "r1 must be a map reference");
    used_[v.map] = 1;
    fact_map(out_.call_map, pc, v.map);
    return v.map;
  }

  void helper(State& s, int pc, int id) {
    if (id == 1) {
      int m = map_arg(s, pc);
      if (maps_[m].type == MAP_RINGBUF) fail(pc, "lookup on a ring buffer");
      mem_arg(s, pc, 2, maps_[m].key_size, out_.arg2_kind, "map key");
      Val r;
      r.t = T_MAPVAL_NULL;
      r.map = m;
      r.b = bconst(0);
      r.lo = r.hi = 0;
      s.r[0] = r;
    } else if (id == 2 || id == 3) {
      int m = map_arg(s, pc);
      const MapShape& ms = maps_[m];
      if (ms.type == MAP_RINGBUF) fail(pc, "update/delete on a ring buffer");
      if (ms.flags & (F_SHARED | F_READ_ONLY)) fail(pc, "update/delete on a shared or read-only map");
      mem_arg(s, pc, 2, ms.key_size, out_.arg2_kind, "map key");
      if (id == 2) {
        mem_arg(s, pc, 3, ms.value_size, out_.arg3_kind, "map update value");
        if (use(s, pc, 4).t != T_SCALAR) fail(pc, "update flags must be a scalar");
      }
      if (ms.type == MAP_HASH)
        for (auto& v : s.r)
          if ((v.t == T_MAPVAL || v.t == T_MAPVAL_NULL) && v.map == m) v = Val{T_CONFLICT};
      s.r[0] = sany();
    } else if (id == 130) {
      int m = map_arg(s, pc);
      if (maps_[m].type != MAP_RINGBUF) fail(pc, "ringbuf_output needs a ring buffer map");
      const Val& z = use(s, pc, 3);
      if (!is_const(z) || z.lo < 1 || z.lo > 4096) fail(pc, "ringbuf_output size must be a constant in [1, 4096]");
      if (out_.ring_size[pc] && out_.ring_size[pc] != z.lo) fail(pc, "ringbuf_output size differs between paths");
      out_.ring_size[pc] = (uint32_t)z.lo;
      mem_arg(s, pc, 2, z.lo, out_.arg2_kind, "ring record");
      if (use(s, pc, 4).t != T_SCALAR) fail(pc, "ringbuf_output flags must be a scalar");
      if (simt_ && use(s, pc, 4).lanes) fail(pc, "SIMT hook: lane-varying ringbuf_output flags");
      s.ring += 8 + ((z.lo + 7) & ~7ull);
      if (s.ring > kMaxRingBytes) fail(pc, "ring-byte budget exceeded");
      s.r[0] = sany();
    } else {
      fail(pc, "helper " + std::to_string(id) + " is not available to device programs");
    }
    for (int r = 1; r <= 5; r++) s.r[r] = Val{};
    if (++s.calls > kMaxCalls) fail(pc, "helper-call budget exceeded");
  }

  // scalar transfer for ALU ops
  Val alu(int pc, bool w64, const Insn& in, const Val& a, const Val& b) {
    int o = opc(in);
    bool x = xsrc(in);
    if (o == 0xb0 && !(x && in.off)) {  // MOV
      if (w64) return b;
      if (b.hi <= 0xffffffffull) return b;
      return is_const(b) ? sconst((uint32_t)b.lo) : scal(btrunc32(b.b), 0, 0xffffffffull);
    }
    bool unary = o == 0x80 || o == 0xd0;
    if (is_const(a) && (unary || is_const(b)) && !(o == 0xb0))
      return sconst(eval_alu(w64, o, in.off, x, in.imm, a.lo, unary ? 0 : b.lo));
    if (o == 0xb0 && is_const(b)) return sconst(eval_alu(w64, o, in.off, x, in.imm, 0, b.lo));
    (void)pc;
    if (!w64) {
      switch (o) {
        case 0x50: {
          Bits r = btrunc32(band(a.b, b.b));
          return scal(r, 0, std::min<uint64_t>(std::min(a.hi, b.hi), 0xffffffffull));
        }
        case 0x00:
          if (a.hi + b.hi <= 0xffffffffull && a.hi <= 0xffffffffull && b.hi <= 0xffffffffull)
            return scal(btrunc32(badd(a.b, b.b)), a.lo + b.lo, a.hi + b.hi);
          return s32any();
        case 0x70:
          if (is_const(b) && a.hi <= 0xffffffffull) {
            int k = (int)(b.lo & 31);
            return scal(Bits{a.b.v >> k, a.b.m >> k}, a.lo >> k, a.hi >> k);
          }
          return s32any();
        case 0x90:
          if (!in.off && is_const(b) && (uint32_t)b.lo) return scal(Bits{0, 0xffffffffull}, 0, std::min<uint64_t>(a.hi, (uint32_t)b.lo - 1));
          return s32any();
        case 0xd0:
          if (in.imm == 64) return sany();
          return scal(Bits{0, (1ull << in.imm) - 1}, 0, (1ull << in.imm) - 1);
      }
      return s32any();
    }
    uint64_t t;
    switch (o) {
      case 0x00:
        if (!__builtin_add_overflow(a.hi, b.hi, &t)) return scal(badd(a.b, b.b), a.lo + b.lo, t);
        return scal(badd(a.b, b.b), 0, ~0ull);
      case 0x10:
        if (a.lo >= b.hi) return scal(bsub(a.b, b.b), a.lo - b.hi, a.hi - b.lo);
        return scal(bsub(a.b, b.b), 0, ~0ull);
      case 0x20:
        if (!__builtin_mul_overflow(a.hi, b.hi, &t)) return scal(kUnknownBits, a.lo * b.lo, t);
        return sany();
      case 0x30:
        if (!in.off && is_const(b) && b.lo) return scal(kUnknownBits, a.lo / b.lo, a.hi / b.lo);
        return sany();
      case 0x90:
        if (!in.off && is_const(b) && b.lo) return scal(kUnknownBits, 0, std::min(a.hi, b.lo - 1));
        return sany();
      case 0x40: return scal(bor(a.b, b.b), std::max(a.lo, b.lo), umax_bits(a.hi | b.hi));
      case 0x50: return scal(band(a.b, b.b), 0, std::min(a.hi, b.hi));
      case 0xa0: return scal(bxor(a.b, b.b), 0, umax_bits(a.hi | b.hi));
      case 0x60:
        if (is_const(b)) {
          int k = (int)(b.lo & 63);
          Bits r{a.b.v << k, a.b.m << k};
          if (k == 0 || (a.hi >> (64 - k)) == 0) return scal(r, a.lo << k, a.hi << k);
          return scal(r, 0, ~0ull);
        }
        return sany();
      case 0x70:
        if (is_const(b)) {
          int k = (int)(b.lo & 63);
          return scal(Bits{a.b.v >> k, a.b.m >> k}, a.lo >> k, a.hi >> k);
        }
        return scal(kUnknownBits, 0, a.hi);
      case 0xc0:
        if (is_const(b) && a.hi < (1ull << 63)) {
          int k = (int)(b.lo & 63);
          return scal(Bits{a.b.v >> k, a.b.m >> k}, a.lo >> k, a.hi >> k);
        }
        return sany();
    }
    return sany();
  }

  // 1 taken, 0 not taken, -1 either
  static int decide(int o, const Val& a, const Val& b, bool w32) {
    if (is_const(a) && is_const(b)) {
      uint64_t p = a.lo, q = b.lo;
      int64_t sp = (int64_t)p, sq = (int64_t)q;
      if (w32) {
        p = (uint32_t)p;
        q = (uint32_t)q;
        sp = (int32_t)p;
        sq = (int32_t)q;
      }
      switch (o) {
        case 0x10: return p == q;
        case 0x50: return p != q;
        case 0x20: return p > q;
        case 0x30: return p >= q;
        case 0xa0: return p < q;
        case 0xb0: return p <= q;
        case 0x40: return (p & q) != 0;
        case 0x60: return sp > sq;
        case 0x70: return sp >= sq;
        case 0xc0: return sp < sq;
        case 0xd0: return sp <= sq;
      }
      return -1;
    }
    if (w32) return -1;
    switch (o) {
      case 0x10: return (a.hi < b.lo || b.hi < a.lo) ? 0 : -1;
      case 0x50: return (a.hi < b.lo || b.hi < a.lo) ? 1 : -1;
      case 0x20: return a.lo > b.hi ? 1 : (a.hi <= b.lo ? 0 : -1);
      case 0x30: return a.lo >= b.hi ? 1 : (a.hi < b.lo ? 0 : -1);
      case 0xa0: return a.hi < b.lo ? 1 : (a.lo >= b.hi ? 0 : -1);
      case 0xb0: return a.hi <= b.lo ? 1 : (a.lo > b.hi ? 0 : -1);
      case 0x40: return (band(a.b, b.b).v != 0) ? 1 : -1;
    }
    return -1;
  }

  // narrow a on the edge where (a op k) has outcome ``taken``
  static bool narrow(Val& a, int o, uint64_t k, bool taken) {
    uint64_t lo = a.lo, hi = a.hi;
    bool eq = (o == 0x10 && taken) || (o == 0x50 && !taken);
    bool ne = (o == 0x10 && !taken) || (o == 0x50 && taken);
    if (eq) {
      if (k < lo || k > hi) return false;
      lo = hi = k;
    } else if (ne) {
      if (lo == hi && lo == k) return false;
      if (lo == k) lo++;
      else if (hi == k) hi--;
    } else if ((o == 0x20 && taken) || (o == 0xb0 && !taken)) {  // a > k
      if (k == ~0ull) return false;
      lo = std::max(lo, k + 1);
    } else if ((o == 0x20 && !taken) || (o == 0xb0 && taken)) {  // a <= k
      hi = std::min(hi, k);
    } else if ((o == 0x30 && taken) || (o == 0xa0 && !taken)) {  // a >= k
      lo = std::max(lo, k);
    } else if ((o == 0x30 && !taken) || (o == 0xa0 && taken)) {  // a < k
      if (k == 0) return false;
      hi = std::min(hi, k - 1);
    } else {
      return true;
    }
    if (lo > hi) return false;
    a = scal(a.b, lo, hi);
    return true;
  }

  using Edges = std::vector<std::pair<int, State>>;

  Edges step(int pc, State s) {
    const Insn& in = P[pc];
    seen_[pc] = 1;
    if (++s.steps > kMaxDynInsns) fail(pc, "dynamic instruction budget exceeded");
    Edges e;
    int nx = pc + 1;
    int c = cls(in), o = opc(in);
    bool x = xsrc(in);
    static const int kSize[4] = {4, 2, 1, 8};
    switch (c) {
      case 4:
      case 7: {
        bool w64 = c == 7;
        if (o == 0x80 || o == 0xd0) {
          const Val& a = use(s, pc, in.dst);
          if (a.t != T_SCALAR) fail(pc, "arithmetic on a pointer");
          const bool ln = a.lanes;
          s.r[in.dst] = alu(pc, w64, in, a, sconst(0));
          s.r[in.dst].lanes = ln;
          break;
        }
        Val b = x ? use(s, pc, in.src) : sconst(w64 ? (uint64_t)(int64_t)in.imm : (uint64_t)(uint32_t)in.imm);
        if (o == 0xb0 && w64 && in.off == 0) {
          s.r[in.dst] = b;
          break;
        }
        if (o == 0xb0) {
          if (b.t != T_SCALAR) fail(pc, "pointer truncated or sign-extended");
          s.r[in.dst] = alu(pc, w64, in, sconst(0), b);
          s.r[in.dst].lanes = b.lanes;
          break;
        }
        const Val a = use(s, pc, in.dst);
        if (a.t == T_SCALAR && b.t == T_SCALAR) {
          s.r[in.dst] = alu(pc, w64, in, a, b);
          s.r[in.dst].lanes = a.lanes || b.lanes;
          break;
        }
        if (!w64 || b.t != T_SCALAR || (o != 0x00 && o != 0x10) || (a.t != T_STACK && a.t != T_MAPVAL))
          fail(pc, "invalid pointer arithmetic");
        Val r = a;
        if (is_const(b)) {
          int64_t d = (int64_t)b.lo;
          if (o == 0x10) d = -d;
          r.lo = (uint64_t)((int64_t)a.lo + d);
          r.hi = (uint64_t)((int64_t)a.hi + d);
          r.b = badd(a.b, bconst((uint64_t)d));
        } else if (b.hi < (1ull << 32)) {
          if (o == 0x00) {
            r.lo = (uint64_t)((int64_t)a.lo + (int64_t)b.lo);
            r.hi = (uint64_t)((int64_t)a.hi + (int64_t)b.hi);
            r.b = badd(a.b, b.b);
          } else {
            r.lo = (uint64_t)((int64_t)a.lo - (int64_t)b.hi);
            r.hi = (uint64_t)((int64_t)a.hi - (int64_t)b.lo);
            r.b = bsub(a.b, b.b);
          }
        } else {
          fail(pc, "pointer offset is unbounded");
        }
        if ((int64_t)r.lo < -(1ll << 32) || (int64_t)r.hi > (1ll << 32)) fail(pc, "pointer offset out of range");
        r.lanes = a.lanes || b.lanes;
        s.r[in.dst] = r;
        break;
      }
      case 5:
      case 6: {
        bool w32 = c == 6;
        if (o == 0x90) {
          if (use(s, pc, 0).t != T_SCALAR) fail(pc, "r0 must hold a scalar at exit");
          out_.max_insns = std::max(out_.max_insns, s.steps);
          out_.max_calls = std::max(out_.max_calls, s.calls);
          out_.max_ring = std::max(out_.max_ring, s.ring);
          return e;
        }
        if (o == 0x80) {
          helper(s, pc, in.imm);
          break;
        }
        int t = target(pc);
        if (o == 0x00) {
          e.push_back({t, s});
          return e;
        }
        const Val& a = use(s, pc, in.dst);
        Val b = x ? use(s, pc, in.src) : sconst(w32 ? (uint64_t)(uint32_t)in.imm : (uint64_t)(int64_t)in.imm);
        if (simt_ && (a.lanes || b.lanes)) fail(pc, "SIMT hook: the branch condition varies by lane");
        if (a.t == T_MAPVAL || a.t == T_MAPVAL_NULL) {
          if (w32 || x || in.imm || (o != 0x10 && o != 0x50)) fail(pc, "only a null check may compare a pointer");
          State nonnull = s, null = s;
          nonnull.r[in.dst].t = T_MAPVAL;
          null.r[in.dst] = sconst(0);
          bool maybe_null = a.t == T_MAPVAL_NULL;
          int tk = o == 0x10 ? 1 : 0;  // jeq: taken when null
          if (tk) {
            if (maybe_null) e.push_back({t, null});
            e.push_back({nx, nonnull});
          } else {
            e.push_back({t, nonnull});
            if (maybe_null) e.push_back({nx, null});
          }
          return e;
        }
        if (a.t != T_SCALAR || b.t != T_SCALAR) fail(pc, "comparison with a pointer");
        int d = decide(o, a, b, w32);
        bool nar = !w32 && is_const(b);
        if (d != 0) {
          State st = s;
          if (!nar || narrow(st.r[in.dst], o, b.lo, true)) e.push_back({t, st});
        }
        if (d != 1) {
          State sf = s;
          if (!nar || narrow(sf.r[in.dst], o, b.lo, false)) e.push_back({nx, sf});
        }
        return e;
      }
      case 1: {
        int sz = kSize[(in.op >> 3) & 3];
        Val base = use(s, pc, in.src);
        const bool ln = access(s, pc, base, in.off, sz, 0);
        bool sx = (in.op & 0xe0) == 0x80;
        s.r[in.dst] = (sz == 8 || sx) ? sany() : scal(Bits{0, (1ull << (8 * sz)) - 1}, 0, (1ull << (8 * sz)) - 1);
        s.r[in.dst].lanes = ln;
        break;
      }
      case 2: {
        int sz = kSize[(in.op >> 3) & 3];
        Val base = use(s, pc, in.dst);
        access(s, pc, base, in.off, sz, 1);
        break;
      }
      case 3: {
        int sz = kSize[(in.op >> 3) & 3];
        Val base = use(s, pc, in.dst);
        const Val& sv = use(s, pc, in.src);
        if (sv.t != T_SCALAR) fail(pc, "pointers cannot be stored to memory");
        const bool sl = sv.lanes;
        if ((in.op & 0xe0) == 0x60) {
          access(s, pc, base, in.off, sz, 1, sl);
          break;
        }
        bool reads = in.imm & 1;
        if (in.imm == 0xf1 && use(s, pc, 0).t != T_SCALAR) fail(pc, "cmpxchg compares against a scalar r0");
        const bool ol = access(s, pc, base, in.off, sz, reads ? 3 : 2, sl || (in.imm == 0xf1 && s.r[0].lanes));
        Val old = sz == 8 ? sany() : s32any();
        old.lanes = ol;
        if (in.imm == 0xf1) s.r[0] = old;
        else if (reads) s.r[in.src] = old;
        break;
      }
      case 0: {
        if (in.src == 0) {
          s.r[in.dst] = sconst((uint64_t)(uint32_t)in.imm | ((uint64_t)(uint32_t)P[pc + 1].imm << 32));
        } else {
          int m = -1;
          if (in.src == 5) {
            if (in.imm >= 0 && in.imm < (int)maps_.size()) m = in.imm;
          } else {
            for (size_t k = 0; k < fds_.size(); k++)
              if (fds_[k] == in.imm) m = (int)k;
          }
          if (m < 0) fail(pc, "unknown map reference");
          if (out_.ld_map[pc] >= 0 && out_.ld_map[pc] != m) fail(pc, "map reference differs");
          out_.ld_map[pc] = m;
          Val v;
          v.t = T_MAP;
          v.map = m;
          v.b = bconst(0);
          v.lo = v.hi = 0;
          s.r[in.dst] = v;
        }
        nx = pc + 2;
        break;
      }
    }
    e.push_back({nx, s});
    return e;
  }

  // Walk slots lo..hi in order from ``in`` at ``lo``; edges beyond hi go to
  // ``out``; the back-edge hi -> lo (when ``back``) is joined into *back.
  void walk(int lo, int hi, const State& in, std::map<int, State>& out, State* back) {
    std::map<int, State> pend;
    pend[lo] = in;
    int pc = lo;
    while (pc <= hi) {
      auto it = pend.find(pc);
      if (it == pend.end()) {
        pc += is_lddw(pc) ? 2 : 1;
        continue;
      }
      State s = std::move(it->second);
      pend.erase(it);
      int j = back_of_head_[pc];
      if (j >= 0 && !(back && pc == lo)) {
        loop(pc, j, s, pend, hi, out);
        pc = j + 1;
        continue;
      }
      for (auto& ed : step(pc, std::move(s))) {
        int t = ed.first;
        if (back && pc == hi && t == lo) sjoin(*back, ed.second);
        else if (t > pc && t <= hi) sjoin(pend[t], ed.second);
        else if (t > hi) sjoin(out[t], ed.second);
        else fail(pc, "backward jump outside a counted loop");
      }
      pc += is_lddw(pc) ? 2 : 1;
    }
  }

  void loop(int h, int j, State s, std::map<int, State>& pend, int hi, std::map<int, State>& out) {
    int c = P[j].dst;
    if (!is_const(s.r[c])) fail(h, "loop counter is not a constant when the loop is entered");
    std::map<int, State> ex;
    for (uint64_t trip = 0;; trip++) {
      if (trip > kMaxDynInsns) fail(j, "loop runs too many times");
      State nb;
      walk(h, j, s, ex, &nb);
      if (!nb.live) break;
      s = std::move(nb);
    }
    for (auto& kv : ex) {
      if (kv.first <= hi) sjoin(pend[kv.first], kv.second);
      else sjoin(out[kv.first], kv.second);
    }
  }
};

}  // namespace

Verdict verify(const std::vector<Insn>& prog, int hook, const std::vector<MapShape>& table,
               const std::vector<int>& fds) {
  Verifier v(prog, hook, table, fds);
  return v.run();
}

}  // namespace gx
