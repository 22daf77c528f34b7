// CPU oracle: bounds and termination checker.  Test infrastructure only.
//
// Rule classes follow the paper's verification model (section 4.4): the
// program must terminate (bounded loops), access memory safely and type-
// correctly, and stay within per-hook resource budgets; device code may not
// use global synchronisation, and shared state takes only commutative
// updates.  Concrete rules:
//   * at most 4096 slots; valid encodings; jump targets in range and not into
//     the second slot of lddw; every slot reachable; no fall-through past the
//     end;
//   * back-edges only in canonical counted form: the back-edge is a 64-bit
//     conditional jump comparing a counter register with a constant, directly
//     preceded by the only write of that counter inside the loop (add/sub of a
//     non-zero constant); loops nest properly and are entered at their head;
//   * abstract interpretation over unsigned intervals plus known trailing
//     zero bits; loops are unrolled iteration by iteration with the exact
//     counter value, so the dynamic instruction bound is exact per path;
//   * ctx is read-only at exact field offsets and sizes; the stack is
//     r10 + [-512, 0) at constant, naturally aligned offsets and must be
//     written before it is read; map values need a null check and an offset
//     range inside the value, naturally aligned; pointers may not be stored,
//     compared (other than the null check) or leaked into r0;
//   * shared maps take only lookups and commutative atomics without fetch;
//     read-only maps take only lookups and loads; value pointers into a hash
//     map die at the next update or delete of that map;
//   * budgets: 65536 dynamic instructions, 64 helper calls and 4096 ring
//     bytes per invocation;
//   * SIMT hook: every value is warp-uniform or lane-varying (the record's
//     fields vary, its tile's aggregate is uniform; results vary if an
//     operand does; stack bytes carry the kind of what was stored); branch
//     conditions (loop bounds included), map keys, ring records and their
//     flags, and the addresses of map atomics must be uniform; the maps must
//     be shared, read-only or ring buffers; fetching atomics on maps are
//     refused; an atomic's operand may vary (the device combines a wave's
//     operands into one update).
#include <algorithm>
#include <functional>
#include <map>
#include <sstream>

#include "gxo.h"

namespace gxo {
namespace {

constexpr uint64_t kMaxSteps = 65536;
constexpr uint64_t kMaxCalls = 64;
constexpr uint64_t kMaxRing = 4096;
constexpr uint64_t kMaxTrips = 65536;
const int kSz[4] = {4, 2, 1, 8};

enum AK : uint8_t { A_UNINIT, A_SCALAR, A_CTX, A_STACK, A_MAPVAL, A_MAPVAL_OR_NULL, A_MAP, A_BAD };

struct AV {
  AK k = A_UNINIT;
  uint64_t lo = 0, hi = 0;  // scalar: unsigned range; pointer: signed offset range
  int tz = 0;               // known trailing zero bits
  int map = -1;
  bool var = false;         // lane-varying (SIMT hook)
};

int ctz64(uint64_t v) { return v ? __builtin_ctzll(v) : 64; }

AV exact(uint64_t v) { return AV{A_SCALAR, v, v, ctz64(v), -1}; }
AV unknown() { return AV{A_SCALAR, 0, ~0ull, 0, -1}; }
AV range(uint64_t lo, uint64_t hi, int tz) { return AV{A_SCALAR, lo, hi, std::min(tz, 64), -1}; }

struct AState {
  bool live = false;
  AV r[11];
  uint8_t stk[STACK_BYTES];
  uint8_t stkvar[STACK_BYTES];  // byte holds a lane-varying value (SIMT hook)
  uint64_t steps = 0, calls = 0, ring = 0;
};

AV join_v(const AV& a, const AV& b) {
  if (a.k == A_UNINIT || b.k == A_UNINIT) return AV{};
  if (a.k == A_BAD || b.k == A_BAD) return AV{A_BAD};
  AK k = a.k;
  if (a.k != b.k) {
    bool mv = (a.k == A_MAPVAL || a.k == A_MAPVAL_OR_NULL) && (b.k == A_MAPVAL || b.k == A_MAPVAL_OR_NULL);
    if (!mv || a.map != b.map) return AV{A_BAD};
    k = A_MAPVAL_OR_NULL;
  }
  if (k != A_SCALAR && a.map != b.map) return AV{A_BAD};
  AV r = a;
  r.k = k;
  if (k == A_SCALAR) {
    r.lo = std::min(a.lo, b.lo);
    r.hi = std::max(a.hi, b.hi);
  } else {
    r.lo = (uint64_t)std::min((int64_t)a.lo, (int64_t)b.lo);
    r.hi = (uint64_t)std::max((int64_t)a.hi, (int64_t)b.hi);
  }
  r.tz = std::min(a.tz, b.tz);
  r.var = a.var || b.var;
  return r;
}

void join_into(AState& dst, const AState& src) {
  if (!src.live) return;
  if (!dst.live) {
    dst = src;
    return;
  }
  for (int i = 0; i < 11; i++) dst.r[i] = join_v(dst.r[i], src.r[i]);
  for (int i = 0; i < STACK_BYTES; i++) dst.stk[i] = dst.stk[i] && src.stk[i];
  for (int i = 0; i < STACK_BYTES; i++) dst.stkvar[i] = dst.stkvar[i] || src.stkvar[i];
  dst.steps = std::max(dst.steps, src.steps);
  dst.calls = std::max(dst.calls, src.calls);
  dst.ring = std::max(dst.ring, src.ring);
}

struct Reject {
  std::string msg;
};

bool mul_ovf(uint64_t a, uint64_t b, uint64_t* r) { return __builtin_mul_overflow(a, b, r); }

uint64_t bits_mask(uint64_t hi) {  // smallest 2^k - 1 >= hi
  uint64_t m = hi;
  for (int s = 1; s < 64; s <<= 1) m |= m >> s;
  return m;
}

// Concrete semantics for exact operands (same definitions as the interpreter,
// written out again here so the checker stands on its own).
uint64_t c_sext(uint64_t v, int bits) {
  if (bits >= 64) return v;
  uint64_t m = 1ull << (bits - 1);
  v &= (1ull << bits) - 1;
  return (v ^ m) - m;
}
uint64_t c_bswap(uint64_t v, int bits) {
  uint64_t r = 0;
  for (int i = 0; i < bits / 8; i++) r = (r << 8) | ((v >> (8 * i)) & 0xff);
  return r;
}
uint64_t concrete(bool is64, int code, int16_t off, bool x, int32_t imm, uint64_t a, uint64_t b) {
  if (is64) {
    int64_t sa = (int64_t)a, sb = (int64_t)b;
    switch (code) {
      case 0x00: return a + b;
      case 0x10: return a - b;
      case 0x20: return a * b;
      case 0x30: return b == 0 ? 0 : off == 0 ? a / b : (sa == INT64_MIN && sb == -1) ? a : (uint64_t)(sa / sb);
      case 0x40: return a | b;
      case 0x50: return a & b;
      case 0x60: return a << (b & 63);
      case 0x70: return a >> (b & 63);
      case 0x80: return 0 - a;
      case 0x90: return b == 0 ? a : off == 0 ? a % b : sb == -1 ? 0 : (uint64_t)(sa % sb);
      case 0xa0: return a ^ b;
      case 0xb0: return (x && off) ? c_sext(b, off) : b;
      case 0xc0: return (uint64_t)(sa >> (b & 63));
      case 0xd0: return c_bswap(a, imm);
    }
    return 0;
  }
  uint32_t a3 = (uint32_t)a, b3 = (uint32_t)b;
  int32_t sa = (int32_t)a3, sb = (int32_t)b3;
  switch (code) {
    case 0x00: return (uint32_t)(a3 + b3);
    case 0x10: return (uint32_t)(a3 - b3);
    case 0x20: return (uint32_t)(a3 * b3);
    case 0x30: return b3 == 0 ? 0 : off == 0 ? a3 / b3 : (sa == INT32_MIN && sb == -1) ? a3 : (uint32_t)(sa / sb);
    case 0x40: return a3 | b3;
    case 0x50: return a3 & b3;
    case 0x60: return (uint32_t)(a3 << (b3 & 31));
    case 0x70: return a3 >> (b3 & 31);
    case 0x80: return (uint32_t)(0u - a3);
    case 0x90: return b3 == 0 ? a3 : off == 0 ? a3 % b3 : sb == -1 ? 0 : (uint32_t)(sa % sb);
    case 0xa0: return a3 ^ b3;
    case 0xb0: return (x && off) ? (uint32_t)c_sext(b, off) : b3;
    case 0xc0: return (uint32_t)(sa >> (b3 & 31));
    case 0xd0: return x ? c_bswap(a, imm) : (imm == 64 ? a : a & ((1ull << imm) - 1));
  }
  return 0;
}

// Abstract transfer for scalar ALU operations.
AV alu_scalar(bool is64, int code, int16_t off, bool x, int32_t imm, const AV& a, const AV& b) {
  bool ae = a.lo == a.hi, be = b.lo == b.hi;
  if (code == 0xb0 && !(x && off)) {  // plain MOV
    if (is64) return b;
    if (b.hi <= 0xffffffffull) return b;
    return be ? exact((uint32_t)b.lo) : range(0, 0xffffffffull, b.tz);
  }
  if ((ae || code == 0xd0 || code == 0x80) && be) {
    if (code == 0xd0 || code == 0x80) {
      if (ae) return exact(concrete(is64, code, off, x, imm, a.lo, 0));
    } else {
      return exact(concrete(is64, code, off, x, imm, a.lo, b.lo));
    }
  }
  uint64_t r;
  if (is64) {
    switch (code) {
      case 0x00:
        if (!__builtin_add_overflow(a.hi, b.hi, &r)) return range(a.lo + b.lo, r, std::min(a.tz, b.tz));
        return range(0, ~0ull, std::min(a.tz, b.tz));
      case 0x10:
        if (a.lo >= b.hi) return range(a.lo - b.hi, a.hi - b.lo, std::min(a.tz, b.tz));
        return range(0, ~0ull, std::min(a.tz, b.tz));
      case 0x20:
        if (!mul_ovf(a.hi, b.hi, &r)) return range(a.lo * b.lo, r, a.tz + b.tz);
        return range(0, ~0ull, a.tz + b.tz);
      case 0x30:
        if (off == 0 && be && b.lo) return range(a.lo / b.lo, a.hi / b.lo, 0);
        return unknown();
      case 0x90:
        if (off == 0 && be && b.lo) return range(0, std::min(a.hi, b.lo - 1), 0);
        return unknown();
      case 0x50:
        return range(0, std::min(a.hi, b.hi), std::max(a.tz, b.tz));
      case 0x40:
      case 0xa0:
        return range(0, bits_mask(std::max(a.hi, b.hi)), std::min(a.tz, b.tz));
      case 0x60:
        if (be) {
          int k = (int)(b.lo & 63);
          if (k == 0 || (a.hi >> (64 - k)) == 0) return range(a.lo << k, a.hi << k, a.tz + k);
          return range(0, ~0ull, a.tz + k);
        }
        return unknown();
      case 0x70:
        if (be) {
          int k = (int)(b.lo & 63);
          return range(a.lo >> k, a.hi >> k, std::max(0, a.tz - k));
        }
        return range(0, a.hi, 0);
      case 0xc0:
        if (be && a.hi < (1ull << 63)) {
          int k = (int)(b.lo & 63);
          return range(a.lo >> k, a.hi >> k, std::max(0, a.tz - k));
        }
        return unknown();
    }
    return unknown();
  }
  // 32-bit: result is always zero-extended
  AV full = range(0, 0xffffffffull, 0);
  switch (code) {
    case 0x00:
      if (a.hi <= 0xffffffffull && b.hi <= 0xffffffffull && a.hi + b.hi <= 0xffffffffull)
        return range(a.lo + b.lo, a.hi + b.hi, std::min(a.tz, b.tz));
      return range(0, 0xffffffffull, std::min({a.tz, b.tz, 32}));
    case 0x50: {
      uint64_t h = std::min({a.hi, b.hi, (uint64_t)0xffffffffull});
      return range(0, h, std::min(32, std::max(a.tz, b.tz)));
    }
    case 0x70:
      if (be && a.hi <= 0xffffffffull) {
        int k = (int)(b.lo & 31);
        return range(a.lo >> k, a.hi >> k, std::max(0, a.tz - k));
      }
      return full;
    case 0x90:
      if (off == 0 && be && (uint32_t)b.lo) return range(0, std::min<uint64_t>(a.hi, (uint32_t)b.lo - 1), 0);
      return full;
    case 0xd0:  // END in the 32-bit class keeps imm bits, up to 64
      return imm >= 64 ? unknown() : range(0, (1ull << imm) - 1, 0);
  }
  return full;
}

struct Checker {
  const std::vector<Insn>& ins;
  int n;
  int hook;
  bool simt;  // SIMT hook: uniformity rules apply
  HookInfo hi;
  const std::vector<MapShape>& maps;
  const std::vector<int>& table;
  std::vector<int> loop_end;  // header -> back-edge pc
  std::vector<char> is_second;
  CheckResult res;
  int min_stack = STACK_BYTES;
  std::vector<char> map_used;
  std::vector<int> shared_op;  // per shared map: the one (atomic op, size) it takes, or -1

  Checker(const std::vector<Insn>& i, int h, const std::vector<MapShape>& m, const std::vector<int>& t)
      : ins(i), n((int)i.size()), hook(h), simt(h == HOOK_SIMT_MEM), maps(m), table(t) {}

  [[noreturn]] void rej(int pc, const std::string& m) {
    std::ostringstream os;
    os << "insn " << pc << ": " << m;
    throw Reject{os.str()};
  }

  static bool is_lddw(const Insn& in) { return in.op == 0x18; }

  // ---------------- structural checks ----------------
  void check_encoding(int pc) {
    const Insn& in = ins[pc];
    int cls = in.op & 7, code = in.op & 0xf0;
    bool x = in.op & 8;
    if (in.dst > 10 || in.src > 10) rej(pc, "bad register");
    switch (cls) {
      case 4:
      case 7: {
        bool is64 = cls == 7;
        if (code == 0xe0 || code == 0xf0) rej(pc, "unknown ALU op");
        if (code == 0x80) {
          if (x || in.src || in.off || in.imm) rej(pc, "bad NEG encoding");
        } else if (code == 0xd0) {
          if (in.src || in.off || (in.imm != 16 && in.imm != 32 && in.imm != 64)) rej(pc, "bad END encoding");
          if (is64 && x) rej(pc, "bad BSWAP encoding");
        } else {
          if (!x && in.src) rej(pc, "reserved src field set");
          if (x && in.imm) rej(pc, "reserved imm field set");
          bool okoff = in.off == 0;
          if ((code == 0x30 || code == 0x90) && in.off == 1) okoff = true;
          if (code == 0xb0 && x && (in.off == 8 || in.off == 16 || (is64 && in.off == 32))) okoff = true;
          if (!okoff) rej(pc, "reserved off field set");
          if (!x && (code == 0x30 || code == 0x90) && in.imm == 0) rej(pc, "division by constant zero");
          if (!x && (code == 0x60 || code == 0x70 || code == 0xc0) &&
              (in.imm < 0 || in.imm >= (is64 ? 64 : 32)))
            rej(pc, "constant shift out of range");
        }
        if (in.dst == 10) rej(pc, "write to r10");
        break;
      }
      case 5:
      case 6: {
        bool is32 = cls == 6;
        if (code == 0xe0 || code == 0xf0) rej(pc, "unknown jump op");
        if (code == 0x80) {
          if (is32 || x || in.src || in.dst || in.off) rej(pc, "bad CALL encoding");
        } else if (code == 0x90) {
          if (is32 || x || in.src || in.dst || in.off || in.imm) rej(pc, "bad EXIT encoding");
        } else if (code == 0x00) {
          if (x || in.src || in.dst || (is32 ? in.off : in.imm)) rej(pc, "bad JA encoding");
        } else {
          if (!x && in.src) rej(pc, "reserved src field set");
          if (x && in.imm) rej(pc, "reserved imm field set");
        }
        break;
      }
      case 1: {
        int mode = in.op & 0xe0;
        if (mode != 0x60 && mode != 0x80) rej(pc, "unsupported load mode");
        if (mode == 0x80 && (in.op & 0x18) == 0x18) rej(pc, "bad sign-extending load size");
        if (in.imm) rej(pc, "reserved imm field set");
        if (in.dst == 10) rej(pc, "write to r10");
        break;
      }
      case 2:
        if ((in.op & 0xe0) != 0x60 || in.src) rej(pc, "bad ST encoding");
        break;
      case 3: {
        int mode = in.op & 0xe0;
        if (mode == 0x60) {
          if (in.imm) rej(pc, "reserved imm field set");
        } else if (mode == 0xc0) {
          int sz = in.op & 0x18;
          if (sz != 0x00 && sz != 0x18) rej(pc, "bad atomic size");
          switch (in.imm) {
            case 0x00: case 0x40: case 0x50: case 0xa0:
            case 0x01: case 0x41: case 0x51: case 0xa1:
            case 0xe1: case 0xf1: break;
            default: rej(pc, "bad atomic op");
          }
        } else {
          rej(pc, "unsupported store mode");
        }
        break;
      }
      case 0:
        if (in.op != 0x18) rej(pc, "unsupported LD instruction");
        if (in.off) rej(pc, "reserved off field set");
        if (in.src != 0 && in.src != 1 && in.src != 5) rej(pc, "unsupported lddw source");
        if (pc + 1 >= n) rej(pc, "truncated lddw");
        {
          const Insn& s2 = ins[pc + 1];
          if (s2.op || s2.dst || s2.src || s2.off) rej(pc + 1, "bad second lddw slot");
          if (in.src && s2.imm) rej(pc + 1, "map reference with high bits");
        }
        if (in.dst == 10) rej(pc, "write to r10");
        break;
    }
  }

  int jump_target(int pc) {
    const Insn& in = ins[pc];
    int cls = in.op & 7;
    return pc + 1 + ((cls == 6 && (in.op & 0xf0) == 0) ? in.imm : in.off);
  }
  bool is_jump(const Insn& in) {
    int cls = in.op & 7, code = in.op & 0xf0;
    return (cls == 5 || cls == 6) && code != 0x80 && code != 0x90;
  }
  bool falls_through(const Insn& in) {
    int cls = in.op & 7, code = in.op & 0xf0;
    if (cls == 5 || cls == 6) return !(code == 0x90 || code == 0x00);
    return true;
  }

  bool writes_reg(const Insn& in, int r) {
    int cls = in.op & 7, code = in.op & 0xf0;
    switch (cls) {
      case 4: case 7: case 1: case 0: return in.dst == r;
      case 5: return code == 0x80 && r <= 5;
      case 3:
        if ((in.op & 0xe0) == 0xc0) {
          if (in.imm == 0xf1) return r == 0;
          if (in.imm & 1) return in.src == r;
        }
        return false;
    }
    return false;
  }

  void structure() {
    if (n == 0) throw Reject{"empty program"};
    if (n > MAX_INSNS) throw Reject{"too many instructions"};
    is_second.assign(n, 0);
    for (int pc = 0; pc < n; pc++) {
      if (is_second[pc]) continue;
      check_encoding(pc);
      if (is_lddw(ins[pc])) is_second[pc + 1] = 1;
    }
    // jump targets, fall-through past the end, reachability
    std::vector<char> reach(n, 0);
    std::vector<int> work{0};
    reach[0] = 1;
    while (!work.empty()) {
      int pc = work.back();
      work.pop_back();
      const Insn& in = ins[pc];
      int next = pc + (is_lddw(in) ? 2 : 1);
      std::vector<int> succ;
      if (is_jump(in)) {
        int t = jump_target(pc);
        if (t < 0 || t >= n) rej(pc, "jump out of range");
        if (is_second[t]) rej(pc, "jump into the middle of lddw");
        succ.push_back(t);
      }
      if (falls_through(in)) {
        if (next >= n) rej(pc, "falls off the end of the program");
        succ.push_back(next);
      }
      for (int t : succ)
        if (!reach[t]) {
          reach[t] = 1;
          work.push_back(t);
        }
    }
    for (int pc = 0; pc < n; pc++)
      if (!is_second[pc] && !reach[pc]) rej(pc, "unreachable instruction");
    // loops
    loop_end.assign(n, -1);
    std::vector<std::pair<int, int>> loops;
    for (int j = 0; j < n; j++) {
      if (is_second[j] || !is_jump(ins[j])) continue;
      int h = jump_target(j);
      if (h > j) continue;
      const Insn& be = ins[j];
      int cls = be.op & 7, code = be.op & 0xf0;
      if (cls != 5 || code == 0x00 || (be.op & 8)) rej(j, "unbounded loop (back-edge is not a counted compare with a constant)");
      int c = be.dst;
      if (j - 1 < h) rej(j, "unbounded loop (no counter update)");
      const Insn& inc = ins[j - 1];
      bool add_or_sub_k = inc.op == 0x07 || inc.op == 0x17;  // ALU64 ADD K / SUB K
      if (is_second[j - 1] || !add_or_sub_k || inc.dst != c || inc.imm == 0)
        rej(j, "unbounded loop (counter update must directly precede the back-edge)");
      if (loop_end[h] >= 0) rej(j, "two back-edges to one loop head");
      for (int p = h; p < j - 1; p++)
        if (!is_second[p] && writes_reg(ins[p], c)) rej(p, "loop counter written inside the loop body");
      loop_end[h] = j;
      loops.push_back({h, j});
    }
    for (auto& a : loops)
      for (auto& b : loops) {
        if (&a == &b) continue;
        bool disjoint = a.second < b.first || b.second < a.first;
        bool nested = (a.first <= b.first && b.second <= a.second) || (b.first <= a.first && a.second <= b.second);
        if (!disjoint && !nested) rej(a.first, "overlapping loops");
        if (a.first == b.first) rej(a.first, "two loops share a head");
      }
    for (int p = 0; p < n; p++) {
      if (is_second[p] || !is_jump(ins[p])) continue;
      int t = jump_target(p);
      for (auto& L : loops) {
        bool inside = p >= L.first && p <= L.second;
        if (!inside && t > L.first && t <= L.second) rej(p, "jump into the middle of a loop");
        if (inside && p != L.second && t == L.second) rej(p, "jump skips the loop counter update");
      }
    }
  }

  // ---------------- abstract interpretation ----------------
  const AV& rd(const AState& s, int pc, int r) {
    const AV& v = s.r[r];
    if (v.k == A_UNINIT) rej(pc, "read of uninitialised r" + std::to_string(r));
    if (v.k == A_BAD) rej(pc, "r" + std::to_string(r) + " has no single type here (or was invalidated)");
    return v;
  }

  int map_of_ref(int pc, const Insn& in) {
    int id = -1;
    if (in.src == 5) {
      if (in.imm < 0 || in.imm >= (int)table.size()) rej(pc, "bad map index");
      id = table[in.imm];
    } else {
      for (int t : table)
        if (t == in.imm) id = t;
    }
    if (id < 0 || id >= (int)maps.size()) rej(pc, "bad map reference");
    return id;
  }

  // Check an access of ``size`` bytes at base + off; mode 0 load, 1 store,
  // 2 commutative atomic, 3 fetching atomic.  ``sv``: whether the stored
  // value is lane-varying.  Returns whether the bytes read are.
  bool access(AState& s, int pc, const AV& b, int64_t off, int size, int mode, bool sv = false) {
    if (b.k == A_CTX) {
      if (mode != 0) rej(pc, "write to ctx");
      for (auto& f : hi.fields)
        if ((int64_t)f.first == off && (int)f.second == size) return simt && (uint64_t)off < hi.uniform_off;
      rej(pc, "bad ctx access");
    }
    if (b.k == A_STACK) {
      if (b.lo != b.hi) rej(pc, "variable-offset stack access");
      int64_t o = (int64_t)b.lo + off;
      if (o < 0 || o + size > STACK_BYTES) rej(pc, "stack access out of bounds");
      if (o % size) rej(pc, "misaligned stack access");
      if (mode != 1)
        for (int i = 0; i < size; i++)
          if (!s.stk[o + i]) rej(pc, "read of uninitialised stack");
      bool v = false;
      if (mode != 1)
        for (int i = 0; i < size; i++) v = v || s.stkvar[o + i];
      if (mode != 0)
        for (int i = 0; i < size; i++) {
          s.stk[o + i] = 1;
          s.stkvar[o + i] = mode == 1 ? sv : (s.stkvar[o + i] || sv);
        }
      min_stack = std::min<int>(min_stack, (int)o);
      return v;
    }
    if (b.k == A_MAPVAL) {
      const MapShape& m = maps[b.map];
      int64_t lo = (int64_t)b.lo + off, hi2 = (int64_t)b.hi + off;
      if (lo < 0 || hi2 + size > (int64_t)m.value_size) rej(pc, "map value access out of bounds");
      if (lo % size) rej(pc, "misaligned map value access");
      if (b.lo != b.hi && b.tz < __builtin_ctz(size)) rej(pc, "possibly misaligned map value access");
      if (simt && mode != 0 && b.var) rej(pc, "lane-varying map address of an update (SIMT hook)");
      if (simt && mode == 3) rej(pc, "fetching atomic on a map (SIMT hook: non-uniform atomic)");
      if ((m.flags & F_READ_ONLY) && mode != 0) rej(pc, "write to read-only map");
      if ((m.flags & F_SHARED) && mode != 2) rej(pc, "shared map takes only commutative atomics");
      if (m.flags & F_SHARED) {
        // updates commute only if every update of the map is the same
        // operation at the same width
        int key = (ins[pc].imm & 0xff) | (size << 8);
        if (shared_op[b.map] < 0) shared_op[b.map] = key;
        else if (shared_op[b.map] != key) rej(pc, "shared map updated with different atomic operations");
      }
      return b.var;
    }
    if (b.k == A_MAPVAL_OR_NULL) rej(pc, "map value access without null check");
    rej(pc, "memory access through non-pointer");
  }

  // A helper's memory argument; ``what`` names it when the SIMT hook needs
  // it warp-uniform (nullptr: it may vary).
  void arg_mem(AState& s, int pc, int reg, uint32_t nbytes, const char* what = nullptr) {
    const AV& b = rd(s, pc, reg);
    if (b.k == A_STACK) {
      if (b.lo != b.hi) rej(pc, "variable-offset stack argument");
      int64_t o = (int64_t)b.lo;
      if (o < 0 || o + (int64_t)nbytes > STACK_BYTES) rej(pc, "stack argument out of bounds");
      for (uint32_t i = 0; i < nbytes; i++)
        if (!s.stk[o + i]) rej(pc, "helper reads uninitialised stack");
      if (simt && what)
        for (uint32_t i = 0; i < nbytes; i++)
          if (s.stkvar[o + i]) rej(pc, std::string("lane-varying ") + what + " (SIMT hook)");
      min_stack = std::min<int>(min_stack, (int)o);
      return;
    }
    if (b.k == A_MAPVAL) {
      const MapShape& m = maps[b.map];
      if ((int64_t)b.lo < 0 || (int64_t)b.hi + (int64_t)nbytes > (int64_t)m.value_size)
        rej(pc, "map value argument out of bounds");
      if (m.flags & F_SHARED) rej(pc, "shared map value used as helper input");
      if (simt && what && b.var) rej(pc, std::string("lane-varying ") + what + " (SIMT hook)");
      return;
    }
    rej(pc, "helper memory argument must point to stack or a map value");
  }

  int map_arg(const AState& s, int pc, int reg) {
    const AV& b = rd(s, pc, reg);
    if (b.k != A_MAP) rej(pc, "helper argument r" + std::to_string(reg) + " is not a map");
    map_used[b.map] = 1;
    return b.map;
  }

  void call(AState& s, int pc, int32_t id) {
    if (id == H_LOOKUP) {
      int m = map_arg(s, pc, 1);
      if (maps[m].type == MAP_RINGBUF) rej(pc, "lookup on a ring buffer");
      arg_mem(s, pc, 2, maps[m].key_size, "map key");
      s.r[0] = AV{A_MAPVAL_OR_NULL, 0, 0, 64, m};
    } else if (id == H_UPDATE || id == H_DELETE) {
      int m = map_arg(s, pc, 1);
      if (maps[m].type == MAP_RINGBUF) rej(pc, "update/delete on a ring buffer");
      if (maps[m].flags & (F_SHARED | F_READ_ONLY)) rej(pc, "update/delete on a shared or read-only map");
      arg_mem(s, pc, 2, maps[m].key_size, "map key");
      if (id == H_UPDATE) {
        arg_mem(s, pc, 3, maps[m].value_size, "map update value");
        if (rd(s, pc, 4).k != A_SCALAR) rej(pc, "update flags must be a scalar");
      }
      if (maps[m].type == MAP_HASH)
        for (auto& v : s.r)
          if ((v.k == A_MAPVAL || v.k == A_MAPVAL_OR_NULL) && v.map == m) v = AV{A_BAD};
      s.r[0] = unknown();
    } else if (id == H_RINGBUF_OUTPUT) {
      int m = map_arg(s, pc, 1);
      if (maps[m].type != MAP_RINGBUF) rej(pc, "ringbuf_output needs a ring buffer");
      const AV& sz = rd(s, pc, 3);
      if (sz.k != A_SCALAR || sz.lo != sz.hi) rej(pc, "ringbuf_output size must be a constant");
      if (sz.lo == 0 || sz.lo > 4096) rej(pc, "ringbuf_output size out of range");
      arg_mem(s, pc, 2, (uint32_t)sz.lo, "ring record");
      if (rd(s, pc, 4).k != A_SCALAR) rej(pc, "ringbuf_output flags must be a scalar");
      if (simt && rd(s, pc, 4).var) rej(pc, "lane-varying ringbuf_output flags (SIMT hook)");
      s.ring += 8 + ((sz.lo + 7) & ~7ull);
      if (s.ring > kMaxRing) rej(pc, "ring byte budget exceeded");
      s.r[0] = unknown();
    } else {
      rej(pc, "unknown helper " + std::to_string(id));
    }
    for (int i = 1; i <= 5; i++) s.r[i] = AV{};
    if (++s.calls > kMaxCalls) rej(pc, "helper call budget exceeded");
  }

  // Decide a scalar condition: 1 always, 0 never, -1 unknown.
  static int decide(int code, const AV& a, const AV& b, bool is32) {
    if (a.lo == a.hi && b.lo == b.hi) {
      uint64_t x = a.lo, y = b.lo;
      if (is32) {
        x = (uint32_t)x;
        y = (uint32_t)y;
      }
      int64_t sx = is32 ? (int32_t)x : (int64_t)x, sy = is32 ? (int32_t)y : (int64_t)y;
      switch (code) {
        case 0x10: return x == y;
        case 0x20: return x > y;
        case 0x30: return x >= y;
        case 0x40: return (x & y) != 0;
        case 0x50: return x != y;
        case 0x60: return sx > sy;
        case 0x70: return sx >= sy;
        case 0xa0: return x < y;
        case 0xb0: return x <= y;
        case 0xc0: return sx < sy;
        case 0xd0: return sx <= sy;
      }
      return -1;
    }
    if (is32) return -1;
    uint64_t alo = a.lo, ahi = a.hi, blo = b.lo, bhi = b.hi;
    bool nonneg = ahi < (1ull << 63) && bhi < (1ull << 63);
    switch (code) {
      case 0x10: if (ahi < blo || bhi < alo) return 0; return -1;
      case 0x50: if (ahi < blo || bhi < alo) return 1; return -1;
      case 0x20: case 0x60:
        if (code == 0x60 && !nonneg) return -1;
        if (alo > bhi) return 1;
        if (ahi <= blo) return 0;
        return -1;
      case 0x30: case 0x70:
        if (code == 0x70 && !nonneg) return -1;
        if (alo >= bhi) return 1;
        if (ahi < blo) return 0;
        return -1;
      case 0xa0: case 0xc0:
        if (code == 0xc0 && !nonneg) return -1;
        if (ahi < blo) return 1;
        if (alo >= bhi) return 0;
        return -1;
      case 0xb0: case 0xd0:
        if (code == 0xd0 && !nonneg) return -1;
        if (ahi <= blo) return 1;
        if (alo > bhi) return 0;
        return -1;
    }
    return -1;
  }

  // Narrow ``a`` on the edge where (a code c) is ``taken``; false if empty.
  static bool refine(AV& a, int code, uint64_t c, bool taken) {
    uint64_t lo = a.lo, hi = a.hi;
    switch (code) {
      case 0x10:
        if (taken) lo = hi = c;
        else {
          if (lo == c && hi == c) return false;
          if (lo == c) lo++;
          if (hi == c) hi--;
        }
        break;
      case 0x50:
        if (!taken) lo = hi = c;
        else {
          if (lo == c && hi == c) return false;
          if (lo == c) lo++;
          if (hi == c) hi--;
        }
        break;
      case 0x20:  // a > c
        if (taken) { if (c == ~0ull) return false; lo = std::max(lo, c + 1); }
        else hi = std::min(hi, c);
        break;
      case 0x30:  // a >= c
        if (taken) lo = std::max(lo, c);
        else { if (c == 0) return false; hi = std::min(hi, c - 1); }
        break;
      case 0xa0:  // a < c
        if (taken) { if (c == 0) return false; hi = std::min(hi, c - 1); }
        else lo = std::max(lo, c);
        break;
      case 0xb0:  // a <= c
        if (taken) hi = std::min(hi, c);
        else { if (c == ~0ull) return false; lo = std::max(lo, c + 1); }
        break;
      default:
        return true;
    }
    if (lo > hi) return false;
    a.lo = lo;
    a.hi = hi;
    if (lo == hi) a.tz = ctz64(lo);
    return true;
  }

  // Execute one instruction; returns successor (pc, state) pairs.
  std::vector<std::pair<int, AState>> step(int pc, AState s) {
    const Insn& in = ins[pc];
    int cls = in.op & 7, code = in.op & 0xf0;
    bool x = in.op & 8;
    if (++s.steps > kMaxSteps) rej(pc, "dynamic instruction budget exceeded");
    std::vector<std::pair<int, AState>> out;
    int next = pc + 1;
    switch (cls) {
      case 4:
      case 7: {
        bool is64 = cls == 7;
        const AV& a0 = s.r[in.dst];
        if (code == 0xd0 || code == 0x80) {
          const AV& a = rd(s, pc, in.dst);
          if (a.k != A_SCALAR) rej(pc, "ALU on a pointer");
          const bool v = a.var;
          s.r[in.dst] = alu_scalar(is64, code, in.off, x, in.imm, a, exact(0));
          s.r[in.dst].var = v;
          break;
        }
        AV b = x ? rd(s, pc, in.src) : exact(is64 ? (uint64_t)(int64_t)in.imm : (uint64_t)(uint32_t)in.imm);
        if (code == 0xb0 && in.off == 0 && is64) {  // MOV64 copies pointers too
          s.r[in.dst] = b;
          break;
        }
        if (code == 0xb0) {
          if (b.k != A_SCALAR) rej(pc, "pointer leaked through 32-bit or sign-extending move");
          const bool v = b.var;
          s.r[in.dst] = alu_scalar(is64, code, in.off, x, in.imm, exact(0), b);
          s.r[in.dst].var = v;
          break;
        }
        const AV& a = rd(s, pc, in.dst);
        (void)a0;
        const bool var = a.var || b.var;
        if (a.k == A_SCALAR && b.k == A_SCALAR) {
          s.r[in.dst] = alu_scalar(is64, code, in.off, x, in.imm, a, b);
          s.r[in.dst].var = var;
          break;
        }
        if (!is64 || b.k != A_SCALAR || (code != 0x00 && code != 0x10) || (a.k != A_STACK && a.k != A_MAPVAL))
          rej(pc, "illegal pointer arithmetic");
        AV r = a;
        bool sneg = b.hi >= (1ull << 63);  // possibly negative as signed
        if (b.lo == b.hi) {
          int64_t d = (int64_t)b.lo;
          if (code == 0x10) d = -d;
          r.lo = (uint64_t)((int64_t)a.lo + d);
          r.hi = (uint64_t)((int64_t)a.hi + d);
          r.tz = std::min(a.tz, ctz64(b.lo));
        } else if (!sneg && b.hi < (1ull << 40)) {
          if (code == 0x00) {
            r.lo = (uint64_t)((int64_t)a.lo + (int64_t)b.lo);
            r.hi = (uint64_t)((int64_t)a.hi + (int64_t)b.hi);
          } else {
            r.lo = (uint64_t)((int64_t)a.lo - (int64_t)b.hi);
            r.hi = (uint64_t)((int64_t)a.hi - (int64_t)b.lo);
          }
          r.tz = std::min(a.tz, b.tz);
        } else {
          rej(pc, "unbounded pointer arithmetic");
        }
        if ((int64_t)r.lo < -(1ll << 40) || (int64_t)r.hi > (1ll << 40)) rej(pc, "pointer offset out of range");
        r.var = var;
        s.r[in.dst] = r;
        break;
      }
      case 5:
      case 6: {
        bool is32 = cls == 6;
        if (code == 0x90) {
          if (rd(s, pc, 0).k != A_SCALAR) rej(pc, "r0 at exit is not a scalar");
          res.max_insns = std::max(res.max_insns, s.steps);
          res.max_calls = std::max(res.max_calls, s.calls);
          res.max_ring_bytes = std::max(res.max_ring_bytes, s.ring);
          return out;
        }
        if (code == 0x80) {
          call(s, pc, in.imm);
          break;
        }
        int t = jump_target(pc);
        if (code == 0x00) {
          out.push_back({t, s});
          return out;
        }
        const AV& a = rd(s, pc, in.dst);
        AV b = x ? rd(s, pc, in.src) : exact(is32 ? (uint64_t)(uint32_t)in.imm : (uint64_t)(int64_t)in.imm);
        if (simt && (a.var || b.var)) rej(pc, "lane-varying branch condition (SIMT hook)");
        if (a.k == A_MAPVAL_OR_NULL || a.k == A_MAPVAL) {
          if (is32 || x || in.imm != 0 || (code != 0x10 && code != 0x50))
            rej(pc, "pointer comparison other than a null check");
          AState nn = s, nul = s;
          nn.r[in.dst].k = A_MAPVAL;
          nul.r[in.dst] = exact(0);
          bool null_possible = a.k == A_MAPVAL_OR_NULL;
          if (code == 0x10) {  // jeq ptr, 0
            if (null_possible) out.push_back({t, nul});
            out.push_back({next, nn});
          } else {
            out.push_back({t, nn});
            if (null_possible) out.push_back({next, nul});
          }
          return out;
        }
        if (a.k != A_SCALAR || b.k != A_SCALAR) rej(pc, "comparison involving a pointer");
        int d = decide(code, a, b, is32);
        bool can_refine = !is32 && b.lo == b.hi;
        if (d != 0) {
          AState st = s;
          if (!can_refine || refine(st.r[in.dst], code, b.lo, true)) out.push_back({t, st});
        }
        if (d != 1) {
          AState sf = s;
          if (!can_refine || refine(sf.r[in.dst], code, b.lo, false)) out.push_back({next, sf});
        }
        return out;
      }
      case 1: {
        int size = kSz[(in.op >> 3) & 3];
        const AV& b = rd(s, pc, in.src);
        const bool v = access(s, pc, b, in.off, size, 0);
        bool sx = (in.op & 0xe0) == 0x80;
        s.r[in.dst] = (size == 8 || sx) ? unknown() : range(0, (1ull << (8 * size)) - 1, 0);
        s.r[in.dst].var = v;
        break;
      }
      case 2: {
        int size = kSz[(in.op >> 3) & 3];
        const AV& b = rd(s, pc, in.dst);
        access(s, pc, b, in.off, size, 1);
        break;
      }
      case 3: {
        int size = kSz[(in.op >> 3) & 3];
        const AV& b = rd(s, pc, in.dst);
        const AV& v = rd(s, pc, in.src);
        if (v.k != A_SCALAR) rej(pc, "pointer stored to memory");
        if ((in.op & 0xe0) == 0x60) {
          access(s, pc, b, in.off, size, 1, v.var);
          break;
        }
        bool fetch = in.imm & 1;
        if (in.imm == 0xf1 && rd(s, pc, 0).k != A_SCALAR) rej(pc, "cmpxchg needs a scalar r0");
        const bool ov = access(s, pc, b, in.off, size, fetch ? 3 : 2, v.var || (in.imm == 0xf1 && s.r[0].var));
        if (in.imm == 0xf1) {
          s.r[0] = size == 8 ? unknown() : range(0, 0xffffffffull, 0);
          s.r[0].var = ov;
        } else if (fetch) {
          s.r[in.src] = size == 8 ? unknown() : range(0, 0xffffffffull, 0);
          s.r[in.src].var = ov;
        }
        break;
      }
      case 0: {
        if (in.src == 0) {
          uint64_t v = (uint64_t)(uint32_t)in.imm | ((uint64_t)(uint32_t)ins[pc + 1].imm << 32);
          s.r[in.dst] = exact(v);
        } else {
          int m = map_of_ref(pc, in);
          s.r[in.dst] = AV{A_MAP, 0, 0, 0, m};
        }
        next = pc + 2;
        break;
      }
    }
    out.push_back({next, s});
    return out;
  }

  // Analyse [lo, hi] from ``entry``.  Edges to targets beyond ``hi`` are
  // joined into ``outer``; the back-edge (from ``hi`` to ``lo``) into ``*back``.
  void region(int lo, int hi, const AState& entry, std::map<int, AState>& outer, AState* back) {
    std::map<int, AState> pend;
    pend[lo] = entry;
    for (int pc = lo; pc <= hi; pc += is_lddw(ins[pc]) ? 2 : 1) {
      auto it = pend.find(pc);
      if (it == pend.end()) continue;
      AState s = std::move(it->second);
      pend.erase(it);
      if (loop_end[pc] >= 0 && !(back && pc == lo)) {
        int j = loop_end[pc];
        run_loop(pc, j, s, pend, hi, outer);
        pc = j;  // the loop's exits are already in pend/outer
        continue;
      }
      for (auto& e : step(pc, std::move(s))) {
        int t = e.first;
        if (back && pc == hi && t == lo) {
          join_into(*back, e.second);
        } else if (t > pc && t <= hi) {
          join_into(pend[t], e.second);
        } else if (t > hi) {
          join_into(outer[t], e.second);
        } else {
          rej(pc, "unexpected backward jump");
        }
      }
    }
  }

  void run_loop(int h, int j, AState s, std::map<int, AState>& pend, int hi, std::map<int, AState>& outer) {
    int c = ins[j].dst;
    if (s.r[c].k != A_SCALAR || s.r[c].lo != s.r[c].hi) rej(h, "loop counter r" + std::to_string(c) + " is not a constant on entry");
    std::map<int, AState> exits;
    for (uint64_t trip = 0;; trip++) {
      if (trip > kMaxTrips) rej(j, "loop trip count too large");
      AState back;
      region(h, j, s, exits, &back);
      if (!back.live) break;
      s = std::move(back);
    }
    for (auto& e : exits) {
      if (e.first <= hi)
        join_into(pend[e.first], e.second);
      else
        join_into(outer[e.first], e.second);
    }
  }

  CheckResult run() {
    try {
      if (!hook_info(hook, &hi)) throw Reject{"unknown hook type"};
      for (int id : table)
        if (id < 0 || id >= (int)maps.size()) throw Reject{"bad map table"};
      structure();
      map_used.assign(maps.size(), 0);
      shared_op.assign(maps.size(), -1);
      AState s;
      s.live = true;
      s.r[1] = AV{A_CTX, 0, 0, 64, -1};
      s.r[10] = AV{A_STACK, (uint64_t)STACK_BYTES, (uint64_t)STACK_BYTES, 9, -1};
      std::fill(std::begin(s.stk), std::end(s.stk), 0);
      std::fill(std::begin(s.stkvar), std::end(s.stkvar), 0);
      std::map<int, AState> outer;
      region(0, n - 1, s, outer, nullptr);
      if (!outer.empty()) rej(outer.begin()->first, "edge leaves the program");
      res.ok = true;
      res.stack_bytes = (uint32_t)((STACK_BYTES - min_stack + 7) & ~7);
      bool ep = true;
      for (size_t m = 0; m < maps.size(); m++)
        if (map_used[m] && maps[m].type != MAP_RINGBUF && !(maps[m].flags & (F_SHARED | F_READ_ONLY)))
          ep = false;
      if (hook == HOOK_WAVE_MEM && !ep)
        throw Reject{"a warp-leader hook runs once per wave: its maps must be shared, read-only or ring buffers"};
      if (hook == HOOK_SCHED && !ep)
        throw Reject{"a scheduling hook runs in every worker at once: its maps must be shared, read-only or ring buffers"};
      if (simt && !ep)
        throw Reject{"a SIMT hook's lanes run one wave's events together: its maps must be shared, read-only or ring buffers"};
      res.event_parallel = ep;
      res.log = "accepted";
    } catch (const Reject& r) {
      res = CheckResult{};
      res.ok = false;
      res.log = r.msg;
    }
    return res;
  }
};

}  // namespace

CheckResult check(const std::vector<Insn>& insns, int hook, const std::vector<MapShape>& maps,
                  const std::vector<int>& map_table) {
  Checker c(insns, hook, maps, map_table);
  return c.run();
}

}  // namespace gxo
