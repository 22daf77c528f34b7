// CPU oracle: decoder, sequential interpreter, maps, ring buffer and the
// ownership tracker.  Test infrastructure only (see gxo.h).
//
// Every register carries a dynamic tag (uninitialised, scalar, ctx / stack /
// map-value pointer, map handle), and every memory access is bounds-,
// alignment- and initialisation-checked, so a program that the checker
// wrongly accepts shows up as a counted fault instead of silent corruption.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "gxo.h"

namespace gxo {

std::vector<Insn> decode(const uint8_t* code, uint32_t n_slots) {
  std::vector<Insn> out(n_slots);
  for (uint32_t i = 0; i < n_slots; i++) {
    const uint8_t* p = code + 8 * i;
    Insn& in = out[i];
    in.op = p[0];
    in.dst = p[1] & 0x0f;
    in.src = p[1] >> 4;
    in.off = (int16_t)(uint16_t)(p[2] | (p[3] << 8));
    in.imm = (int32_t)((uint32_t)p[4] | ((uint32_t)p[5] << 8) | ((uint32_t)p[6] << 16) |
                       ((uint32_t)p[7] << 24));
  }
  return out;
}

bool hook_info(int hook, HookInfo* out) {
  if (hook == HOOK_MEM_ACCESS) {
    // {u64 addr @0, u32 stream_id @8, u32 pad @12, u64 timestamp @16}
    *out = {24, 8, 4, {{0, 8}, {8, 4}, {16, 8}}};
    return true;
  }
  if (hook == HOOK_KERNEL_TIMING) {
    // {u32 kernel_id @0, u32 pad @4, u64 latency_ns @8}
    *out = {16, 0, 4, {{0, 4}, {8, 8}}};
    return true;
  }
  if (hook == HOOK_WAVE_MEM) {
    // input: memory-access records (24 B); context of one invocation:
    // {u64 lo = smallest addr @0, u64 hi = largest addr @8, u32 n = records
    // @16, u32 stream of the tile's first record @20}
    *out = {24, 8, 4, {{0, 8}, {8, 8}, {16, 4}, {20, 4}}};
    return true;
  }
  if (hook == HOOK_SIMT_MEM) {
    // input: memory-access records (24 B); context of one invocation: the
    // record's fields, then its tile's aggregate as HOOK_WAVE_MEM's context
    // at offset 24 (warp-uniform)
    *out = {24, 8, 4, {{0, 8}, {8, 4}, {16, 8}, {24, 8}, {32, 8}, {40, 4}, {44, 4}}, 24};
    return true;
  }
  if (hook == HOOK_SCHED) {
    // {u32 worker @0, u32 units done @4, u64 ns since the worker started @8,
    // u64 ns since it began stealing @16, u32 units stolen @24, u32 units
    // left in the victim's range @28}
    *out = {32, 0, 4, {{0, 4}, {4, 4}, {8, 8}, {16, 8}, {24, 4}, {28, 4}}};
    return true;
  }
  return false;
}

// Context of a warp-leader invocation for records [b, e) (24-byte
// memory-access records), laid out as hook_info(HOOK_WAVE_MEM) states.
static void wave_context(const uint8_t* events, uint64_t b, uint64_t e, uint8_t* ctx) {
  uint64_t lo = ~0ull, hi = 0;
  for (uint64_t i = b; i < e; i++) {
    uint64_t a = 0;
    std::memcpy(&a, events + i * 24, 8);
    lo = a < lo ? a : lo;
    hi = a > hi ? a : hi;
  }
  const uint32_t n = (uint32_t)(e - b);
  uint32_t s0 = 0;
  std::memcpy(&s0, events + b * 24 + 8, 4);
  std::memcpy(ctx, &lo, 8);
  std::memcpy(ctx + 8, &hi, 8);
  std::memcpy(ctx + 16, &n, 4);
  std::memcpy(ctx + 20, &s0, 4);
}

static uint64_t load_le(const uint8_t* p, int size) {
  uint64_t v = 0;
  for (int i = size - 1; i >= 0; i--) v = (v << 8) | p[i];
  return v;
}

static void store_le(uint8_t* p, uint64_t v, int size) {
  for (int i = 0; i < size; i++) {
    p[i] = (uint8_t)v;
    v >>= 8;
  }
}

static uint64_t bswap(uint64_t v, int bits) {
  uint64_t r = 0;
  for (int i = 0; i < bits / 8; i++) r = (r << 8) | ((v >> (8 * i)) & 0xff);
  return r;
}

static uint64_t sext(uint64_t v, int bits) {
  if (bits >= 64) return v;
  uint64_t m = 1ull << (bits - 1);
  v &= (1ull << bits) - 1;
  return (v ^ m) - m;
}

// ---------------------------------------------------------------------------
// ALU semantics (RFC 9669 section 4).  ``b`` is the second operand already
// widened: the sign-extended imm for 64-bit K forms, the raw 32-bit imm for
// 32-bit K forms, or the source register.

static uint64_t alu64(int code, int16_t off, uint64_t a, uint64_t b, int32_t imm, bool x) {
  int64_t sa = (int64_t)a, sb = (int64_t)b;
  switch (code) {
    case 0x00: return a + b;
    case 0x10: return a - b;
    case 0x20: return a * b;
    case 0x30:
      if (b == 0) return 0;
      if (off == 0) return a / b;
      if (sa == INT64_MIN && sb == -1) return (uint64_t)INT64_MIN;
      return (uint64_t)(sa / sb);
    case 0x40: return a | b;
    case 0x50: return a & b;
    case 0x60: return a << (b & 63);
    case 0x70: return a >> (b & 63);
    case 0x80: return (uint64_t)0 - a;
    case 0x90:
      if (b == 0) return a;
      if (off == 0) return a % b;
      if (sb == -1) return 0;
      return (uint64_t)(sa % sb);
    case 0xa0: return a ^ b;
    case 0xb0: return (x && off) ? sext(b, off) : b;
    case 0xc0: return (uint64_t)(sa >> (b & 63));
    case 0xd0: return bswap(a, imm);
  }
  return 0;
}

static uint64_t alu32(int code, int16_t off, uint64_t a64, uint64_t b64, int32_t imm, bool x) {
  uint32_t a = (uint32_t)a64, b = (uint32_t)b64;
  int32_t sa = (int32_t)a, sb = (int32_t)b;
  switch (code) {
    case 0x00: return (uint32_t)(a + b);
    case 0x10: return (uint32_t)(a - b);
    case 0x20: return (uint32_t)(a * b);
    case 0x30:
      if (b == 0) return 0;
      if (off == 0) return a / b;
      if (sa == INT32_MIN && sb == -1) return (uint32_t)INT32_MIN;
      return (uint32_t)(sa / sb);
    case 0x40: return a | b;
    case 0x50: return a & b;
    case 0x60: return (uint32_t)(a << (b & 31));
    case 0x70: return a >> (b & 31);
    case 0x80: return (uint32_t)(0u - a);
    case 0x90:
      if (b == 0) return a;
      if (off == 0) return a % b;
      if (sb == -1) return 0;
      return (uint32_t)(sa % sb);
    case 0xa0: return a ^ b;
    case 0xb0: return (x && off) ? (uint32_t)sext(b64, off) : b;
    case 0xc0: return (uint32_t)(sa >> (b & 31));
    case 0xd0:
      // END: to-LE truncates (little-endian host), to-BE swaps; 64-bit result
      if (!x) return imm == 64 ? a64 : (a64 & ((1ull << imm) - 1));
      return bswap(a64, imm);
  }
  return 0;
}

static bool jmp_cond(int code, uint64_t a, uint64_t b, bool is32) {
  if (is32) {
    a = (uint32_t)a;
    b = (uint32_t)b;
  }
  int64_t sa = is32 ? (int64_t)(int32_t)a : (int64_t)a;
  int64_t sb = is32 ? (int64_t)(int32_t)b : (int64_t)b;
  switch (code) {
    case 0x10: return a == b;
    case 0x20: return a > b;
    case 0x30: return a >= b;
    case 0x40: return (a & b) != 0;
    case 0x50: return a != b;
    case 0x60: return sa > sb;
    case 0x70: return sa >= sb;
    case 0xa0: return a < b;
    case 0xb0: return a <= b;
    case 0xc0: return sa < sb;
    case 0xd0: return sa <= sb;
  }
  return false;
}

// ---------------------------------------------------------------------------
// maps

int Oracle::create_map(int type, uint32_t ksz, uint32_t vsz, uint32_t max, uint32_t flags) {
  Map m;
  m.type = type;
  m.key_size = ksz;
  m.value_size = vsz;
  m.max_entries = max;
  m.flags = flags;
  if (type == MAP_ARRAY) {
    if (ksz != 4 || vsz == 0 || max == 0) return -E_INVAL;
    m.array.assign((size_t)max * vsz, 0);
  } else if (type == MAP_HASH) {
    if (ksz == 0 || vsz == 0 || max == 0) return -E_INVAL;
  } else if (type == MAP_RINGBUF) {
    if (ksz || vsz || max < 4096 || (max & (max - 1))) return -E_INVAL;
  } else {
    return -E_INVAL;
  }
  if ((flags & F_SHARED) && (flags & F_READ_ONLY)) return -E_INVAL;
  maps.push_back(std::move(m));
  return (int)maps.size() - 1;
}

static int array_index(const Map& m, const uint8_t* key, uint32_t* idx) {
  *idx = (uint32_t)load_le(key, 4);
  return *idx < m.max_entries ? 0 : -1;
}

static int64_t do_update(Map& m, const uint8_t* key, const uint8_t* val, uint64_t flags,
                         uint64_t* e2big) {
  if (flags > 2) return -E_INVAL;
  if (m.type == MAP_ARRAY) {
    uint32_t idx;
    if (array_index(m, key, &idx)) return -E_2BIG;
    if (flags == 1) return -E_EXIST;  // every array element exists
    std::memcpy(&m.array[(size_t)idx * m.value_size], val, m.value_size);
    return 0;
  }
  if (m.type == MAP_HASH) {
    Bytes k(key, key + m.key_size);
    auto it = m.hash.find(k);
    if (it != m.hash.end()) {
      if (flags == 1) return -E_EXIST;
      std::memcpy(it->second->data(), val, m.value_size);
      return 0;
    }
    if (flags == 2) return -E_NOENT;
    if (m.hash.size() >= m.max_entries) {
      if (e2big) (*e2big)++;
      return -E_2BIG;
    }
    m.hash.emplace(std::move(k), std::make_shared<Bytes>(val, val + m.value_size));
    return 0;
  }
  return -E_INVAL;
}

static int64_t do_delete(Map& m, const uint8_t* key) {
  if (m.type != MAP_HASH) return -E_INVAL;
  Bytes k(key, key + m.key_size);
  auto it = m.hash.find(k);
  if (it == m.hash.end()) return -E_NOENT;
  m.hash.erase(it);
  return 0;
}

int Oracle::map_update(int id, const uint8_t* key, const uint8_t* val, uint64_t flags) {
  if (id < 0 || id >= (int)maps.size()) return -E_INVAL;
  return (int)do_update(maps[id], key, val, flags, nullptr);
}

int Oracle::map_lookup(int id, const uint8_t* key, uint8_t* val_out) {
  if (id < 0 || id >= (int)maps.size()) return -E_INVAL;
  Map& m = maps[id];
  if (m.type == MAP_ARRAY) {
    uint32_t idx;
    if (array_index(m, key, &idx)) return -E_NOENT;
    std::memcpy(val_out, &m.array[(size_t)idx * m.value_size], m.value_size);
    return 0;
  }
  if (m.type == MAP_HASH) {
    auto it = m.hash.find(Bytes(key, key + m.key_size));
    if (it == m.hash.end()) return -E_NOENT;
    std::memcpy(val_out, it->second->data(), m.value_size);
    return 0;
  }
  return -E_INVAL;
}

int Oracle::map_delete(int id, const uint8_t* key) {
  if (id < 0 || id >= (int)maps.size()) return -E_INVAL;
  return (int)do_delete(maps[id], key);
}

int64_t Oracle::map_dump(int id, uint8_t* keys, uint8_t* vals, uint64_t cap) {
  if (id < 0 || id >= (int)maps.size()) return -E_INVAL;
  Map& m = maps[id];
  uint64_t n = 0;
  if (m.type == MAP_ARRAY) {
    for (uint32_t i = 0; i < m.max_entries; i++, n++) {
      if (n >= cap) continue;
      if (keys) store_le(keys + 4 * n, i, 4);
      if (vals) std::memcpy(vals + n * m.value_size, &m.array[(size_t)i * m.value_size], m.value_size);
    }
    return (int64_t)n;
  }
  if (m.type == MAP_HASH) {
    for (auto& kv : m.hash) {
      if (n < cap) {
        if (keys) std::memcpy(keys + n * m.key_size, kv.first.data(), m.key_size);
        if (vals) std::memcpy(vals + n * m.value_size, kv.second->data(), m.value_size);
      }
      n++;
    }
    return (int64_t)n;
  }
  return -E_INVAL;
}

int64_t Oracle::ring_drain(int id, uint8_t* buf, uint64_t cap, uint64_t* n_records) {
  if (id < 0 || id >= (int)maps.size() || maps[id].type != MAP_RINGBUF) return -E_INVAL;
  Map& m = maps[id];
  uint64_t pos = 0, n = 0;
  size_t i = 0;
  for (; i < m.records.size(); i++) {
    const Bytes& r = m.records[i];
    uint64_t sz = 8 + ((r.size() + 7) & ~7ull);
    if (pos + sz > cap) break;
    std::memset(buf + pos, 0, sz);
    store_le(buf + pos, r.size(), 4);
    std::memcpy(buf + pos + 8, r.data(), r.size());
    pos += sz;
    m.ring_used -= sz;
    n++;
  }
  m.records.erase(m.records.begin(), m.records.begin() + i);
  if (n_records) *n_records = n;
  return (int64_t)pos;
}

// ---------------------------------------------------------------------------
// interpreter

namespace {

const int kSizes[4] = {4, 2, 1, 8};

enum Kind : uint8_t { K_UNINIT, K_SCALAR, K_CTX, K_STACK, K_MAPVAL, K_MAPHANDLE, K_DEAD };

struct Reg {
  Kind k = K_UNINIT;
  uint64_t v = 0;    // scalar value or pointer offset
  int map = -1;      // map id for K_MAPVAL / K_MAPHANDLE
  int64_t slot = -1; // array element index, or index into the hash reference table
};

struct HashRef {
  std::shared_ptr<Bytes> val;
  Bytes key;
};

struct Fault {
  std::string msg;
};

struct Exec {
  Oracle& o;
  const Program& p;
  const HookInfo& hi;
  const uint8_t* rec;
  uint64_t stream;
  Reg r[11];
  uint8_t stack[STACK_BYTES];
  bool init[STACK_BYTES];
  std::vector<HashRef> refs;

  Exec(Oracle& o_, const Program& p_, const HookInfo& h_) : o(o_), p(p_), hi(h_) {}

  [[noreturn]] void fault(const std::string& m) { throw Fault{m}; }

  const Reg& rd(int i) {
    if (i > 10) fault("bad register");
    if (r[i].k == K_UNINIT) fault("read of uninitialised r" + std::to_string(i));
    if (r[i].k == K_DEAD) fault("use of invalidated pointer r" + std::to_string(i));
    return r[i];
  }
  uint64_t scalar(int i) {
    const Reg& x = rd(i);
    if (x.k != K_SCALAR) fault("pointer used as scalar r" + std::to_string(i));
    return x.v;
  }
  void wr_scalar(int i, uint64_t v) {
    if (i >= 10) fault("write to r10");
    r[i] = Reg{K_SCALAR, v, -1, -1};
  }

  void touch(int map, const Bytes& slot, bool write) {
    Map& m = o.maps[map];
    if (!o.track_ownership || m.type == MAP_RINGBUF || (m.flags & (F_SHARED | F_READ_ONLY))) return;
    auto it = m.owner.find(slot);
    if (it == m.owner.end()) {
      m.owner.emplace(slot, std::make_pair(stream, write));
      return;
    }
    if (it->second.first != stream) m.multi[slot] = true;
    it->second.second = it->second.second || write;
  }

  Bytes slot_of(const Reg& x) {
    Map& m = o.maps[x.map];
    if (m.type == MAP_ARRAY) {
      Bytes b(4);
      store_le(b.data(), (uint64_t)x.slot, 4);
      return b;
    }
    return refs[x.slot].key;
  }

  // Resolve [base + off, base + off + size) to host bytes with all checks.
  // mode: 0 = load, 1 = store, 2 = commutative atomic, 3 = fetching atomic.
  int atomic_op = 0;  // operation of the atomic being executed (for shared maps)

  uint8_t* mem(int base_reg, int64_t off, int size, int mode) {
    const Reg& b = rd(base_reg);
    if (b.k == K_CTX) {
      if (mode != 0) fault("write to ctx");
      if (b.v != 0) fault("ctx pointer arithmetic");
      for (auto& f : hi.fields)
        if ((int64_t)f.first == off && (int)f.second == size) return const_cast<uint8_t*>(rec) + off;
      fault("bad ctx access");
    }
    int64_t o2 = (int64_t)b.v + off;
    if (o2 % size) fault("misaligned access");
    if (b.k == K_STACK) {
      if (o2 < 0 || o2 + size > STACK_BYTES) fault("stack access out of bounds");
      if (mode == 0 || mode == 2 || mode == 3)
        for (int i = 0; i < size; i++)
          if (!init[o2 + i]) fault("read of uninitialised stack");
      if (mode != 0)
        for (int i = 0; i < size; i++) init[o2 + i] = true;
      return stack + o2;
    }
    if (b.k == K_MAPVAL) {
      Map& m = o.maps[b.map];
      if (o2 < 0 || o2 + size > (int64_t)m.value_size) fault("map value access out of bounds");
      if ((m.flags & F_READ_ONLY) && mode != 0) fault("write to read-only map");
      if ((m.flags & F_SHARED) && mode != 2) fault("non-commutative access to shared map");
      if (m.flags & F_SHARED) {
        int key = atomic_op | (size << 8);
        if (m.shared_op < 0) m.shared_op = key;
        else if (m.shared_op != key) fault("shared map updated with different atomic operations");
      }
      touch(b.map, slot_of(b), mode != 0);
      if (m.type == MAP_ARRAY) return &m.array[(size_t)b.slot * m.value_size + o2];
      return refs[b.slot].val->data() + o2;
    }
    fault("memory access through non-pointer");
  }

  // Pointer argument of a helper: ``n`` readable bytes.
  const uint8_t* arg_bytes(int reg, uint32_t n) {
    const Reg& b = rd(reg);
    if (b.k == K_STACK) {
      int64_t o2 = (int64_t)b.v;
      if (o2 < 0 || o2 + (int64_t)n > STACK_BYTES) fault("helper stack argument out of bounds");
      for (uint32_t i = 0; i < n; i++)
        if (!init[o2 + i]) fault("helper reads uninitialised stack");
      return stack + o2;
    }
    if (b.k == K_MAPVAL) {
      Map& m = o.maps[b.map];
      int64_t o2 = (int64_t)b.v;
      if (o2 < 0 || o2 + (int64_t)n > (int64_t)m.value_size) fault("helper map argument out of bounds");
      if (m.flags & F_SHARED) fault("helper reads shared map value");
      touch(b.map, slot_of(b), false);
      if (m.type == MAP_ARRAY) return &m.array[(size_t)b.slot * m.value_size + o2];
      return refs[b.slot].val->data() + o2;
    }
    fault("helper argument is not a pointer");
  }

  int map_arg(int reg) {
    const Reg& b = rd(reg);
    if (b.k != K_MAPHANDLE) fault("helper map argument is not a map");
    return b.map;
  }

  void invalidate(int map) {
    for (auto& x : r)
      if (x.k == K_MAPVAL && x.map == map) x.k = K_DEAD;
  }

  uint64_t call(int32_t id) {
    o.stats.helper_calls++;
    if (id == H_LOOKUP) {
      int mid = map_arg(1);
      Map& m = o.maps[mid];
      if (m.type == MAP_RINGBUF) fault("lookup on ring buffer");
      const uint8_t* key = arg_bytes(2, m.key_size);
      Bytes k(key, key + m.key_size);
      touch(mid, k, false);
      if (m.type == MAP_ARRAY) {
        uint32_t idx;
        if (array_index(m, key, &idx)) return set_r0_scalar(0);
        r[0] = Reg{K_MAPVAL, 0, mid, idx};
        return 1;
      }
      auto it = m.hash.find(k);
      if (it == m.hash.end()) return set_r0_scalar(0);
      refs.push_back(HashRef{it->second, k});
      r[0] = Reg{K_MAPVAL, 0, mid, (int64_t)refs.size() - 1};
      return 1;
    }
    if (id == H_UPDATE || id == H_DELETE) {
      int mid = map_arg(1);
      Map& m = o.maps[mid];
      if (m.type == MAP_RINGBUF) fault("update/delete on ring buffer");
      if (m.flags & (F_SHARED | F_READ_ONLY)) fault("update/delete on shared or read-only map");
      Bytes k;
      {
        const uint8_t* key = arg_bytes(2, m.key_size);
        k.assign(key, key + m.key_size);
      }
      int64_t ret;
      if (id == H_UPDATE) {
        Bytes v;
        {
          const uint8_t* val = arg_bytes(3, m.value_size);
          v.assign(val, val + m.value_size);
        }
        uint64_t flags = scalar(4);
        touch(mid, k, true);
        ret = do_update(m, k.data(), v.data(), flags, &o.stats.e2big);
      } else {
        touch(mid, k, true);
        ret = do_delete(m, k.data());
      }
      if (m.type == MAP_HASH) invalidate(mid);
      return set_r0_scalar((uint64_t)ret);
    }
    if (id == H_RINGBUF_OUTPUT) {
      int mid = map_arg(1);
      Map& m = o.maps[mid];
      if (m.type != MAP_RINGBUF) fault("ringbuf_output on non-ring map");
      uint64_t size = scalar(3);
      uint64_t flags = scalar(4);
      if (size == 0 || size > 4096) fault("ringbuf_output size");
      const uint8_t* data = arg_bytes(2, (uint32_t)size);
      if (flags != 0) return set_r0_scalar((uint64_t)-E_INVAL);
      uint64_t need = 8 + ((size + 7) & ~7ull);
      if (m.ring_used + need > m.max_entries) {
        o.stats.drops++;
        return set_r0_scalar((uint64_t)-E_AGAIN);
      }
      m.ring_used += need;
      m.records.emplace_back(data, data + size);
      return set_r0_scalar(0);
    }
    fault("unknown helper " + std::to_string(id));
  }

  uint64_t set_r0_scalar(uint64_t v) {
    r[0] = Reg{K_SCALAR, v, -1, -1};
    return 0;
  }

  uint32_t run_event(const uint8_t* record) {
    rec = record;
    stream = load_le(record + hi.stream_off, hi.stream_size);
    for (auto& x : r) x = Reg{};
    r[1] = Reg{K_CTX, 0, -1, -1};
    r[10] = Reg{K_STACK, (uint64_t)STACK_BYTES, -1, -1};
    std::memset(init, 0, sizeof init);
    std::memset(stack, 0, sizeof stack);
    refs.clear();
    const auto& ins = p.insns;
    const int n = (int)ins.size();
    uint64_t steps = 0;
    int pc = 0;
    for (;;) {
      if (pc < 0 || pc >= n) fault("pc out of range");
      if (++steps > (1ull << 24)) fault("runaway program");
      const Insn& in = ins[pc];
      o.stats.insns++;
      int cls = in.op & 7;
      bool x = in.op & 0x08;
      int code = in.op & 0xf0;
      switch (cls) {
        case 7:    // ALU64
        case 4: {  // ALU
          bool is64 = cls == 7;
          if (code == 0xd0 || code == 0x80) {  // END and NEG take no source
            uint64_t a = scalar(in.dst);
            uint64_t v = is64 ? alu64(code, in.off, a, 0, in.imm, x) : alu32(code, in.off, a, 0, in.imm, x);
            wr_scalar(in.dst, v);
            break;
          }
          uint64_t b;
          Reg bsrc;
          if (x) {
            bsrc = rd(in.src);
            b = bsrc.v;
          } else {
            bsrc = Reg{K_SCALAR, 0, -1, -1};
            b = is64 ? (uint64_t)(int64_t)in.imm : (uint64_t)(uint32_t)in.imm;
          }
          if (code == 0xb0 && is64 && in.off == 0) {  // MOV64 copies any tag
            if (in.dst >= 10) fault("write to r10");
            if (x)
              r[in.dst] = bsrc;
            else
              wr_scalar(in.dst, b);
            break;
          }
          const Reg& a = code == 0xb0 ? Reg{K_SCALAR, 0, -1, -1} : rd(in.dst);
          bool aptr = a.k != K_SCALAR, bptr = bsrc.k != K_SCALAR;
          if (aptr || bptr) {
            // pointer +/- scalar on stack and map-value pointers only
            if (!is64 || bptr || (code != 0x00 && code != 0x10) ||
                (a.k != K_STACK && a.k != K_MAPVAL))
              fault("illegal pointer arithmetic");
            Reg res = a;
            res.v = code == 0x00 ? a.v + b : a.v - b;
            if (in.dst >= 10) fault("write to r10");
            r[in.dst] = res;
            break;
          }
          uint64_t v = is64 ? alu64(code, in.off, a.v, b, in.imm, x) : alu32(code, in.off, a.v, b, in.imm, x);
          wr_scalar(in.dst, v);
          break;
        }
        case 5:    // JMP
        case 6: {  // JMP32
          bool is32 = cls == 6;
          if (code == 0x90) {  // EXIT
            return (uint32_t)scalar(0);
          }
          if (code == 0x80) {  // CALL
            call(in.imm);
            for (int i = 1; i <= 5; i++) r[i] = Reg{};
            break;
          }
          if (code == 0x00) {  // JA
            pc += 1 + (is32 ? in.imm : in.off);
            continue;
          }
          const Reg& a = rd(in.dst);
          Reg b = x ? rd(in.src) : Reg{K_SCALAR, is32 ? (uint64_t)(uint32_t)in.imm : (uint64_t)(int64_t)in.imm, -1, -1};
          bool taken;
          if (a.k == K_SCALAR && b.k == K_SCALAR) {
            taken = jmp_cond(code, a.v, b.v, is32);
          } else if (!is32 && (code == 0x10 || code == 0x50) && a.k == K_MAPVAL && b.k == K_SCALAR &&
                     b.v == 0) {
            taken = code == 0x50;  // a non-null map value pointer never equals 0
          } else {
            fault("illegal pointer comparison");
          }
          pc += taken ? 1 + in.off : 1;
          continue;
        }
        case 1: {  // LDX
          int mode = in.op & 0xe0;
          int size = kSizes[(in.op >> 3) & 3];
          uint8_t* p8 = mem(in.src, in.off, size, 0);
          uint64_t v = load_le(p8, size);
          if (mode == 0x80) v = sext(v, 8 * size);
          wr_scalar(in.dst, v);
          break;
        }
        case 2: {  // ST
          int size = kSizes[(in.op >> 3) & 3];
          uint8_t* p8 = mem(in.dst, in.off, size, 1);
          store_le(p8, (uint64_t)(int64_t)in.imm, size);
          break;
        }
        case 3: {  // STX
          int size = kSizes[(in.op >> 3) & 3];
          if ((in.op & 0xe0) == 0x60) {
            uint64_t v = scalar(in.src);
            uint8_t* p8 = mem(in.dst, in.off, size, 1);
            store_le(p8, v, size);
            break;
          }
          // ATOMIC (W, DW)
          int aop = in.imm;
          bool fetch = aop & 1;
          uint64_t v = scalar(in.src);
          uint64_t cmp = aop == 0xf1 ? scalar(0) : 0;
          atomic_op = aop & 0xff;
          uint8_t* p8 = mem(in.dst, in.off, size, fetch ? 3 : 2);
          uint64_t old = load_le(p8, size), nv = old;
          switch (aop & 0xf0) {
            case 0x00: nv = old + v; break;
            case 0x40: nv = old | v; break;
            case 0x50: nv = old & v; break;
            case 0xa0: nv = old ^ v; break;
            case 0xe0: nv = v; break;
            case 0xf0: nv = ((size == 4 ? (uint32_t)cmp : cmp) == old) ? v : old; break;
            default: fault("bad atomic op");
          }
          store_le(p8, nv, size);
          if (aop == 0xf1)
            wr_scalar(0, old);
          else if (fetch)
            wr_scalar(in.src, old);
          break;
        }
        case 0: {  // LD_IMM64
          if (pc + 1 >= n) fault("truncated lddw");
          uint64_t v = (uint64_t)(uint32_t)in.imm | ((uint64_t)(uint32_t)ins[pc + 1].imm << 32);
          if (in.src == 0) {
            wr_scalar(in.dst, v);
          } else {
            int mid = -1;
            if (in.src == 5) {
              if (in.imm < 0 || in.imm >= (int)p.map_table.size()) fault("bad map index");
              mid = p.map_table[in.imm];
            } else if (in.src == 1) {
              for (int id : p.map_table)
                if (id == in.imm) mid = id;
            }
            if (mid < 0 || mid >= (int)o.maps.size()) fault("bad map reference");
            if (in.dst >= 10) fault("write to r10");
            r[in.dst] = Reg{K_MAPHANDLE, 0, mid, -1};
          }
          pc += 2;
          continue;
        }
      }
      pc++;
    }
  }
};

}  // namespace

int Oracle::run(const Program& prog, const uint8_t* events, uint64_t n, int order, uint64_t seed,
                uint32_t* rc_out) {
  HookInfo hi;
  if (!hook_info(prog.hook, &hi)) return -E_INVAL;
  for (int id : prog.map_table)
    if (id < 0 || id >= (int)maps.size()) return -E_INVAL;
  if (prog.hook == HOOK_WAVE_MEM) {
    // one invocation per tile of 64 consecutive records, its return code
    // given to every record of the tile; tiles in index order or shuffled
    const uint64_t tiles = (n + 63) / 64;
    std::vector<uint64_t> tix(tiles);
    std::iota(tix.begin(), tix.end(), 0);
    if (order == 2) {
      uint64_t s = seed;
      for (uint64_t i = tiles; i > 1; i--) {
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        std::swap(tix[i - 1], tix[z % i]);
      }
    }
    Exec ex(*this, prog, hi);
    for (uint64_t t : tix) {
      const uint64_t b = t * 64, e = b + 64 < n ? b + 64 : n;
      uint8_t ctx[24];
      wave_context(events, b, e, ctx);
      uint32_t rc = 0;
      try {
        rc = ex.run_event(ctx);
      } catch (const Fault& f) {
        stats.faults++;
        if (stats.fault_msg.empty()) stats.fault_msg = "tile " + std::to_string(t) + ": " + f.msg;
      }
      if (rc_out)
        for (uint64_t i = b; i < e; i++) rc_out[i] = rc;
    }
    return 0;
  }
  if (prog.hook == HOOK_SIMT_MEM) {
    // one invocation per record on {record, its tile's aggregate}; records
    // in index order or shuffled (the program is event-parallel)
    std::vector<uint64_t> ix(n);
    std::iota(ix.begin(), ix.end(), 0);
    if (order == 2) {
      uint64_t s = seed;
      for (uint64_t i = n; i > 1; i--) {
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        std::swap(ix[i - 1], ix[z % i]);
      }
    }
    std::vector<uint8_t> agg(((n + 63) / 64) * 24);
    for (uint64_t t = 0; t * 64 < n; t++) wave_context(events, t * 64, std::min(n, t * 64 + 64), &agg[t * 24]);
    Exec ex(*this, prog, hi);
    for (uint64_t i : ix) {
      uint8_t ctx[48];
      std::memcpy(ctx, events + i * 24, 24);
      std::memcpy(ctx + 24, &agg[(i / 64) * 24], 24);
      uint32_t rc = 0;
      try {
        rc = ex.run_event(ctx);
      } catch (const Fault& f) {
        stats.faults++;
        if (stats.fault_msg.empty()) stats.fault_msg = "event " + std::to_string(i) + ": " + f.msg;
      }
      if (rc_out) rc_out[i] = rc;
    }
    return 0;
  }
  std::vector<uint64_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  auto key = [&](uint64_t i) { return load_le(events + i * hi.record_size + hi.stream_off, hi.stream_size); };
  if (order == 1 || order == 3) {
    // group by stream (descending key), keep index order within a stream
    std::stable_sort(idx.begin(), idx.end(), [&](uint64_t a, uint64_t b) { return key(a) > key(b); });
    if (order == 1) {
      std::vector<std::vector<uint64_t>> groups;
      for (uint64_t i : idx) {
        if (groups.empty() || key(groups.back()[0]) != key(i)) groups.emplace_back();
        groups.back().push_back(i);
      }
      idx.clear();
      for (size_t round = 0;; round++) {
        bool any = false;
        for (auto& g : groups)
          if (round < g.size()) {
            idx.push_back(g[round]);
            any = true;
          }
        if (!any) break;
      }
    }
  } else if (order == 2) {
    uint64_t s = seed;
    for (uint64_t i = n; i > 1; i--) {  // Fisher-Yates with SplitMix64
      s += 0x9E3779B97F4A7C15ull;
      uint64_t z = s;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      z ^= z >> 31;
      std::swap(idx[i - 1], idx[z % i]);
    }
  }
  for (auto& m : maps) {
    m.owner.clear();
    m.multi.clear();
  }
  Exec ex(*this, prog, hi);
  for (uint64_t i : idx) {
    uint32_t rc = 0;
    try {
      rc = ex.run_event(events + i * hi.record_size);
    } catch (const Fault& f) {
      stats.faults++;
      if (stats.fault_msg.empty()) stats.fault_msg = "event " + std::to_string(i) + ": " + f.msg;
    }
    if (rc_out) rc_out[i] = rc;
  }
  uint64_t v = 0;
  for (auto& m : maps)
    for (auto& kv : m.multi)
      if (kv.second && m.owner[kv.first].second) v++;
  stats.violations = v;
  return 0;
}

}  // namespace gxo
