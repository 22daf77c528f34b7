// Device building blocks of the eBPF runtime for gfx950 (CDNA4, wave64),
// shared by the interpreter and by programs compiled to native code: wave
// utilities, per-lane stack frames in LDS, map helpers with
// wave-aggregated commutative atomics, ring-buffer output and the event
// loops of the two execution modes.
//
// Per lane: the event record's words in VGPRs and a private stack frame in
// LDS laid out word-major per wave (conflict-free for uniform offsets).
// Commutative map atomics that hit one address from every active lane are
// reduced across the wave and issued once (section 4.4, "Warp-level
// Execution Optimizations"); ring-buffer space is reserved once per wave.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#include "gx_internal.h"

namespace gx {

// Map helpers: a compiled program inlines them (its map descriptors are
// constants, so sizes, masks and addresses fold into the code); the
// interpreter calls them.
#ifdef GX_LDS_BYTES
#define GX_HELPER __device__ __forceinline__
#else
#define GX_HELPER __device__
#endif

// Stack frames live in this LDS array.  A compiled program sizes it
// statically (GX_LDS_BYTES); the interpreter's kernels size it at launch.
#ifdef GX_LDS_BYTES
__shared__ __attribute__((aligned(16))) uint8_t g_lds[GX_LDS_BYTES];
#else
extern __shared__ __attribute__((aligned(16))) uint8_t g_lds[];
#endif

// ---------------------------------------------------------------------------
// wave utilities

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ uint32_t rfl(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t rfl64(uint64_t x) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t rdlane(uint32_t x, uint32_t l) { return __builtin_amdgcn_readlane(x, l); }

// Wave-uniform execution (a compiled program run by one lane of a wave, one
// queue per wave): values the compiler cannot prove uniform are read from
// the first active lane, so the program's arithmetic, compares and branches
// run on the scalar unit (one instruction a cycle, no EXEC-mask updates)
// instead of as 64-lane vector operations of which one lane is used.
template <bool UNI>
__device__ __forceinline__ uint64_t uni(uint64_t x) {
  return UNI ? rfl64(x) : x;
}
__device__ __forceinline__ uint32_t popc64(uint64_t m) { return (uint32_t)__builtin_popcountll(m); }
__device__ __forceinline__ uint32_t rank_in(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Largest x over the active lanes (read lane by lane: used once per queue).
__device__ __forceinline__ uint32_t wave_max_active(uint32_t x) {
  uint32_t m = 0;
  for (uint64_t b = ballot(true); b; b &= b - 1) {
    const uint32_t v = __builtin_amdgcn_readlane(x, (uint32_t)__builtin_ctzll(b));
    m = v > m ? v : m;
  }
  return m;
}

// Map memory is device memory.  Its pointers come from descriptors, not
// kernel arguments, so the compiler cannot tell their address space; the
// casts make every access a global_* instruction instead of a flat_* one
// (a flat access also counts against the LDS counter, so a stack access
// after it would wait for the global one to finish).
#define GX_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GX_GLOBAL T* gl(T* p) {
  return (GX_GLOBAL T*)p;
}

// LDS words that lanes of a wave pass to each other (one lane writes, the
// others read later): every access is volatile, so that the compiler keeps
// no lane's own copy in a register, which would see only that lane's
// updates.
template <typename T>
__device__ __forceinline__ volatile __attribute__((address_space(3))) T* lds(T* p) {
  return (volatile __attribute__((address_space(3))) T*)p;
}

template <typename T>
__device__ __forceinline__ T ld_relaxed(T* p) {
  return __hip_atomic_load(gl(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// stack frames in LDS: frame byte o of a lane lives at
//   base + (o >> 3) * 512 + lane * 8 + (o & 7)

struct Stk {
  uint32_t base;   // byte offset of this wave's frames in g_lds
  uint32_t lane8;  // lane * 8
  uint32_t owner;  // global thread index: identifies the hardware lane for the launch
};

__device__ __forceinline__ uint8_t* saddr(const Stk& k, uint32_t o) {
  return g_lds + k.base + (o >> 3) * 512u + k.lane8 + (o & 7u);
}

__device__ __forceinline__ uint64_t sx(uint64_t v, int sc) {
  switch (sc) {
    case 0: return (uint64_t)(int64_t)(int8_t)v;
    case 1: return (uint64_t)(int64_t)(int16_t)v;
    case 2: return (uint64_t)(int64_t)(int32_t)v;
  }
  return v;
}

__device__ __forceinline__ uint64_t load_sized(const uint8_t* p, int sc) {
  switch (sc) {
    case 0: return *p;
    case 1: return *(const uint16_t*)p;
    case 2: return *(const uint32_t*)p;
  }
  return *(const uint64_t*)p;
}
__device__ __forceinline__ void store_sized(uint8_t* p, uint64_t v, int sc) {
  switch (sc) {
    case 0: *p = (uint8_t)v; break;
    case 1: *(uint16_t*)p = (uint16_t)v; break;
    case 2: *(uint32_t*)p = (uint32_t)v; break;
    default: *(uint64_t*)p = v; break;
  }
}
// the same on map memory
__device__ __forceinline__ uint64_t load_sized_g(uint64_t a, int sc) {
  switch (sc) {
    case 0: return *(const GX_GLOBAL uint8_t*)a;
    case 1: return *(const GX_GLOBAL uint16_t*)a;
    case 2: return *(const GX_GLOBAL uint32_t*)a;
  }
  return *(const GX_GLOBAL uint64_t*)a;
}
__device__ __forceinline__ void store_sized_g(uint64_t a, uint64_t v, int sc) {
  switch (sc) {
    case 0: *(GX_GLOBAL uint8_t*)a = (uint8_t)v; break;
    case 1: *(GX_GLOBAL uint16_t*)a = (uint16_t)v; break;
    case 2: *(GX_GLOBAL uint32_t*)a = (uint32_t)v; break;
    default: *(GX_GLOBAL uint64_t*)a = v; break;
  }
}

// Bytes [8w, 8w + 8) of an object of ``n`` bytes at ``p`` (stack offset or
// global address), zero beyond n.
__device__ __forceinline__ uint64_t chunk(int kind, uint64_t p, uint32_t w, uint32_t n, const Stk& stk) {
  uint32_t left = n - 8 * w;
  uint32_t m = left < 8 ? left : 8;
  if (kind == PK_STACK) {
    uint32_t o = (uint32_t)p + 8 * w;
    if (m == 8 && (o & 7) == 0) return *(const uint64_t*)saddr(stk, o);
    if (m == 4 && (o & 3) == 0) return *(const uint32_t*)saddr(stk, o);
    uint64_t v = 0;
    for (uint32_t i = 0; i < m; i++) v |= (uint64_t)*saddr(stk, o + i) << (8 * i);
    return v;
  }
  const GX_GLOBAL uint8_t* q = (const GX_GLOBAL uint8_t*)(p + 8 * w);
  if (m == 8 && ((uintptr_t)q & 7) == 0) return *(const GX_GLOBAL uint64_t*)q;
  if (m == 4 && ((uintptr_t)q & 3) == 0) return *(const GX_GLOBAL uint32_t*)q;
  uint64_t v = 0;
  for (uint32_t i = 0; i < m; i++) v |= (uint64_t)q[i] << (8 * i);
  return v;
}

// Copy n bytes from (kind, p) to global memory dst (8-byte aligned).
__device__ __forceinline__ void copy_in(uint8_t* dst, int kind, uint64_t p, uint32_t n, const Stk& stk) {
  uint32_t full = n / 8;
  for (uint32_t w = 0; w < full; w++) gl((uint64_t*)dst)[w] = chunk(kind, p, w, n, stk);
  for (uint32_t i = full * 8; i < n; i++) {
    uint64_t c = chunk(kind, p, i / 8, n, stk);
    gl(dst)[i] = (uint8_t)(c >> (8 * (i & 7)));
  }
}

// ---------------------------------------------------------------------------
// maps

__device__ __forceinline__ uint64_t key_hash(const MapDev* m, int kind, uint64_t kp, const Stk& stk) {
  uint32_t nw = (m->key_size + 7) / 8;
  uint64_t h = m->key_size;
  for (uint32_t w = 0; w < nw; w++) h = hash_step(h, chunk(kind, kp, w, m->key_size, stk));
  return hash_final(h);
}

// Hash slots.  The header word {u8 state, u24 epoch, u32 tag} and the key
// words are shared between lanes of every XCD, so they are only read and
// written with device-coherent relaxed atomics (no fences: on a multi-XCD
// device a release/acquire fence writes back / invalidates the whole L2).
// Values are written by the one lane that owns the key, with plain accesses.
// A tombstone records the launch (epoch) and the hardware lane (owner) that
// freed it; within that launch only the same lane may reclaim it, so no two
// lanes - possibly on different XCDs, whose L2s write back in no fixed
// order - ever write the same slot's bytes in one launch.  Later launches
// may reclaim any tombstone (a launch boundary writes every L2 back).
__device__ __forceinline__ uint64_t hdr_word(uint32_t state, uint32_t epoch, uint32_t tag) {
  return (uint64_t)state | ((uint64_t)(epoch & 0xffffffu) << 8) | ((uint64_t)tag << 32);
}

// May this launch's lane ``owner`` claim the slot whose header is st?
__device__ __forceinline__ bool claimable(uint64_t st, uint32_t epoch, uint32_t owner) {
  const uint32_t state = (uint32_t)st & 0xff;
  if (state == SLOT_EMPTY) return true;
  if (state != SLOT_TOMB) return false;
  return ((uint32_t)(st >> 8) & 0xffffffu) != (epoch & 0xffffffu) || (uint32_t)(st >> 32) == owner;
}

__device__ __forceinline__ bool key_eq(const MapDev* m, uint8_t* hdr, int kind, uint64_t kp, const Stk& stk) {
  uint32_t nw = (m->key_size + 7) / 8;
  for (uint32_t w = 0; w < nw; w++)
    if (ld_relaxed((uint64_t*)(hdr + 8 + 8 * w)) != chunk(kind, kp, w, m->key_size, stk)) return false;
  return true;
}

// A slot's header word and its one key word (keys of up to 8 bytes: a
// 16-byte slot) read in one device-coherent 16-byte access.  One access
// returns one state of the slot: an inserter's key words are complete at
// the coherence point before its header turns live, so a live header never
// comes with a stale key.  It replaces two dependent device-coherent reads,
// each of which goes past the XCD's L2.  The wait is part of the access
// (the header is needed at once).
typedef uint32_t gx_u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void load_slot16(const uint8_t* hdr, uint64_t* st, uint64_t* key) {
  gx_u32x4 v;
  __asm__ volatile("global_load_dwordx4 %0, %1, off sc1\n\ts_waitcnt vmcnt(0)" : "=v"(v) : "v"(hdr) : "memory");
  *st = (uint64_t)v.x | ((uint64_t)v.y << 32);
  *key = (uint64_t)v.z | ((uint64_t)v.w << 32);
}

// Probe for a key.  Returns the slot index or -1; *free_slot receives the
// first slot this launch may claim (or -1).
GX_HELPER int64_t hash_find(const MapDev* m, uint64_t h, int kind, uint64_t kp, const Stk& stk,
                             uint32_t epoch, int64_t* free_slot) {
  uint32_t mask = m->slot_mask;
  uint32_t i = (uint32_t)h & mask;
  uint32_t tag = (uint32_t)(h >> 32);
  int64_t fr = -1;
  const bool pair = m->sstride == 16;  // key of at most 8 bytes
  const uint64_t k0 = pair ? chunk(kind, kp, 0, m->key_size, stk) : 0;
  for (uint32_t probe = 0; probe <= mask; probe++) {
    uint8_t* hdr = m->slots + (uint64_t)i * m->sstride;
    uint64_t st, sk = 0;
    if (pair)
      load_slot16(hdr, &st, &sk);
    else
      st = ld_relaxed((uint64_t*)hdr);
    uint32_t state = (uint32_t)st & 0xff;
    if (state == SLOT_EMPTY) {
      if (fr < 0) fr = i;
      break;
    }
    if (state == SLOT_TOMB) {
      if (fr < 0 && claimable(st, epoch, stk.owner)) fr = i;
    } else if (state == SLOT_LIVE && (uint32_t)(st >> 32) == tag && (pair ? sk == k0 : key_eq(m, hdr, kind, kp, stk))) {
      if (free_slot) *free_slot = fr;
      return i;
    }
    i = (i + 1) & mask;
  }
  if (free_slot) *free_slot = fr;
  return -1;
}

// Lookup of a key of at most 8 bytes given as a value (compiled programs
// whose key lies in a register of the private frame); slots of 16 bytes.
GX_HELPER uint64_t hash_lookup_k(const MapDev* m, uint64_t k0, uint32_t epoch) {
  (void)epoch;
  const uint64_t h = hash_final(hash_step(m->key_size, k0));
  const uint32_t mask = m->slot_mask, tag = (uint32_t)(h >> 32);
  uint32_t i = (uint32_t)h & mask;
  for (uint32_t probe = 0; probe <= mask; probe++) {
    uint64_t st, sk;
    load_slot16(m->slots + (uint64_t)i * 16u, &st, &sk);
    const uint32_t state = (uint32_t)st & 0xff;
    if (state == SLOT_EMPTY) break;
    if (state == SLOT_LIVE && (uint32_t)(st >> 32) == tag && sk == k0) return (uint64_t)(m->data + (uint64_t)i * m->vstride);
    i = (i + 1) & mask;
  }
  return 0;
}

GX_HELPER uint64_t hash_lookup(const MapDev* m, int kind, uint64_t kp, const Stk& stk, uint32_t epoch) {
  uint64_t h = key_hash(m, kind, kp, stk);
  int64_t s = hash_find(m, h, kind, kp, stk, epoch, nullptr);
  return s < 0 ? 0 : (uint64_t)(m->data + (uint64_t)s * m->vstride);
}

GX_HELPER int64_t hash_update(const MapDev* m, int kkind, uint64_t kp, int vkind, uint64_t vp,
                               uint64_t flags, const Stk& stk, uint32_t epoch) {
  if (flags > 2) return -E_INVAL;
  uint64_t h = key_hash(m, kkind, kp, stk);
  int64_t fr;
  int64_t s = hash_find(m, h, kkind, kp, stk, epoch, &fr);
  if (s >= 0) {
    if (flags == 1) return -E_EXIST;
    copy_in(m->data + (uint64_t)s * m->vstride, vkind, vp, m->value_size, stk);
    return 0;
  }
  if (flags == 2) return -E_NOENT;
  uint64_t live = __hip_atomic_fetch_add(gl(&m->ctrl[0]), 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (live >= m->max_entries) {
    __hip_atomic_fetch_add(gl(&m->ctrl[0]), ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(gl(&m->ctrl[1]), 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return -E_2BIG;
  }
  uint32_t mask = m->slot_mask;
  uint32_t tag = (uint32_t)(h >> 32);
  uint32_t i = fr >= 0 ? (uint32_t)fr : ((uint32_t)h & mask);
  for (uint32_t probe = 0; probe <= mask; probe++) {
    uint64_t* hw = (uint64_t*)(m->slots + (uint64_t)i * m->sstride);
    uint64_t cur = ld_relaxed(hw);
    if (claimable(cur, epoch, stk.owner) &&
        __hip_atomic_compare_exchange_strong(gl(hw), &cur, hdr_word(SLOT_BUSY, epoch, tag), __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      uint32_t nw = (m->key_size + 7) / 8;
      for (uint32_t w = 0; w < nw; w++)
        __hip_atomic_store(gl(hw + 1 + w), chunk(kkind, kp, w, m->key_size, stk), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      copy_in(m->data + (uint64_t)i * m->vstride, vkind, vp, m->value_size, stk);
      // the key words reach the coherence point before the slot turns live
      __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __hip_atomic_store(gl(hw), hdr_word(SLOT_LIVE, epoch, tag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return 0;
    }
    i = (i + 1) & mask;
  }
  // no claimable slot in this launch; undo the reservation
  __hip_atomic_fetch_add(gl(&m->ctrl[0]), ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_fetch_add(gl(&m->ctrl[1]), 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return -E_2BIG;
}

GX_HELPER int64_t hash_delete(const MapDev* m, int kind, uint64_t kp, const Stk& stk, uint32_t epoch) {
  uint64_t h = key_hash(m, kind, kp, stk);
  int64_t s = hash_find(m, h, kind, kp, stk, epoch, nullptr);
  if (s < 0) return -E_NOENT;
  __hip_atomic_store(gl((uint64_t*)(m->slots + (uint64_t)s * m->sstride)),
                     hdr_word(SLOT_TOMB, epoch, stk.owner), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_fetch_add(gl(&m->ctrl[0]), ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return 0;
}

__device__ __forceinline__ uint64_t array_lookup_idx(const MapDev* m, uint32_t idx) {
  return idx < m->max_entries ? (uint64_t)(m->data + (uint64_t)idx * m->vstride) : 0;
}

__device__ __forceinline__ uint64_t array_lookup(const MapDev* m, int kind, uint64_t kp, const Stk& stk) {
  uint32_t idx = (uint32_t)chunk(kind, kp, 0, 4, stk);
  return idx < m->max_entries ? (uint64_t)(m->data + (uint64_t)idx * m->vstride) : 0;
}

GX_HELPER int64_t array_update(const MapDev* m, int kkind, uint64_t kp, int vkind, uint64_t vp, uint64_t flags,
                                const Stk& stk) {
  if (flags > 2) return -E_INVAL;
  uint32_t idx = (uint32_t)chunk(kkind, kp, 0, 4, stk);
  if (idx >= m->max_entries) return -E_2BIG;
  if (flags == 1) return -E_EXIST;
  copy_in(m->data + (uint64_t)idx * m->vstride, vkind, vp, m->value_size, stk);
  return 0;
}

// Ring space.  ctrl[0] head (bytes reserved so far), ctrl[1] tail (bytes
// the host consumed), ctrl[2] drops, ctrl[3] = ~(start of the first
// reservation that overflowed), 0 if none; from ctrl[kRingCount] on, the
// bytes of discard records and the records written since the last drain
// (summed per block in LDS, added once per block), so that a drain that
// takes the whole range need not walk it; ctrl[kRingUnknown] = 1 when a
// writer did not count (the interpreter's per-wave outputs).  A reservation is one fetch-add
// on the head (no compare-and-swap retries under contention); the head
// and tail are read first, so a request that cannot fit moves nothing.
// When two requests race past the end, the late one finds its range beyond
// the space, gives it up and records where it started: every later
// reservation lies further out and fails too, so the committed data ends
// exactly at the smallest such start, and the host's drain cuts the head
// back to it.
__device__ __forceinline__ bool ring_reserve(const MapDev* m, uint64_t total, uint64_t* base) {
  const uint64_t cap = (uint64_t)m->slot_mask + 1;
  const uint64_t t = ld_relaxed(&m->ctrl[1]);
  const uint64_t h = ld_relaxed(&m->ctrl[0]);
  if (h + total - t > cap) return false;
  const uint64_t old = __hip_atomic_fetch_add(gl(&m->ctrl[0]), total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (old + total - t > cap) {
    __hip_atomic_fetch_max(gl(&m->ctrl[3]), ~old, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
  }
  *base = old;
  return true;
}


// A record's payload word w, from the stack or map memory (``kind``, ``dp``)
// or, in compiled programs whose record lies in the private frame, from the
// caller's registers.
struct RecSrc {
  int kind;
  uint64_t dp;
  const Stk& stk;
  __device__ __forceinline__ uint64_t operator()(uint32_t w, uint32_t size) const { return chunk(kind, dp, w, size, stk); }
};
struct RecVal {
  uint64_t w[8];  // up to 64 bytes
  __device__ __forceinline__ uint64_t operator()(uint32_t j, uint32_t size) const {
    const uint32_t left = size - 8 * j;
    return left >= 8 ? w[j] : w[j] & ((1ull << (8 * left)) - 1);
  }
};

template <class Src>
__device__ __forceinline__ void ring_put(const MapDev* m, uint64_t pos, const Src& src, uint32_t size) {
  const uint64_t mask = m->slot_mask;
  const uint32_t nw = (size + 7) / 8;
  for (uint32_t w = 0; w < nw; w++) *gl((uint64_t*)(m->data + ((pos + 8 + 8 * w) & mask))) = src(w, size);
  // records are read by the host once the producing launch has completed
  *gl((uint64_t*)(m->data + (pos & mask))) = (uint64_t)size;
}

// ringbuf_output for the whole wave; ``act`` lanes take part.  Space for all
// outputs of the wave is reserved at once by the first active lane.
GX_HELPER uint64_t ring_output(const MapDev* m, int kind, uint64_t dp, uint32_t size, uint64_t flags,
                                bool act, const Stk& stk) {
  uint64_t res = 0;
  bool want = act && flags == 0;
  if (act && flags != 0) res = (uint64_t)-E_INVAL;
  uint64_t wm = ballot(want);
  if (wm == 0) return res;
  uint32_t need = 8 + ((size + 7) & ~7u);
  uint32_t cnt = popc64(wm);
  uint32_t leader = (uint32_t)__builtin_ctzll(wm);
  uint64_t total = (uint64_t)need * cnt;
  uint32_t ok = 0, base_lo = 0, base_hi = 0;
  if (lane_id() == leader) {
    uint64_t b = 0;
    ok = ring_reserve(m, total, &b) ? 1u : 0u;
    base_lo = (uint32_t)b;
    base_hi = (uint32_t)(b >> 32);
    if (!ok) __hip_atomic_fetch_add(gl(&m->ctrl[2]), (uint64_t)cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *gl(&m->ctrl[kRingUnknown]) = 1;  // records not counted: the drain walks them
  }
  ok = rdlane(ok, leader);
  uint64_t base = ((uint64_t)rdlane(base_hi, leader) << 32) | rdlane(base_lo, leader);
  if (!ok) {
    if (want) res = (uint64_t)-E_AGAIN;
    return res;
  }
  if (want) {
    ring_put(m, base + (uint64_t)need * rank_in(wm), RecSrc{kind, dp, stk}, size);
    res = 0;
  }
  return res;
}

// Ring space for compiled programs is handed out in two levels, so that the
// ring's head (one device-wide atomic counter, which every reservation
// serialises on) is touched rarely: a block reserves a large chunk from the
// ring, and each of its waves carves its own smaller chunk from the block's
// under a block-local lock in LDS; ring outputs carve their records from
// the wave's chunk.  The chunks live in LDS, one per (wave, ring) and one
// per (block, ring): a wave's lanes may reach a ring output under
// different EXEC masks, and LDS keeps one copy that every lane sees.
// Unused rest of a chunk becomes one discarded record when it is closed.
// A wave's chunk counts the records carved from it and adds them to the
// ring's record count when it is closed or replaced.
struct RingChunk {
  uint64_t pos;
  uint64_t left;
  uint64_t recs;
};

#ifdef GX_RING_SLOTS
__shared__ RingChunk g_rchunk[GX_RING_SLOTS];
__device__ __forceinline__ void chunk_store(uint32_t slot, uint64_t pos, uint64_t left, uint64_t recs) {
  *lds(&g_rchunk[slot].pos) = pos;
  *lds(&g_rchunk[slot].left) = left;
  *lds(&g_rchunk[slot].recs) = recs;
}
__shared__ RingChunk g_rblock[GX_NRINGS];
__shared__ uint32_t g_rlock[GX_NRINGS];
__shared__ uint64_t g_rcount[2 * GX_NRINGS];  // the block's discard bytes and records, per ring

// Chunk sizes: blocks' chunks and waves' chunks in flight each hold at most
// an eighth of the ring, so reserved-but-unused space never exceeds a
// quarter of it.
__device__ __forceinline__ uint64_t ring_chunk_bytes(uint64_t cap, uint64_t waves) {
  uint64_t c = cap / (8 * (waves ? waves : 1));
  c = c < 64 ? 64 : c > 8192 ? 8192 : c;
  return c & ~7ull;
}
__device__ __forceinline__ uint64_t ring_block_bytes(uint64_t cap, uint64_t blocks) {
  uint64_t c = cap / (8 * (blocks ? blocks : 1));
  c = c < 256 ? 256 : c > (1u << 20) ? (1u << 20) : c;
  return c & ~7ull;
}

__device__ __forceinline__ void ring_chunk_init(uint32_t slot) {
  if (lane_id() == 0) g_rchunk[slot] = RingChunk{0, 0, 0};
}
// by one wave of the block, before any wave uses the ring
__device__ __forceinline__ void ring_block_init(uint32_t r) {
  if (lane_id() == 0) {
    g_rblock[r] = RingChunk{0, 0, 0};
    g_rlock[r] = 0;
    g_rcount[2 * r] = 0;
    g_rcount[2 * r + 1] = 0;
  }
}

// (one lane) the unused rest of a chunk of ring r as a discard record
__device__ __forceinline__ void ring_discard(const MapDev* m, uint32_t r, uint64_t pos, uint64_t left) {
  if (left >= 8) {
    *gl((uint64_t*)(m->data + (pos & (uint64_t)m->slot_mask))) = (uint64_t)(left - 8) | ((uint64_t)RING_DISCARD << 32);
    __hip_atomic_fetch_add(&g_rcount[2 * r], left, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}
// (one lane) records carved from a wave's chunk of ring r
__device__ __forceinline__ void ring_count(uint32_t r, uint64_t recs) {
  if (recs) __hip_atomic_fetch_add(&g_rcount[2 * r + 1], recs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Close a wave's chunk (every wave) / the block's chunk (one wave, after
// every wave of the block has closed its own), which also adds the block's
// counts to the ring's.
__device__ __forceinline__ void ring_chunk_close(const MapDev* m, uint32_t slot) {
  const uint32_t r = slot % GX_NRINGS;
  const uint64_t left = *lds(&g_rchunk[slot].left), pos = *lds(&g_rchunk[slot].pos), recs = *lds(&g_rchunk[slot].recs);
  if (lane_id() == (uint32_t)__builtin_ctzll(ballot(true))) {
    ring_discard(m, r, pos, left);
    ring_count(r, recs);
    *lds(&g_rchunk[slot].left) = 0;
    *lds(&g_rchunk[slot].recs) = 0;
  }
}
__device__ __forceinline__ void ring_block_close(const MapDev* m, uint32_t r) {
  if (lane_id() == (uint32_t)__builtin_ctzll(ballot(true))) {
    ring_discard(m, r, g_rblock[r].pos, g_rblock[r].left);
    g_rblock[r].left = 0;
    const uint64_t d = g_rcount[2 * r], n = g_rcount[2 * r + 1];
    uint64_t* c = m->ctrl + kRingCount + 2 * (blockIdx.x % kRingCountSlots);
    if (d) __hip_atomic_fetch_add(gl(c), d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (n) __hip_atomic_fetch_add(gl(c + 1), n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    g_rcount[2 * r] = 0;
    g_rcount[2 * r + 1] = 0;
  }
}

// A wave's new chunk of ``ask`` bytes (by one lane): cut from the block's
// chunk, which is refilled from the ring when short.  false: the ring has
// no room (not even for ``need``, the wave's request itself).
__device__ __forceinline__ bool ring_block_take(const MapDev* m, uint32_t r, uint64_t block_bytes, uint64_t ask,
                                                uint64_t need, uint64_t* pos, uint64_t* got) {
  while (__hip_atomic_exchange(&g_rlock[r], 1u, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) != 0)
    __builtin_amdgcn_s_sleep(1);
  RingChunk b = g_rblock[r];
  bool ok = true;
  if (b.left < ask) {
    uint64_t base = 0;
    const uint64_t bask = ask > block_bytes ? ask : block_bytes;
    if (ring_reserve(m, bask, &base)) {
      ring_discard(m, r, b.pos, b.left);
      b = RingChunk{base, bask, 0};
    } else if (b.left >= need) {
      ask = need;  // the ring is nearly full: finish the block's chunk
    } else if (ring_reserve(m, need, &base)) {
      ring_discard(m, r, b.pos, b.left);
      b = RingChunk{base, need, 0};
      ask = need;
    } else {
      ok = false;
    }
  }
  if (ok) {
    *pos = b.pos;
    *got = ask;
    b.pos += ask;
    b.left -= ask;
    g_rblock[r] = b;
  }
  __hip_atomic_store(&g_rlock[r], 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  return ok;
}

// ringbuf_output carving from the wave's chunk, for active lanes that all
// pass one ring slot and one size; a new chunk of ``chunk_bytes`` (or the
// wave's whole request, if larger) is taken from the block's chunk when
// this one is short.  Same results as ring_output while space lasts; near a
// full ring a request may fail a little earlier (the unused parts of chunks
// count as used until the drain).
template <class Src>
__device__ __forceinline__ uint64_t ring_output_group(const MapDev* m, uint32_t slot, uint32_t r,
                                                       uint64_t chunk_bytes, uint64_t block_bytes, const Src& src,
                                                       uint32_t size, uint64_t flags) {
  uint64_t res = 0;
  const bool want = flags == 0;
  if (!want) res = (uint64_t)-E_INVAL;
  const uint64_t wm = ballot(want);
  if (wm == 0) return res;
  const uint32_t leader = (uint32_t)__builtin_ctzll(ballot(true));
  const uint32_t need = 8 + ((size + 7) & ~7u);
  const uint32_t cnt = popc64(wm);
  const uint64_t total = (uint64_t)need * cnt;
  uint64_t pos = *lds(&g_rchunk[slot].pos), left = *lds(&g_rchunk[slot].left), recs = *lds(&g_rchunk[slot].recs);
  if (total > left) {
    uint32_t ok = 0, lo = 0, hi = 0, glo = 0, ghi = 0;
    if (lane_id() == leader) {
      ring_discard(m, r, pos, left);
      ring_count(r, recs);
      uint64_t b = 0, got = 0;
      ok = ring_block_take(m, r, block_bytes, total > chunk_bytes ? total : chunk_bytes, total, &b, &got) ? 1u : 0u;
      lo = (uint32_t)b;
      hi = (uint32_t)(b >> 32);
      glo = (uint32_t)got;
      ghi = (uint32_t)(got >> 32);
      if (!ok) __hip_atomic_fetch_add(gl(&m->ctrl[2]), (uint64_t)cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    ok = rdlane(ok, leader);
    if (!ok) {
      if (lane_id() == leader) chunk_store(slot, pos, 0, 0);
      return want ? (uint64_t)-E_AGAIN : res;
    }
    pos = ((uint64_t)rdlane(hi, leader) << 32) | rdlane(lo, leader);
    left = ((uint64_t)rdlane(ghi, leader) << 32) | rdlane(glo, leader);
    recs = 0;
  }
  if (want) {
    ring_put(m, pos + (uint64_t)need * rank_in(wm), src, size);
    res = 0;
  }
  if (lane_id() == leader) chunk_store(slot, pos + total, left - total, recs + cnt);
  return res;
}

// ringbuf_output of compiled programs.  The compiler may merge call sites
// that differ in record size or ring (their arguments then vary by lane),
// so the active lanes are served one (slot, size) group at a time; each
// group's records are carved as one wave request.
template <class Src>
__device__ __forceinline__ uint64_t ring_output_src(const MapDev* m, uint32_t slot, uint32_t r, uint64_t chunk_bytes,
                                                     uint64_t block_bytes, const Src& src, uint32_t size,
                                                     uint64_t flags) {
  uint64_t res = 0;
  for (uint64_t todo = ballot(true); todo;) {
    const uint32_t l0 = (uint32_t)__builtin_ctzll(todo);
    const bool mine = slot == rdlane(slot, l0) && size == rdlane(size, l0);
    todo &= ~ballot(mine);
    if (mine) res = ring_output_group(m, slot, r, chunk_bytes, block_bytes, src, size, flags);
  }
  return res;
}
__device__ __forceinline__ uint64_t ring_output_chunked(const MapDev* m, uint32_t slot, uint32_t r,
                                                         uint64_t chunk_bytes, uint64_t block_bytes, int kind,
                                                         uint64_t dp, uint32_t size, uint64_t flags,
                                                         const Stk& stk) {
  return ring_output_src(m, slot, r, chunk_bytes, block_bytes, RecSrc{kind, dp, stk}, size, flags);
}
// The record's words passed by value (a record in the private frame of a
// compiled program: no stack memory is read).
__device__ __forceinline__ uint64_t ring_output_words(const MapDev* m, uint32_t slot, uint32_t r,
                                                       uint64_t chunk_bytes, uint64_t block_bytes, const RecVal& v,
                                                       uint32_t size, uint64_t flags) {
  return ring_output_src(m, slot, r, chunk_bytes, block_bytes, v, size, flags);
}
#endif

// ---------------------------------------------------------------------------
// Wave aggregation of commutative map updates by distinct address (section
// 4.4: duplicate map updates that SIMT execution causes).  The active lanes
// are taken group by group: the lowest remaining lane's address and every
// lane that shares it.  A group of two or more lanes is combined into one
// value, which its lowest lane applies once; the first singleton group ends
// the search (the addresses are then mostly distinct: uniformly spread
// updates pay one comparison), and so does the 8th group.  Combining equal
// addends takes a closed form (n * v for add, v for or/and, v or 0 for
// xor); unequal addends over a full wave take a DPP reduction; otherwise
// they are read lane by lane.

constexpr int kAggGroups = 8;

__device__ __forceinline__ uint64_t agg_identity(uint32_t op) { return op == 0x50 ? ~0ull : 0ull; }
__device__ __forceinline__ uint64_t agg_apply(uint64_t a, uint64_t b, uint32_t op) {
  switch (op) {
    case 0x00: return a + b;
    case 0x40: return a | b;
    case 0x50: return a & b;
    default: return a ^ b;
  }
}

__device__ __forceinline__ uint64_t rdlane_u64(uint64_t x, uint32_t j) {
  return ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(x >> 32), j) << 32) |
         __builtin_amdgcn_readlane((uint32_t)x, j);
}

// One DPP step of a wave reduction: every lane combines its value with the
// source lane's (row shift, or a row broadcast into the rows ROWS enables);
// lanes without a source combine with the identity.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_combine(uint64_t x, uint32_t op) {
  const uint64_t id = agg_identity(op);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)id, (int)(uint32_t)x, CTRL, ROWS, 0xf, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(id >> 32), (int)(uint32_t)(x >> 32), CTRL, ROWS, 0xf, false);
  return agg_apply(x, ((uint64_t)hi << 32) | lo, op);
}

// op over all 64 lanes (every lane active): inclusive scans of the rows of
// 16 by shifts of 1, 2, 4 and 8 lanes, then row 0 broadcast into row 1 and
// row 2 into row 3, then rows 0-1 into rows 2-3: lane 63 holds the total.
__device__ __forceinline__ uint64_t wave_reduce_full(uint64_t x, uint32_t op) {
  x = dpp_combine<0x111, 0xf>(x, op);  // row_shr:1
  x = dpp_combine<0x112, 0xf>(x, op);  // row_shr:2
  x = dpp_combine<0x114, 0xf>(x, op);  // row_shr:4
  x = dpp_combine<0x118, 0xf>(x, op);  // row_shr:8
  x = dpp_combine<0x142, 0xa>(x, op);  // row_bcast:15
  x = dpp_combine<0x143, 0xc>(x, op);  // row_bcast:31
  return rdlane_u64(x, 63);
}

// op over the lanes of group ``grp`` (active lanes, lowest lane l0).
__device__ __forceinline__ uint64_t group_combine(uint64_t v, uint32_t op, uint64_t grp, uint32_t l0) {
  const uint64_t v0 = rdlane_u64(v, l0);
  if ((ballot(v != v0) & grp) == 0) {
    const uint32_t n = popc64(grp);
    return op == 0x00 ? v0 * n : op == 0xa0 ? ((n & 1) ? v0 : 0) : v0;
  }
  if (grp == ~0ull) return wave_reduce_full(v, op);
  uint64_t acc = agg_identity(op);
  for (uint64_t m = grp; m; m &= m - 1) acc = agg_apply(acc, rdlane_u64(v, (uint32_t)__builtin_ctzll(m)), op);
  return acc;
}

// Aggregate this wave's commutative updates (op, addend v at addr): group
// leaders call apply(addr, combined) for their groups.  Returns true for a
// lane whose update is still its own to apply.
template <class F>
__device__ __forceinline__ bool wave_aggregate(uint64_t addr, uint64_t v, uint32_t op, F&& apply) {
  uint64_t todo = ballot(true);
  const uint32_t me = lane_id();
  for (int g = 0; g < kAggGroups && todo; g++) {
    const uint32_t l0 = (uint32_t)__builtin_ctzll(todo);
    const uint64_t grp = ballot(addr == rdlane_u64(addr, l0)) & todo;
    if (grp == (1ull << l0)) break;
    const uint64_t agg = group_combine(v, op, grp, l0);
    if (me == l0) apply(addr, agg);
    todo &= ~grp;
  }
  return (todo >> me) & 1;
}

template <typename T>
__device__ __forceinline__ void global_rmw_op(uint64_t addr, T v, uint32_t op) {
  GX_GLOBAL T* p = (GX_GLOBAL T*)addr;
  switch (op) {
    case 0x00: __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); break;
    case 0x40: __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); break;
    case 0x50: __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); break;
    default: __hip_atomic_fetch_xor(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); break;
  }
}

// The wave aggregation of a commutative non-fetching atomic on global
// memory; true for a lane whose update is still its own.  (Kept inline: a
// call out of the interpreter's dispatch loop costs register saves around
// every call, measured far worse than the grouping's own registers.)
__device__ __forceinline__ bool atomic_aggregate(uint64_t addr, uint64_t v, uint32_t op, int sc) {
  const bool w64 = sc == 3;
  return wave_aggregate(addr, v, op, [&](uint64_t a, uint64_t x) {
    if (w64)
      global_rmw_op<uint64_t>(a, x, op);
    else
      global_rmw_op<uint32_t>(a, (uint32_t)x, op);
  });
}

// Atomic read-modify-write on global memory; the commutative non-fetching
// forms are aggregated per wave by distinct address first.
__device__ __forceinline__ uint64_t atomic_global(uint64_t addr, uint64_t v, uint32_t op, int sc, uint64_t r0) {
  bool w64 = sc == 3;
  if (!(op & 1) && !atomic_aggregate(addr, v, op, sc)) return 0;  // ADD / OR / AND / XOR without fetch
  if (w64) {
    GX_GLOBAL uint64_t* p = (GX_GLOBAL uint64_t*)addr;
    switch (op) {
      case 0x00: case 0x01: return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      case 0x40: case 0x41: return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      case 0x50: case 0x51: return __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      case 0xa0: case 0xa1: return __hip_atomic_fetch_xor(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      case 0xe1: return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      default: {
        uint64_t e = r0;
        __hip_atomic_compare_exchange_strong(p, &e, v, __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return e;
      }
    }
  }
  GX_GLOBAL uint32_t* p = (GX_GLOBAL uint32_t*)addr;
  uint32_t x = (uint32_t)v;
  switch (op) {
    case 0x00: case 0x01: return __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    case 0x40: case 0x41: return __hip_atomic_fetch_or(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    case 0x50: case 0x51: return __hip_atomic_fetch_and(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    case 0xa0: case 0xa1: return __hip_atomic_fetch_xor(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    case 0xe1: return __hip_atomic_exchange(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    default: {
      uint32_t e = (uint32_t)r0;
      __hip_atomic_compare_exchange_strong(p, &e, x, __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return e;
    }
  }
}

// Load from memory that is constant for the launch: a scalar load when
// every active lane reads the same address, else a vector load.
template <typename T>
__device__ __forceinline__ T load_uniform(uint64_t addr) {
  typedef const __attribute__((address_space(4))) T cT;
  const uint64_t u = rfl64(addr);
  if (ballot(addr != u) == 0) return *(const cT*)u;
  // lanes apart: a global (not flat) vector load, consumed on this path, so
  // that the scalar path above never waits for the wave's vector memory
  uint64_t v = *(const GX_GLOBAL T*)addr;
  __asm__ volatile("" : "+v"(v));
  return (T)v;
}

// ---------------------------------------------------------------------------
// LDS accumulation of a shared map's commutative atomics (compiled programs,
// event-parallel kernels; section 4.4's aggregation of duplicate map
// updates taken from the wave to the workgroup).  A shared map takes one
// commutative operation at one width and is never read during a run, so a
// block may sum its updates in LDS and apply them to the map once, when it
// finishes: the map's final contents are the same.  Small maps are mirrored
// whole (word i of the LDS copy is word i of the value area); larger ones
// get a tagged cache keyed by address, whose misses go to the map directly.

template <typename T>
__device__ __forceinline__ T op_identity(uint32_t op) {
  return op == 0x50 ? (T)~(T)0 : (T)0;
}

template <typename T>
__device__ __forceinline__ void lds_rmw(T* p, T v, uint32_t op) {
  switch (op) {
    case 0x00: __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); break;
    case 0x40: __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); break;
    case 0x50: __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); break;
    default: __hip_atomic_fetch_xor(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); break;
  }
}

template <typename T>
__device__ __forceinline__ void global_rmw(T* q, T v, uint32_t op) {
  GX_GLOBAL T* p = gl(q);
  switch (op) {
    case 0x00: __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); break;
    case 0x40: __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); break;
    case 0x50: __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); break;
    default: __hip_atomic_fetch_xor(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); break;
  }
}

// whole-map mirror: acc[0..words) starts at the identity
template <typename T>
__device__ __forceinline__ void mirror_init(T* acc, uint32_t words, uint32_t op) {
  for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) acc[i] = op_identity<T>(op);
}
// consecutive threads flush consecutive words: coalesced device atomics
template <typename T>
__device__ __forceinline__ void mirror_flush(const T* acc, uint32_t words, uint32_t op, uint8_t* data) {
  const T id = op_identity<T>(op);
  for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) {
    const T v = acc[i];
    if (v != id) global_rmw((T*)data + i, v, op);
  }
}

// tagged cache, 4-way set associative: slot s*4 + w holds the partial sum
// of the word its tag names in set s (tag 0: free); a word claims the first
// free way of its set and keeps it for the block's lifetime, so a word whose
// set is full goes to the map directly.  Two tag formats: 32-bit tags (the
// word index + 1, one per slot), or 8-bit tags (the word index divided by
// the set count, + 1; the set's four packed in one 32-bit word), which hold
// 1.6x the slots in the same LDS when the quotient stays below 255.
constexpr uint32_t kCacheWays = 4;

// Set of a key (a word index) in a cache of ``sets`` 4-way sets: the index
// modulo an odd set count, so neighbouring words sit in neighbouring sets
// (the flush below then updates them with neighbouring lanes) while
// power-of-two strides still spread over all sets.
__device__ __forceinline__ uint32_t cache_set(uint32_t key, uint32_t sets) {
  return key % sets;
}

// Tag words of a cache of ``sets`` sets.
template <bool TAG8>
__device__ __forceinline__ uint32_t cache_tag_words(uint32_t sets) {
  return TAG8 ? sets : sets * kCacheWays;
}

template <typename TV, bool TAG8>
__device__ __forceinline__ void cache_init(uint32_t* tag, TV* val, uint32_t sets, uint32_t op) {
  for (uint32_t i = threadIdx.x; i < sets * kCacheWays; i += blockDim.x) {
    if (i < cache_tag_words<TAG8>(sets)) tag[i] = 0;
    val[i] = op_identity<TV>(op);
  }
}

// Way of ``key`` in its set, claiming an empty way if the key has none
// (-1: the set is full).  A tag goes from 0 to a key once, by compare-and-
// swap; the set's four tags are first read in one LDS access, and a stale
// 0 there only sends the lane to the compare-and-swap, which sees the truth.
__device__ __forceinline__ int cache_way(uint32_t* tag, uint32_t base, uint32_t key) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  typedef volatile __attribute__((address_space(3))) u32x4 lds_u32x4;
  const u32x4 t4 = *(lds_u32x4*)&tag[base];  // an LDS read, not a flat one
  const uint32_t t[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
  for (int w = 0; w < (int)kCacheWays; w++) {
    uint32_t c = t[w];
    if (c == 0) {
      uint32_t e = 0;
      c = __hip_atomic_compare_exchange_strong(&tag[base + w], &e, key, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP)
              ? key
              : e;
    }
    if (c == key) return w;
  }
  return -1;
}

// The same with 8-bit tags: t8 (1..255) in set s's tag word.  Ways fill in
// order, so a set's free ways are its last ones; the lowest byte equal to
// t8, or the lowest zero byte, is found with the zero-byte test on the
// word (exact for the lowest such byte).  A claim swaps the whole word and
// is retried when another lane changed it first; at most four claims ever
// succeed on a set, so a lane tries at most five times.
__device__ __forceinline__ int cache_way8(uint32_t* tag, uint32_t s, uint32_t t8) {
  uint32_t cur = *lds(&tag[s]);
  for (int tries = 0; tries < 5; tries++) {
    const uint32_t x = cur ^ (t8 * 0x01010101u);
    const uint32_t hit = (x - 0x01010101u) & ~x & 0x80808080u;
    if (hit) return (int)(__builtin_ctz(hit) >> 3);
    const uint32_t fr = (cur - 0x01010101u) & ~cur & 0x80808080u;
    if (!fr) return -1;
    const uint32_t w = __builtin_ctz(fr) >> 3;
    uint32_t e = cur;
    if (__hip_atomic_compare_exchange_strong(&tag[s], &e, cur | (t8 << (8 * w)), __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP))
      return (int)w;
    cur = e;
  }
  return -1;
}

// Slot of word index ``x`` (claimed if need be), or -1 when its set is full.
template <bool TAG8>
__device__ __forceinline__ int cache_slot(uint32_t* tag, uint32_t sets, uint32_t x) {
  const uint32_t s = cache_set(x, sets);
  const int w = TAG8 ? cache_way8(tag, s, x / sets + 1) : cache_way(tag, s * kCacheWays, x + 1);
  return w < 0 ? -1 : (int)(s * kCacheWays) + w;
}

template <typename T, bool TAG8>
__device__ __forceinline__ void cache_rmw(uint32_t* tag, T* val, uint32_t sets, uint8_t* data, uint64_t addr, T v,
                                          uint32_t op) {
  const int k = cache_slot<TAG8>(tag, sets, (uint32_t)((addr - (uint64_t)(uintptr_t)data) / sizeof(T)));
  if (k >= 0)
    lds_rmw(&val[k], v, op);
  else
    global_rmw((T*)addr, v, op);
}

// 64-bit sums kept as 32-bit partial sums (twice the slots in the same LDS):
// only addends up to ``vmax`` are summed in LDS, where vmax times the most
// updates a block can make (its events times the program's updates per
// invocation) stays below 2^32, so no partial sum can wrap and the LDS add
// needs no returned value; larger addends go to the map directly.
template <bool TAG8>
__device__ __forceinline__ void cache_add_narrow(uint32_t* tag, uint32_t* val, uint32_t sets, uint8_t* data,
                                                 uint64_t addr, uint64_t v, uint32_t vmax) {
  const int k = v <= vmax ? cache_slot<TAG8>(tag, sets, (uint32_t)((addr - (uint64_t)(uintptr_t)data) / 8)) : -1;
  if (k < 0)
    global_rmw((uint64_t*)addr, v, 0u);
  else
    __hip_atomic_fetch_add(&val[k], (uint32_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Largest addend a block's narrow caches sum in LDS (see cache_add_narrow):
// the block's waves take tiles t0, t0 + waves, ... of 64 events, and each
// invocation makes at most ``per_inv`` updates.
__device__ __forceinline__ uint32_t narrow_vmax(uint64_t n_events, uint64_t per_inv) {
  const uint64_t nw = blockDim.x / 64u, waves = (uint64_t)gridDim.x * nw;
  const uint64_t tiles = (n_events + 63) / 64;
  const uint64_t most = (tiles + waves - 1) / waves * nw * 64u * per_inv;
  return most ? (uint32_t)(0xffffffffull / most) : 0xffffffffu;
}

// Word index held by way w of set s, or -1 for a free way.
template <bool TAG8>
__device__ __forceinline__ int64_t cache_word(const uint32_t* tag, uint32_t sets, uint32_t s, uint32_t w) {
  const uint32_t t = TAG8 ? (tag[s] >> (8 * w)) & 0xffu : tag[s * kCacheWays + w];
  return t == 0 ? -1 : TAG8 ? (int64_t)(t - 1) * sets + s : (int64_t)t - 1;
}

// Consecutive threads flush one way of consecutive sets, which mostly hold
// neighbouring words (the first keys of a region to arrive take way 0):
// their device atomics then share cache lines.  T is the map word, TV the
// slot.
template <typename T, typename TV, bool TAG8>
__device__ __forceinline__ void cache_flush(const uint32_t* tag, const TV* val, uint32_t sets, uint32_t op,
                                            uint8_t* data) {
  const TV id = op_identity<TV>(op);
  for (uint32_t i = threadIdx.x; i < sets * kCacheWays; i += blockDim.x) {
    const uint32_t w = i / sets, s = i - w * sets;
    const int64_t x = cache_word<TAG8>(tag, sets, s, w);
    const TV v = val[s * kCacheWays + w];
    if (x >= 0 && v != id) global_rmw((T*)data + x, (T)v, op);
  }
}

// The block's cache written out for the reduce kernel: tags [sets][nb][4]
// (32-bit tags) or [sets][nb] (8-bit tags, a set's four in one word), then
// slots [sets][nb][4], this block's four ways of each set side by side.
template <typename TV, bool TAG8>
__device__ __forceinline__ void cache_spill(const uint32_t* tag, const TV* val, uint32_t sets, uint8_t* spill,
                                            uint32_t b, uint32_t nb) {
  uint32_t* st = (uint32_t*)spill;
  TV* sv = (TV*)(spill + (uint64_t)cache_tag_words<TAG8>(sets) * nb * 4);
  for (uint32_t i = threadIdx.x; i < sets * kCacheWays; i += blockDim.x) {
    const uint32_t s = i / kCacheWays, w = i - s * kCacheWays;
    const uint64_t at = ((uint64_t)s * nb + b) * kCacheWays + w;
    if (!TAG8) gl(st)[at] = tag[i];
    else if (w == 0) gl(st)[(uint64_t)s * nb + b] = tag[s];
    gl(sv)[at] = val[i];
  }
}

// One cache set over all blocks of a launch (one reduce block per set):
// every word of the set is summed in LDS - word x of set s is s + q * sets,
// so q indexes the LDS sums - and applied to the map with one device atomic.
template <typename T, typename TV, uint32_t QMAX, bool TAG8>
__device__ __forceinline__ void cache_reduce(const uint8_t* spill, uint32_t sets, uint32_t s, uint32_t nb,
                                             uint32_t op, uint8_t* data, uint32_t words) {
  __shared__ T sum[QMAX];
  const uint32_t* st = (const uint32_t*)spill;
  const TV* sv = (const TV*)(spill + (uint64_t)cache_tag_words<TAG8>(sets) * nb * 4);
  const T id = op_identity<T>(op);
  for (uint32_t q = threadIdx.x; q < QMAX; q += blockDim.x) sum[q] = id;
  __syncthreads();
  const uint64_t base = (uint64_t)s * nb * kCacheWays;
  for (uint32_t j = threadIdx.x; j < nb * kCacheWays; j += blockDim.x) {
    // q + 1 for the word of this way: the 8-bit tag itself, or x / sets + 1
    const uint32_t t = TAG8 ? (gl(st)[(uint64_t)s * nb + j / kCacheWays] >> (8 * (j % kCacheWays))) & 0xffu
                            : gl(st)[base + j];
    if (!t) continue;
    const TV v = gl(sv)[base + j];
    if (v != op_identity<TV>(op)) lds_rmw<T>(&sum[TAG8 ? t - 1 : (t - 1) / sets], (T)v, op);
  }
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < QMAX; q += blockDim.x) {
    const T v = sum[q];
    const uint64_t w = (uint64_t)q * sets + s;
    if (v != id && w < words) global_rmw((T*)data + w, v, op);
  }
}

// Lookup-memo table entries of compiled programs: the generation word's top
// bit marks an entry whose window words are newer than the map's memory.
constexpr uint64_t kMemoGen = ~0ull >> 1;

// Read-modify-write of the bytes at bit shift sh of a private-frame word
// (compiled programs; the frame is the lane's own): returns the old value.
__device__ __forceinline__ uint64_t frame_rmw(uint64_t& w, uint32_t sh, uint64_t v, uint32_t op, int sc, uint64_t r0) {
  const uint64_t mask = sc == 3 ? ~0ull : ((1ull << (8u << sc)) - 1);
  const uint64_t old = (w >> sh) & mask;
  uint64_t nv;
  switch (op & 0xf0) {
    case 0x00: nv = old + v; break;
    case 0x40: nv = old | v; break;
    case 0x50: nv = old & v; break;
    case 0xa0: nv = old ^ v; break;
    case 0xe0: nv = v; break;
    default: nv = ((sc == 3 ? r0 : (uint32_t)r0) == old) ? v : old; break;
  }
  w = (w & ~(mask << sh)) | ((nv & mask) << sh);
  return old;
}

// Read-modify-write on the lane's own stack (private: no atomicity needed).
__device__ __forceinline__ uint64_t atomic_stack(uint8_t* p, uint64_t v, uint32_t op, int sc, uint64_t r0) {
  uint64_t old = load_sized(p, sc), nv;
  switch (op & 0xf0) {
    case 0x00: nv = old + v; break;
    case 0x40: nv = old | v; break;
    case 0x50: nv = old & v; break;
    case 0xa0: nv = old ^ v; break;
    case 0xe0: nv = v; break;
    default: nv = ((sc == 3 ? r0 : (uint32_t)r0) == old) ? v : old; break;
  }
  store_sized(p, nv, sc);
  return old;
}

__device__ __forceinline__ uint64_t bswap_bits(uint64_t a, uint32_t bits) {
  if (bits == 16) return __builtin_bswap16((uint16_t)a);
  if (bits == 32) return __builtin_bswap32((uint32_t)a);
  return __builtin_bswap64(a);
}

// Minimum over all 64 lanes (every lane active) with DPP row operations:
// swap neighbours, swap pairs, mirror halves of 8, mirror rows of 16, then
// broadcast lane 15 into odd rows and lane 31 into the upper half; lane 63
// ends with the minimum of the wave.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_min(uint32_t x) {
  uint32_t y = (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, CTRL, ROW_MASK, 0xf, false);
  return y < x ? y : x;
}
__device__ __forceinline__ uint32_t wave_min_all(uint32_t x) {
  x = dpp_min<0xb1, 0xf>(x);   // quad_perm [1,0,3,2]
  x = dpp_min<0x4e, 0xf>(x);   // quad_perm [2,3,0,1]
  x = dpp_min<0x141, 0xf>(x);  // row_half_mirror
  x = dpp_min<0x140, 0xf>(x);  // row_mirror
  x = dpp_min<0x142, 0xa>(x);  // row_bcast:15
  x = dpp_min<0x143, 0xc>(x);  // row_bcast:31
  return __builtin_amdgcn_readlane(x, 63);
}

// Checked mode: a map-value access must stay inside the map it was verified
// against; a violation is counted and the access skipped.
__device__ __forceinline__ bool guard_ok(const RunArgs& A, uint32_t pc, uint64_t addr, uint32_t size) {
  typedef const __attribute__((address_space(4))) uint64_t cu64;
  const cu64* g = (const cu64*)(A.guards + 2 * pc);
  bool ok = addr >= g[0] && addr + size <= g[1];
  if (!ok) __hip_atomic_fetch_add(gl(A.err), 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return ok;
}

// ---------------------------------------------------------------------------
// event loops.  ``R.run(A, live, c0, c1, c2, g, stk, steps)`` executes one
// invocation per live lane and returns its rc; c0..c2 are the lane's
// context words, g the tile aggregate's (SIMT hook; zero otherwise).

struct Ctx {
  uint64_t c0, c1, c2;  // event record words
};

__device__ __forceinline__ Ctx load_record(const RunArgs& A, uint64_t i) {
  const uint64_t* p = (const uint64_t*)(A.events + i * A.record_size);
  Ctx c;
  c.c0 = p[0];
  c.c1 = p[1];
  c.c2 = A.record_size > 16 ? p[2] : 0;
  return c;
}

// One row-level DPP step of a wave-wide 64-bit min and max: every lane whose
// source lane (row shift, or row broadcast into the rows ROWS enables) exists
// combines that lane's values with its own; the others keep their own.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  const int l = (int)(uint32_t)v, h = (int)(uint32_t)(v >> 32);
  const uint32_t l2 = (uint32_t)__builtin_amdgcn_update_dpp(l, l, CTRL, ROWS, 0xf, false);
  const uint32_t h2 = (uint32_t)__builtin_amdgcn_update_dpp(h, h, CTRL, ROWS, 0xf, false);
  return ((uint64_t)h2 << 32) | l2;
}
template <int CTRL, int ROWS>
__device__ __forceinline__ void minmax_step(uint64_t& lo, uint64_t& hi) {
  const uint64_t a = dpp_u64<CTRL, ROWS>(lo), b = dpp_u64<CTRL, ROWS>(hi);
  lo = a < lo ? a : lo;
  hi = b > hi ? b : hi;
}

// One wave-tile of an event-parallel run: lane l runs event first + l.
// Warp-leader hook (section 4.4's warp-level execution): the context of one
// invocation for the wave's tile of memory-access records, from every
// lane's record - the smallest and largest address, the number of records,
// the stream of the tile's first record (lane 0's) - identical in every
// lane.  The extremes take four row shifts (1, 2, 4, 8 lanes: the last lane
// of each 16-lane row then holds its row's) and two row broadcasts (row 0
// into row 1, row 1 into rows 2 and 3: lane 63 then holds the wave's), all
// in the vector ALU, and one read of lane 63.
__device__ __forceinline__ Ctx wave_context(const Ctx& c, bool live) {
  uint64_t lo = live ? c.c0 : ~0ull, hi = live ? c.c0 : 0;
  minmax_step<0x111, 0xf>(lo, hi);  // row_shr:1
  minmax_step<0x112, 0xf>(lo, hi);  // row_shr:2
  minmax_step<0x114, 0xf>(lo, hi);  // row_shr:4
  minmax_step<0x118, 0xf>(lo, hi);  // row_shr:8
  minmax_step<0x142, 0xa>(lo, hi);  // row_bcast:15 into rows 1 and 3
  minmax_step<0x143, 0xc>(lo, hi);  // row_bcast:31 into rows 2 and 3
  const uint64_t wlo = ((uint64_t)rdlane((uint32_t)(lo >> 32), 63) << 32) | rdlane((uint32_t)lo, 63);
  const uint64_t whi = ((uint64_t)rdlane((uint32_t)(hi >> 32), 63) << 32) | rdlane((uint32_t)hi, 63);
  const uint32_t n = popc64(ballot(live));
  const uint32_t s0 = __builtin_amdgcn_readlane((uint32_t)c.c1, 0);
  return Ctx{wlo, whi, (uint64_t)n | ((uint64_t)s0 << 32)};
}

// One tile of an event-parallel run: every lane runs its record, or, for the
// warp-leader hook, lane 0 runs the tile's aggregate and every record of the
// tile receives its return code.
// (One call of R.run: the interpreter's body is large, and a second inlined
// copy of it would crowd the instruction cache.)
template <class Run>
__device__ __forceinline__ uint32_t tile_run(Run& R, const RunArgs& A, bool live, const Ctx& c, const Stk& stk,
                                             uint64_t& steps) {
  Ctx w = c, g{0, 0, 0};
  bool go = live;
  if (A.leader) {
    w = wave_context(c, live);
    go = lane_id() == 0 && live;
  } else if (A.simt) {
    g = wave_context(c, live);  // every lane runs its record, with the tile's aggregate
  }
  const uint32_t rc = R.run(A, go, w.c0, w.c1, w.c2, g, stk, steps);
  return A.leader ? __builtin_amdgcn_readlane(rc, 0) : rc;
}

template <class Run>
__device__ __forceinline__ void event_tile(Run& R, const RunArgs& A, uint64_t first, const Stk& stk, uint64_t& steps) {
  const uint64_t i = first + lane_id();
  const bool live = i < A.n_events;
  Ctx c{0, 0, 0};
  if (live) c = load_record(A, i);
  uint32_t rc = tile_run(R, A, live, c, stk, steps);
  if (live && A.rc) A.rc[i] = rc;
}

// A wave's share of an event-parallel run: tiles t0, t0 + tstep, ...
// (The interpreter loads one tile at a time: its flat accesses to the
// stack and maps wait for every outstanding vector load, so a tile loaded
// ahead would only be waited for sooner, and measured slower.)
template <class Run>
__device__ __forceinline__ void event_loop(Run& R, const RunArgs& A, uint64_t t0, uint64_t tstep, const Stk& stk) {
  uint64_t steps = 0;
  const uint64_t tiles = (A.n_events + 63) / 64;
  const uint32_t l = lane_id();
  for (uint64_t t = t0; t < tiles; t += tstep) {
    const uint64_t i = t * 64 + l;
    const bool live = i < A.n_events;
    Ctx c{0, 0, 0};
    if (live) c = load_record(A, i);
    const uint32_t rc = tile_run(R, A, live, c, stk, steps);
    if (live && A.rc) A.rc[i] = rc;
  }
}

// The same with the records of the next AHEAD tiles loaded while the
// current tile runs (compiled programs: their tiles issue no flat
// accesses, so no wait inside a tile holds the loads back).  AHEAD + 1
// record sets take turns (the loop body is unrolled over them) and every
// load is unconditional (a lane past the end reads the last record and
// runs no invocation), so that no register copy has to wait for a load.
template <int AHEAD, class Run>
__device__ __forceinline__ void event_loop_ahead(Run& R, const RunArgs& A, uint64_t t0, uint64_t tstep,
                                                 const Stk& stk) {
  constexpr int K = AHEAD + 1;
  uint64_t steps = 0;
  const uint64_t n = A.n_events, d = tstep * 64;
  if (n == 0) return;
  const uint64_t last = n - 1;
  uint64_t i = t0 * 64 + lane_id();  // this lane's event of the current tile
  Ctx set[K];
#pragma unroll
  for (int u = 0; u < AHEAD; u++) set[u] = load_record(A, i + u * d < last ? i + u * d : last);
  // every lane takes the same trips: t is lane 0's event
  for (uint64_t t = t0 * 64; t < n;) {
#pragma unroll
    for (int u = 0; u < K; u++) {
      const uint64_t j = i + AHEAD * d;
      set[(u + AHEAD) % K] = load_record(A, j < last ? j : last);
      const uint32_t rc = tile_run(R, A, i < n, set[u], stk, steps);
      if (i < n && A.rc) A.rc[i] = rc;
      i += d;
      t += d;
      if (t >= n) break;
    }
  }
}

// Record k of the queue-ordered copy.
__device__ __forceinline__ Ctx load_sorted(const RunArgs& A, uint64_t k) {
  const uint64_t* p = (const uint64_t*)(A.sorted + k * kSortedStride);
  Ctx c;
  c.c0 = p[0];
  c.c1 = p[1];
  c.c2 = A.record_size > 16 ? p[2] : 0;
  return c;
}

// One wave of a stream-sequential run: lane l < lanes owns queue q0 + l and
// runs that queue's events in index order.  The partition left each queue's
// records together (sorted[qstart[q] ..]) and their event indices in
// order[].  A lane's next kStreamBlock records and indices are loaded in
// one go while the current block runs: loads complete in issue order on
// this hardware, so one wait per block replaces one per event.  Return
// codes are kept in registers and stored once per block.
constexpr uint32_t kStreamBlock = 8;

template <class Run>
__device__ __forceinline__ void stream_wave(Run& R, const RunArgs& A, uint32_t q0, uint32_t lanes, uint32_t qstride,
                                            uint32_t qend_last, const Stk& stk, uint64_t& steps) {
  constexpr uint32_t B = kStreamBlock;
  const uint32_t l = lane_id();
  const uint32_t q = q0 + l;
  const bool own = l < lanes && q < A.n_queues;
  uint32_t beg = 0, end = 0;
  if (own) {
    beg = A.qstart[(uint64_t)q * qstride];
    end = q + 1 < A.n_queues ? A.qstart[(uint64_t)(q + 1) * qstride] : qend_last;
  }
  const uint32_t cnt = end - beg;
  const uint32_t rounds = wave_max_active(cnt);
  Ctx nx[B];
  uint32_t ni[B];
#pragma unroll
  for (uint32_t j = 0; j < B; j++) {
    nx[j] = Ctx{0, 0, 0};
    ni[j] = 0;
    if (j < cnt) {
      nx[j] = load_sorted(A, (uint64_t)beg + j);
      ni[j] = A.order[beg + j];
    }
  }
  for (uint32_t k0 = 0; k0 < rounds; k0 += B) {
    Ctx cu[B];
    uint32_t si[B], crc[B];
#pragma unroll
    for (uint32_t j = 0; j < B; j++) {
      cu[j] = nx[j];
      si[j] = ni[j];
      crc[j] = 0;
    }
    if (k0 + B < rounds) {
#pragma unroll
      for (uint32_t j = 0; j < B; j++)
        if (k0 + B + j < cnt) {
          nx[j] = load_sorted(A, (uint64_t)beg + k0 + B + j);
          ni[j] = A.order[beg + k0 + B + j];
        }
    }
    for (uint32_t j = 0; j < B; j++) {
      const Ctx c = cu[0];
#pragma unroll
      for (uint32_t x = 0; x + 1 < B; x++) cu[x] = cu[x + 1];
      uint32_t rc = 0;
      if (k0 + j < rounds) rc = R.run(A, k0 + j < cnt, c.c0, c.c1, c.c2, Ctx{0, 0, 0}, stk, steps);
#pragma unroll
      for (uint32_t x = 0; x + 1 < B; x++) crc[x] = crc[x + 1];
      crc[B - 1] = rc;
    }
    if (A.rc) {
#pragma unroll
      for (uint32_t j = 0; j < B; j++)
        if (k0 + j < cnt) A.rc[si[j]] = crc[j];
    }
    if (steps > A.step_limit) break;
  }
}

// One queue of a stream-sequential run, by lane 0 of the wave with
// wave-uniform values (compiled programs, one queue per wave; the kernels
// that call this have one wave per block).  The other 63 lanes fetch the
// queue's records: each lane loads one record of the next block of 64 with
// vector loads while lane 0 runs the current block, and lane 0 takes event
// j's record from lane j's registers (cross-lane reads: no memory access on
// the event chain).  The wait for a block's records thus comes once per 64
// events, long after they were requested.  (Holding records in scalar
// registers, the earlier design, ran out of scalar registers: the compiler
// spilled them as soon as they arrived, which made every record fetch a
// full memory round trip on the event chain.)  Return codes are gathered
// in LDS and stored by the whole wave after each block.
struct UniStage {
  uint32_t rc[64];
};

__device__ __forceinline__ uint64_t rdlane64(uint64_t x, uint32_t j) {
  return ((uint64_t)rdlane((uint32_t)(x >> 32), j) << 32) | rdlane((uint32_t)x, j);
}

template <bool GATHER, class Run>
__device__ __forceinline__ void stream_uni(Run& R, const RunArgs& A, uint32_t q, uint32_t qstride,
                                           uint32_t qend_last, const Stk& stk, uint64_t& steps) {
  typedef const __attribute__((address_space(4))) uint32_t cu32;
  __shared__ __attribute__((aligned(16))) UniStage st;
  if (q >= A.n_queues) return;
  const uint32_t beg = ((const cu32*)A.qstart)[(uint64_t)q * qstride];
  const uint32_t end = q + 1 < A.n_queues ? ((const cu32*)A.qstart)[(uint64_t)(q + 1) * qstride] : qend_last;
  if (beg >= end) return;
  const bool wide = A.record_size > 16;
  const uint32_t l = lane_id(), w2 = wide ? 2u : 1u;
  Ctx nc{0, 0, 0};
  uint32_t ni = 0;
  // With the queue-ordered copy, lane l reads record k0 + l of it and its
  // index; without it (A.sorted null), lane l gathers event order[k0 + l]
  // from the input: the indices are read a block earlier than the records
  // (ni2), so neither load waits inside the loop.  Every load is
  // unconditional (a lane past the queue's end reads its last event; a
  // 16-byte record's third word is its second, cleared where it is used),
  // so that no register copy of a load in flight waits for it.
  constexpr bool gather = GATHER;  // A.sorted is null exactly when GATHER
  const uint64_t last = end - 1;
  uint32_t ni2 = 0;
  auto index_of = [&](uint64_t k) { return ((const GX_GLOBAL uint32_t*)A.order)[k < last ? k : last]; };
  auto fetch = [&](uint64_t k0) {  // lane l: record k0 + l
    const uint64_t k = k0 + l;
    const GX_GLOBAL uint64_t* p;
    if (gather) {
      ni = ni2;
      ni2 = index_of(k + 64);
      p = (const GX_GLOBAL uint64_t*)(A.events + (uint64_t)ni * A.record_size);
    } else {
      p = (const GX_GLOBAL uint64_t*)(A.sorted + (k < last ? k : last) * kSortedStride);
      ni = index_of(k);
    }
    nc.c0 = p[0];
    nc.c1 = p[1];
    nc.c2 = p[w2];
  };
  if (gather) ni2 = index_of((uint64_t)beg + l);
  fetch(beg);
  for (uint64_t k0 = beg; k0 < end; k0 += 64) {
    Ctx cc{nc.c0, nc.c1, wide ? nc.c2 : 0};  // this block's records, one per lane
    // formed here, with every lane active: lane 0 reads them below by lane
    // index inside a branch only it takes, so their computation must not
    // move into that branch
    __asm__ volatile("" : "+v"(cc.c0), "+v"(cc.c1), "+v"(cc.c2));
    const uint32_t ci = ni;
    fetch(k0 + 64);
    const uint32_t n = end - k0 < 64 ? (uint32_t)(end - k0) : 64u;
    if (l == 0) {
      for (uint32_t j = 0; j < n; j++)
        st.rc[j] = (uint32_t)uni<true>(
            R.run(A, true, rdlane64(cc.c0, j), rdlane64(cc.c1, j), rdlane64(cc.c2, j), Ctx{0, 0, 0}, stk, steps));
    }
    R.uniformize();  // state lane 0 carries from event to event, back to wave-uniform
    if (A.rc && l < n) A.rc[ci] = st.rc[l];
    const uint64_t s0 = ((uint64_t)rdlane((uint32_t)(steps >> 32), 0) << 32) | rdlane((uint32_t)steps, 0);
    if (s0 > A.step_limit) break;
  }
}

// Persistent loop of the batched form: each wave claims work items (run,
// chunk) from a counter until none is left and calls f(batch, chunk).  The
// tables are read-only for the launch, so they are read with scalar loads.
template <class F>
__device__ __forceinline__ void batched_items(const BatchDev* B, const uint2* items, uint32_t n_items,
                                              uint32_t* next, F&& f) {
  typedef const __attribute__((address_space(4))) uint64_t cu64;
  static_assert(sizeof(BatchDev) % 8 == 0, "BatchDev is loaded as 8-byte words");
  for (;;) {
    uint32_t it = 0;
    if (lane_id() == 0) it = atomicAdd(next, 1u);
    it = __builtin_amdgcn_readlane(it, 0);
    if (it >= n_items) break;
    const uint64_t wv = ((const cu64*)items)[it];
    const uint32_t run = (uint32_t)wv, chunk = (uint32_t)(wv >> 32);
    uint64_t words[sizeof(BatchDev) / 8];
    const cu64* src = (const cu64*)(B + run);
#pragma unroll
    for (uint32_t k = 0; k < sizeof(BatchDev) / 8; k++) words[k] = src[k];
    BatchDev bd;
    __builtin_memcpy(&bd, words, sizeof(BatchDev));
    f(bd, chunk);
  }
}


// ---------------------------------------------------------------------------
// Hooks inside application kernels (section 5.3: trampolines at a kernel's
// memory instructions; persistent workers that claim logical work units).

// x mod n by Barrett reduction with mu = floor((2^64 - 1) / n): the quotient
// estimate is at most two below the true one, so two corrections suffice.
__device__ __forceinline__ uint64_t mod_n(uint64_t x, uint64_t n, uint64_t mu) {
  const uint64_t q = (uint64_t)(((unsigned __int128)x * mu) >> 64);
  uint64_t r = x - q * n;
  r = r >= n ? r - n : r;
  return r >= n ? r - n : r;
}

// One 64-iteration tile t of the instrumented vector add: lane l runs
// iteration i = 64 t + l, c[j] = a[j] + b[j] with j = (i stride) mod n.  With
// HOOK, a trampoline at the load of a[j] builds the access's memory-access
// record {addr = 8 j, stream = t, ts = i} and runs the program on it (per
// lane, once per tile on the tile's aggregate for the warp-leader hook, per
// lane with the aggregate for the SIMT hook).  A non-zero return code d is
// a prefetch hint for a[(j + d) mod n]: gfx950 has no data-prefetch
// instruction, so the lane loads that element and folds it into ``sink``,
// which only an empty asm statement at the kernel's end reads (the load is
// issued with the tile's own and waited for with them).
template <bool HOOK, class Run>
__device__ __forceinline__ void app_vadd_tile(Run& R, const RunArgs& A, const AppArgs& P, uint64_t t, const Stk& stk,
                                              uint64_t& steps, uint64_t& sink) {
  const uint64_t i = t * 64 + lane_id();
  const bool live = i < P.n;
  const uint64_t j = live ? mod_n(i * P.stride, P.n, P.mu) : 0;
  if (HOOK) {
    const uint32_t rc = tile_run(R, A, live, Ctx{8 * j, (uint64_t)(uint32_t)t, i}, stk, steps);
    if (live) {
      if (rc) sink ^= __builtin_bit_cast(uint64_t, P.a[mod_n(j + rc, P.n, P.mu)]);
      if (A.rc) A.rc[i] = rc;
    }
  }
  if (live) P.c[j] = P.a[j] + P.b[j];
}

// A wave's share of the vector add: tiles t0, t0 + tstep, ...
template <bool HOOK, class Run>
__device__ __forceinline__ void app_vadd_loop(Run& R, const RunArgs& A, const AppArgs& P, uint64_t t0, uint64_t tstep,
                                              const Stk& stk) {
  uint64_t sink = 0;
  const uint64_t tiles = (P.n + 63) / 64;
  for (uint64_t t = t0; t < tiles; t += tstep) {
    uint64_t steps = 0;  // the runaway guard's budget is per tile
    app_vadd_tile<HOOK>(R, A, P, t, stk, steps, sink);
  }
  asm volatile("" ::"v"(sink));
}

// Work unit u of the block scheduler's workload (a stand-in for one tile of
// an imbalanced kernel): lane l iterates a 64-bit linear congruential
// generator (Knuth's MMIX constants) cost[u] times from 64 u + l and stores
// the result at out[64 u + l].
__device__ __forceinline__ void sched_unit(const SchedArgs& S, uint32_t u) {
  uint64_t x = 64ull * u + lane_id();
  const uint32_t k = rfl(S.cost[u]);
  for (uint32_t m = 0; m < k; m++) x = x * 6364136223846793005ull + 1442695040888963407ull;
  S.out[64ull * u + lane_id()] = x;
}

__device__ __forceinline__ uint64_t wall_ticks() { return __builtin_amdgcn_s_memrealtime(); }

// Persistent worker w of the block scheduler (one wave; section 4.3.2's
// work-stealing scheduler).  Worker w owns units [w N / W, (w + 1) N / W)
// of the N units and claims them in order from its counter.  Once its range
// is empty, with HOOK, it asks the program before each steal whether to
// take one more unit; the victim is the first worker after w (cyclically)
// with units left, found 64 workers at a time.  The decision's context
// {u32 worker, u32 units done, u64 ns since the worker started, u64 ns
// since it began stealing, u32 units stolen, u32 units left in the
// victim's range} and return code are appended to the log.  A claim is a
// fetch-add on the owner's counter, so every unit runs exactly once
// whichever worker takes it: the results never depend on the policy, only
// the time does.  Without HOOK (static assignment) the worker stops once
// its range is empty.
template <bool HOOK, class Run>
__device__ __forceinline__ void sched_worker(Run& R, const RunArgs& A, const SchedArgs& S, uint32_t w,
                                             const Stk& stk) {
  const uint32_t W = S.workers, l = lane_id();
  auto first = [&](uint32_t v) { return (uint32_t)((uint64_t)v * S.n_units / W); };
  auto claim = [&](uint32_t v) -> uint32_t {
    uint32_t k = 0;
    if (l == 0) k = __hip_atomic_fetch_add(gl(&S.next[v]), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t u = first(v) + rdlane(k, 0);
    return u < first(v + 1) ? u : ~0u;
  };
  const uint64_t t0 = wall_ticks();
  uint32_t done = 0, stolen = 0;
  for (uint32_t u = claim(w); u != ~0u; u = claim(w)) {
    sched_unit(S, u);
    done++;
  }
  if (!HOOK) return;
  const uint64_t t1 = wall_ticks();
  for (;;) {
    uint32_t victim = ~0u, left = 0;
    for (uint32_t d0 = 1; d0 < W && victim == ~0u; d0 += 64) {
      const uint32_t d = d0 + l;
      uint32_t v = 0, rem = 0;
      if (d < W) {
        v = w + d >= W ? w + d - W : w + d;
        const uint32_t taken = __hip_atomic_load(gl(&S.next[v]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t size = first(v + 1) - first(v);
        rem = taken < size ? size - taken : 0;
      }
      if (ballot(rem > 0)) {
        // the candidate with the most units left (the nearest among
        // equals): thieves spread over the slow workers instead of all
        // claiming from the first one they find
        uint64_t lo = ((uint64_t)rem << 6) | (63u - l), hi = lo;
        minmax_step<0x111, 0xf>(lo, hi);  // row_shr:1
        minmax_step<0x112, 0xf>(lo, hi);  // row_shr:2
        minmax_step<0x114, 0xf>(lo, hi);  // row_shr:4
        minmax_step<0x118, 0xf>(lo, hi);  // row_shr:8
        minmax_step<0x142, 0xa>(lo, hi);  // row_bcast:15 into rows 1 and 3
        minmax_step<0x143, 0xc>(lo, hi);  // row_bcast:31 into rows 2 and 3
        const uint32_t f = 63u - (rdlane((uint32_t)hi, 63) & 63u);
        victim = rdlane(v, f);
        left = rdlane(rem, f);
      }
    }
    if (victim == ~0u) break;
    const uint64_t now = wall_ticks();
    const uint64_t c0 = w | ((uint64_t)done << 32);
    const uint64_t c1 = (now - t0) * S.tick_num / S.tick_den;
    const uint64_t c2 = (now - t1) * S.tick_num / S.tick_den;
    const uint64_t c3 = stolen | ((uint64_t)left << 32);
    // the record's fourth word travels as the aggregate's first; the
    // runaway guard's budget is per decision
    uint64_t steps = 0;
    const uint32_t rc = rdlane(R.run(A, l == 0, c0, c1, c2, Ctx{c3, 0, 0}, stk, steps), 0);
    if (l == 0) {
      const uint32_t at = __hip_atomic_fetch_add(gl(S.log_n), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (S.log && at < S.log_cap) {
        S.log[4ull * at] = c0;
        S.log[4ull * at + 1] = c1;
        S.log[4ull * at + 2] = c2;
        S.log[4ull * at + 3] = c3;
        S.log_rc[at] = rc;
      }
    }
    if (!rc) break;
    const uint32_t u = claim(victim);
    if (u != ~0u) {
      sched_unit(S, u);
      done++;
      stolen++;
    }
  }
}
}  // namespace gx
