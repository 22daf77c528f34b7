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
__device__ __forceinline__ uint32_t popc64(uint64_t m) { return (uint32_t)__builtin_popcountll(m); }
__device__ __forceinline__ uint32_t rank_in(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Wave reductions over the active lanes.  Older device compilers (such as
// the run-time compiler some PyTorch builds bundle) lack the builtins; they
// then get a lane loop here and per-lane map atomics without aggregation.
#if __has_builtin(__builtin_amdgcn_wave_reduce_add_u64) && __has_builtin(__builtin_amdgcn_wave_reduce_max_u32)
#define GX_HAS_WAVE_REDUCE 1
#else
#define GX_HAS_WAVE_REDUCE 0
#endif

__device__ __forceinline__ uint32_t wave_max_active(uint32_t x) {
#if GX_HAS_WAVE_REDUCE
  return __builtin_amdgcn_wave_reduce_max_u32(x, 0);
#else
  uint32_t m = 0;
  for (uint64_t b = ballot(true); b; b &= b - 1) {
    const uint32_t v = __builtin_amdgcn_readlane(x, (uint32_t)__builtin_ctzll(b));
    m = v > m ? v : m;
  }
  return m;
#endif
}

template <typename T>
__device__ __forceinline__ T ld_relaxed(T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
  const uint8_t* q = (const uint8_t*)p + 8 * w;
  if (m == 8 && ((uintptr_t)q & 7) == 0) return *(const uint64_t*)q;
  if (m == 4 && ((uintptr_t)q & 3) == 0) return *(const uint32_t*)q;
  uint64_t v = 0;
  for (uint32_t i = 0; i < m; i++) v |= (uint64_t)q[i] << (8 * i);
  return v;
}

// Copy n bytes from (kind, p) to global memory dst (8-byte aligned).
__device__ __forceinline__ void copy_in(uint8_t* dst, int kind, uint64_t p, uint32_t n, const Stk& stk) {
  uint32_t full = n / 8;
  for (uint32_t w = 0; w < full; w++) ((uint64_t*)dst)[w] = chunk(kind, p, w, n, stk);
  for (uint32_t i = full * 8; i < n; i++) {
    uint64_t c = chunk(kind, p, i / 8, n, stk);
    dst[i] = (uint8_t)(c >> (8 * (i & 7)));
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

// Probe for a key.  Returns the slot index or -1; *free_slot receives the
// first slot this launch may claim (or -1).
GX_HELPER int64_t hash_find(const MapDev* m, uint64_t h, int kind, uint64_t kp, const Stk& stk,
                             uint32_t epoch, int64_t* free_slot) {
  uint32_t mask = m->slot_mask;
  uint32_t i = (uint32_t)h & mask;
  uint32_t tag = (uint32_t)(h >> 32);
  int64_t fr = -1;
  for (uint32_t probe = 0; probe <= mask; probe++) {
    uint8_t* hdr = m->slots + (uint64_t)i * m->sstride;
    uint64_t st = ld_relaxed((uint64_t*)hdr);
    uint32_t state = (uint32_t)st & 0xff;
    if (state == SLOT_EMPTY) {
      if (fr < 0) fr = i;
      break;
    }
    if (state == SLOT_TOMB) {
      if (fr < 0 && claimable(st, epoch, stk.owner)) fr = i;
    } else if (state == SLOT_LIVE && (uint32_t)(st >> 32) == tag && key_eq(m, hdr, kind, kp, stk)) {
      if (free_slot) *free_slot = fr;
      return i;
    }
    i = (i + 1) & mask;
  }
  if (free_slot) *free_slot = fr;
  return -1;
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
  uint64_t live = __hip_atomic_fetch_add(&m->ctrl[0], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (live >= m->max_entries) {
    __hip_atomic_fetch_add(&m->ctrl[0], ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&m->ctrl[1], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return -E_2BIG;
  }
  uint32_t mask = m->slot_mask;
  uint32_t tag = (uint32_t)(h >> 32);
  uint32_t i = fr >= 0 ? (uint32_t)fr : ((uint32_t)h & mask);
  for (uint32_t probe = 0; probe <= mask; probe++) {
    uint64_t* hw = (uint64_t*)(m->slots + (uint64_t)i * m->sstride);
    uint64_t cur = ld_relaxed(hw);
    if (claimable(cur, epoch, stk.owner) &&
        __hip_atomic_compare_exchange_strong(hw, &cur, hdr_word(SLOT_BUSY, epoch, tag), __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      uint32_t nw = (m->key_size + 7) / 8;
      for (uint32_t w = 0; w < nw; w++)
        __hip_atomic_store(hw + 1 + w, chunk(kkind, kp, w, m->key_size, stk), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      copy_in(m->data + (uint64_t)i * m->vstride, vkind, vp, m->value_size, stk);
      // the key words reach the coherence point before the slot turns live
      __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __hip_atomic_store(hw, hdr_word(SLOT_LIVE, epoch, tag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return 0;
    }
    i = (i + 1) & mask;
  }
  // no claimable slot in this launch; undo the reservation
  __hip_atomic_fetch_add(&m->ctrl[0], ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_fetch_add(&m->ctrl[1], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return -E_2BIG;
}

GX_HELPER int64_t hash_delete(const MapDev* m, int kind, uint64_t kp, const Stk& stk, uint32_t epoch) {
  uint64_t h = key_hash(m, kind, kp, stk);
  int64_t s = hash_find(m, h, kind, kp, stk, epoch, nullptr);
  if (s < 0) return -E_NOENT;
  __hip_atomic_store((uint64_t*)(m->slots + (uint64_t)s * m->sstride),
                     hdr_word(SLOT_TOMB, epoch, stk.owner), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_fetch_add(&m->ctrl[0], ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return 0;
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

// ringbuf_output for the whole wave; ``act`` lanes take part.  Space for all
// outputs of the wave is reserved with one compare-and-swap on the head.
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
  uint64_t cap = (uint64_t)m->slot_mask + 1;
  uint32_t ok = 0, base_lo = 0, base_hi = 0;
  if (lane_id() == leader) {
    uint64_t* head = &m->ctrl[0];
    uint64_t h = ld_relaxed(head);
    for (int tries = 0; tries < 1 << 20; tries++) {
      uint64_t t = ld_relaxed(&m->ctrl[1]);
      if (h + total - t > cap) break;
      if (__hip_atomic_compare_exchange_strong(head, &h, h + total, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 1;
        break;
      }
    }
    base_lo = (uint32_t)h;
    base_hi = (uint32_t)(h >> 32);
    if (!ok) __hip_atomic_fetch_add(&m->ctrl[2], (uint64_t)cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  ok = rdlane(ok, leader);
  uint64_t base = ((uint64_t)rdlane(base_hi, leader) << 32) | rdlane(base_lo, leader);
  if (!ok) {
    if (want) res = (uint64_t)-E_AGAIN;
    return res;
  }
  if (want) {
    uint64_t pos = base + (uint64_t)need * rank_in(wm);
    uint64_t mask = cap - 1;
    uint32_t nw = (size + 7) / 8;
    for (uint32_t w = 0; w < nw; w++)
      *(uint64_t*)(m->data + ((pos + 8 + 8 * w) & mask)) = chunk(kind, dp, w, size, stk);
    // records are read by the host once the producing launch has completed
    *(uint64_t*)(m->data + (pos & mask)) = (uint64_t)size;
    res = 0;
  }
  return res;
}

// Atomic read-modify-write on global memory; commutative non-fetching forms
// are reduced across the active lanes when they all hit one address.
__device__ __forceinline__ uint64_t atomic_global(uint64_t addr, uint64_t v, uint32_t op, int sc, uint64_t r0) {
  bool w64 = sc == 3;
#if GX_HAS_WAVE_REDUCE
  if (!(op & 1)) {  // ADD / OR / AND / XOR without fetch
    uint64_t first = rfl64(addr);
    if (ballot(addr == first) == ballot(true)) {
      uint64_t agg;
      switch (op) {
        case 0x00: agg = w64 ? __builtin_amdgcn_wave_reduce_add_u64(v, 0) : __builtin_amdgcn_wave_reduce_add_u32((uint32_t)v, 0); break;
        case 0x40: agg = w64 ? __builtin_amdgcn_wave_reduce_or_b64(v, 0) : __builtin_amdgcn_wave_reduce_or_b32((uint32_t)v, 0); break;
        case 0x50: agg = w64 ? __builtin_amdgcn_wave_reduce_and_b64(v, 0) : __builtin_amdgcn_wave_reduce_and_b32((uint32_t)v, 0); break;
        default: agg = w64 ? __builtin_amdgcn_wave_reduce_xor_b64(v, 0) : __builtin_amdgcn_wave_reduce_xor_b32((uint32_t)v, 0); break;
      }
      if (lane_id() == (uint32_t)__builtin_ctzll(ballot(true))) {
        v = agg;
      } else {
        return 0;
      }
    }
  }
#endif
  if (w64) {
    uint64_t* p = (uint64_t*)addr;
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
  uint32_t* p = (uint32_t*)addr;
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
  if (!ok) __hip_atomic_fetch_add(A.err, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return ok;
}

// ---------------------------------------------------------------------------
// event loops.  ``Run::run(A, live, c0, c1, c2, stk, steps)`` executes one
// invocation per live lane and returns its rc.

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

// One wave-tile of an event-parallel run: lane l runs event first + l.
template <class Run>
__device__ __forceinline__ void event_tile(const RunArgs& A, uint64_t first, const Stk& stk, uint64_t& steps) {
  const uint64_t i = first + lane_id();
  const bool live = i < A.n_events;
  Ctx c{0, 0, 0};
  if (live) c = load_record(A, i);
  uint32_t rc = Run::run(A, live, c.c0, c.c1, c.c2, stk, steps);
  if (live && A.rc) A.rc[i] = rc;
}

// One wave of a stream-sequential run: lane l < lanes owns queue q0 + l and
// runs that queue's events (order[qstart[q] ..]) in index order.
template <class Run>
__device__ __forceinline__ void stream_wave(const RunArgs& A, uint32_t q0, uint32_t lanes, uint32_t qstride,
                                            uint32_t qend_last, const Stk& stk, uint64_t& steps) {
  const uint32_t l = lane_id();
  const uint32_t q = q0 + l;
  const bool own = l < lanes && q < A.n_queues;
  uint32_t beg = 0, end = 0;
  if (own) {
    beg = A.qstart[(uint64_t)q * qstride];
    end = q + 1 < A.n_queues ? A.qstart[(uint64_t)(q + 1) * qstride] : qend_last;
  }
  uint32_t cnt = end - beg;
  const uint32_t rounds = wave_max_active(cnt);
  // the next event's index and record are loaded while this one runs
  uint64_t ni = cnt > 0 ? A.order[beg] : 0;
  Ctx nc{0, 0, 0};
  if (cnt > 0) nc = load_record(A, ni);
  for (uint32_t k = 0; k < rounds; k++) {
    const bool live = k < cnt;
    const uint64_t i = ni;
    const Ctx c = nc;
    if (k + 1 < cnt) {
      ni = A.order[beg + k + 1];
      nc = load_record(A, ni);
    }
    uint32_t rc = Run::run(A, live, c.c0, c.c1, c.c2, stk, steps);
    if (live && A.rc) A.rc[i] = rc;
    if (steps > A.step_limit) break;
  }
}

}  // namespace gx
