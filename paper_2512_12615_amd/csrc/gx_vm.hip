// Interpreter of the device-side eBPF runtime for gfx950 (CDNA4, wave64),
// and the runtime's other kernels (stream partition, scans, map operations).
//
// One lane runs one event's invocation (paper section 5.3 runs the handler
// per warp; the deterministic per-event reading is documented with the
// boundary).  Per lane: r0-r10 as a 16 x u64 register vector held in VGPRs.
// Per wave: one uniform pc; the pre-decoded micro-op is fetched through the
// scalar cache.  Branches that all live lanes take the same way keep the wave
// in uniform mode; a split branch switches the wave to minimum-pc scheduling
// until the lanes meet again.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "gx_dev.h"

namespace gx {

typedef uint64_t rf_t __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// The interpreter: runs one invocation per live lane and returns rc.

// A shared map's commutative atomic into the block's LDS mirror (only
// commutative non-fetching operations reach a shared map, all of one
// operation at one width, so the old value is never needed).
__device__ __forceinline__ void acc_rmw(const RunArgs& A, uint64_t ad, uint64_t v) {
  uint8_t* base = g_lds + A.acc_lds;
  const uint64_t i = (ad - A.acc_lo) >> A.acc_sc;
  if (A.acc_sc == 3)
    lds_rmw<uint64_t>((uint64_t*)base + i, v, A.acc_op);
  else
    lds_rmw<uint32_t>((uint32_t*)base + i, (uint32_t)v, A.acc_op);
}

__device__ __forceinline__ uint32_t vm_run(const RunArgs& A, bool live, uint64_t c0, uint64_t c1, uint64_t c2,
                                           const Ctx& g, const Stk stk, uint64_t& steps) {
  const Uop* __restrict__ U = A.uops;
  rf_t r = (rf_t)(0);
  r[10] = A.stack_bytes;
  bool alive = live;
  uint32_t rc = 0;
  uint32_t pc = 0;
  bool div = false;
  uint32_t mypc = 0;
  uint32_t wd = 15;
  uint64_t wres = 0;
  if (ballot(alive) == 0) return 0;
  for (;;) {
    // pc and wd are wave-uniform; say so, so that register indexing and the
    // micro-op fetch stay scalar
    pc = rfl(pc);
    wd = rfl(wd);
    r[wd] = wres;
    if (++steps > A.step_limit) {
      if (lane_id() == (uint32_t)__builtin_ctzll(ballot(true)))
        __hip_atomic_fetch_add(A.err, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    // constant address space: invariant for the kernel's lifetime, so the
    // uniform fetch becomes a scalar load
    typedef const __attribute__((address_space(4))) uint64_t cu64;
    const cu64* up = (const cu64*)(U + pc);
    const uint64_t q0 = up[0], imm = up[1];
    const uint32_t w0 = (uint32_t)q0;
    const int32_t aux = (int32_t)(q0 >> 32);
    const uint32_t h = w0 & 0xff, d = (w0 >> 8) & 15, s = (w0 >> 12) & 15, a8 = (w0 >> 16) & 0xff;
    const bool K = (w0 >> 24) & 1;
    bool act = alive && (!div || mypc == pc);
    const uint64_t a = r[d];
    uint64_t b;
    if (K) b = imm;
    else b = r[s];
    uint64_t res = a, wold = a;
    uint32_t nwd = 15;
    uint32_t npc = pc + 1;
    int br = 0;
    bool tk = false;
    const uint32_t xa = (uint32_t)a, xb = (uint32_t)b;
    const int sc = a8 & 3;
    switch (h) {
      case H_ADD64: res = a + b; nwd = d; break;
      case H_SUB64: res = a - b; nwd = d; break;
      case H_MUL64: res = a * b; nwd = d; break;
      case H_DIV64: res = b ? a / b : 0; nwd = d; break;
      case H_SDIV64:
        res = !b ? 0 : ((int64_t)a == INT64_MIN && (int64_t)b == -1) ? a : (uint64_t)((int64_t)a / (int64_t)b);
        nwd = d;
        break;
      case H_OR64: res = a | b; nwd = d; break;
      case H_AND64: res = a & b; nwd = d; break;
      case H_LSH64: res = a << (b & 63); nwd = d; break;
      case H_RSH64: res = a >> (b & 63); nwd = d; break;
      case H_NEG64: res = 0 - a; nwd = d; break;
      case H_MOD64: res = b ? a % b : a; nwd = d; break;
      case H_SMOD64: res = !b ? a : ((int64_t)b == -1) ? 0 : (uint64_t)((int64_t)a % (int64_t)b); nwd = d; break;
      case H_XOR64: res = a ^ b; nwd = d; break;
      case H_MOV64: res = b; nwd = d; break;
      case H_ARSH64: res = (uint64_t)((int64_t)a >> (b & 63)); nwd = d; break;
      case H_MOVSX64: res = a8 == 8 ? sx(b, 0) : a8 == 16 ? sx(b, 1) : sx(b, 2); nwd = d; break;
      case H_BSWAP: res = bswap_bits(a, a8); nwd = d; break;
      case H_TRUNC: res = a8 == 16 ? (a & 0xffff) : a8 == 32 ? (a & 0xffffffffull) : a; nwd = d; break;
      case H_ADD32: res = (uint32_t)(xa + xb); nwd = d; break;
      case H_SUB32: res = (uint32_t)(xa - xb); nwd = d; break;
      case H_MUL32: res = (uint32_t)(xa * xb); nwd = d; break;
      case H_DIV32: res = xb ? xa / xb : 0; nwd = d; break;
      case H_SDIV32:
        res = !xb ? 0 : ((int32_t)xa == INT32_MIN && (int32_t)xb == -1) ? xa : (uint32_t)((int32_t)xa / (int32_t)xb);
        nwd = d;
        break;
      case H_OR32: res = xa | xb; nwd = d; break;
      case H_AND32: res = xa & xb; nwd = d; break;
      case H_LSH32: res = (uint32_t)(xa << (xb & 31)); nwd = d; break;
      case H_RSH32: res = xa >> (xb & 31); nwd = d; break;
      case H_NEG32: res = (uint32_t)(0u - xa); nwd = d; break;
      case H_MOD32: res = xb ? xa % xb : xa; nwd = d; break;
      case H_SMOD32: res = !xb ? xa : ((int32_t)xb == -1) ? 0u : (uint32_t)((int32_t)xa % (int32_t)xb); nwd = d; break;
      case H_XOR32: res = xa ^ xb; nwd = d; break;
      case H_MOV32: res = xb; nwd = d; break;
      case H_ARSH32: res = (uint32_t)((int32_t)xa >> (xb & 31)); nwd = d; break;
      case H_MOVSX32: res = (uint32_t)(a8 == 8 ? sx(b, 0) : sx(b, 1)); nwd = d; break;
      // jumps
      case H_JA: npc = (uint32_t)aux; break;
      case H_JEQ: br = 1; tk = a == b; break;
      case H_JGT: br = 1; tk = a > b; break;
      case H_JGE: br = 1; tk = a >= b; break;
      case H_JSET: br = 1; tk = (a & b) != 0; break;
      case H_JNE: br = 1; tk = a != b; break;
      case H_JSGT: br = 1; tk = (int64_t)a > (int64_t)b; break;
      case H_JSGE: br = 1; tk = (int64_t)a >= (int64_t)b; break;
      case H_JLT: br = 1; tk = a < b; break;
      case H_JLE: br = 1; tk = a <= b; break;
      case H_JSLT: br = 1; tk = (int64_t)a < (int64_t)b; break;
      case H_JSLE: br = 1; tk = (int64_t)a <= (int64_t)b; break;
      case H_JEQ32: br = 1; tk = xa == xb; break;
      case H_JGT32: br = 1; tk = xa > xb; break;
      case H_JGE32: br = 1; tk = xa >= xb; break;
      case H_JSET32: br = 1; tk = (xa & xb) != 0; break;
      case H_JNE32: br = 1; tk = xa != xb; break;
      case H_JSGT32: br = 1; tk = (int32_t)xa > (int32_t)xb; break;
      case H_JSGE32: br = 1; tk = (int32_t)xa >= (int32_t)xb; break;
      case H_JLT32: br = 1; tk = xa < xb; break;
      case H_JLE32: br = 1; tk = xa <= xb; break;
      case H_JSLT32: br = 1; tk = (int32_t)xa < (int32_t)xb; break;
      case H_JSLE32: br = 1; tk = (int32_t)xa <= (int32_t)xb; break;
      // memory
      case H_LDX_CTX: {
        const uint32_t wi = (uint32_t)aux >> 3;
        uint64_t wv = c0;
        if (wi == 1) wv = c1;
        if (wi == 2) wv = c2;
        if (wi == 3) wv = g.c0;  // the tile's aggregate (SIMT hook)
        if (wi == 4) wv = g.c1;
        if (wi == 5) wv = g.c2;
        wv >>= 8 * ((uint32_t)aux & 7);
        uint64_t v = sc == 3 ? wv : (wv & ((1ull << (8 << sc)) - 1));
        res = (a8 & 4) ? sx(v, sc) : v;
        nwd = d;
        break;
      }
      case H_LDX_STACK:
        if (act) {
          uint64_t v = load_sized(saddr(stk, (uint32_t)b + aux), sc);
          res = (a8 & 4) ? sx(v, sc) : v;
        }
        nwd = d;
        break;
      case H_LDX_MAP:
        if (A.checked) act = act && guard_ok(A, pc, b + (int64_t)aux, 1u << sc);
        if (act) {
          uint64_t v = load_sized_g(b + (uint64_t)(int64_t)aux, sc);
          res = (a8 & 4) ? sx(v, sc) : v;
        }
        nwd = d;
        break;
      case H_ST_STACK:
      case H_STX_STACK:
        if (act) store_sized(saddr(stk, (uint32_t)a + aux), b, sc);
        break;
      case H_ST_MAP:
      case H_STX_MAP:
        if (A.checked) act = act && guard_ok(A, pc, a + (int64_t)aux, 1u << sc);
        if (act) store_sized_g(a + (uint64_t)(int64_t)aux, b, sc);
        break;
      case H_ATOMIC_STACK:
      case H_ATOMIC_MAP: {
        uint32_t op = (uint32_t)imm;
        uint64_t r0 = r[0];
        uint64_t v = r[s];
        uint64_t old = 0;
        if (A.checked && h == H_ATOMIC_MAP) act = act && guard_ok(A, pc, a + (int64_t)aux, 1u << sc);
        if (act) {
          const uint64_t ad = a + (int64_t)aux;
          if (h == H_ATOMIC_STACK)
            old = atomic_stack(saddr(stk, (uint32_t)a + aux), v, op, sc, r0);
          else if (ad - A.acc_lo < A.acc_hi - A.acc_lo)
            acc_rmw(A, ad, v);  // the block's LDS mirror of a shared map
          else
            old = atomic_global(ad, v, op, sc, r0);
        }
        if (op == 0xf1) {
          res = old;
          wold = r0;
          nwd = 0;
        } else if (op & 1) {
          res = old;
          wold = v;
          nwd = s;
        }
        break;
      }
      case H_LDIMM: res = imm; nwd = d; npc = pc + 2; break;
      // helpers (dst field is 0, so a == r0)
      case H_LOOKUP_ARRAY: {
        const MapDev* m = (const MapDev*)imm;
        if (act) res = array_lookup(m, a8 & 1, r[2], stk);
        nwd = 0;
        break;
      }
      case H_LOOKUP_HASH: {
        const MapDev* m = (const MapDev*)imm;
        if (act) res = hash_lookup(m, a8 & 1, r[2], stk, A.epoch);
        nwd = 0;
        break;
      }
      case H_UPDATE_ARRAY: {
        const MapDev* m = (const MapDev*)imm;
        if (act) res = (uint64_t)array_update(m, a8 & 1, r[2], (a8 >> 1) & 1, r[3], r[4], stk);
        nwd = 0;
        break;
      }
      case H_UPDATE_HASH: {
        const MapDev* m = (const MapDev*)imm;
        if (act) res = (uint64_t)hash_update(m, a8 & 1, r[2], (a8 >> 1) & 1, r[3], r[4], stk, A.epoch);
        nwd = 0;
        break;
      }
      case H_DELETE_HASH: {
        const MapDev* m = (const MapDev*)imm;
        if (act) res = (uint64_t)hash_delete(m, a8 & 1, r[2], stk, A.epoch);
        nwd = 0;
        break;
      }
      case H_RET_EINVAL: res = (uint64_t)-E_INVAL; nwd = 0; break;
      case H_RINGBUF_OUTPUT: {
        const MapDev* m = (const MapDev*)imm;
        uint64_t rr = ring_output(m, a8 & 1, r[2], (uint32_t)aux, r[4], act, stk);
        if (act) res = rr;
        nwd = 0;
        break;
      }
      case H_EXIT: br = 2; break;
      default: br = 2; break;
    }
    wd = nwd;
    wres = res;
    if (div && !act) wres = wold;
    if (br == 2) {
      if (act) {
        rc = (uint32_t)a;
        alive = false;
      }
      if (!div || ballot(alive) == 0) {
        r[wd] = wres;
        break;
      }
    }
    if (!div) {
      if (br == 1) {
        uint64_t am = ballot(alive), tm = ballot(alive && tk);
        if (tm == 0) {
          pc = pc + 1;
        } else if (tm == am) {
          pc = (uint32_t)aux;
        } else {
          div = true;
          mypc = tk ? (uint32_t)aux : pc + 1;
          pc = (uint32_t)aux < pc + 1 ? (uint32_t)aux : pc + 1;
        }
      } else {
        pc = npc;
      }
    } else {
      // minimum-pc scheduling.  Lanes not active here wait at pcs above pc,
      // so when any active lane continues at pc + 1 (or at pc + 2 after an
      // lddw, whose second slot no lane can wait at) that is the new minimum;
      // a taken back-edge is below every waiting lane.  Only a forward jump
      // taken by every active lane, or an exit, needs a reduction.
      if (act) mypc = br == 1 ? (tk ? (uint32_t)aux : pc + 1) : npc;
      bool known = false;
      if (br == 1) {
        uint64_t tm = ballot(act && tk), fm = ballot(act && !tk);
        if (tm != 0 && (uint32_t)aux <= pc) {
          pc = (uint32_t)aux;
          known = true;
        } else if (fm != 0) {
          pc = pc + 1;
          known = true;
        }
      } else if (br == 0 && h != H_JA) {
        pc = npc;
        known = true;
      }
      if (!known) pc = wave_min_all(alive ? mypc : 0xffffffffu);
      if (ballot(alive && mypc != pc) == 0) div = false;
    }
  }
  return rc;
}

struct Interp {
  __device__ __forceinline__ uint32_t run(const RunArgs& A, bool live, uint64_t c0, uint64_t c1, uint64_t c2,
                                          const Ctx& g, const Stk stk, uint64_t& steps) {
    return vm_run(A, live, c0, c1, c2, g, stk, steps);
  }
};

// Event-parallel mode: lane = event.
extern "C" __global__ void __launch_bounds__(256) gx_k_event_parallel(RunArgs A) {
  const uint32_t wave = threadIdx.x >> 6;
  Stk stk{wave * 64u * A.stack_bytes, lane_id() * 8u, blockIdx.x * blockDim.x + threadIdx.x};
  uint64_t steps = 0;
  Interp I;
  event_tile(I, A, (uint64_t)blockIdx.x * blockDim.x + wave * 64u, stk, steps);
}

// Event-parallel mode with a shared map summed in LDS: each block mirrors
// the map's value area (starting at the operation's identity), its waves
// take tiles t, t + stride, ... of the run, and the block applies its sums
// to the map once at the end (consecutive threads, consecutive words: one
// coalesced device atomic per word it touched).  The grid is sized so that
// each block runs at least as many events as the mirror has words.
extern "C" __global__ void __launch_bounds__(1024) gx_k_event_parallel_acc(RunArgs A) {
  const uint32_t wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  Stk stk{wave * 64u * A.stack_bytes, lane_id() * 8u, blockIdx.x * blockDim.x + threadIdx.x};
  const uint32_t words = (uint32_t)((A.acc_hi - A.acc_lo) >> A.acc_sc);
  uint8_t* mirror = g_lds + A.acc_lds;
  if (A.acc_sc == 3)
    mirror_init<uint64_t>((uint64_t*)mirror, words, A.acc_op);
  else
    mirror_init<uint32_t>((uint32_t*)mirror, words, A.acc_op);
  __syncthreads();
  Interp I;
  event_loop(I, A, (uint64_t)blockIdx.x * nw + wave, (uint64_t)gridDim.x * nw, stk);
  __syncthreads();
  if (A.acc_sc == 3)
    mirror_flush<uint64_t>((const uint64_t*)mirror, words, A.acc_op, (uint8_t*)A.acc_lo);
  else
    mirror_flush<uint32_t>((const uint32_t*)mirror, words, A.acc_op, (uint8_t*)A.acc_lo);
}

// The instrumented vector add, interpreted: one 64-iteration tile per wave.
extern "C" __global__ void __launch_bounds__(256) gx_k_app_vadd(RunArgs A, AppArgs P) {
  const uint32_t wave = threadIdx.x >> 6;
  Stk stk{wave * 64u * A.stack_bytes, lane_id() * 8u, blockIdx.x * blockDim.x + threadIdx.x};
  uint64_t steps = 0, sink = 0;
  Interp I;
  app_vadd_tile<true>(I, A, P, (uint64_t)blockIdx.x * 4u + wave, stk, steps, sink);
  asm volatile("" ::"v"(sink));
}

// The same with a shared map summed in the block's LDS mirror (as
// gx_k_event_parallel_acc): waves loop over tiles grid-stride and the block
// applies its sums once at the end.
extern "C" __global__ void __launch_bounds__(1024) gx_k_app_vadd_acc(RunArgs A, AppArgs P) {
  const uint32_t wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  Stk stk{wave * 64u * A.stack_bytes, lane_id() * 8u, blockIdx.x * blockDim.x + threadIdx.x};
  const uint32_t words = (uint32_t)((A.acc_hi - A.acc_lo) >> A.acc_sc);
  uint8_t* mirror = g_lds + A.acc_lds;
  if (A.acc_sc == 3)
    mirror_init<uint64_t>((uint64_t*)mirror, words, A.acc_op);
  else
    mirror_init<uint32_t>((uint32_t*)mirror, words, A.acc_op);
  __syncthreads();
  Interp I;
  app_vadd_loop<true>(I, A, P, (uint64_t)blockIdx.x * nw + wave, (uint64_t)gridDim.x * nw, stk);
  __syncthreads();
  if (A.acc_sc == 3)
    mirror_flush<uint64_t>((const uint64_t*)mirror, words, A.acc_op, (uint8_t*)A.acc_lo);
  else
    mirror_flush<uint32_t>((const uint32_t*)mirror, words, A.acc_op, (uint8_t*)A.acc_lo);
}

// The vector add without a hook (grid-stride over tiles).
extern "C" __global__ void __launch_bounds__(256) gx_k_app_plain(AppArgs P) {
  const RunArgs A{};
  Interp I;
  const Stk stk{0, 0, 0};
  app_vadd_loop<false>(I, A, P, (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6), (uint64_t)gridDim.x * 4u, stk);
}

// The block scheduler's workers, interpreted: one one-wave block per worker.
extern "C" __global__ void __launch_bounds__(64) gx_k_sched(RunArgs A, SchedArgs S) {
  Stk stk{0, lane_id() * 8u, blockIdx.x * 64u + threadIdx.x};
  Interp I;
  sched_worker<true>(I, A, S, blockIdx.x, stk);
}

// Static assignment (no scheduling hook): each worker runs its own range.
extern "C" __global__ void __launch_bounds__(64) gx_k_sched_plain(SchedArgs S) {
  const RunArgs A{};
  Interp I;
  const Stk stk{0, 0, 0};
  sched_worker<false>(I, A, S, blockIdx.x, stk);
}

// Stream-sequential mode: ``lanes`` lanes of each one-wave block own queues.
extern "C" __global__ void __launch_bounds__(64) gx_k_stream_seq(RunArgs A, uint32_t lanes, uint32_t qstride) {
  Stk stk{0, lane_id() * 8u, blockIdx.x * blockDim.x + threadIdx.x};
  uint64_t steps = 0;
  Interp I;
  stream_wave(I, A, blockIdx.x * lanes, lanes, qstride, (uint32_t)A.n_events, stk, steps);
}

// ---------------------------------------------------------------------------
// Batched form: one persistent launch over work items of many runs.  Each
// item is (run, chunk): a 64-event tile of an event-parallel run, or a group
// of ``lanes`` queues of a stream-sequential run.  Waves claim items from a
// counter in the order the host sorted them (largest first).

extern "C" __global__ void __launch_bounds__(64) gx_k_batched(const BatchDev* B, const uint2* items, uint32_t n_items,
                                                              uint32_t* next) {
  Stk stk{0, lane_id() * 8u, blockIdx.x * blockDim.x + threadIdx.x};
  Interp I;
  batched_items(B, items, n_items, next, [&](const BatchDev& bd, uint32_t chunk) {
    uint64_t steps = 0;
    if (bd.mode == 0)
      event_tile(I, bd.A, (uint64_t)chunk * 64u, stk, steps);
    else
      stream_wave(I, bd.A, chunk * bd.lanes, bd.lanes, bd.qstride, bd.qend_last, stk, steps);
  });
}

extern "C" __global__ void gx_k_zero(uint32_t* p, uint32_t n) {
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// ---------------------------------------------------------------------------
// stable partition of event indices by queue = stream key & (L - 1)

__device__ __forceinline__ uint32_t stream_key_of(const uint8_t* events, uint32_t rs, uint32_t soff, uint64_t i) {
  return *(const uint32_t*)(events + i * rs + soff);
}

__device__ __forceinline__ void part_count(const PartJob& J, uint32_t t, uint32_t* counts) {
  uint32_t* cnt = (uint32_t*)g_lds;
  const uint32_t L = 1u << J.lbits, l = lane_id();
  for (uint32_t q = l; q < L; q += 64) cnt[q] = 0;
  __syncthreads();
  uint64_t b = (uint64_t)t * J.tile, e = b + J.tile < J.n_events ? b + J.tile : J.n_events;
  // four rounds of keys are loaded before their LDS counts are added
  for (uint64_t c = b; c < e; c += 256) {
    uint32_t k[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const uint64_t i = c + 64 * u + l;
      k[u] = i < e ? stream_key_of(J.events, J.record_size, J.stream_off, i) : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; u++)
      if (c + 64 * u + l < e) atomicAdd(&cnt[k[u] & (L - 1)], 1u);
  }
  __syncthreads();
  for (uint32_t q = l; q < L; q += 64) counts[J.cbase + (uint64_t)q * J.nt + t] = cnt[q];
}

__device__ __forceinline__ void part_scatter(const PartJob& J, uint32_t t, const uint32_t* offs, uint32_t* order,
                                             uint8_t* sorted) {
  uint32_t* base = (uint32_t*)g_lds;
  const uint32_t L = 1u << J.lbits, l = lane_id();
  for (uint32_t q = l; q < L; q += 64) base[q] = offs[J.cbase + (uint64_t)q * J.nt + t];
  __syncthreads();
  uint64_t b = (uint64_t)t * J.tile, e = b + J.tile < J.n_events ? b + J.tile : J.n_events;
  // the next round's keys are loaded while this round ranks and writes
  uint32_t nkey = b + l < e ? stream_key_of(J.events, J.record_size, J.stream_off, b + l) : 0;
  for (uint64_t c = b; c < e; c += 64) {
    uint64_t i = c + l;
    bool v = i < e;
    uint32_t key = v ? (nkey & (L - 1)) : 0;
    if (c + 64 + l < e) nkey = stream_key_of(J.events, J.record_size, J.stream_off, c + 64 + l);
    uint64_t peers = ballot(v);
    for (uint32_t bit = 0; bit < J.lbits; bit++) {
      uint64_t m = ballot(v && ((key >> bit) & 1));
      peers &= ((key >> bit) & 1) ? m : ~m;
    }
    uint32_t rank = rank_in(peers);
    uint32_t pos = 0;
    if (v) pos = base[key] + rank;
    // every lane has read its base before a group leader advances it: one
    // wave executes the LDS read and the LDS write in program order
    if (v) {
      order[pos] = (uint32_t)i;
      if (rank == 0) base[key] = pos + popc64(peers);
      // the record itself, so that each queue's records lie together
      // (null sorted: the consumer gathers the records through order[])
      if (sorted) {
        const uint64_t* src = (const uint64_t*)(J.events + i * J.record_size);
        uint64_t* dst = (uint64_t*)(sorted + (uint64_t)pos * kSortedStride);
        dst[0] = src[0];
        dst[1] = src[1];
        if (J.record_size > 16) dst[2] = src[2];
      }
    }
  }
}

// One wave per tile; ``tiles`` maps block -> (job, tile) for batched runs.
extern "C" __global__ void __launch_bounds__(64) gx_k_part_count(const PartJob* jobs, const uint2* tiles,
                                                                 uint32_t* counts) {
  const uint2 jt = tiles[blockIdx.x];
  const PartJob J = jobs[jt.x];
  part_count(J, jt.y, counts);
}

extern "C" __global__ void __launch_bounds__(64) gx_k_part_scatter(const PartJob* jobs, const uint2* tiles,
                                                                   const uint32_t* offs, uint32_t* order,
                                                                   uint8_t* sorted) {
  const uint2 jt = tiles[blockIdx.x];
  const PartJob J = jobs[jt.x];
  part_scatter(J, jt.y, offs, order, sorted);
}

// Single-run forms take the job by value.
extern "C" __global__ void __launch_bounds__(64) gx_k_part_count1(PartJob J, uint32_t* counts) {
  part_count(J, blockIdx.x, counts);
}

extern "C" __global__ void __launch_bounds__(64) gx_k_part_scatter1(PartJob J, const uint32_t* offs, uint32_t* order,
                                                                    uint8_t* sorted) {
  part_scatter(J, blockIdx.x, offs, order, sorted);
}

// exclusive scan of u32 data[0..n): block sums, then the sums, then add back
constexpr uint32_t kScanItems = 16;
constexpr uint32_t kScanBlock = 256 * kScanItems;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* tmp, uint32_t* total) {
  // 256 threads; tmp has 256 entries
  const uint32_t t = threadIdx.x;
  tmp[t] = v;
  __syncthreads();
  for (uint32_t off = 1; off < 256; off <<= 1) {
    uint32_t x = t >= off ? tmp[t - off] : 0;
    __syncthreads();
    tmp[t] += x;
    __syncthreads();
  }
  uint32_t incl = tmp[t];
  *total = tmp[255];
  __syncthreads();
  return incl - v;
}

extern "C" __global__ void __launch_bounds__(256) gx_k_scan_local(uint32_t* data, uint64_t n, uint32_t* sums) {
  __shared__ uint32_t tmp[256];
  uint64_t base = (uint64_t)blockIdx.x * kScanBlock + (uint64_t)threadIdx.x * kScanItems;
  uint32_t vals[kScanItems];
  uint32_t acc = 0;
#pragma unroll
  for (uint32_t k = 0; k < kScanItems; k++) {
    vals[k] = base + k < n ? data[base + k] : 0;
    acc += vals[k];
  }
  uint32_t total;
  uint32_t pre = block_exclusive_scan(acc, tmp, &total);
#pragma unroll
  for (uint32_t k = 0; k < kScanItems; k++) {
    if (base + k < n) data[base + k] = pre;
    pre += vals[k];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

extern "C" __global__ void __launch_bounds__(256) gx_k_scan_sums(uint32_t* sums, uint32_t nb) {
  __shared__ uint32_t tmp[256];
  uint32_t carry = 0;
  for (uint32_t c = 0; c < nb; c += 256) {
    uint32_t i = c + threadIdx.x;
    uint32_t v = i < nb ? sums[i] : 0;
    uint32_t total;
    uint32_t pre = block_exclusive_scan(v, tmp, &total);
    if (i < nb) sums[i] = pre + carry;
    carry += total;
    __syncthreads();
  }
}

extern "C" __global__ void __launch_bounds__(256) gx_k_scan_add(uint32_t* data, uint64_t n, const uint32_t* sums) {
  uint64_t base = (uint64_t)blockIdx.x * kScanBlock;
  uint32_t add = sums[blockIdx.x];
  for (uint32_t k = threadIdx.x; k < kScanBlock; k += 256)
    if (base + k < n) data[base + k] += add;
}

// ---------------------------------------------------------------------------
// control-plane map operations (one lane): op 0 lookup, 1 update, 2 delete
extern "C" __global__ void gx_k_map_op(const MapDev* m, int op, const uint8_t* key, const uint8_t* val,
                                       uint64_t flags, int64_t* ret, uint8_t* val_out, uint32_t epoch) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Stk stk{0, 0, 0xffffffffu};
  uint64_t kp = (uint64_t)key, vp = (uint64_t)val;
  int64_t r = -E_INVAL;
  if (m->type == MAP_ARRAY) {
    if (op == 0) {
      uint64_t p = array_lookup(m, PK_MAPVAL, kp, stk);
      if (p) {
        for (uint32_t i = 0; i < m->value_size; i++) val_out[i] = ((const uint8_t*)p)[i];
        r = 0;
      } else {
        r = -E_NOENT;
      }
    } else if (op == 1) {
      r = array_update(m, PK_MAPVAL, kp, PK_MAPVAL, vp, flags, stk);
    }
  } else if (m->type == MAP_HASH) {
    if (op == 0) {
      uint64_t p = hash_lookup(m, PK_MAPVAL, kp, stk, epoch);
      if (p) {
        for (uint32_t i = 0; i < m->value_size; i++) val_out[i] = ((const uint8_t*)p)[i];
        r = 0;
      } else {
        r = -E_NOENT;
      }
    } else if (op == 1) {
      r = hash_update(m, PK_MAPVAL, kp, PK_MAPVAL, vp, flags, stk, epoch);
    } else {
      r = hash_delete(m, PK_MAPVAL, kp, stk, epoch);
    }
  }
  *ret = r;
}

}  // namespace gx

// ---------------------------------------------------------------------------
// Workspace of the allocation-free run entry point (gx_run_batch_noalloc):
// one fixed array per device, held until the process ends.  Its device
// address is looked up once per device; host code uses that address only
// (the array's name is a host-side stand-in, not device memory).

namespace gx {
constexpr uint64_t kScratchBytes = 16ull << 20;
}

static __device__ __align__(256) uint8_t scratch[gx::kScratchBytes];

// ---------------------------------------------------------------------------
// host-side launchers

namespace gx {

// Device address of the current device's scratch array (device ``dev``),
// looked up on the first call for that device.  0 or the HIP error.
hipError_t scratch_region(int dev, uint8_t** ptr, uint64_t* bytes) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static uint8_t* addr[kMaxDevices] = {};
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = (uint8_t*)p;
  }
  *ptr = addr[dev];
  *bytes = kScratchBytes;
  return hipSuccess;
}

hipError_t vm_init() {
  hipError_t e = hipFuncSetAttribute((const void*)gx_k_event_parallel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     256 * kStackMax);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)gx_k_event_parallel_acc, hipFuncAttributeMaxDynamicSharedMemorySize,
                          kAccLdsMax);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)gx_k_stream_seq, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * kStackMax);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)gx_k_app_vadd, hipFuncAttributeMaxDynamicSharedMemorySize, 256 * kStackMax);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)gx_k_app_vadd_acc, hipFuncAttributeMaxDynamicSharedMemorySize, kAccLdsMax);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)gx_k_sched, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * kStackMax);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)gx_k_batched, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * kStackMax);
}

hipError_t launch_event_parallel(const RunArgs& A, hipStream_t s) {
  uint64_t blocks = (A.n_events + 255) / 256;
  hipLaunchKernelGGL(gx_k_event_parallel, dim3((uint32_t)blocks), dim3(256), 256 * A.stack_bytes, s, A);
  return hipGetLastError();
}

// The mirrored form: as many waves per block (up to 16) as the LDS holds
// next to the mirror, and blocks enough to fill the device but no more
// than one per ``words`` events.
hipError_t launch_event_parallel_acc(RunArgs A, uint32_t n_cu, hipStream_t s) {
  const uint64_t acc_bytes = A.acc_hi - A.acc_lo;
  uint32_t nw = 16;
  while (nw > 1 && (uint64_t)nw * 64 * A.stack_bytes + acc_bytes > kAccLdsMax) nw /= 2;
  A.acc_lds = nw * 64u * A.stack_bytes;
  const uint64_t words = acc_bytes >> A.acc_sc;
  const uint64_t tiles = (A.n_events + 63) / 64;
  const uint64_t per_words = A.n_events / words > n_cu ? A.n_events / words : n_cu;
  uint64_t nb = (tiles + nw - 1) / nw;
  if (nb > per_words) nb = per_words;
  if (nb == 0) nb = 1;
  hipLaunchKernelGGL(gx_k_event_parallel_acc, dim3((uint32_t)nb), dim3(64 * nw), A.acc_lds + acc_bytes, s, A);
  return hipGetLastError();
}

hipError_t launch_app_vadd(const RunArgs& A, const AppArgs& P, hipStream_t s) {
  const uint64_t blocks = (P.n + 255) / 256;
  hipLaunchKernelGGL(gx_k_app_vadd, dim3((uint32_t)blocks), dim3(256), 256 * A.stack_bytes, s, A, P);
  return hipGetLastError();
}

// The mirrored form's shape as launch_event_parallel_acc's, over n tiles.
hipError_t launch_app_vadd_acc(RunArgs A, const AppArgs& P, uint32_t n_cu, hipStream_t s) {
  const uint64_t acc_bytes = A.acc_hi - A.acc_lo;
  uint32_t nw = 16;
  while (nw > 1 && (uint64_t)nw * 64 * A.stack_bytes + acc_bytes > kAccLdsMax) nw /= 2;
  A.acc_lds = nw * 64u * A.stack_bytes;
  const uint64_t words = acc_bytes >> A.acc_sc;
  const uint64_t tiles = (P.n + 63) / 64;
  const uint64_t per_words = P.n / words > n_cu ? P.n / words : n_cu;
  uint64_t nb = (tiles + nw - 1) / nw;
  if (nb > per_words) nb = per_words;
  if (nb == 0) nb = 1;
  hipLaunchKernelGGL(gx_k_app_vadd_acc, dim3((uint32_t)nb), dim3(64 * nw), A.acc_lds + acc_bytes, s, A, P);
  return hipGetLastError();
}

hipError_t launch_app_plain(const AppArgs& P, uint32_t n_cu, hipStream_t s) {
  const uint64_t tiles = (P.n + 63) / 64;
  const uint64_t blocks = std::min<uint64_t>((tiles + 3) / 4, (uint64_t)n_cu * 8);
  hipLaunchKernelGGL(gx_k_app_plain, dim3((uint32_t)std::max<uint64_t>(blocks, 1)), dim3(256), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_sched(const RunArgs& A, const SchedArgs& S, hipStream_t s) {
  hipLaunchKernelGGL(gx_k_sched, dim3(S.workers), dim3(64), 64 * A.stack_bytes, s, A, S);
  return hipGetLastError();
}

hipError_t launch_sched_plain(const SchedArgs& S, hipStream_t s) {
  hipLaunchKernelGGL(gx_k_sched_plain, dim3(S.workers), dim3(64), 0, s, S);
  return hipGetLastError();
}

hipError_t launch_stream_seq(const RunArgs& A, uint32_t lanes, uint32_t qstride, hipStream_t s) {
  uint32_t blocks = (A.n_queues + lanes - 1) / lanes;
  hipLaunchKernelGGL(gx_k_stream_seq, dim3(blocks), dim3(64), 64 * A.stack_bytes, s, A, lanes, qstride);
  return hipGetLastError();
}

// Exclusive scan of u32 data[0..m) in place (sums: ceil(m / 4096) entries).
hipError_t launch_scan(uint32_t* data, uint64_t m, uint32_t* sums, hipStream_t s) {
  uint32_t nb = (uint32_t)((m + kScanBlock - 1) / kScanBlock);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(gx_k_scan_local, dim3(nb), dim3(256), 0, s, data, m, sums);
  hipLaunchKernelGGL(gx_k_scan_sums, dim3(1), dim3(256), 0, s, sums, nb);
  hipLaunchKernelGGL(gx_k_scan_add, dim3(nb), dim3(256), 0, s, data, m, (const uint32_t*)sums);
  return hipGetLastError();
}

// Stable partition of one run's event indices into 2^lbits queues.  counts
// must hold 2^lbits * nt entries, sums ceil(2^lbits * nt / 4096), order n.
hipError_t launch_partition(const RunArgs& A, uint32_t lbits, uint32_t tile, uint32_t nt, uint32_t* counts,
                            uint32_t* sums, uint32_t* order, uint8_t* sorted, hipStream_t s) {
  uint32_t L = 1u << lbits;
  PartJob J{A.events, A.n_events, A.record_size, A.stream_off, lbits, tile, nt, 0, 0};
  hipLaunchKernelGGL(gx_k_part_count1, dim3(nt), dim3(64), L * 4, s, J, counts);
  hipError_t e = launch_scan(counts, (uint64_t)L * nt, sums, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gx_k_part_scatter1, dim3(nt), dim3(64), L * 4, s, J, (const uint32_t*)counts, order, sorted);
  return hipGetLastError();
}

// Combined partition of several runs: jobs/tiles are device tables; counts
// of all runs are concatenated, so one scan yields positions in one global
// order array in which run j's events occupy a contiguous range.
hipError_t launch_partition_jobs(const PartJob* d_jobs, const uint2* d_tiles, uint32_t n_tiles, uint32_t max_lbits,
                                 uint64_t total_counts, uint32_t* counts, uint32_t* sums, uint32_t* order,
                                 uint8_t* sorted, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  uint32_t L = 1u << max_lbits;
  hipLaunchKernelGGL(gx_k_part_count, dim3(n_tiles), dim3(64), L * 4, s, d_jobs, d_tiles, counts);
  hipError_t e = launch_scan(counts, total_counts, sums, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gx_k_part_scatter, dim3(n_tiles), dim3(64), L * 4, s, d_jobs, d_tiles,
                     (const uint32_t*)counts, order, sorted);
  return hipGetLastError();
}

hipError_t launch_zero(uint32_t* p, uint32_t n, hipStream_t s) {
  hipLaunchKernelGGL(gx_k_zero, dim3(1), dim3(64), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_batched(const BatchDev* d_batches, const uint2* d_items, uint32_t n_items, uint32_t* d_next,
                          uint32_t waves, uint32_t stack_max, hipStream_t s) {
  hipLaunchKernelGGL(gx_k_zero, dim3(1), dim3(64), 0, s, d_next, 1u);
  hipLaunchKernelGGL(gx_k_batched, dim3(waves), dim3(64), 64 * stack_max, s, d_batches, d_items, n_items, d_next);
  return hipGetLastError();
}

hipError_t launch_map_op(const MapDev* m, int op, const uint8_t* key, const uint8_t* val, uint64_t flags,
                         int64_t* ret, uint8_t* val_out, uint32_t epoch, hipStream_t s) {
  hipLaunchKernelGGL(gx_k_map_op, dim3(1), dim3(64), 0, s, m, op, key, val, flags, ret, val_out, epoch);
  return hipGetLastError();
}

}  // namespace gx
