// Compilation of verified programs to native gfx950 code (host side).
#pragma once
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "gx_internal.h"

namespace gx {

// Waves per block of a compiled program's event-parallel kernel (each block
// loops over 64-event tiles, grid-stride): as many as 64 KiB of LDS stack
// frames allow, at most kJitMaxWaves.  More waves per block share one LDS
// accumulator, so each block flushes it over more events.
constexpr uint32_t kJitMaxWaves = 16;
uint32_t jit_waves(uint32_t stack_bytes, bool event_parallel);

// A verified program as the code generator sees it: its micro-ops, frame
// size, maps as (descriptor device address, descriptor contents) in its
// map-table order, the verifier's map of each map-value access and of each
// lddw map reference (by slot), and its execution mode.
struct JitProg {
  const std::vector<Uop>* U;
  uint32_t stack_bytes;
  const std::vector<std::pair<uint64_t, MapDev>>* maps;
  const std::vector<int>* mem_map;
  const std::vector<int>* ld_map;
  bool event_parallel;
  bool leader = false;  // warp-leader hook: one lane runs each tile, on wave-uniform values
  bool simt = false;    // SIMT hook: shared-map updates are wave-uniform, combined per wave
  // the kernel the source holds besides the program: 0, the run kernels of
  // its mode; 1, the instrumented vector add gx_j_app_vadd (event-parallel
  // memory hooks); 2, the block scheduler's workers gx_j_sched (HOOK_SCHED)
  int kernel = 0;
  uint64_t max_insns = 0;  // the verifier's bound on instructions per invocation (0: unknown)
};

// HIP source of one program: its micro-ops written out as straight-line
// code with labels at jump targets, helpers called directly with each map's
// shape as constants (sizes, masks and strides fold into the code), and the
// event-loop kernel of its mode: gx_j_event_parallel (jit_waves() waves per
// block, grid-stride over 64-event tiles; shared-map atomics summed in LDS)
// or gx_j_stream_seq (one wave per block).  Stack frames live in a static
// LDS array; each wave carves ring records from its own chunk of reserved
// ring space.  The source holds no map address (those come from
// RunArgs::maptab), so instances with same-shaped maps share it.
// With JitProg::kernel 1 the source holds, in place of the run kernels,
// gx_j_app_vadd(RunArgs, AppArgs) with the event-parallel kernel's block
// shape and LDS accumulators (and gx_j_reduce when the program spills);
// with kernel 2, gx_j_sched(RunArgs, SchedArgs): one worker (one wave) per
// block, shared-map updates straight to the map.
// *info receives what the launch needs to know: the LDS accumulator words a
// block flushes at its end (0: none), which sizes the grid; and, when the
// program has LDS caches, the spill bytes per block and the blocks of the
// reduce kernel gx_j_reduce (see JitInfo).
struct JitInfo {
  uint64_t acc_words = 0;
  // Event-parallel programs with LDS caches: at its end each block writes
  // its caches to a spill area (spill_block_bytes per block of the launch,
  // RunArgs::spill) instead of applying every slot to the map with a device
  // atomic; gx_j_reduce(A, blocks) then sums each cache set over all blocks
  // in LDS and applies one atomic per word (reduce_blocks blocks of 256
  // threads).  0: no spill (caches flush directly).
  uint64_t spill_block_bytes = 0;
  uint32_t reduce_blocks = 0;
};
std::string jit_source(const JitProg& p, JitInfo* info = nullptr);

// HIP source of a program set: every program in its own namespace and one
// persistent kernel gx_j_set over the batched form's work items, which picks
// the program by BatchDev::slot (one wave per block; no LDS accumulators).
std::string jit_set_source(const std::vector<JitProg>& progs);

// Compile a generated source for gfx950.  Returns 0 and the code object, or
// -EIO with the compiler log.
int jit_compile(const std::string& src, std::vector<char>* code, std::string* log);

// Text of the device headers the generated source includes (embedded into
// the library when it is built).
extern const char kJitHdrDev[];
extern const char kJitHdrInternal[];

}  // namespace gx
