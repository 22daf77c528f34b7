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

// HIP source of one program: its micro-ops written out as straight-line
// code with labels at jump targets, helpers called directly with the map
// descriptors as constants, and the event-loop kernel of its mode:
// gx_j_event_parallel (jit_waves() waves per block, grid-stride over
// 64-event tiles) or gx_j_stream_seq (one wave per block).  Stack frames live in a
// static LDS array; each wave carves ring records from its own chunk of
// reserved ring space.
// ``maps`` holds (descriptor device address, descriptor contents) of every
// map the program uses, in its map-table order; the generated code gets each
// map's shape as constants, so key sizes, slot masks and strides fold into
// the code.
// ``mem_map`` is the verifier's map of each map-value access (by slot):
// the event-parallel kernel sums the atomics of shared maps in LDS.
// *acc_words receives the LDS accumulator words a block flushes at its end
// (0: no accumulators), which the launch uses to size its grid.
// ``ld_map`` is the verifier's map of each lddw map reference.  Only the
// kernel of the program's execution mode is emitted.  The source holds the
// maps' shapes but none of their addresses (those come from RunArgs::maptab),
// so program instances with same-shaped maps compile to the same source.
std::string jit_source(const std::vector<Uop>& U, uint32_t stack_bytes,
                       const std::vector<std::pair<uint64_t, MapDev>>& maps, const std::vector<int>& mem_map,
                       const std::vector<int>& ld_map, bool event_parallel, uint64_t* acc_words = nullptr);

// Compile a generated source for gfx950.  Returns 0 and the code object, or
// -EIO with the compiler log.
int jit_compile(const std::string& src, std::vector<char>* code, std::string* log);

// Text of the device headers the generated source includes (embedded into
// the library when it is built).
extern const char kJitHdrDev[];
extern const char kJitHdrInternal[];

}  // namespace gx
