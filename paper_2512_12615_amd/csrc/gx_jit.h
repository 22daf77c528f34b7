// Compilation of verified programs to native gfx950 code (host side).
#pragma once
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "gx_internal.h"

namespace gx {

// HIP source of one program: its micro-ops written out as straight-line
// code with labels at jump targets, helpers called directly with the map
// descriptors as constants, and the two event-loop kernels
// (gx_j_event_parallel, gx_j_stream_seq; 64 threads per block, stack frames
// in a static LDS array).
// ``maps`` holds (descriptor device address, descriptor contents) of every
// map the program uses; the generated code gets each descriptor as a
// constant, so key sizes, slot masks and addresses fold into the code.
std::string jit_source(const std::vector<Uop>& U, uint32_t stack_bytes,
                       const std::vector<std::pair<uint64_t, MapDev>>& maps);

// Compile a generated source for gfx950.  Returns 0 and the code object, or
// -EIO with the compiler log.
int jit_compile(const std::string& src, std::vector<char>* code, std::string* log);

// Text of the device headers the generated source includes (embedded into
// the library when it is built).
extern const char kJitHdrDev[];
extern const char kJitHdrInternal[];

}  // namespace gx
