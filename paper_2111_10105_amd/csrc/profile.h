// HIP-event timing of one kernel family at a time (measurement support for
// the benchmark).  Process-wide, meant for one thread; when no family is
// selected begin/end cost one comparison.
#pragma once

#include <hip/hip_runtime.h>

namespace dmc {
namespace prof {

void begin(hipStream_t s, int kernel);
void end(hipStream_t s, int kernel);
// suspend event recording (while a stream is captured into a graph)
void pause(bool on);

}  // namespace prof
}  // namespace dmc
