// Optional per-kernel timing with HIP events (off unless vx_profile_begin()
// was called).  Each recorded launch is bracketed by two events on the
// launching stream; vx_profile_end() waits for them and sums the durations
// and the algorithmic work per kernel name.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vx {

bool profiling();
// Returns a slot to close with prof_stop(), or -1 when profiling is off.
int prof_start(const char* name, double units, hipStream_t st);
void prof_stop(int slot, hipStream_t st);

}  // namespace vx
