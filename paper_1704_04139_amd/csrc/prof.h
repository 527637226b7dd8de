// prof.h — opt-in per-kernel timing with HIP events on the launch stream.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mbx {

enum ProfKernel { PK_NONE = 0, PK_RESIDUAL = 1, PK_MATVEC = 2, PK_SMOOTH0 = 3, PK_PRECOND = 4, PK_GRAM = 5 };

// True when launches of kernel class k are being timed.
bool prof_on(int k);
// True while any kernel class is being timed.
bool prof_active();
// Brackets one launch: records an event pair on stream s and the launch's
// algorithmic bytes.
void prof_begin(int k, hipStream_t s);
void prof_end(int k, hipStream_t s, double bytes);
// Closes a bracket around `launches` back-to-back launches of class k
// (their summed algorithmic bytes): the per-launch average then carries one
// event pair's overhead divided among them.
void prof_end_n(int k, hipStream_t s, double bytes, int launches);

}  // namespace mbx
