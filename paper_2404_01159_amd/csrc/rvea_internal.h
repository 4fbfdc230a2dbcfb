// rvea_internal.h -- host-side launchers of the library's kernels (one per
// kernel group; each enqueues on the given stream and returns the launch
// error, if any).
#pragma once

#include <hip/hip_runtime.h>

#include "rvea_dev.h"

namespace rvea {

int pick_segment(int d);
int assoc_rows_per_block();

hipError_t launch_lattice(const RunView &R, hipStream_t s, int H);
hipError_t launch_vec_aux(const RunView &R, hipStream_t s);
hipError_t launch_gamma(const RunView &R, hipStream_t s, int force);
hipError_t launch_init(const RunView &R, hipStream_t s);
hipError_t launch_prepare(const RunView &R, hipStream_t s);
hipError_t launch_offspring(const RunView &R, hipStream_t s);
hipError_t launch_select_front(const RunView &R, hipStream_t s);
hipError_t launch_assoc(const RunView &R, hipStream_t s);
hipError_t launch_rerank(const RunView &R, hipStream_t s);
hipError_t launch_select_back(const RunView &R, hipStream_t s);
hipError_t launch_adapt(const RunView &R, hipStream_t s);

}  // namespace rvea
