// Deterministic two-stage FP64 reductions without atomics or device-scope
// fences: every workgroup stores its partial (fixed shuffle tree, fixed order
// across waves) to partials[blockIdx.x]; a one-workgroup finalize kernel
// launched next on the same stream sums the partials in index order and
// applies the CG scalar update.  (A device-scope fence per workgroup would
// force the XCD's L2 to write back, which costs far more than one extra
// launch.)
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace cta {

// All threads of the workgroup call this once; thread 0 stores the partial.
__device__ __forceinline__ void block_partial(double v, double* partials, double* red) {
    const double s = block_sum(v, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

}  // namespace cta
