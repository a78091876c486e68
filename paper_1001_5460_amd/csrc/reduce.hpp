// Deterministic two-stage FP64 grid reduction.
//
// Every workgroup reduces its partial (fixed shuffle tree, then fixed order
// across waves), stores it to partials[blockIdx.x] and counts itself in with a
// device-scope atomic.  The last workgroup to arrive sums the partials in
// index order (thread i takes i, i+256, ...; then the fixed block tree), so
// the total does not depend on which workgroup finishes last.  It then resets
// the counter for the next launch.
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace cta {

__device__ __forceinline__ double load_relaxed(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// All threads of every workgroup call this once per launch.  Returns true on
// all threads of the last workgroup, with the grid total in `total`.
__device__ __forceinline__ bool grid_reduce(double v, double* partials, unsigned* counter,
                                            double* red, double& total) {
    __shared__ int s_last;
    const double s = block_sum(v, red);
    if (threadIdx.x == 0) {
        __hip_atomic_store(&partials[blockIdx.x], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const unsigned prev = atomicAdd(counter, 1u);
        s_last = (prev == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!s_last) return false;
    __threadfence();
    double acc = 0.0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += CTA_WG) acc += load_relaxed(&partials[i]);
    total = block_sum(acc, red);
    if (threadIdx.x == 0) *counter = 0u;
    return true;
}

}  // namespace cta
