// Device side of the persistent kernels' work queues (the layout of tiles,
// runs, bounds and counters is described with MF_QUEUES in gf_types.h).
// Included by every kernel file whose kernels claim tiles from the queues.
#pragma once

#include <hip/hip_runtime.h>

#include "gf_types.h"

namespace gfnc {
namespace {

// Next run for a workgroup or wave (one lane calls), or -1 when every queue
// is empty: the home queue of this workgroup's XCD first, then the others in
// turn; q counts the queues found empty so far.
__device__ __forceinline__ int queue_take_run(unsigned *counters, const unsigned *__restrict__ bounds, int &q)
{
    const int home = (int)(blockIdx.x % MF_QUEUES);
    while (q < MF_QUEUES) {
        const int qi = (home + q) % MF_QUEUES;
        const unsigned lo = bounds[qi], hi = bounds[qi + 1];
        if (lo < hi) {
            const unsigned t = atomicAdd(&counters[MF_CTR_STRIDE * qi], 1u);
            if (t < hi - lo)
                return (int)(lo + t);
        }
        q++;
    }
    return -1;
}

// Tile cursor of a claimant: the rest of its current run, then the next run.
// runs == nullptr means every run is one tile (run r is tile r).
struct QueueCursor {
    int q = 0;
    unsigned next = 0, end = 0;
};

__device__ __forceinline__ int queue_next_tile(unsigned *counters, const unsigned *__restrict__ runs,
                                               const unsigned *__restrict__ bounds, QueueCursor &c)
{
    while (c.next == c.end) {
        const int r = queue_take_run(counters, bounds, c.q);
        if (r < 0)
            return -1;
        c.next = runs ? runs[r] : (unsigned)r;
        c.end = runs ? runs[r + 1] : (unsigned)r + 1;
    }
    return (int)c.next++;
}

// The last of `claimants` to finish sets every counter back to zero.
__device__ __forceinline__ void queue_retire(unsigned *counters, unsigned claimants)
{
    __threadfence();
    if (atomicAdd(&counters[MF_CTR_RETIRED], 1u) == claimants - 1) {
        for (int i = 0; i < MF_QUEUES; i++)
            atomicExch(&counters[MF_CTR_STRIDE * i], 0u);
        atomicExch(&counters[MF_CTR_RETIRED], 0u);
    }
}

}  // namespace
}  // namespace gfnc
