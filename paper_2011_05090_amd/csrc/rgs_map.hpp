// Workgroup -> (item, local block) for the implicit launch maps of batched
// calls (BlockMap): a two-level search by the first wave over the listed
// items' first blocks (64 candidates per level, so two dependent loads for up
// to 4096 items), shared with the workgroup through LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rgs_types.hpp"

namespace rgs {

__device__ __forceinline__ int64_t map_first(const BlockMap& m, int p) {
    return (m.base ? m.base[p] : 0) + (int64_t)m.uniform * p;
}

// Every thread of the workgroup must call it (it contains a barrier).
__device__ __forceinline__ int2 locate(const BlockMap& m, int64_t id) {
    __shared__ int2 found;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        int lo = 0, hi = m.count;   // first(lo) <= id < first(hi)
        while (hi - lo > 1) {
            const int step = (hi - lo + 63) / 64;
            const int p = lo + lane * step;
            const bool ok = p < hi && map_first(m, p) <= id;
            const uint64_t bal = __ballot(ok);
            const int last = 63 - __clzll((long long)bal);
            lo += last * step;
            hi = min(hi, lo + step);
        }
        if (lane == 0) found = make_int2(m.ids ? m.ids[lo] : lo, (int)(id - map_first(m, lo)));
    }
    __syncthreads();
    return found;
}

}  // namespace rgs
