// ss_pivot.h -- the quicksort's pivot rule (Section 5.2 applies the parallel
// partition at each level of a quicksort but leaves the choice of pivot
// open).  A segment's pivot is the lower median of 64 of its keys at equally
// spaced positions: one wavefront loads one key per lane and every lane
// counts the keys ranked before its own.  The pivot is always a key of the
// segment, so a segment with no key below it has that key as its minimum.
#pragma once

#include "ss_common.h"
#include "ss_device.h"

namespace ss {

// Called by all 64 lanes of a wavefront for the same segment A[0, l), l >= 1;
// every lane returns the pivot.
template <typename T>
__device__ __forceinline__ uint64_t sample_median64(const T *A, uint64_t l, int lane)
{
    const uint64_t x = key_of(A[(uint64_t)lane * l / 64]);
    uint32_t before = 0;  // keys ranked before lane's: smaller, or equal at a lower lane
#pragma unroll 8
    for (int j = 0; j < 64; j++) {
        const uint64_t y = __shfl(x, j, 64);
        before += (y < x) | ((y == x) & (j < lane));
    }
    const uint64_t at = __ballot(before == 31);  // exactly one lane holds rank 31
    return __shfl(x, __builtin_ctzll(at), 64);
}

}  // namespace ss
