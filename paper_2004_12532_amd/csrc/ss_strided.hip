// ss_strided.hip -- the Serial Cleanup Step of the Strided Algorithm
// (Section 4, "The Strided Algorithm"): after the Partial Partition Step with
// every chunk offset 0, the subarray between the smallest and the largest
// splitting position is partitioned serially -- here by a single workgroup,
// the GPU's unit of serial execution (the block two-pointer exchange of
// ss_cleanup.h).
#include "ss_cleanup.h"
#include "ss_common.h"
#include "ss_device.h"
#include "ss_internal.h"

namespace ss {

template <typename T, int NT, int BB>
__global__ void __launch_bounds__(NT) k_cleanup(char *base, uint64_t pivot, const uint64_t *prev,
                                                 uint32_t count, uint64_t *result, uint64_t *d_split,
                                                 const uint64_t *ctl, uint32_t nctl, uint64_t *host)
{
    constexpr int NW = NT / 64;
    __shared__ CleanupSmem<T, NT, BB> S;
    __shared__ uint64_t red[2 * NW];

    const int tid = threadIdx.x;
    uint64_t lo, hi;
    reduce_partials<NT>(prev, count, red, lo, hi);
    if (tid == 0) {
        result[2] = lo;
        result[3] = hi;
    }
    const uint64_t split = cleanup_region<T, NT, BB>(reinterpret_cast<T *>(base), pivot, lo, hi, S);
    if (tid == 0) {
        result[0] = 1;
        result[1] = split;
        if (d_split)
            *d_split = split;
        if (host) {
            host[0] = 1;
            host[1] = split;
            host[2] = lo;
            host[3] = hi;
        }
    }
    if (host)
        for (uint32_t k = tid; k < nctl * kCtlWords; k += NT)
            host[kResultWordsDev + k] = ctl[k];
    if (host && tid >= 4 && tid < kResultWordsDev)
        host[tid] = result[tid];
}

constexpr int kCleanupNT = 1024, kCleanupBB = 32768;  // 32 KiB blocks: twice the bytes per serial step of 16 KiB

uint64_t cleanup_pass_elems(int w) { return 2ull * kCleanupBB / (uint64_t)w; }

hipError_t launch_cleanup(int dtype, char *base, uint64_t pivot, const uint64_t *prev, uint32_t count,
                          uint64_t *result, uint64_t *d_split, const uint64_t *ctl, uint32_t nctl, uint64_t *host,
                          hipStream_t st)
{
    constexpr int NT = kCleanupNT, BB = kCleanupBB;
    switch (dtype) {
    case SS_U32:
        hipLaunchKernelGGL((k_cleanup<uint32_t, NT, BB>), dim3(1), dim3(NT), 0, st, base, pivot, prev, count,
                           result, d_split, ctl, nctl, host);
        break;
    case SS_U64:
        hipLaunchKernelGGL((k_cleanup<uint64_t, NT, BB>), dim3(1), dim3(NT), 0, st, base, pivot, prev, count,
                           result, d_split, ctl, nctl, host);
        break;
    default:
        hipLaunchKernelGGL((k_cleanup<KV, NT, BB>), dim3(1), dim3(NT), 0, st, base, pivot, prev, count, result,
                           d_split, ctl, nctl, host);
        break;
    }
    return hipGetLastError();
}

}  // namespace ss
