// ss_level_xch.hip -- instantiations of the register-resident Partial
// Partition Step in its write-minimal exchange form (only the misplaced
// pairs of each group are swapped and written).  A translation unit of its
// own, so that the exchange code's register allocation stays out of the
// stable kernels.
#include "ss_level_rs.h"

namespace ss {

template <typename T, int NT, int NV>
hipError_t launch_level_xch(bool first, uint32_t grid, const LevelArgs &a, hipStream_t st)
{
    return launch_level_rs_t<T, NT, NV, kFormExchange>(first, grid, a, st);
}

template <typename T, int NT, int NV>
const void *level_xch_fn(bool first)
{
    return level_rs_fn_t<T, NT, NV, kFormExchange>(first);
}

#define SS_INSTANTIATE_XCH(T, NT, NV)                                                              \
    template hipError_t launch_level_xch<T, NT, NV>(bool, uint32_t, const LevelArgs &, hipStream_t); \
    template const void *level_xch_fn<T, NT, NV>(bool);

SS_RS_VARIANTS(SS_INSTANTIATE_XCH, uint32_t)
SS_RS_VARIANTS(SS_INSTANTIATE_XCH, uint64_t)
SS_RS_VARIANTS(SS_INSTANTIATE_XCH, KV)

}  // namespace ss

namespace ss {

namespace {

// Sample size and skew threshold of the automatic choice.  A group of S
// slots has about q (1 - q) S misplaced pairs when a fraction q of the keys
// are predecessors, so near q = 0 or 1 only a few percent of the lines are
// written and the exchange form of the first level (with 32 KiB groups)
// wins; towards the middle the scattered swaps dirty nearly every line and
// the stable form with 128 KiB groups is faster.  Measured crossovers at
// 2^30 elements: q between 1/16 and 1/10 for 8-byte keys, above 1/10 for
// 16-byte records (fewer elements share a line), so the exchange is chosen
// when the sampled q is at most 1/den or at least 1 - 1/den.
// The sample is 64 runs of 64 consecutive keys, run c starting at c n / 64:
// 4096 keys from 64 pages, so one workgroup reads it with coalesced loads
// and few address translations (16384 keys at scattered positions took
// 40 us, nearly all of it translation misses).
constexpr uint32_t kSkewRuns = 64;
constexpr uint32_t kRunLen = 64;
constexpr uint32_t kSkewSamples = kSkewRuns * kRunLen;
constexpr int kPrepNT = 1024;
constexpr int kPrepPerThread = kSkewSamples / kPrepNT;

template <typename T>
__global__ void __launch_bounds__(kPrepNT) k_xch_prepare(const T *A, uint64_t n, uint64_t pivot, uint64_t *result,
                                                          uint32_t force)
{
    constexpr uint64_t den = sizeof(T) >= 16 ? 10 : 16;
    __shared__ uint32_t total;
    if (threadIdx.x == 0)
        total = 0;
    __syncthreads();
    if (!force) {
        // wave w reads runs w, w + 16, w + 32 and w + 48, one key per lane;
        // all of a thread's loads are issued before any is used
        const uint32_t lane = threadIdx.x % 64, wave = threadIdx.x / 64;
        T v[kPrepPerThread];
#pragma unroll
        for (int r = 0; r < kPrepPerThread; r++) {
            const uint64_t run = wave + (uint64_t)r * (kPrepNT / 64);
            const uint64_t pos = run * n / kSkewRuns + lane;
            v[r] = A[pos < n ? pos : n - 1];
        }
        uint32_t mine = 0;
#pragma unroll
        for (int r = 0; r < kPrepPerThread; r++)
            mine += key_of(v[r]) < pivot;
        atomicAdd(&total, mine);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint64_t c = total;
        const bool skewed = c * den <= kSkewSamples || c * den >= (den - 1) * kSkewSamples;
        result[kResultGate] = force || skewed ? 1ull : 0ull;
        result[kResultWritten] = 0ull;
        result[kResultWrittenFirst] = 0ull;
    }
}

}  // namespace

hipError_t launch_xch_prepare(int dtype, const char *base, uint64_t n, uint64_t pivot, uint64_t *result, bool force,
                              hipStream_t st)
{
    const uint32_t f = force ? 1u : 0u;
    switch (dtype) {
    case SS_U32:
        hipLaunchKernelGGL(k_xch_prepare<uint32_t>, dim3(1), dim3(kPrepNT), 0, st,
                           reinterpret_cast<const uint32_t *>(base), n, pivot, result, f);
        break;
    case SS_U64:
        hipLaunchKernelGGL(k_xch_prepare<uint64_t>, dim3(1), dim3(kPrepNT), 0, st,
                           reinterpret_cast<const uint64_t *>(base), n, pivot, result, f);
        break;
    default:
        hipLaunchKernelGGL(k_xch_prepare<KV>, dim3(1), dim3(kPrepNT), 0, st, reinterpret_cast<const KV *>(base), n,
                           pivot, result, f);
        break;
    }
    return hipGetLastError();
}

}  // namespace ss
