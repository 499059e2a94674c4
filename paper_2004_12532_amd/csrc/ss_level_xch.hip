// ss_level_xch.hip -- instantiations of the register-resident Partial
// Partition Step in its write-minimal exchange form (only the misplaced
// pairs of each group are swapped and written).  A translation unit of its
// own, so that the exchange code's register allocation stays out of the
// stable kernels.
#include "ss_level_rs.h"

namespace ss {

#define SS_INSTANTIATE_FORM(T, NT, NV, FORM)                                                                  \
    template hipError_t launch_level_rs_t<T, NT, NV, FORM>(bool, uint32_t, const LevelArgs &, hipStream_t); \
    template const void *level_rs_fn_t<T, NT, NV, FORM>(bool);                                              \
    template size_t level_form_lds<T, NT, NV, FORM>();
#define SS_INSTANTIATE_XCH(T, NT, NV) SS_INSTANTIATE_FORM(T, NT, NV, kFormExchange)

SS_RS_VARIANTS(SS_INSTANTIATE_XCH, uint32_t)
SS_RS_VARIANTS(SS_INSTANTIATE_XCH, uint64_t)
SS_RS_VARIANTS(SS_INSTANTIATE_XCH, KV)
SS_INSTANTIATE_XCH(uint64_t, 512, 4)
SS_INSTANTIATE_XCH(KV, 512, 4)

}  // namespace ss

namespace ss {

namespace {

// The sample of the automatic choice (kGateRuns runs of kGateRunLen keys,
// ss_common.h): a skewed pivot leaves only a few percent of the lines to
// write, and the exchange form of the first level (with 32 KiB groups) wins;
// towards the middle the scattered swaps dirty nearly every line and the
// stable form with 128 KiB groups is faster.  Runs cost few address
// translations: 16384 keys at scattered positions took 40 us, nearly all of
// it translation misses.  This kernel serves calls that force the exchange
// form (it only clears the counts then); the automatic choice samples
// inside the stable first-level kernel.
constexpr int kPrepNT = 1024;
constexpr int kPrepPerThread = kGateSamples / kPrepNT;

template <typename T>
__global__ void __launch_bounds__(kPrepNT) k_xch_prepare(const T *A, uint64_t n, uint64_t pivot, uint64_t *result,
                                                          uint32_t force)
{
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
            const uint64_t pos = run * n / kGateRuns + lane;
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
        const bool skewed = gate_skewed(total, (int)sizeof(T));
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
