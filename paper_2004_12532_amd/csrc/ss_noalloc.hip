// ss_noalloc.hip -- ss_partition_noalloc: the single-array partition
// without any allocation, for callers that cannot allocate device memory
// (code under HIP graph capture, serving loops that forbid allocation).
//
// The per-call device state of a partition -- the (v_min, v_max) partials
// of every level, the level records and the result words -- lives in one
// file-scope device array per GPU instead of the hipMalloc'd per-stream
// workspace, and no host memory is mapped: the call is asynchronous and its
// split lands in the caller's device word.  The array's address is looked up
// once per device with hipGetSymbolAddress (the array's name in host code
// is not a device address).  Nothing in it has to start at zero: every
// level writes all the partials the next one reads, the first level's
// kernel clears the exchange form's counts, and the base case writes the
// result words.  Calls that overlap on one GPU share the array and race.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "ss.h"
#include "ss_common.h"
#include "ss_internal.h"

namespace ss {

namespace {

// Level slots of the array: the longest planned chain for n <= 2^40 elements
// is well below this (the plan stops once the expected region is a few
// thousand elements; each level after the first shrinks it about ninefold).
constexpr uint32_t kNoAllocLevels = 16;
constexpr size_t kNoAllocPartWords = (size_t)kNoAllocLevels * 2 * kMaxGrid;
constexpr size_t kNoAllocCtlWords = (size_t)kNoAllocLevels * kCtlWords;
constexpr size_t kNoAllocWords = kNoAllocPartWords + kNoAllocCtlWords + kResultWords;

__device__ __align__(256) uint64_t scratch[kNoAllocWords];  // 1 MiB + 1 KiB + 64 B per GPU

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint64_t *g_ptr[kMaxDevices];  // the array's device address on each GPU (null until looked up)

// The array's address on the current device, looked up on the device's
// first call.
int scratch_of(int dev, uint64_t **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return fail_msg(SS_EUNSUPPORTED, "device index beyond the no-allocation table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail_device(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_ptr[dev] = static_cast<uint64_t *>(ptr);
    }
    *out = g_ptr[dev];
    return SS_OK;
}

__global__ void k_zero_word(uint64_t *w) { *w = 0ull; }

}  // namespace

}  // namespace ss

using namespace ss;

extern "C" int ss_partition_noalloc(void *d_ptr, size_t n, int dtype, uint64_t pivot, const ss_params *p,
                                    void *stream, uint64_t *d_split)
{
    int rc = check_array(d_ptr, n, dtype);
    if (rc)
        return rc;
    if (!d_split || ((uintptr_t)d_split % 8))
        return fail_msg(SS_EINVAL, "d_split must be an 8-byte aligned device word");
    Resolved R;
    if ((rc = resolve_params(p, dtype, &R, SS_ENGINE_STAGED)))
        return rc;
    if (R.algo != SS_SMOOTHED && R.algo != SS_STRIDED)
        return fail_msg(SS_EINVAL, "ss_partition_noalloc runs Smoothed Striding or Strided");
    if (R.flags & (SS_FLAG_TIME | SS_FLAG_GRAPH))
        return fail_msg(SS_EINVAL, "ss_partition_noalloc takes no timing or graph flags");
    if (R.levels > kNoAllocLevels)
        return fail_msg(SS_EINVAL, "max_levels above the no-allocation limit of 16");
    if ((rc = check_lines(n, R)))
        return rc;
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {
        // the split of an empty array, written by a one-thread kernel (no
        // host buffer to keep alive, no memset node under graph capture)
        hipLaunchKernelGGL(k_zero_word, dim3(1), dim3(1), 0, st, d_split);
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? SS_OK : fail_device(e, "zero-word kernel launch");
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail_device(e, "hipGetDevice");
    uint64_t *base = nullptr;
    if ((rc = scratch_of(dev, &base)))
        return rc;
    Workspace ws;
    ws.part = base;
    ws.ctl = base + kNoAllocPartWords;
    ws.result = ws.ctl + kNoAllocCtlWords;
    ws.part_words = kNoAllocPartWords;
    ws.ctl_words = kNoAllocCtlWords;
    ws.bytes = kNoAllocWords * sizeof(uint64_t);
    ws.levels_cap = kNoAllocLevels;
    RunOut ro;
    std::memset(&ro, 0, sizeof(ro));
    return run_partition((char *)d_ptr, n, dtype, pivot, R, st, d_split, false, &ro, &ws);
}
