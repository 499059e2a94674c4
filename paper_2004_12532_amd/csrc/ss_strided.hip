// ss_strided.hip -- the Serial Cleanup Step of the Strided Algorithm
// (Section 4, "The Strided Algorithm"): after the Partial Partition Step with
// every chunk offset 0, the subarray between the smallest and the largest
// splitting position is partitioned serially -- here by a single workgroup,
// the GPU's unit of serial execution.
//
// The workgroup runs a block version of the two-pointer partition: it keeps
// one block of B elements from the left end and one from the right end of
// the unresolved range in LDS, exchanges the k-th successor of the left block
// with the k-th predecessor of the right block for as many pairs as both
// have, writes back whichever block has become clean (only predecessors on
// the left, only successors on the right) and fetches the next block on that
// side.  When at most 2B elements remain they are partitioned in one pass.
#include "ss_common.h"
#include "ss_device.h"
#include "ss_internal.h"

namespace ss {

template <typename T, int NT, int BB>
__global__ void __launch_bounds__(NT) k_cleanup(char *base, uint64_t pivot, const uint64_t *prev,
                                                 uint32_t count, uint64_t *result, uint64_t *d_split,
                                                 const uint64_t *ctl, uint64_t *host)
{
    constexpr int W = sizeof(T);
    constexpr int B = BB / W;      // elements per block
    constexpr int K = B / NT;      // block elements per thread
    constexpr int K2 = 2 * K;      // final pass
    constexpr int NW = NT / 64;
    static_assert(K * NT == B && K >= 1, "block shape");

    __shared__ T buf[2 * B];
    __shared__ uint16_t il[B], ir[B];
    __shared__ uint32_t sh[K2 * NW + 1];
    __shared__ uint64_t red[2 * NW];

    const int tid = threadIdx.x;
    T *const A = reinterpret_cast<T *>(base);
    T *const lb = buf;
    T *const rb = buf + B;

    uint64_t lo, hi;
    reduce_partials<NT>(prev, count, red, lo, hi);
    if (tid == 0) {
        result[2] = lo;
        result[3] = hi;
    }
    uint64_t L = lo, R = hi > lo ? hi : lo;
    bool lload = false, rload = false;
    uint32_t nL = 0, nR = 0;

    while (R - L > 2ull * B) {
        if (!lload) {
            bool f[K];
            uint32_t rk[K], tot;
#pragma unroll
            for (int r = 0; r < K; r++) {
                const T x = A[L + r * NT + tid];
                lb[r * NT + tid] = x;
                f[r] = !(key_of(x) < pivot);
            }
            block_rank<NT, K>(f, rk, tot, sh);
            nL = tot;
            lload = true;
        }
        if (!rload) {
            bool f[K];
            uint32_t rk[K], tot;
#pragma unroll
            for (int r = 0; r < K; r++) {
                const T x = A[R - B + r * NT + tid];
                rb[r * NT + tid] = x;
                f[r] = key_of(x) < pivot;
            }
            block_rank<NT, K>(f, rk, tot, sh);
            nR = tot;
            rload = true;
        }
        const uint32_t m = nL < nR ? nL : nR;
        if (m) {
            bool f[K];
            uint32_t rk[K], tot;
#pragma unroll
            for (int r = 0; r < K; r++)
                f[r] = !(key_of(lb[r * NT + tid]) < pivot);
            block_rank<NT, K>(f, rk, tot, sh);
#pragma unroll
            for (int r = 0; r < K; r++)
                if (f[r] && rk[r] < m)
                    il[rk[r]] = (uint16_t)(r * NT + tid);
#pragma unroll
            for (int r = 0; r < K; r++)
                f[r] = key_of(rb[r * NT + tid]) < pivot;
            block_rank<NT, K>(f, rk, tot, sh);
#pragma unroll
            for (int r = 0; r < K; r++)
                if (f[r] && rk[r] < m)
                    ir[rk[r]] = (uint16_t)(r * NT + tid);
            __syncthreads();
            for (uint32_t k = tid; k < m; k += NT) {
                const T x = lb[il[k]];
                lb[il[k]] = rb[ir[k]];
                rb[ir[k]] = x;
            }
            __syncthreads();
        }
        nL -= m;
        nR -= m;
        if (nL == 0) {
#pragma unroll
            for (int r = 0; r < K; r++)
                A[L + r * NT + tid] = lb[r * NT + tid];
            L += B;
            lload = false;
        }
        if (nR == 0) {
#pragma unroll
            for (int r = 0; r < K; r++)
                A[R - B + r * NT + tid] = rb[r * NT + tid];
            R -= B;
            rload = false;
        }
        __syncthreads();
    }
    if (lload) {
#pragma unroll
        for (int r = 0; r < K; r++)
            A[L + r * NT + tid] = lb[r * NT + tid];
    }
    if (rload) {
#pragma unroll
        for (int r = 0; r < K; r++)
            A[R - B + r * NT + tid] = rb[r * NT + tid];
    }
    __syncthreads();

    // Final pass over [L, R), at most 2B elements: stable partition through LDS.
    const uint32_t n = (uint32_t)(R - L);
    T x[K2];
    bool f[K2];
    uint32_t rk[K2], tot;
#pragma unroll
    for (int r = 0; r < K2; r++) {
        const uint32_t k = r * NT + tid;
        f[r] = false;
        if (k < n) {
            x[r] = A[L + k];
            f[r] = key_of(x[r]) < pivot;
        }
    }
    block_rank<NT, K2>(f, rk, tot, sh);
#pragma unroll
    for (int r = 0; r < K2; r++) {
        const uint32_t k = r * NT + tid;
        if (k < n)
            buf[f[r] ? rk[r] : tot + k - rk[r]] = x[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < K2; r++) {
        const uint32_t k = r * NT + tid;
        if (k < n)
            A[L + k] = buf[k];
    }
    if (tid == 0) {
        result[0] = 1;
        result[1] = L + tot;
        if (d_split)
            *d_split = L + tot;
        if (host) {
            host[0] = 1;
            host[1] = L + tot;
            host[2] = lo;
            host[3] = hi;
        }
    }
    if (host && tid < kCtlWords)
        host[kResultWordsDev + tid] = ctl[tid];
}

hipError_t launch_cleanup(int dtype, char *base, uint64_t pivot, const uint64_t *prev, uint32_t count,
                          uint64_t *result, uint64_t *d_split, const uint64_t *ctl, uint64_t *host, hipStream_t st)
{
    constexpr int NT = 1024, BB = 16384;
    switch (dtype) {
    case SS_U32:
        hipLaunchKernelGGL((k_cleanup<uint32_t, NT, BB>), dim3(1), dim3(NT), 0, st, base, pivot, prev, count,
                           result, d_split, ctl, host);
        break;
    case SS_U64:
        hipLaunchKernelGGL((k_cleanup<uint64_t, NT, BB>), dim3(1), dim3(NT), 0, st, base, pivot, prev, count,
                           result, d_split, ctl, host);
        break;
    default:
        hipLaunchKernelGGL((k_cleanup<KV, NT, BB>), dim3(1), dim3(NT), 0, st, base, pivot, prev, count, result,
                           d_split, ctl, host);
        break;
    }
    return hipGetLastError();
}

}  // namespace ss
