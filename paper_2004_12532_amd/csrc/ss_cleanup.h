// ss_cleanup.h -- serial partition of an unresolved range by one workgroup
// (the Serial Cleanup Step of the Strided Algorithm, Section 4).
//
// The workgroup runs a block version of the two-pointer partition: it keeps
// one block of B elements from the left end and one from the right end of
// the unresolved range in LDS, exchanges the k-th successor of the left block
// with the k-th predecessor of the right block for as many pairs as both
// have, writes back whichever block has become clean (only predecessors on
// the left, only successors on the right) and fetches the next block on that
// side.  When at most 2B elements remain they are partitioned in one pass.
#pragma once

#include "ss_common.h"
#include "ss_device.h"

namespace ss {

template <typename T, int NT, int BB>
struct CleanupSmem {
    static constexpr int B = BB / (int)sizeof(T);  // elements per block
    static constexpr int K2 = 2 * (B / NT);
    T buf[2 * B];
    uint16_t il[B], ir[B];
    uint32_t sh[K2 * (NT / 64) + 1];
};

// Partition A[lo, hi) by key < pivot; every thread of the workgroup calls it.
// Returns the split (absolute index) in every thread.
template <typename T, int NT, int BB>
__device__ uint64_t cleanup_region(T *const A, uint64_t pivot, uint64_t lo, uint64_t hi, CleanupSmem<T, NT, BB> &S)
{
    constexpr int B = CleanupSmem<T, NT, BB>::B;
    constexpr int K = B / NT;      // block elements per thread
    constexpr int K2 = 2 * K;      // final pass
    static_assert(K * NT == B && K >= 1, "block shape");
    const int tid = threadIdx.x;
    T *const lb = S.buf;
    T *const rb = S.buf + B;
    uint16_t *const il = S.il;
    uint16_t *const ir = S.ir;
    uint32_t *const sh = S.sh;
    T *const buf = S.buf;

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
    __syncthreads();  // the LDS buffer may be reused by the caller
    return L + tot;
}

}  // namespace ss
