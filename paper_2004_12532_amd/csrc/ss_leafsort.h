// ss_leafsort.h -- workgroup-local sort of a short segment in LDS (the
// quicksort's leaves, Section 5.2: a small subproblem is finished without
// the parallel partition).  Least-significant-digit radix sort with 9- or
// 10-bit digits over the bits in which the segment's keys differ; KV16
// records move with their key.  Within a pass, each wavefront ranks 64 elements at a time:
// eight ballots give each lane the mask of lanes holding the same digit, the
// lowest lane of that mask advances the wavefront's counter for the digit,
// and a scan over (digit, wavefront) turns the counters into destinations.
// The sort is stable and needs no atomics.
#pragma once

#include "ss_common.h"
#include "ss_device.h"

namespace ss {

template <typename T>
__device__ __forceinline__ uint64_t qkey(const T &x)
{
    return key_of(x);
}

// One workgroup (1024 threads) sorts A[0, n), n <= CAP, by key.  Digits are
// DBITS wide: 10 bits when the keys fit a 64 KiB tile (the counters of 16
// wavefronts x 1024 digits then fit beside it in LDS), else 9.
template <typename T, int CAP, int KEYBITS>
__device__ void qleaf_sort(T *A, uint32_t n)
{
    constexpr int NT = 1024, NW = NT / 64;
    constexpr int E = CAP / NT;  // elements per thread
    constexpr int DBITS = (int)sizeof(T) * CAP <= 65536 ? 10 : 9;
    constexpr int ND = 1 << DBITS;
    static_assert(ND <= NT && 64 * E < 65536, "digit counters: one digit per thread, 16-bit counts");
    __shared__ T buf[CAP];
    __shared__ uint16_t cnt[NW][ND];  // per wavefront and digit; then destinations
    __shared__ uint32_t wsum[NW];
    __shared__ uint64_t red[2 * NW];

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const uint64_t lt = (1ull << lane) - 1;

    // Striped arrangement: element r of thread (wid, lane) is at
    // index wid * 64 * E + r * 64 + lane, so element order is (wave, round, lane).
    T x[E];
    bool valid[E];
    uint64_t kmin = ~0ull, kmax = 0;
    for (int r = 0; r < E; r++) {
        const uint32_t idx = wid * 64 * E + r * 64 + lane;
        valid[r] = idx < n;
        if (valid[r]) {
            x[r] = A[idx];
            const uint64_t k = qkey(x[r]);
            kmin = k < kmin ? k : kmin;
            kmax = k > kmax ? k : kmax;
        }
    }
    // Only the bits in which the leaf's keys differ need sorting: above the
    // highest bit where the smallest and the largest key differ, every key
    // has the same bits.
    kmin = wave_min(kmin);
    kmax = wave_max(kmax);
    if (lane == 0) {
        red[wid] = kmin;
        red[NW + wid] = kmax;
    }
    __syncthreads();
    kmin = red[0];
    kmax = red[NW];
    for (int w = 1; w < NW; w++) {
        kmin = red[w] < kmin ? red[w] : kmin;
        kmax = red[NW + w] > kmax ? red[NW + w] : kmax;
    }
    const uint64_t diff = kmin ^ kmax;
    const uint32_t nbits = diff ? 64u - (uint32_t)__clzll(diff) : 0u;
    if (nbits == 0) {
        __syncthreads();  // red is rewritten by the next leaf
        return;           // every key is equal: the leaf is sorted
    }
    for (uint32_t sh = 0; sh < nbits && sh < (uint32_t)KEYBITS; sh += DBITS) {
        for (int d = lane; d < ND; d += 64)
            cnt[wid][d] = 0;
        // rank within the wavefront: lanes holding the same digit, in (round, lane) order
        uint32_t pos[E];
        for (int r = 0; r < E; r++) {
            const uint32_t d = valid[r] ? (uint32_t)(qkey(x[r]) >> sh) & (ND - 1) : 0u;
            uint64_t m = __ballot(valid[r]);
#pragma unroll
            for (int bit = 0; bit < DBITS; bit++) {
                const uint64_t bb = __ballot((d >> bit) & 1);
                m &= ((d >> bit) & 1) ? bb : ~bb;
            }
            const uint32_t before = (uint32_t)__popcll(m & lt);
            const uint32_t old = valid[r] ? cnt[wid][d] : 0u;
            pos[r] = old + before;
            if (valid[r] && before == 0)
                cnt[wid][d] = (uint16_t)(old + (uint32_t)__popcll(m));
        }
        __syncthreads();
        // destinations: digit-major, then wavefront, then rank within the wavefront.
        // Thread t owns digit t: its total over the wavefronts, a scan over digits.
        uint32_t tot = 0;
        if (tid < ND)
            for (int w = 0; w < NW; w++)
                tot += cnt[w][tid];
        uint32_t inc = tot;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const uint32_t y = __shfl_up(inc, dd, 64);
            if (lane >= dd)
                inc += y;
        }
        if (lane == 63)
            wsum[wid] = inc;
        __syncthreads();
        if (tid < ND) {
            uint32_t run = inc - tot;
            for (int w = 0; w < wid; w++)
                run += wsum[w];
            for (int w = 0; w < NW; w++) {
                const uint32_t c = cnt[w][tid];
                cnt[w][tid] = (uint16_t)run;
                run += c;
            }
        }
        __syncthreads();
        for (int r = 0; r < E; r++)
            if (valid[r])
                buf[cnt[wid][(uint32_t)(qkey(x[r]) >> sh) & (ND - 1)] + pos[r]] = x[r];
        __syncthreads();
        for (int r = 0; r < E; r++) {
            const uint32_t idx = wid * 64 * E + r * 64 + lane;
            if (valid[r])
                x[r] = buf[idx];
        }
        __syncthreads();
    }
    for (int r = 0; r < E; r++) {
        const uint32_t idx = wid * 64 * E + r * 64 + lane;
        if (valid[r])
            A[idx] = x[r];
    }
    __syncthreads();  // LDS is reused by the next leaf
}

}  // namespace ss
