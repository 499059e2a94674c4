// ss_leafsort.h -- workgroup-local sort of a short segment in LDS (the
// quicksort's leaves, Section 5.2: a small subproblem is finished without
// the parallel partition).  Least-significant-digit radix sort with 8-bit
// digits over the bits in which the segment's keys differ; KV16 records move
// with their key.  Within a pass, each wavefront ranks 64 elements at a time:
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

template <typename T>
struct Digit {
    __device__ static __forceinline__ uint32_t of(const T &x, uint32_t sh) { return (uint32_t)(qkey(x) >> sh) & 255u; }
};

// One workgroup (1024 threads) sorts A[0, n), n <= CAP, by key.
template <typename T, int CAP, int KEYBITS>
__device__ void qleaf_sort(T *A, uint32_t n)
{
    constexpr int NT = 1024, NW = NT / 64;
    constexpr int E = CAP / NT;  // elements per thread
    __shared__ T buf[CAP];
    __shared__ uint32_t cnt[NW][256];
    __shared__ uint32_t dig_base[256];

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
    {
        __shared__ uint64_t red[2 * NW];
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
        __syncthreads();  // red is rewritten by the next leaf
    }
    const uint64_t diff = kmin ^ kmax;
    const uint32_t nbits = diff ? 64u - (uint32_t)__clzll(diff) : 0u;
    if (nbits == 0)
        return;  // every key is equal: the leaf is sorted
    for (uint32_t sh = 0; sh < nbits && sh < KEYBITS; sh += 8) {
        for (int d = lane; d < 256; d += 64)
            cnt[wid][d] = 0;
        uint32_t pos[E];
        for (int r = 0; r < E; r++) {
            const uint32_t d = valid[r] ? Digit<T>::of(x[r], sh) : 0u;
            uint64_t m = __ballot(valid[r]);
            for (int bit = 0; bit < 8; bit++) {
                const uint64_t bb = __ballot((d >> bit) & 1);
                m &= ((d >> bit) & 1) ? bb : ~bb;
            }
            // m: valid lanes of this round holding digit d
            const uint32_t before = (uint32_t)__popcll(m & lt);
            const uint32_t old = valid[r] ? cnt[wid][d] : 0u;
            pos[r] = old + before;
            if (valid[r] && before == 0)
                cnt[wid][d] = old + (uint32_t)__popcll(m);
        }
        __syncthreads();
        // destinations: digit-major, then wavefront, then position within the wavefront
        if (tid < 256) {
            uint32_t tot = 0;
            for (int w = 0; w < NW; w++)
                tot += cnt[w][tid];
            dig_base[tid] = tot;
        }
        __syncthreads();
        if (tid < 64) {
            uint32_t v[4], s = 0;
            for (int k = 0; k < 4; k++) {
                v[k] = dig_base[tid * 4 + k];
                s += v[k];
            }
            uint32_t inc = s;
            for (int dd = 1; dd < 64; dd <<= 1) {
                const uint32_t y = __shfl_up(inc, dd, 64);
                if (lane >= dd)
                    inc += y;
            }
            uint32_t run = inc - s;
            for (int k = 0; k < 4; k++) {
                dig_base[tid * 4 + k] = run;
                run += v[k];
            }
        }
        __syncthreads();
        if (tid < 256) {
            uint32_t run = dig_base[tid];
            for (int w = 0; w < NW; w++) {
                const uint32_t c = cnt[w][tid];
                cnt[w][tid] = run;
                run += c;
            }
        }
        __syncthreads();
        for (int r = 0; r < E; r++)
            if (valid[r])
                buf[cnt[wid][Digit<T>::of(x[r], sh)] + pos[r]] = x[r];
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
