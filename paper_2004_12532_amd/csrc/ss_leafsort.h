// ss_leafsort.h -- workgroup-local sort of a short segment in LDS (the
// quicksort's leaves, Section 5.2: a small subproblem is finished without
// the parallel partition).  Least-significant-digit radix sort with 9- or
// 10-bit digits of key - min, over the bits of the segment's key span; KV16
// records move with their key.  Within a pass, each wavefront ranks 64
// elements at a time: one ballot per digit bit gives each lane the mask of
// lanes holding the same digit, the lowest lane of that mask advances the
// wavefront's counter for the digit, and a scan over (digit, wavefront)
// turns the counters into destinations.
// The sort is stable and needs no atomics.
#pragma once

#include "ss_common.h"
#include "ss_device.h"

#include <type_traits>

namespace ss {

template <typename T>
__device__ __forceinline__ uint64_t qkey(const T &x)
{
    return key_of(x);
}

// Threads of the workgroups that sort leaves: the bucket sort of 4-byte keys
// runs 512 threads in 80 KiB of LDS, so two workgroups share a compute unit
// and one's loads and barriers overlap the other's work; 8-byte keys (144 KiB
// of LDS) and the radix sort run 1024.
template <typename T>
constexpr int leaf_bucket_nt()
{
    return sizeof(T) == 4 ? 512 : 1024;
}
constexpr int kLeafRadixNT = 1024;

// Plain keys (4 or 8 bytes), where equal keys are identical and stability
// cannot be observed, are bucketed; records (KV16) take the radix sort.
template <typename T>
constexpr bool leaf_buckets()
{
    return sizeof(T) <= 8;
}

// Largest bucket the bucket sort below sorts by insertion; a leaf with a
// larger one (and keys not all equal within buckets) is left to the radix sort.
constexpr uint32_t kLeafBucketMax = 32;

// One workgroup (NT threads) sorts A[0, n), n <= CAP, by key.  Returns true
// when A is sorted; false only from the bucket sort, for a leaf it leaves
// untouched because a bucket is crowded (the caller queues it for the radix
// sort, which is a separate kernel so that the bucket kernel keeps few
// registers).
//
// Bucket sort (RADIX false): bucket = (key - min) >> shift with 4096 buckets
// over the leaf's span, counted and scattered with LDS atomics, and every
// bucket finished by an insertion sort (none is needed when shift is 0: a
// bucket then holds one key value).  A leaf's keys come from a narrow,
// evenly filled key range (the parts left by the partitions above it), so
// buckets hold a few keys each.
//
// Radix sort (RADIX true): stable, 9-bit digits of key - min.
//
// The per-wavefront minimum, maximum and scan totals sit in the element
// buffer, which holds no element while they are live.
template <typename T, int CAP, int KEYBITS, int NT, bool RADIX>
__device__ bool qleaf_sort(T *A, uint32_t n)
{
    constexpr int NW = NT / 64;
    constexpr int E = CAP / NT;  // elements per thread
    constexpr int LOG2NB = 12, NB = 1 << LOG2NB, PB = NB / NT;
    constexpr int DBITS = 9, ND = 1 << DBITS;
    constexpr int CW = RADIX ? NW * ND / 2 : NB;  // 32-bit counter words
    static_assert(!RADIX || (ND <= NT && 64 * E < 65536), "digit counters: one digit per thread, 16-bit counts");
    static_assert(RADIX || (leaf_buckets<T>() && NB % NT == 0), "bucket sort: plain keys, whole buckets per thread");
    static_assert(CAP * sizeof(T) >= 2 * NW * 8 + 2 * NW * 4, "scratch inside the element buffer");
    __shared__ __align__(16) T buf[CAP];
    __shared__ uint32_t cw[CW];
    uint16_t(*cnt)[ND] = reinterpret_cast<uint16_t(*)[ND]>(cw);  // radix: per wavefront and digit
    uint64_t *red = reinterpret_cast<uint64_t *>(buf);              // [2 * NW]: minima, maxima
    uint32_t *wsum = reinterpret_cast<uint32_t *>(red + 2 * NW);     // [NW]
    uint32_t *wmax = wsum + NW;                                      // [NW]

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const uint64_t lt = (1ull << lane) - 1;

    // Striped arrangement: element r of thread (wid, lane) is at
    // index wid * 64 * E + r * 64 + lane, so element order is (wave, round, lane).
    const uint32_t base = wid * 64 * E + lane;
    auto valid = [&](int r) { return base + r * 64 < n; };
    T x[E];
    uint64_t kmin = ~0ull, kmax = 0;
    for (int r = 0; r < E; r++) {
        const uint32_t idx = base + r * 64;
        if (idx < n) {
            x[r] = A[idx];
            const uint64_t k = qkey(x[r]);
            kmin = k < kmin ? k : kmin;
            kmax = k > kmax ? k : kmax;
        }
    }
    kmin = wave_min(kmin);
    kmax = wave_max(kmax);
    if (lane == 0) {
        red[wid] = kmin;
        red[NW + wid] = kmax;
    }
    if constexpr (!RADIX)
        for (int j = tid; j < NB; j += NT)
            cw[j] = 0;
    __syncthreads();
    kmin = red[0];
    kmax = red[NW];
    for (int w = 1; w < NW; w++) {
        kmin = red[w] < kmin ? red[w] : kmin;
        kmax = red[NW + w] > kmax ? red[NW + w] : kmax;
    }
    // Digits and buckets are taken from key - kmin, which is at most
    // kmax - kmin: only the bits of that span need sorting.  (4-byte keys
    // compute it in 32 bits.)
    const uint64_t span = kmax - kmin;
    const uint32_t nbits = span ? 64u - (uint32_t)__clzll(span) : 0u;
    using K = typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type;
    const K kmin_k = (K)kmin;
    auto rel = [&](const T &v) { return (K)qkey(v) - kmin_k; };
    if (nbits == 0) {
        __syncthreads();  // red is rewritten by the next leaf
        return true;      // every key is equal: the leaf is sorted
    }
    if constexpr (!RADIX) {
        const uint32_t shift = nbits > (uint32_t)LOG2NB ? nbits - (uint32_t)LOG2NB : 0u;
        for (int r = 0; r < E; r++)
            if (valid(r))
                atomicAdd(&cw[(uint32_t)(rel(x[r]) >> shift)], 1u);
        __syncthreads();
        // bucket starts: thread t owns buckets [t * PB, t * PB + PB)
        uint32_t c[PB], tot = 0, mx = 0;
#pragma unroll
        for (int i = 0; i < PB; i++) {
            c[i] = cw[tid * PB + i];
            tot += c[i];
            mx = c[i] > mx ? c[i] : mx;
        }
        uint32_t inc = tot;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const uint32_t y = __shfl_up(inc, dd, 64);
            if (lane >= dd)
                inc += y;
        }
        mx = (uint32_t)wave_max((uint64_t)mx);
        if (lane == 63)
            wsum[wid] = inc;
        if (lane == 0)
            wmax[wid] = mx;
        __syncthreads();
        uint32_t run = inc - tot, bmax = 0;
        for (int w = 0; w < NW; w++) {
            if (w < wid)
                run += wsum[w];
            bmax = wmax[w] > bmax ? wmax[w] : bmax;
        }
#pragma unroll
        for (int i = 0; i < PB; i++) {
            cw[tid * PB + i] = run;
            run += c[i];
        }
        __syncthreads();  // starts written; wsum and wmax read
        if (shift == 0 || bmax <= kLeafBucketMax) {
            for (int r = 0; r < E; r++)
                if (valid(r))
                    buf[atomicAdd(&cw[(uint32_t)(rel(x[r]) >> shift)], 1u)] = x[r];
            __syncthreads();  // cw[b] is now the end of bucket b, the start of bucket b + 1
            if (shift) {
                for (int b = tid; b < NB; b += NT) {
                    const uint32_t s0 = b ? cw[b - 1] : 0u, e0 = cw[b];
                    for (uint32_t i = s0 + 1; i < e0; i++) {
                        const T v = buf[i];
                        uint32_t j = i;
                        while (j > s0 && buf[j - 1] > v) {
                            buf[j] = buf[j - 1];
                            j--;
                        }
                        buf[j] = v;
                    }
                }
                __syncthreads();
            }
            for (int r = 0; r < E; r++) {
                const uint32_t idx = base + r * 64;
                if (valid(r))
                    A[idx] = buf[idx];
            }
            __syncthreads();  // LDS is reused by the next leaf
            return true;
        }
        return false;  // a crowded bucket: A is untouched (the barrier above let every thread read wmax)
    } else {
        for (uint32_t sh = 0; sh < nbits && sh < (uint32_t)KEYBITS; sh += DBITS) {
            for (int d = lane; d < ND; d += 64)
                cnt[wid][d] = 0;
            // rank within the wavefront: lanes holding the same digit, in (round, lane) order
            uint32_t pos[E];
            for (int r = 0; r < E; r++) {
                const uint32_t d = valid(r) ? (uint32_t)(rel(x[r]) >> sh) & (ND - 1) : 0u;
                uint64_t m = __ballot(valid(r));
#pragma unroll
                for (int bit = 0; bit < DBITS; bit++) {
                    const uint64_t bb = __ballot((d >> bit) & 1);
                    m &= ((d >> bit) & 1) ? bb : ~bb;
                }
                const uint32_t before = (uint32_t)__popcll(m & lt);
                const uint32_t old = valid(r) ? cnt[wid][d] : 0u;
                pos[r] = old + before;
                if (valid(r) && before == 0)
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
                if (valid(r))
                    buf[cnt[wid][(uint32_t)(rel(x[r]) >> sh) & (ND - 1)] + pos[r]] = x[r];
            __syncthreads();
            for (int r = 0; r < E; r++) {
                const uint32_t idx = base + r * 64;
                if (valid(r))
                    x[r] = buf[idx];
            }
            __syncthreads();
        }
        for (int r = 0; r < E; r++) {
            const uint32_t idx = base + r * 64;
            if (valid(r))
                A[idx] = x[r];
        }
        __syncthreads();  // LDS is reused by the next leaf
        return true;
    }
}

}  // namespace ss
