// ss_device.h -- device-side helpers shared by the library's kernels:
// 16-byte register vectors, per-dtype element access, wavefront reductions
// and the reduction of per-workgroup (v_min, v_max) partials.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ss_common.h"

namespace ss {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));  // one 16-byte vector in registers

template <typename T>
struct Elem;
template <>
struct Elem<uint32_t> {
    static constexpr int V = 4;
    __device__ static __forceinline__ uint64_t key(const v4u &v, int e)
    {
        return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
    }
    __device__ static __forceinline__ void put(v4u *tile, uint32_t d, const v4u &v, int e)
    {
        reinterpret_cast<uint32_t *>(tile)[d] = e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
    }
    __device__ static __forceinline__ void load1(v4u &v, int e, const char *p)
    {
        const uint32_t x = *reinterpret_cast<const uint32_t *>(p);
        if (e == 0) v.x = x; else if (e == 1) v.y = x; else if (e == 2) v.z = x; else v.w = x;
    }
    __device__ static __forceinline__ void store1(const v4u &v, int e, char *p)
    {
        *reinterpret_cast<uint32_t *>(p) = e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
    }
};
template <>
struct Elem<uint64_t> {
    static constexpr int V = 2;
    __device__ static __forceinline__ uint64_t key(const v4u &v, int e)
    {
        return e == 0 ? ((uint64_t)v.y << 32 | v.x) : ((uint64_t)v.w << 32 | v.z);
    }
    __device__ static __forceinline__ void put(v4u *tile, uint32_t d, const v4u &v, int e)
    {
        reinterpret_cast<uint2 *>(tile)[d] = e == 0 ? make_uint2(v.x, v.y) : make_uint2(v.z, v.w);
    }
    __device__ static __forceinline__ void load1(v4u &v, int e, const char *p)
    {
        const uint2 x = *reinterpret_cast<const uint2 *>(p);
        if (e == 0) { v.x = x.x; v.y = x.y; } else { v.z = x.x; v.w = x.y; }
    }
    __device__ static __forceinline__ void store1(const v4u &v, int e, char *p)
    {
        *reinterpret_cast<uint2 *>(p) = e == 0 ? make_uint2(v.x, v.y) : make_uint2(v.z, v.w);
    }
};
template <>
struct Elem<KV> {
    static constexpr int V = 1;
    __device__ static __forceinline__ uint64_t key(const v4u &v, int) { return (uint64_t)v.y << 32 | v.x; }
    __device__ static __forceinline__ void put(v4u *tile, uint32_t d, const v4u &v, int) { tile[d] = v; }
    __device__ static __forceinline__ void load1(v4u &v, int, const char *p) { v = *reinterpret_cast<const v4u *>(p); }
    __device__ static __forceinline__ void store1(const v4u &v, int, char *p) { *reinterpret_cast<v4u *>(p) = v; }
};

// Inclusive prefix sum over the wavefront's 64 lanes: Hillis-Steele steps
// inside each row of 16 lanes (DPP row shifts by 1, 2, 4 and 8; a lane
// whose source lies before its row's start adds 0), then the totals of the
// rows below, read from lanes 15, 31 and 47.
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t x, int lane)
{
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
    const uint32_t t0 = (uint32_t)__builtin_amdgcn_readlane((int)x, 15);
    const uint32_t t1 = (uint32_t)__builtin_amdgcn_readlane((int)x, 31);
    const uint32_t t2 = (uint32_t)__builtin_amdgcn_readlane((int)x, 47);
    const int row = lane >> 4;
    return x + (row >= 1 ? t0 : 0u) + (row >= 2 ? t1 : 0u) + (row >= 3 ? t2 : 0u);
}

// A workgroup barrier that orders LDS accesses only: every wavefront's LDS
// reads and writes before it are complete, and the compiler moves no memory
// access across it.  Global loads and stores stay in flight (a barrier with
// the default fence waits for them).
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xf | 0x3 << 14 | 0x7 << 4);  // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t wave_min(uint64_t x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint64_t y = __shfl_xor(x, d, 64);
        x = y < x ? y : x;
    }
    return x;
}

__device__ __forceinline__ uint64_t wave_max(uint64_t x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint64_t y = __shfl_xor(x, d, 64);
        x = y > x ? y : x;
    }
    return x;
}

// Reduce the previous level's partials to the region [vmin, vmax) (all
// threads receive it).  `red` holds 2 * waves words of LDS.
template <int NT>
__device__ __forceinline__ void reduce_partials(const uint64_t *prev, uint32_t count, uint64_t *red,
                                                uint64_t &lo, uint64_t &hi)
{
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    uint64_t mn = ~0ull, mx = 0;
    for (uint32_t k = tid; k < count; k += NT) {
        const uint64_t a = prev[2 * k], b = prev[2 * k + 1];
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    if (lane == 0) {
        red[wid] = mn;
        red[NW + wid] = mx;
    }
    __syncthreads();
    mn = red[0];
    mx = red[NW];
#pragma unroll
    for (int w = 1; w < NW; w++) {
        mn = red[w] < mn ? red[w] : mn;
        mx = red[NW + w] > mx ? red[NW + w] : mx;
    }
    lo = mn;
    hi = mx;
}

// Region of a non-first level: [v_min, v_max) of the previous level.  When
// the previous level had at most one group (g <= 1: it finished the
// partition, or had nothing left to do), workgroup 0's partial is the whole
// answer and the other partials need not be read.
template <int NT>
__device__ __forceinline__ void prev_region(const uint64_t *prev, uint32_t count, const uint64_t *prev_ctl,
                                            uint64_t *red, uint64_t &lo, uint64_t &hi)
{
    if (prev_ctl && prev_ctl[2] <= 1) {
        lo = prev[0];
        hi = prev[1] > prev[0] ? prev[1] : prev[0];
        return;
    }
    reduce_partials<NT>(prev, count, red, lo, hi);
}

// Key of an element held as its own type.
__device__ __forceinline__ uint64_t key_of(uint32_t x) { return x; }
__device__ __forceinline__ uint64_t key_of(uint64_t x) { return x; }
__device__ __forceinline__ uint64_t key_of(const KV &x) { return x.key; }

// Exclusive ranks among flagged items of one workgroup pass: item k is held
// by thread k % NT in round k / NT, and items are ranked in k order.  `sh`
// needs K * NT / 64 + 1 words of LDS (at most 512 counts).  Ends with a barrier.
template <int NT, int K>
__device__ __forceinline__ void block_rank(const bool (&flag)[K], uint32_t (&rank)[K], uint32_t &total,
                                           uint32_t *sh)
{
    constexpr int NW = NT / 64;
    constexpr int E = K * NW;              // per-(round, wave) counts to scan
    constexpr int C = (E + 63) / 64;       // counts per lane of the scanning wave
    static_assert(C <= 8, "rank scan size");
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int r = 0; r < K; r++) {
        const uint64_t m = __ballot(flag[r]);
        rank[r] = lanes_below(m);
        if (lane == 0)
            sh[r * NW + wid] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (wid == 0) {
        uint32_t x[C], sum = 0;
#pragma unroll
        for (int c = 0; c < C; c++) {
            const int k = lane * C + c;
            x[c] = k < E ? sh[k] : 0u;
            sum += x[c];
        }
        uint32_t inc = sum;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(inc, d, 64);
            if (lane >= d)
                inc += y;
        }
        uint32_t run = inc - sum;
#pragma unroll
        for (int c = 0; c < C; c++) {
            const int k = lane * C + c;
            if (k < E)
                sh[k] = run;
            run += x[c];
        }
        if (lane == 63)
            sh[E] = inc;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < K; r++)
        rank[r] += sh[r * NW + wid];
    total = sh[E];
    __syncthreads();
}

}  // namespace ss
