// ss_batched.hip -- Smoothed Striding partition of many independent arrays
// with one persistent launch per recursion level (Section 4's Partial
// Partition Step applied to every array at once).
//
// Device state, one entry per array k: its current region [lo_k, hi_k)
// (absolute element indices into the base), its pivot, its size class, its
// number of groups g_k at this level, and its split once found.  A level is
// three launches with no host decision in between:
//   k_binit / k_bstep  per array (one wavefront): fold the previous level's
//             splitting positions of its groups into [v_min, v_max) -- a
//             region left with one group or none is finished (split = v_min),
//             otherwise it is the next region -- and plan the next level's
//             geometry g_k from that region;
//   k_bscan   one workgroup: exclusive scan of g_k -> the array's first item,
//             staged through LDS so that every global access is coalesced;
//   k_blevel  persistent: every workgroup takes items t = bid, bid + grid, ...,
//             finds the array k of item t (binary search over the first-item
//             offsets in LDS; for very large batches an item map written by
//             k_bfill), partitions group t - first_k of array k exactly as the
//             single-array kernel does and writes the group's splitting
//             position v.
// The number of levels is planned on the host from the longest array (each
// level shrinks a region by more than 16x once it spans several groups).  An
// array still open after the last level -- unlikely, but not excluded by the
// randomness of the offsets -- is finished by k_bcleanup, one workgroup per
// such array running the serial block two-pointer exchange over its small
// remaining region, so a call is a fixed chain of launches that never needs a
// host decision.
// Arrays that fit one group are whole-array tiles (g = 1) and finish at the
// first level.  The chunk offsets depend on (seed, level, j, g) only, never on
// an array's position in the batch, so an array gets the same bytes alone and
// inside any batch.
#include "ss_cleanup.h"
#include "ss_common.h"
#include "ss_device.h"
#include "ss_internal.h"
#include "ss_ldsctx.h"
#include "ss_levelctx.h"

#include <algorithm>
#include <cmath>
#include <tuple>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

namespace ss {

// With search set, the level kernel finds an item's array by binary search
// over the first-item offsets, copied into dynamic LDS at its start, instead
// of reading an item map: for up to 16399 arrays with the 128 KiB-group
// kernel (one workgroup per CU either way; 128 KiB of LDS), up to 4095 with
// the smaller ones (whose occupancy the LDS must not cut).
constexpr uint32_t kSearchMaxBig = 16400, kSearchMaxSmall = 4096;

struct BatchGeom {
    char *base;
    uint64_t seed;
    uint32_t level;
    uint32_t search;
    BatchClasses C;
};

__device__ __forceinline__ uint32_t bnum(const BatchState &B)
{
    return B.count ? *B.count : B.num;
}

// Element at which array k's line grid starts.
__device__ __forceinline__ uint64_t line_origin(const BatchState &B, uint32_t k)
{
    return B.base_lines ? 0ull : B.start[k];
}

__device__ __forceinline__ uint32_t plan_groups(const BatchState &B, const BatchGeom &Gm, uint32_t k, uint64_t lo,
                                                uint64_t hi)
{
    const uint32_t c = B.cls[k];
    const uint64_t o = line_origin(B, k);
    return plan_geo(lo - o, hi - o, Gm.C.log2b[c], Gm.C.s_max[c]).g;
}

// First level: every array's region is the whole array.
__global__ void __launch_bounds__(256) k_binit(BatchState B, BatchGeom Gm)
{
    const uint32_t num = bnum(B);
    for (uint32_t k = blockIdx.x * 256 + threadIdx.x; k < num; k += gridDim.x * 256) {
        const uint64_t s = B.start[k], l = B.len[k];
        uint32_t c = 0;
        while (c + 1 < Gm.C.n && l > Gm.C.max_len[c])
            c++;
        B.cls[k] = (uint8_t)c;
        B.lo[k] = s;
        B.hi[k] = s + l;
        B.split[k] = l ? ~0ull : s;
        B.g[k] = l ? plan_groups(B, Gm, k, s, s + l) : 0u;
    }
}

// Exclusive scan of g over all arrays (first item of every array), the item
// count ctl[0] and the count of open arrays ctl[1].  One workgroup; chunks of
// kScanChunk entries are staged through LDS so that global reads and writes
// are coalesced, and each thread scans kScanPer consecutive entries.
constexpr int kScanNT = 1024, kScanPer = 20, kScanChunk = kScanNT * kScanPer;

struct ScanSmem {
    uint64_t wsum[kScanNT / 64], wopen[kScanNT / 64];
};

// Exclusive scan of g over all arrays by one workgroup of kScanNT threads.
// Each thread takes kScanPer consecutive entries of a chunk with 16-byte
// loads and writes their kScanPer first-item offsets as 16-byte stores, so a
// wavefront reads 5 KiB and writes 10 KiB contiguously per chunk; a chunk
// covers 20480 arrays, so a batch of 20000 takes one round of the loop (each
// round waits for its loads once).
__device__ void scan_groups(const BatchState &B, ScanSmem &S)
{
    static_assert(kScanPer % 4 == 0, "16-byte loads of g");
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    uint64_t carry = 0, ocarry = 0;
    const uint32_t num = bnum(B);
    for (uint32_t c0 = 0; c0 < num; c0 += kScanChunk) {
        const uint32_t j0 = c0 + (uint32_t)tid * kScanPer;
        uint32_t v[kScanPer];
        if (j0 + kScanPer <= num) {
#pragma unroll
            for (int r = 0; r < kScanPer; r += 4) {
                const v4u a = *reinterpret_cast<const v4u *>(B.g + j0 + r);
                v[r] = a.x;
                v[r + 1] = a.y;
                v[r + 2] = a.z;
                v[r + 3] = a.w;
            }
        } else {
#pragma unroll
            for (int r = 0; r < kScanPer; r++)
                v[r] = j0 + r < num ? B.g[j0 + r] : 0u;
        }
        uint64_t s = 0, open = 0;
#pragma unroll
        for (int r = 0; r < kScanPer; r++) {
            s += v[r];
            open += v[r] != 0;
        }
        uint64_t inc = s, oinc = open;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t y = __shfl_up(inc, d, 64), z = __shfl_up(oinc, d, 64);
            if (lane >= d) {
                inc += y;
                oinc += z;
            }
        }
        if (lane == 63) {
            S.wsum[wid] = inc;
            S.wopen[wid] = oinc;
        }
        __syncthreads();
        uint64_t off = carry, tot = 0, otot = 0;
        for (int w = 0; w < kScanNT / 64; w++) {
            if (w < wid)
                off += S.wsum[w];
            tot += S.wsum[w];
            otot += S.wopen[w];
        }
        uint64_t run = off + inc - s;
        uint64_t f[kScanPer];
#pragma unroll
        for (int r = 0; r < kScanPer; r++) {
            f[r] = run;
            run += v[r];
        }
        if (j0 + kScanPer <= num) {
            typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
#pragma unroll
            for (int r = 0; r < kScanPer; r += 2)
                *reinterpret_cast<u64x2 *>(B.first + j0 + r) = u64x2{f[r], f[r + 1]};
        } else {
#pragma unroll
            for (int r = 0; r < kScanPer; r++)
                if (j0 + r < num)
                    B.first[j0 + r] = f[r];
        }
        carry += tot;
        ocarry += otot;
        __syncthreads();  // wsum is rewritten by the next chunk
    }
    if (tid == 0) {
        B.first[num] = carry;
        B.ctl[0] = carry;
        B.ctl[1] = ocarry;
    }
}

__global__ void __launch_bounds__(kScanNT) k_bscan(BatchState B)
{
    __shared__ ScanSmem S;
    scan_groups(B, S);
}

// Later levels: fold the previous level's splitting positions of array k
// (one wavefront per array), then plan the next level.  (A separate
// single-workgroup scan follows: handing the scan to the last workgroup to
// finish here would need device-scope fences and a shared ticket, which cost
// more than the launch they save on a GPU whose XCDs have separate L2s.)
__global__ void __launch_bounds__(256) k_bstep(BatchState B, BatchGeom Gm)
{
    const uint32_t num = bnum(B);
    for (uint32_t k = blockIdx.x * 4 + (threadIdx.x >> 6); k < num; k += gridDim.x * 4) {
        const uint32_t g = B.g[k];
        if (g == 0)
            continue;
        const uint64_t f = B.first[k];
        uint64_t mn = ~0ull, mx = 0;
        for (uint32_t i = threadIdx.x & 63; i < g; i += 64) {
            const uint64_t v = B.vout[f + i];
            mn = v < mn ? v : mn;
            mx = v > mx ? v : mx;
        }
        mn = wave_min(mn);
        mx = wave_max(mx);
        if ((threadIdx.x & 63) == 0) {
            if (g == 1 || !(mn < mx)) {
                B.split[k] = mn;
                B.g[k] = 0;
            } else {
                B.lo[k] = mn;
                B.hi[k] = mx;
                B.g[k] = plan_groups(B, Gm, k, mn, mx);
            }
        }
    }
}

__global__ void __launch_bounds__(256) k_bfill(BatchState B)
{
    const uint32_t num = bnum(B);
    for (uint32_t k = blockIdx.x * 4 + (threadIdx.x >> 6); k < num; k += gridDim.x * 4) {
        const uint64_t f = B.first[k];
        const uint32_t g = B.g[k];
        for (uint32_t i = threadIdx.x & 63; i < g; i += 64)
            B.imap[f + i] = k;
    }
}

template <typename T, int NT, int NV>
__global__ void __launch_bounds__(NT) k_blevel(BatchState B, BatchGeom Gm)
{
    using Ctx = LevelCtx<T, NT, NV>;
    constexpr int W = Ctx::W;
    constexpr int MAXS = Ctx::NVEC * 16 / 64;
    __shared__ uint32_t xoff[MAXS];
    __shared__ uint32_t cnt[Ctx::E + 1];
    extern __shared__ uint64_t sfirst[];  // num + 1 entries when Gm.search

    const int tid = threadIdx.x;
    const uint64_t total = B.ctl[0];
    uint32_t num = 0;
    if (Gm.search) {
        num = bnum(B);
        for (uint32_t j = tid; j <= num; j += NT)
            sfirst[j] = B.first[j];
        __syncthreads();
    }
    for (uint64_t t = blockIdx.x; t < total; t += gridDim.x) {
        uint32_t k;
        if (Gm.search) {
            // the last array whose first item is <= t (arrays with no items share their successor's offset)
            uint32_t lo = 0, hi = num;  // sfirst[lo] <= t < sfirst[hi]
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (sfirst[mid] <= t)
                    lo = mid;
                else
                    hi = mid;
            }
            k = lo;
        } else {
            k = B.imap[t];
        }
        const uint32_t i = (uint32_t)(t - B.first[k]);
        const uint64_t lo = B.lo[k], hi = B.hi[k], start = line_origin(B, k);
        const uint32_t cl = B.cls[k], log2b = Gm.C.log2b[cl];
        const Geo G = plan_geo(lo - start, hi - start, log2b, Gm.C.s_max[cl]);
        Ctx x;
        x.g = G.g;
        x.s = G.s;
        x.fp = G.fp;
        x.real_end = (uint64_t)G.fp + (hi - lo);
        x.A0 = Gm.base + (lo - G.fp) * W;  // line grid counted from the array's line origin
        x.log2b = log2b;
        x.vpl_log2 = log2b + Ctx::LOG2W - 4;
        x.nvec = G.s << x.vpl_log2;
        x.pivot = B.pivot[k];
        x.xoff = xoff;
        x.cnt = cnt;
        x.tid = tid;
        x.lane = tid & 63;
        x.wid = tid >> 6;
        for (uint32_t j = tid; j < G.s; j += NT)
            xoff[j] = G.g > 1 ? chunk_offset(Gm.seed, Gm.level, j, G.g) : 0u;
        __syncthreads();
        v4u buf[NV];
        typename Ctx::Mask m;
        const bool fast = x.fast(i);
        uint32_t c;
        if (fast) {
            x.template load<true>(buf, i, m);
            c = x.template partition<true>(buf, i, m);
        } else {
            x.template load<false>(buf, i, m);
            c = x.template partition<false>(buf, i, m);
        }
        if (tid == 0) {
            uint64_t vi;
            if (c >= (G.s << log2b)) {
                vi = hi;
            } else {
                const uint64_t vp =
                    ((uint64_t)x.line_of(c >> log2b, i) << log2b) + (c & ((1u << log2b) - 1));
                vi = vp >= x.real_end ? hi : lo + (vp - G.fp);
            }
            B.vout[t] = vi;
        }
        __syncthreads();  // LDS reused by the next item
    }
}

// The same level with the LDS-tile group body (ss_ldsctx.h).
template <typename T, int NT, int TILE>
__global__ void __launch_bounds__(NT, 4) k_blevel_lds(BatchState B, BatchGeom Gm)
{
    using Ctx = LdsCtx<T, NT, TILE>;
    constexpr int W = Ctx::W;
    constexpr int MAXS = TILE / 64;
    __shared__ v4u tile[Ctx::NVEC];
    __shared__ uint32_t xoff[MAXS];
    __shared__ uint32_t wtot[Ctx::E], wpre[Ctx::E + 1];
    extern __shared__ uint64_t sfirst[];  // num + 1 entries when Gm.search

    const int tid = threadIdx.x;
    const uint64_t total = B.ctl[0];
    uint32_t num = 0;
    if (Gm.search) {
        num = bnum(B);
        for (uint32_t j = tid; j <= num; j += NT)
            sfirst[j] = B.first[j];
        __syncthreads();
    }
    for (uint64_t t = blockIdx.x; t < total; t += gridDim.x) {
        uint32_t k;
        if (Gm.search) {
            uint32_t lo = 0, hi = num;  // sfirst[lo] <= t < sfirst[hi]
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (sfirst[mid] <= t)
                    lo = mid;
                else
                    hi = mid;
            }
            k = lo;
        } else {
            k = B.imap[t];
        }
        const uint32_t i = (uint32_t)(t - B.first[k]);
        const uint64_t lo = B.lo[k], hi = B.hi[k], start = line_origin(B, k);
        const uint32_t cl = B.cls[k], log2b = Gm.C.log2b[cl];
        const Geo G = plan_geo(lo - start, hi - start, log2b, Gm.C.s_max[cl]);
        Ctx x;
        x.g = G.g;
        x.s = G.s;
        x.fp = G.fp;
        x.real_end = (uint64_t)G.fp + (hi - lo);
        x.A0 = Gm.base + (lo - G.fp) * W;
        x.log2b = log2b;
        x.vpl_log2 = log2b + Ctx::LOG2W - 4;
        x.nvec = G.s << x.vpl_log2;
        x.pivot = B.pivot[k];
        x.xoff = xoff;
        x.tile = tile;
        x.wtot = wtot;
        x.wpre = wpre;
        x.tid = tid;
        x.lane = tid & 63;
        x.wid = tid >> 6;
        for (uint32_t j = tid; j < G.s; j += NT)
            xoff[j] = G.g > 1 ? chunk_offset(Gm.seed, Gm.level, j, G.g) : 0u;
        __syncthreads();
        v4u buf[Ctx::NV];
        typename Ctx::Mask m;
        uint32_t c;
        if (x.fast(i)) {
            x.template load<true>(buf, i, m);
            c = x.template partition_store<true>(buf, i, m);
        } else {
            x.template load<false>(buf, i, m);
            c = x.template partition_store<false>(buf, i, m);
        }
        if (tid == 0) {
            uint64_t vi;
            if (c >= (G.s << log2b)) {
                vi = hi;
            } else {
                const uint32_t j = c >> log2b;
                uint32_t r = xoff[j] + i;
                r = r >= G.g ? r - G.g : r;
                const uint64_t vp = (((uint64_t)j * G.g + r) << log2b) + (c & ((1u << log2b) - 1));
                vi = vp >= x.real_end ? hi : lo + (vp - G.fp);
            }
            B.vout[t] = vi;
        }
        __syncthreads();  // LDS reused by the next item
    }
}

// Arrays still open after the last level: one workgroup each partitions the
// remaining region serially (block two-pointer exchange).
// 32 KiB blocks per serial step, as in the single-array cleanup.  Workgroup b
// takes arrays b, b + grid, ...: it reads the splits of 1024 of them at once
// (one per thread) to find the open ones, then partitions those in turn.
template <typename T>
__global__ void __launch_bounds__(1024) k_bcleanup(BatchState B, BatchGeom Gm)
{
    __shared__ CleanupSmem<T, 1024, 32768> S;
    __shared__ uint32_t open[1024];
    __shared__ uint32_t n_open;
    const uint32_t num = bnum(B), tid = threadIdx.x, step = gridDim.x;
    for (uint64_t k0 = blockIdx.x; k0 < num; k0 += 1024ull * step) {
        if (tid == 0)
            n_open = 0;
        __syncthreads();
        const uint64_t k = k0 + (uint64_t)tid * step;
        if (k < num && B.split[k] == ~0ull)
            open[atomicAdd(&n_open, 1u)] = (uint32_t)k;
        __syncthreads();
        const uint32_t m = n_open;
        for (uint32_t j = 0; j < m; j++) {
            const uint32_t a = open[j];
            const uint64_t sp =
                cleanup_region<T, 1024, 32768>(reinterpret_cast<T *>(Gm.base), B.pivot[a], B.lo[a], B.hi[a], S);
            if (tid == 0)
                B.split[a] = sp;
        }
        __syncthreads();  // open and n_open are rewritten for the next arrays
    }
}

__global__ void __launch_bounds__(256) k_bfinish(BatchState B, uint64_t *d_splits)
{
    const uint32_t num = bnum(B);
    for (uint32_t k = blockIdx.x * 256 + threadIdx.x; k < num; k += gridDim.x * 256) {
        const uint64_t s = B.split[k];
        d_splits[k] = s == ~0ull ? ~0ull : s - B.start[k];
    }
}

// ------------------------------------------------------------------ host side

namespace {

// Per (device, stream): the device state of a batched call, and two pinned
// host staging buffers for the starts and lengths, used alternately.  A call
// waits only for the copy issued from its buffer two calls earlier (its
// event), never for the whole stream, so back-to-back calls queue on the
// device without a host stall.
struct BatchWork {
    char *dev = nullptr;
    size_t dev_bytes = 0;
    uint64_t *host[2] = {nullptr, nullptr};
    hipEvent_t copied[2] = {nullptr, nullptr};
    size_t host_words = 0;
    uint32_t next = 0;
};
std::mutex g_b_mu;
std::map<std::pair<int, void *>, BatchWork> g_b;

template <typename T, int NT, int NV>
hipError_t launch_blevel(uint32_t grid, const BatchState &B, const BatchGeom &G, hipStream_t st)
{
    const size_t shmem = G.search ? ((size_t)B.num + 1) * sizeof(uint64_t) : 0;
    if (shmem > 32768) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_blevel<T, NT, NV>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL((k_blevel<T, NT, NV>), dim3(grid), dim3(NT), shmem, st, B, G);
    return hipGetLastError();
}

template <typename T, int NT, int NV>
const void *blevel_fn()
{
    return reinterpret_cast<const void *>(&k_blevel<T, NT, NV>);
}

template <typename T, int NT, int TILE>
hipError_t launch_blevel_lds(uint32_t grid, const BatchState &B, const BatchGeom &G, hipStream_t st)
{
    const size_t shmem = G.search ? ((size_t)B.num + 1) * sizeof(uint64_t) : 0;
    if (shmem > 32768) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_blevel_lds<T, NT, TILE>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL((k_blevel_lds<T, NT, TILE>), dim3(grid), dim3(NT), shmem, st, B, G);
    return hipGetLastError();
}

template <typename T, int NT, int TILE>
const void *blevel_lds_fn()
{
    return reinterpret_cast<const void *>(&k_blevel_lds<T, NT, TILE>);
}

struct BVariant {
    int dtype;
    uint32_t engine;
    uint32_t tile;
    int nt;
    hipError_t (*launch)(uint32_t, const BatchState &, const BatchGeom &, hipStream_t);
    const void *(*fn)();
};

#define SS_BV(D, T, NT, NV) \
    {D, SS_ENGINE_REGS, NT * NV * 16, NT, &launch_blevel<T, NT, NV>, &blevel_fn<T, NT, NV>}
#define SS_BVL(D, T, NT, TILE) \
    {D, SS_ENGINE_LDS, TILE, NT, &launch_blevel_lds<T, NT, TILE>, &blevel_lds_fn<T, NT, TILE>}

const BVariant *pick_bvariant(int dtype, uint32_t engine, uint32_t tile)
{
    static const BVariant v[] = {
        SS_BV(SS_U32, uint32_t, 256, 8),         SS_BV(SS_U64, uint64_t, 256, 8),
        SS_BV(SS_KV16, KV, 256, 8),              SS_BV(SS_U32, uint32_t, 512, 8),
        SS_BV(SS_U64, uint64_t, 512, 8),         SS_BV(SS_KV16, KV, 512, 8),
        SS_BV(SS_U32, uint32_t, 512, 16),        SS_BV(SS_U64, uint64_t, 512, 16),
        SS_BV(SS_KV16, KV, 512, 16),             SS_BVL(SS_U32, uint32_t, 256, 32768),
        SS_BVL(SS_U64, uint64_t, 256, 32768),    SS_BVL(SS_KV16, KV, 256, 32768),
        SS_BVL(SS_U32, uint32_t, 512, 65536),    SS_BVL(SS_U64, uint64_t, 512, 65536),
        SS_BVL(SS_KV16, KV, 512, 65536),
    };
    for (const BVariant &x : v)
        if (x.dtype == dtype && x.engine == engine && x.tile == tile)
            return &x;
    return nullptr;
}

}  // namespace

// Levels of the batched recursion for arrays of at most max_len elements:
// one level finishes a region of one group; a region of several groups
// shrinks by well over 16x per level (its middle region is a few percent of
// it plus at most one group's worth of lines), so the chain plans
// 2 + ceil(log16(max_len / group)) levels.  A region still open after them is
// finished by the cleanup kernel.
uint32_t batched_levels(uint64_t max_len, uint64_t tile_elems)
{
    uint32_t lv = 1;
    uint64_t r = max_len;
    while (r > tile_elems && lv < 16) {
        r = r / 16;
        lv++;
    }
    return lv == 1 ? 1u : lv + 1;
}

// Levels of a batched call with the tail geometry, planned as for a single
// array: the first level leaves about 4.4 / sqrt(S0) of an array of max_len
// elements, each later one about 0.11 of the region before it, until the
// expected region fits two passes of the closing serial cleanup (k_bcleanup),
// which partitions whatever is still open.
uint32_t batched_planned_levels(uint64_t max_len, uint64_t S0, int w)
{
    if (max_len <= S0)
        return 1;
    const double base = 2.0 * (double)cleanup_pass_elems(w);
    double r = (double)max_len * 4.4 / std::sqrt((double)S0);
    uint32_t lv = 1;
    while (r > base && lv < 16) {
        r *= 0.11;
        lv++;
    }
    return lv;
}

// Run the batched recursion for `num` arrays whose start/len are already in
// device memory (B.start, B.len): `levels` persistent level launches, then
// the cleanup of any array still open, then (if d_splits) the splits
// relative to each start.  A fixed chain of launches with no host decision.
BatchClasses batched_default_classes(const Resolved &R)
{
    BatchClasses C;
    std::memset(&C, 0, sizeof(C));
    C.n = 1;
    C.max_len[0] = ~0ull;
    C.log2b[0] = R.log2b;
    C.s_max[0] = (uint32_t)(R.tile / ((uint64_t)R.b * R.w));
    return C;
}

// The geometry of a batched call's levels from the second on: every class
// (the table keeps its class count, so each array's class index stays valid)
// takes 32 KiB groups of 128-byte lines, as the single-array path does for
// its small late regions.  There the regions are small and a group is bound
// by latency, so more, shorter groups keep more of them in flight.
BatchClasses batched_tail_classes(const BatchClasses &BC, int w)
{
    BatchClasses T = BC;
    for (uint32_t c = 0; c < T.n; c++) {
        T.log2b[c] = (uint32_t)ilog2(128u / (uint32_t)w);
        T.s_max[c] = kTailGroupBytes / 128u;
    }
    return T;
}

int batched_core(char *base, int dtype, const Resolved &R, const BatchClasses &BC, BatchState &B, uint32_t levels,
                 hipStream_t st, uint64_t *d_splits, uint32_t *launches, const BatchClasses *tailC)
{
    hipError_t e;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess)
        return fail_device(e, "hipGetDevice");
    int cus = 0, lds = 0;
    int rc = device_info(dev, &cus, &lds);
    if (rc)
        return rc;
    const uint32_t engine = R.engine == SS_ENGINE_LDS ? (uint32_t)SS_ENGINE_LDS : (uint32_t)SS_ENGINE_REGS;
    const uint32_t tile = R.tile ? R.tile : 131072u;
    const BVariant *V = pick_bvariant(dtype, engine, tile);
    if (!V)
        return fail_msg(SS_EUNSUPPORTED, "no batched kernel variant for dtype/tile");
    int occ = 0;
    if ((rc = occupancy(dev, V->fn(), V->nt, &occ)))
        return rc;
    const uint32_t P = (uint32_t)(occ * cus);
    for (uint32_t c = 0; c < BC.n; c++)
        if (((uint64_t)BC.s_max[c] << BC.log2b[c]) * R.w > tile || !BC.s_max[c])
            return fail_msg(SS_EINVAL, "size class geometry exceeds the batched kernel's tile");
    // Levels from the second on with the tail geometry (tailC): its own kernel
    // variant of 32 KiB groups.
    const BVariant *Vt = tailC ? pick_bvariant(dtype, SS_ENGINE_REGS, kTailGroupBytes) : nullptr;
    uint32_t Pt = 0;
    if (tailC) {
        if (!Vt)
            return fail_msg(SS_EUNSUPPORTED, "no batched tail kernel variant");
        if ((rc = occupancy(dev, Vt->fn(), Vt->nt, &occ)))
            return rc;
        Pt = (uint32_t)(occ * cus);
    }
    BatchGeom Gm;
    Gm.base = base;
    Gm.seed = R.seed;
    Gm.level = 0;
    Gm.C = BC;
    // per-array kernels loop over the arrays; their grids are capped
    const uint32_t nb256 = std::min<uint32_t>((B.num + 255) / 256, 1024u),
                   nb4 = std::min<uint32_t>((B.num + 3) / 4, 2048u);
    if (levels < 1)
        levels = 1;
    // (the LDS-tile kernel keeps its table small: its occupancy is bound by LDS)
    Gm.search = B.num < (engine == SS_ENGINE_LDS ? 1024u : tile == 131072u ? kSearchMaxBig : kSearchMaxSmall);
    const bool search0 = Gm.search;
    for (uint32_t level = 0; level < levels; level++) {
        Gm.level = level;
        const bool tail = tailC && level >= 1;
        if (tail) {
            Gm.C = *tailC;
            Gm.search = B.num < kSearchMaxSmall;
        } else {
            Gm.search = search0;
        }
        if (level == 0)
            hipLaunchKernelGGL(k_binit, dim3(nb256), dim3(256), 0, st, B, Gm);
        else
            hipLaunchKernelGGL(k_bstep, dim3(nb4), dim3(256), 0, st, B, Gm);
        hipLaunchKernelGGL(k_bscan, dim3(1), dim3(kScanNT), 0, st, B);
        *launches += 2;
        if (!Gm.search) {
            hipLaunchKernelGGL(k_bfill, dim3(nb4), dim3(256), 0, st, B);
            (*launches)++;
        }
        if ((e = tail ? Vt->launch(Pt, B, Gm, st) : V->launch(P, B, Gm, st)) != hipSuccess)
            return fail_device(e, "batched level launch");
        (*launches)++;
    }
    Gm.level = levels;
    hipLaunchKernelGGL(k_bstep, dim3(nb4), dim3(256), 0, st, B, Gm);
    const uint32_t ncl = B.num < (uint32_t)cus ? B.num : (uint32_t)cus;  // open arrays are rare: one pass per CU
    switch (dtype) {
    case SS_U32: hipLaunchKernelGGL(k_bcleanup<uint32_t>, dim3(ncl), dim3(1024), 0, st, B, Gm); break;
    case SS_U64: hipLaunchKernelGGL(k_bcleanup<uint64_t>, dim3(ncl), dim3(1024), 0, st, B, Gm); break;
    default: hipLaunchKernelGGL(k_bcleanup<KV>, dim3(ncl), dim3(1024), 0, st, B, Gm); break;
    }
    (*launches)++;
    if (d_splits) {
        hipLaunchKernelGGL(k_bfinish, dim3(nb256), dim3(256), 0, st, B, d_splits);
        (*launches)++;
    }
    if ((e = hipGetLastError()) != hipSuccess)
        return fail_device(e, "batched launch");
    return SS_OK;
}

int batched_state(int dev, void *stream, uint32_t num, uint64_t items_cap, BatchState *B, uint64_t **host_stage,
                  hipEvent_t *stage_copied)
{
    std::lock_guard<std::mutex> lk(g_b_mu);
    BatchWork &w = g_b[std::make_pair(dev, stream)];
    const size_t words = 8 + (size_t)num * 6 + (num + 1) + items_cap + (items_cap + 1) / 2 + (size_t)(num + 1) / 2 +
                         (size_t)num / 8 + 1 + 16;
    const size_t bytes = words * sizeof(uint64_t);
    hipError_t e;
    if (w.dev_bytes < bytes) {
        if (w.dev) {
            batched_graphs_forget(w.dev);
            (void)hipFree(w.dev);  // synchronizes the device: no earlier call still uses it
        }
        w.dev = nullptr;
        w.dev_bytes = 0;
        if ((e = hipMalloc((void **)&w.dev, bytes)) != hipSuccess) {
            (void)hipGetLastError();
            return fail_msg(SS_ENOMEM, std::string("batched state hipMalloc: ") + hipGetErrorString(e));
        }
        w.dev_bytes = bytes;
    }
    for (auto &ev : w.copied)
        if (!ev && (e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
            return fail_device(e, "hipEventCreate");
    const size_t hwords = 2 * (size_t)num + 2;
    if (w.host_words < hwords) {
        for (int k = 0; k < 2; k++) {
            if (w.host[k]) {
                if ((e = hipEventSynchronize(w.copied[k])) != hipSuccess)  // its last copy has been read
                    return fail_device(e, "hipEventSynchronize");
                (void)hipHostFree(w.host[k]);
            }
            w.host[k] = nullptr;
        }
        w.host_words = 0;
        for (int k = 0; k < 2; k++)
            if ((e = hipHostMalloc((void **)&w.host[k], hwords * sizeof(uint64_t), hipHostMallocDefault)) !=
                hipSuccess) {
                (void)hipGetLastError();
                return fail_msg(SS_ENOMEM, std::string("batched staging hipHostMalloc: ") + hipGetErrorString(e));
            }
        w.host_words = hwords;
    }
    const uint32_t k = w.next;
    w.next ^= 1u;
    // the copy issued from this buffer two calls ago must have been read
    if ((e = hipEventSynchronize(w.copied[k])) != hipSuccess)
        return fail_device(e, "hipEventSynchronize");
    *host_stage = w.host[k];
    *stage_copied = w.copied[k];
    uint64_t *p = reinterpret_cast<uint64_t *>(w.dev);
    B->ctl = p;
    p += 8;
    B->start = p;
    p += num;
    B->len = p;
    p += num;
    B->lo = p;
    p += num;
    B->hi = p;
    p += num;
    B->split = p;
    p += num;
    B->first = p;
    p += num + 1;
    B->vout = p;
    p += items_cap;
    B->g = reinterpret_cast<uint32_t *>(p);
    p += (num + 1) / 2 + 1;
    B->imap = reinterpret_cast<uint32_t *>(p);
    p += (items_cap + 1) / 2;
    B->cls = reinterpret_cast<uint8_t *>(p);
    B->count = nullptr;
    B->num = num;
    return SS_OK;
}

uint64_t batched_items_cap(const uint64_t *lens, uint32_t num, uint64_t tile_elems)
{
    uint64_t cap = 64;
    for (uint32_t k = 0; k < num; k++)
        cap += lens[k] / tile_elems + 3;
    return cap;
}

// ------------------------------------------------------------ graph replay

// The level chain of a batched call is a fixed sequence of kernel launches
// whose arguments depend only on the buffers and the batch shape, so it is
// captured once into a HIP graph (on a private stream; the legacy default
// stream cannot be captured) and replayed with one hipGraphLaunch whenever
// the same (stream, buffers, shape) recurs.  The graph holds kernel nodes
// only; the descriptor upload stays outside it.
namespace {

struct GraphKey {
    int dev;
    void *stream;
    const void *base, *pivots, *splits, *state;
    int dtype;
    uint32_t num, levels, tile, engine, flags;
    uint64_t items_cap, seed, classes;  // classes: hash of the size-class table baked into the arguments
    bool operator<(const GraphKey &o) const
    {
        return std::tie(dev, stream, base, pivots, splits, state, dtype, num, levels, tile, engine, flags, items_cap,
                        seed, classes) < std::tie(o.dev, o.stream, o.base, o.pivots, o.splits, o.state, o.dtype,
                                                  o.num, o.levels, o.tile, o.engine, o.flags, o.items_cap, o.seed,
                                                  o.classes);
    }
};

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    uint32_t launches = 0;
    uint64_t last_use = 0;
};

std::mutex g_gr_mu;
std::map<GraphKey, GraphEntry> g_graphs;
std::map<int, hipStream_t> g_capture_stream;
uint64_t g_graph_clock = 0;
constexpr size_t kMaxGraphs = 64;

}  // namespace

int batched_graph(int dev, char *base, int dtype, const Resolved &R, const BatchClasses &BC, BatchState &B,
                  uint64_t items_cap, uint32_t levels, hipStream_t st, uint64_t *d_splits, uint32_t *launches,
                  const BatchClasses *tailC)
{
    std::lock_guard<std::mutex> lk(g_gr_mu);
    // The engine picks the kernel bodies and the class table is baked into the
    // kernel arguments: both are part of the key (the table as an FNV-1a hash).
    uint64_t h = 1469598103934665603ull;
    const unsigned char *cb = reinterpret_cast<const unsigned char *>(&BC);
    for (size_t j = 0; j < sizeof(BC); j++)
        h = (h ^ cb[j]) * 1099511628211ull;
    h = (h ^ (tailC ? 1u : 0u)) * 1099511628211ull;  // the tail geometry changes the kernels of later levels
    GraphKey key{dev, (void *)st, base, B.pivot, d_splits, B.ctl, dtype, B.num, levels, R.tile, R.engine,
                 R.flags & ~(uint32_t)SS_FLAG_TIME, items_cap, R.seed, h};
    hipError_t e;
    auto it = g_graphs.find(key);
    if (it == g_graphs.end()) {
        hipStream_t &cs = g_capture_stream[dev];
        if (!cs && (e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess)
            return fail_device(e, "hipStreamCreateWithFlags");
        if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return fail_device(e, "hipStreamBeginCapture");
        uint32_t n_launch = 0;
        const int rc = batched_core(base, dtype, R, BC, B, levels, cs, d_splits, &n_launch, tailC);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cs, &graph);
        if (rc) {
            if (graph)
                (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess)
            return fail_device(e, "hipStreamEndCapture");
        GraphEntry ge;
        ge.launches = n_launch;
        e = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess)
            return fail_device(e, "hipGraphInstantiate");
        if (g_graphs.size() >= kMaxGraphs) {
            auto old = g_graphs.begin();
            for (auto j = g_graphs.begin(); j != g_graphs.end(); ++j)
                if (j->second.last_use < old->second.last_use)
                    old = j;
            (void)hipGraphExecDestroy(old->second.exec);
            g_graphs.erase(old);
        }
        it = g_graphs.emplace(key, ge).first;
    }
    it->second.last_use = ++g_graph_clock;
    if ((e = hipGraphLaunch(it->second.exec, st)) != hipSuccess)
        return fail_device(e, "hipGraphLaunch");
    *launches += it->second.launches;
    return SS_OK;
}

// Drop cached graphs that refer to a batched workspace about to be freed.
void batched_graphs_forget(const void *state)
{
    std::lock_guard<std::mutex> lk(g_gr_mu);
    for (auto j = g_graphs.begin(); j != g_graphs.end();) {
        if (j->first.state == state) {
            (void)hipGraphExecDestroy(j->second.exec);
            j = g_graphs.erase(j);
        } else {
            ++j;
        }
    }
}

// Batched partition of segments [starts[k], starts[k] + lens[k]) of d_base
// given on the host; shared by both batched entry points.
static int batched_segments(void *d_base, const uint64_t *starts, const uint64_t *lens, size_t num, int dtype,
                            const uint64_t *d_pivots, uint64_t *d_splits, const ss_params *p, void *stream,
                            ss_stats *stats)
{
    if (((uintptr_t)d_splits % 8) || ((uintptr_t)d_pivots % 8))
        return fail_msg(SS_EINVAL, "pivots and splits must be 8-byte aligned");
    Resolved R;
    int rc = resolve_params(p, dtype, &R, batched_auto_engine(dtype));
    if (rc)
        return rc;
    if (R.algo != SS_SMOOTHED)
        return fail_msg(SS_EUNSUPPORTED, "batched partition uses Smoothed Striding");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess)
        return fail_device(e, "hipGetDevice");
    // size classes: the installed tuning, measured on the register body, for calls
    // that use the register body (the default except for 4-byte keys, whose LDS
    // body is faster than any register geometry) and leave the geometry open
    BatchClasses BC = batched_default_classes(R);
    const uint32_t want_engine = p && p->engine ? p->engine : batched_auto_engine(dtype);
    if (!(p && (p->b || p->tile_bytes)) && want_engine == SS_ENGINE_REGS && batched_has_tuning(dev, dtype)) {
        Resolved Rr;
        if ((rc = resolve_params(p, dtype, &Rr, SS_ENGINE_REGS)))
            return rc;
        R = Rr;
        BC = batched_default_classes(R);
        batched_installed_classes(dev, dtype, R, &BC);
    }
    // Levels from the second on take the tail geometry (32 KiB groups of
    // 128-byte lines) on the 128 KiB register body: a batch's arrays are
    // mostly short, their middle regions after the first level hold a few
    // hundred elements, and a level over them is bound by the latency of its
    // groups.  The choice depends only on the parameters, never on the batch,
    // so an array's bytes stay the same alone and in any batch.
    const BatchClasses TC = batched_tail_classes(BC, R.w);
    const bool use_tail = R.engine == SS_ENGINE_REGS && R.tile == 131072u;
    // Items (groups) per array at any level: at most len / (group elements) + 3.
    uint64_t max_len[kMaxClasses] = {0};
    uint64_t items_cap = 64, items_tail = 64;
    for (size_t k = 0; k < num; k++) {
        if ((rc = check_lines(lens[k], R)))
            return rc;
        uint32_t c = 0;
        while (c + 1 < BC.n && lens[k] > BC.max_len[c])
            c++;
        max_len[c] = lens[k] > max_len[c] ? lens[k] : max_len[c];
        const uint64_t S0 = (uint64_t)BC.s_max[c] << BC.log2b[c];
        items_cap += lens[k] / S0 + 3;
        items_tail += lens[k] / ((uint64_t)TC.s_max[c] << TC.log2b[c]) + 3;
    }
    if (use_tail && items_tail > items_cap)
        items_cap = items_tail;
    uint32_t levels = 1;
    for (uint32_t c = 0; c < BC.n; c++) {
        const uint64_t S0 = (uint64_t)BC.s_max[c] << BC.log2b[c];
        const uint32_t lv = use_tail ? batched_planned_levels(max_len[c], S0, R.w) : batched_levels(max_len[c], S0);
        levels = lv > levels ? lv : levels;
    }
    if (p && p->max_levels)
        levels = R.levels;
    BatchState B;
    uint64_t *stage = nullptr;
    hipEvent_t stage_copied = nullptr;
    if ((rc = batched_state(dev, stream, (uint32_t)num, items_cap, &B, &stage, &stage_copied)))
        return rc;
    B.pivot = d_pivots;
    std::memcpy(stage, starts, num * sizeof(uint64_t));
    std::memcpy(stage + num, lens, num * sizeof(uint64_t));
    if ((e = hipMemcpyAsync(B.start, stage, 2 * num * sizeof(uint64_t), hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipEventRecord(stage_copied, st)) != hipSuccess)
        return fail_device(e, "hipMemcpyAsync");
    RunOut ro;
    std::memset(&ro, 0, sizeof(ro));
    hipEvent_t t0 = nullptr, t1 = nullptr;
    const bool timing = (R.flags & SS_FLAG_TIME) != 0;
    if (timing) {
        if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
            return fail_msg(SS_EDEVICE, "hipEventCreate");
        (void)hipEventRecord(t0, st);
    }
    const BatchClasses *tc = use_tail ? &TC : nullptr;
    if (R.flags & SS_FLAG_GRAPH)
        rc = batched_graph(dev, (char *)d_base, dtype, R, BC, B, items_cap, levels, st, d_splits, &ro.launches, tc);
    else
        rc = batched_core((char *)d_base, dtype, R, BC, B, levels, st, d_splits, &ro.launches, tc);
    if (rc)
        return rc;
    if (timing) {
        (void)hipEventRecord(t1, st);
        (void)hipEventSynchronize(t1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, t0, t1);
        ro.total_ms = ms;
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
    }
    if (stats) {
        if ((e = hipStreamSynchronize(st)) != hipSuccess)
            return fail_device(e, "hipStreamSynchronize");
        fill_stats(stats, ro, R, dtype);
        stats->levels = levels;
        std::lock_guard<std::mutex> lk(g_b_mu);
        stats->aux_bytes = g_b[std::make_pair(dev, stream)].dev_bytes;
    }
    return SS_OK;
}

// ------------------------------------------------------------ size classes

namespace {

std::mutex g_tune_mu;
std::map<std::pair<int, int>, BatchClasses> g_tuned;  // (device, dtype)

static_assert(sizeof(ss_batched_tuning) == 168, "ss_batched_tuning layout");

int classes_from_table(const ss_batched_tuning *t, int w, BatchClasses *C)
{
    if (!t || t->nclass < 1 || t->nclass > (uint32_t)kMaxClasses || kMaxClasses != SS_MAX_CLASSES)
        return fail_msg(SS_EINVAL, "tuning table: nclass out of range");
    std::memset(C, 0, sizeof(*C));
    C->n = t->nclass;
    for (uint32_t c = 0; c < t->nclass; c++) {
        const uint64_t b = t->b[c], line = b * (uint64_t)w, grp = t->group_bytes[c];
        if (!b || (b & (b - 1)) || line < 64 || line > 4096)
            return fail_msg(SS_EINVAL, "tuning table: b * element size must be a power of two in [64, 4096]");
        if (grp < line || grp > 131072u || grp % line)
            return fail_msg(SS_EINVAL, "tuning table: group_bytes must be a multiple of the line, at most 128 KiB");
        if (c && t->max_len[c] < t->max_len[c - 1])
            return fail_msg(SS_EINVAL, "tuning table: max_len must be non-decreasing");
        C->log2b[c] = (uint32_t)ilog2(b);
        C->s_max[c] = (uint32_t)(grp / line);
        C->max_len[c] = c + 1 == t->nclass ? ~0ull : t->max_len[c];
    }
    return SS_OK;
}

void table_from_classes(const BatchClasses &C, int w, ss_batched_tuning *t)
{
    std::memset(t, 0, sizeof(*t));
    t->nclass = C.n;
    for (uint32_t c = 0; c < C.n; c++) {
        t->b[c] = 1u << C.log2b[c];
        t->group_bytes[c] = (uint32_t)(((uint64_t)C.s_max[c] << C.log2b[c]) * (uint64_t)w);
        t->max_len[c] = C.max_len[c];
    }
}

// A synthetic batch for one length class: keys from a SplitMix64 stream,
// lengths log-uniform in (lo, hi], pivots at uniform quantiles of the key
// range.
__global__ void __launch_bounds__(256) k_tune_fill(char *base, uint64_t n, int w, uint64_t seed)
{
    for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
        const uint64_t z = splitmix64_at(seed, i);
        if (w == 4)
            reinterpret_cast<uint32_t *>(base)[i] = (uint32_t)(z >> 32);
        else if (w == 8)
            reinterpret_cast<uint64_t *>(base)[i] = z;
        else {
            reinterpret_cast<uint64_t *>(base)[2 * i] = z;
            reinterpret_cast<uint64_t *>(base)[2 * i + 1] = i;
        }
    }
}

}  // namespace

bool batched_has_tuning(int dev, int dtype)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tuned.count(std::make_pair(dev, dtype)) != 0;
}

// Default group body of the batched calls: 4-byte keys go through an LDS tile
// (32 KiB groups; measured 24% faster than the register body on 20000 u32
// arrays, whose four 4-byte scattered stores per vector cost more than the
// staging), wider keys stay in registers with 128 KiB groups.
uint32_t batched_auto_engine(int dtype)
{
    return dtype == SS_U32 ? (uint32_t)SS_ENGINE_LDS : (uint32_t)SS_ENGINE_REGS;
}

void batched_installed_classes(int dev, int dtype, const Resolved &R, BatchClasses *C)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(std::make_pair(dev, dtype));
    if (it == g_tuned.end())
        return;
    for (uint32_t c = 0; c < it->second.n; c++)
        if (((uint64_t)it->second.s_max[c] << it->second.log2b[c]) * R.w > R.tile)
            return;  // the call's kernel tile is smaller than a tuned group
    *C = it->second;
}

constexpr float kTuneMargin = 0.97f;  // a candidate must be 3% faster than the default geometry

static int autotune(int dtype, hipStream_t st, ss_batched_tuning *out)
{
    const int w = elem_size(dtype);
    hipError_t e;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess)
        return fail_device(e, "hipGetDevice");
    Resolved R;
    int rc = resolve_params(nullptr, dtype, &R);
    if (rc)
        return rc;
    constexpr uint32_t NC = 7;
    const uint64_t bound[NC] = {1ull << 10, 1ull << 12, 1ull << 14, 1ull << 16, 1ull << 18, 1ull << 20, 1ull << 22};
    const uint64_t lower[NC] = {1ull << 8, 1ull << 10, 1ull << 12, 1ull << 14, 1ull << 16, 1ull << 18, 1ull << 20};
    const uint64_t total_target = 1ull << 24;
    const uint32_t lines[4] = {128, 256, 512, 1024};
    const uint32_t groups[3] = {32768, 65536, 131072};
    // scratch: the batch, a pristine copy, pivots, splits
    const size_t data_bytes = (size_t)(total_target + bound[NC - 1]) * w;
    const size_t max_arrays = total_target / lower[0] + 2;
    char *scratch = nullptr;
    if ((e = hipMalloc((void **)&scratch, 2 * data_bytes + 2 * max_arrays * sizeof(uint64_t))) != hipSuccess) {
        (void)hipGetLastError();
        return fail_msg(SS_ENOMEM, std::string("autotune scratch: ") + hipGetErrorString(e));
    }
    char *data = scratch, *pristine = scratch + data_bytes;
    uint64_t *d_piv = reinterpret_cast<uint64_t *>(scratch + 2 * data_bytes);
    uint64_t *d_split = d_piv + max_arrays;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipFree(scratch);
        return fail_msg(SS_EDEVICE, "hipEventCreate");
    }
    ss_batched_tuning T;
    std::memset(&T, 0, sizeof(T));
    T.nclass = NC;
    std::vector<uint64_t> starts, lens, piv;
    for (uint32_t c = 0; c < NC && rc == SS_OK; c++) {
        // lengths: log-uniform in (lower, bound], from a counter-based stream
        starts.clear();
        lens.clear();
        piv.clear();
        uint64_t total = 0, cnt = 0;
        const double l0 = std::log2((double)lower[c]), l1 = std::log2((double)bound[c]);
        while (total < total_target || cnt == 0) {
            const uint64_t z = splitmix64_at(0x7A11 + c, cnt);
            const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
            uint64_t l = (uint64_t)std::exp2(l0 + (l1 - l0) * u);
            l = l <= lower[c] ? lower[c] + 1 : l > bound[c] ? bound[c] : l;
            const double q = 0.05 + 0.9 * (double)(splitmix64_at(0x9A11 + c, cnt) >> 11) * (1.0 / 9007199254740992.0);
            starts.push_back(total);
            lens.push_back(l);
            piv.push_back(w == 4 ? (uint64_t)(q * 4294967296.0) : (uint64_t)(q * 18446744073709551615.0));
            total += l;
            cnt++;
        }
        const uint32_t num = (uint32_t)cnt;
        if ((e = hipMemcpyAsync(d_piv, piv.data(), num * sizeof(uint64_t), hipMemcpyHostToDevice, st)) != hipSuccess) {
            rc = fail_device(e, "hipMemcpyAsync");
            break;
        }
        hipLaunchKernelGGL(k_tune_fill, dim3(1024), dim3(256), 0, st, pristine, total, w, 0x5EED0000ull + c);
        const uint64_t items_cap = batched_items_cap(lens.data(), num, 32768 / w);
        float best = 1e30f, t_default = 1e30f;
        uint32_t best_line = 512, best_group = 131072;
        const uint32_t def_line = kDefaultLineBytes, def_group = R.tile;
        for (uint32_t li = 0; li < 4 && rc == SS_OK; li++) {
            for (uint32_t gi = 0; gi < 3 && rc == SS_OK; gi++) {
                const uint32_t line = lines[li], grp = groups[gi];
                if (line < (uint32_t)w || line < 64)
                    continue;
                BatchClasses BC;
                std::memset(&BC, 0, sizeof(BC));
                BC.n = 1;
                BC.max_len[0] = ~0ull;
                BC.log2b[0] = (uint32_t)ilog2(line / w);
                BC.s_max[0] = grp / line;
                const uint32_t levels = batched_levels(bound[c], grp / w);
                float t_best = 1e30f;
                for (int rep = 0; rep < 3 && rc == SS_OK; rep++) {
                    BatchState B;
                    uint64_t *stage = nullptr;
                    hipEvent_t stage_copied = nullptr;
                    if ((rc = batched_state(dev, st, num, items_cap, &B, &stage, &stage_copied)))
                        break;
                    B.pivot = d_piv;
                    std::memcpy(stage, starts.data(), num * sizeof(uint64_t));
                    std::memcpy(stage + num, lens.data(), num * sizeof(uint64_t));
                    if ((e = hipMemcpyAsync(B.start, stage, 2 * (size_t)num * sizeof(uint64_t),
                                            hipMemcpyHostToDevice, st)) != hipSuccess ||
                        (e = hipEventRecord(stage_copied, st)) != hipSuccess ||
                        (e = hipMemcpyAsync(data, pristine, (size_t)total * w, hipMemcpyDeviceToDevice, st)) !=
                            hipSuccess) {
                        rc = fail_device(e, "hipMemcpyAsync");
                        break;
                    }
                    uint32_t launches = 0;
                    (void)hipEventRecord(e0, st);
                    if ((rc = batched_core(data, dtype, R, BC, B, levels, st, d_split, &launches)))
                        break;
                    (void)hipEventRecord(e1, st);
                    if ((e = hipEventSynchronize(e1)) != hipSuccess) {
                        rc = fail_device(e, "hipEventSynchronize");
                        break;
                    }
                    float ms = 0;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    t_best = ms < t_best ? ms : t_best;
                }
                if (line == def_line && grp == def_group)
                    t_default = t_best;
                if (t_best < best) {
                    best = t_best;
                    best_line = line;
                    best_group = grp;
                }
            }
        }
        // Keep the default geometry unless a candidate beats it clearly: the
        // candidates' times differ by little more than run-to-run noise near
        // the optimum, and a noisy pick cost the joint batch 1-4%.
        if (t_default < 1e30f && !(best < kTuneMargin * t_default)) {
            best = t_default;
            best_line = def_line;
            best_group = def_group;
        }
        T.b[c] = best_line / w;
        T.group_bytes[c] = best_group;
        T.max_len[c] = c + 1 == NC ? ~0ull : bound[c];
        T.ms[c] = best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    (void)hipFree(scratch);
    if (rc)
        return rc;
    BatchClasses C;
    if ((rc = classes_from_table(&T, w, &C)))
        return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[std::make_pair(dev, dtype)] = C;
    }
    if (out)
        *out = T;
    return SS_OK;
}

}  // namespace ss

using namespace ss;

extern "C" int ss_autotune_batched(int dtype, void *stream, ss_batched_tuning *out)
{
    if (!elem_size(dtype))
        return fail_msg(SS_EINVAL, "unknown dtype");
    return autotune(dtype, (hipStream_t)stream, out);
}

extern "C" int ss_set_batched_tuning(int dtype, const ss_batched_tuning *t)
{
    const int w = elem_size(dtype);
    if (!w)
        return fail_msg(SS_EINVAL, "unknown dtype");
    int dev = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess)
        return fail_device(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!t) {
        g_tuned.erase(std::make_pair(dev, dtype));
        return SS_OK;
    }
    BatchClasses C;
    const int rc = classes_from_table(t, w, &C);
    if (rc)
        return rc;
    g_tuned[std::make_pair(dev, dtype)] = C;
    return SS_OK;
}

extern "C" int ss_get_batched_tuning(int dtype, ss_batched_tuning *t)
{
    const int w = elem_size(dtype);
    if (!w || !t)
        return fail_msg(SS_EINVAL, "unknown dtype or null table");
    int dev = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess)
        return fail_device(e, "hipGetDevice");
    Resolved R;
    int rc = resolve_params(nullptr, dtype, &R);
    if (rc)
        return rc;
    BatchClasses C = batched_default_classes(R);
    batched_installed_classes(dev, dtype, R, &C);
    table_from_classes(C, w, t);
    return SS_OK;
}

extern "C" int ss_partition_batched(void *d_base, const uint64_t *h_offsets, size_t num, int dtype,
                                    const uint64_t *d_pivots, uint64_t *d_splits, const ss_params *p,
                                    void *stream, ss_stats *stats)
{
    const int w = elem_size(dtype);
    if (!w)
        return fail_msg(SS_EINVAL, "unknown dtype");
    if (num == 0)
        return SS_OK;
    if (!h_offsets || !d_pivots || !d_splits)
        return fail_msg(SS_EINVAL, "null offsets, pivots or splits");
    if (num > (1u << 30))
        return fail_msg(SS_EINVAL, "too many arrays");
    for (size_t k = 0; k < num; k++)
        if (h_offsets[k + 1] < h_offsets[k])
            return fail_msg(SS_EINVAL, "offsets must be non-decreasing");
    int rc = check_array(d_base, (size_t)h_offsets[num], dtype);
    if (rc)
        return rc;
    std::vector<uint64_t> lens(num);
    for (size_t k = 0; k < num; k++)
        lens[k] = h_offsets[k + 1] - h_offsets[k];
    return batched_segments(d_base, h_offsets, lens.data(), num, dtype, d_pivots, d_splits, p, stream, stats);
}

extern "C" int ss_partition_segments(void *d_base, const uint64_t *h_starts, const uint64_t *h_lens, size_t num,
                                     int dtype, const uint64_t *d_pivots, uint64_t *d_splits, const ss_params *p,
                                     void *stream, ss_stats *stats)
{
    const int w = elem_size(dtype);
    if (!w)
        return fail_msg(SS_EINVAL, "unknown dtype");
    if (num == 0)
        return SS_OK;
    if (!h_starts || !h_lens || !d_pivots || !d_splits)
        return fail_msg(SS_EINVAL, "null starts, lengths, pivots or splits");
    if (num > (1u << 30))
        return fail_msg(SS_EINVAL, "too many segments");
    uint64_t end = 0;
    {
        // segments must be disjoint: check on a sorted copy of (start, end)
        std::vector<std::pair<uint64_t, uint64_t>> iv(num);
        for (size_t k = 0; k < num; k++) {
            if (h_starts[k] + h_lens[k] < h_starts[k])
                return fail_msg(SS_EINVAL, "segment overflows");
            iv[k] = std::make_pair(h_starts[k], h_starts[k] + h_lens[k]);
            end = iv[k].second > end ? iv[k].second : end;
        }
        std::sort(iv.begin(), iv.end());
        for (size_t k = 1; k < num; k++)
            if (iv[k].first < iv[k - 1].second && iv[k].second > iv[k].first && iv[k - 1].second > iv[k - 1].first)
                return fail_msg(SS_EINVAL, "segments overlap");
    }
    int rc = check_array(d_base, (size_t)end, dtype);
    if (rc)
        return rc;
    return batched_segments(d_base, h_starts, h_lens, num, dtype, d_pivots, d_splits, p, stream, stats);
}
