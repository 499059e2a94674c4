// ss_lowspace.hip -- the Low-Space Blocked-Prefix-Sum partition (Section 3,
// with the explicit block-count array of the Low-Space implementation in
// Section 5.1).  Comparator of the Smoothed Striding path.
//
// Steps (each a launch or a short chain of launches on one stream, with no
// host decision in between):
//   1. Count the predecessors while performing the top level of the
//      preprocessing phase (MakeSuccessorHeavy at m = n swaps A[x] and
//      A[n-1-x] when the first is a predecessor and the second a successor;
//      the rule is the same whichever role ends up being the majority, so
//      counting and this level share one pass, as Section 5.1 does).
//   2. If predecessors are the majority the roles are swapped and the array
//      is read logically reversed (Section 3, "ParallelPartition"): every
//      later kernel reads that decision from a device word.  The logical
//      array L satisfies #successors >= n/2.
//   3. The remaining preprocessing levels m = ceil(n/2), ceil(n/4), ...
//      (Lemma preprocessingphase): one launch per level while the level's
//      prefix is larger than an LDS buffer, then one workgroup finishes every
//      remaining level in LDS.
//   4. Block counts of B = 64 elements (one wavefront ballot per block) and
//      their exclusive prefix sums, stored explicitly (Section 5.1): per-block
//      local prefixes within a workgroup's 1024 blocks plus one prefix per
//      workgroup.
//   5. In-place reordering (Section 3, "In-Place Reordering"): the prefix is
//      cut repeatedly to its smallest block prefix holding more than 4/5 of
//      its elements; the innermost prefix (at most one LDS buffer) is
//      partitioned by one workgroup, then each tail, innermost first, swaps
//      its j-th predecessor with the element at the predecessor's global
//      rank, which lies in the already partitioned prefix's successor part.
//   6. split = #predecessors of L, mapped back through the reversal.
#include "ss_common.h"
#include "ss_device.h"
#include "ss_internal.h"

#include <cstring>
#include <mutex>
#include <map>
#include <vector>

namespace ss {

namespace ls {

constexpr int kBlock = 64;            // elements per block (one wavefront)
constexpr int kBlocksPerWg = 1024;    // blocks per workgroup of the counting pass
constexpr int kNT = 256;
constexpr int kSmallBytes = 65536;    // LDS buffer of the single-workgroup kernels

// Control words (device): [0] predecessor count c, [1] reversed flag,
// [2] #predecessors of L, [3] split.
struct Args {
    char *base;
    uint64_t n;
    uint64_t pivot;
    uint64_t *ctl;
    uint64_t *wg_part;    // per-workgroup partial counts of step 1
    uint32_t part_count;
    uint32_t *blk;        // per-block exclusive prefix within its workgroup's 1024 blocks
    uint64_t *wgsum;      // per-workgroup block totals, then their exclusive prefix
    uint64_t nwg;         // workgroups of the counting pass
    uint64_t m;           // preprocessing level size, or reorder prefix size
    uint64_t lo_blk, hi_blk;  // reorder tail blocks [lo_blk, hi_blk)
    uint64_t *d_split;
    uint64_t *host;       // mapped host memory for the result (nullable)
};

template <typename T>
__device__ __forceinline__ T *phys(const Args &a, bool rev, uint64_t x)
{
    return reinterpret_cast<T *>(a.base) + (rev ? a.n - 1 - x : x);
}

template <typename T>
__device__ __forceinline__ bool is_pred(const T &v, uint64_t pivot)
{
    return key_of(v) < pivot;
}

// Step 1: count predecessors and apply the top preprocessing level.
template <typename T>
__global__ void __launch_bounds__(kNT) k_count_top(Args a)
{
    __shared__ uint64_t red[kNT / 64];
    T *A = reinterpret_cast<T *>(a.base);
    const uint64_t half = a.n / 2;
    uint64_t c = 0;
    for (uint64_t x = (uint64_t)blockIdx.x * kNT + threadIdx.x; x < half; x += (uint64_t)gridDim.x * kNT) {
        const T u = A[x], v = A[a.n - 1 - x];
        const bool pu = is_pred(u, a.pivot), pv = is_pred(v, a.pivot);
        c += (uint64_t)pu + (uint64_t)pv;
        if (pu && !pv) {
            A[x] = v;
            A[a.n - 1 - x] = u;
        }
    }
    if ((a.n & 1) && blockIdx.x == 0 && threadIdx.x == 0)
        c += is_pred(A[half], a.pivot);
    for (int d = 32; d >= 1; d >>= 1)
        c += __shfl_xor(c, d, 64);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s = 0;
        for (int w = 0; w < kNT / 64; w++)
            s += red[w];
        a.wg_part[blockIdx.x] = s;
    }
}

// Sum of the step-1 partials; decide the roles.
__global__ void __launch_bounds__(kNT) k_decide(Args a)
{
    __shared__ uint64_t red[kNT / 64];
    uint64_t c = 0;
    for (uint32_t k = threadIdx.x; k < a.part_count; k += kNT)
        c += a.wg_part[k];
    for (int d = 32; d >= 1; d >>= 1)
        c += __shfl_xor(c, d, 64);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s = 0;
        for (int w = 0; w < kNT / 64; w++)
            s += red[w];
        a.ctl[0] = s;
        a.ctl[1] = 2 * s > a.n ? 1 : 0;  // predecessors are the majority: swap roles, reverse
        if (a.host) {
            a.host[0] = 0;
            a.host[1] = 0;
            a.host[2] = s;
            a.host[3] = a.ctl[1];
        }
    }
}

// Step 3: one preprocessing level on L[0, m).
template <typename T>
__global__ void __launch_bounds__(kNT) k_pre_level(Args a)
{
    const bool rev = a.ctl[1] != 0;
    const uint64_t half = a.m / 2;
    for (uint64_t x = (uint64_t)blockIdx.x * kNT + threadIdx.x; x < half; x += (uint64_t)gridDim.x * kNT) {
        T *pu = phys<T>(a, rev, x), *pv = phys<T>(a, rev, a.m - 1 - x);
        const T u = *pu, v = *pv;
        // logical decider: a predecessor of L is an original predecessor, or a successor when reversed
        if ((is_pred(u, a.pivot) != rev) && !(is_pred(v, a.pivot) != rev)) {
            *pu = v;
            *pv = u;
        }
    }
}

// Step 3, tail: every remaining level on L[0, m) in LDS (m * sizeof(T) <= kSmallBytes).
template <typename T>
__global__ void __launch_bounds__(1024) k_pre_small(Args a)
{
    constexpr int CAP = kSmallBytes / sizeof(T);
    __shared__ T buf[CAP];
    const bool rev = a.ctl[1] != 0;
    const uint32_t m0 = (uint32_t)a.m;
    for (uint32_t x = threadIdx.x; x < m0; x += 1024)
        buf[x] = *phys<T>(a, rev, x);
    __syncthreads();
    for (uint32_t m = m0; m >= 2; m = (m + 1) / 2) {
        for (uint32_t x = threadIdx.x; x < m / 2; x += 1024) {
            const T u = buf[x], v = buf[m - 1 - x];
            if ((is_pred(u, a.pivot) != rev) && !(is_pred(v, a.pivot) != rev)) {
                buf[x] = v;
                buf[m - 1 - x] = u;
            }
        }
        __syncthreads();
    }
    for (uint32_t x = threadIdx.x; x < m0; x += 1024)
        *phys<T>(a, rev, x) = buf[x];
}

// Step 4a: per-block predecessor counts of L and their exclusive prefix
// within this workgroup's kBlocksPerWg blocks; the workgroup total.
template <typename T>
__global__ void __launch_bounds__(kNT) k_block_counts(Args a)
{
    __shared__ uint32_t cnt[kBlocksPerWg];
    __shared__ uint32_t wsum[kNT / 64];
    const bool rev = a.ctl[1] != 0;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint64_t blk0 = (uint64_t)blockIdx.x * kBlocksPerWg;
    const uint64_t nblk = (a.n + kBlock - 1) / kBlock;
    for (uint32_t k = wid; k < (uint32_t)kBlocksPerWg; k += kNT / 64) {
        const uint64_t b = blk0 + k;
        bool p = false;
        if (b < nblk) {
            const uint64_t x = b * kBlock + lane;
            if (x < a.n)
                p = is_pred(*phys<T>(a, rev, x), a.pivot) != rev;
        }
        const uint32_t c = (uint32_t)__popcll(__ballot(p));
        if (lane == 0)
            cnt[k] = c;
    }
    __syncthreads();
    // exclusive scan of the 1024 counts: 4 per thread, then across threads
    constexpr int PER = kBlocksPerWg / kNT;
    uint32_t v[PER], s = 0;
    for (int k = 0; k < PER; k++) {
        v[k] = cnt[threadIdx.x * PER + k];
        s += v[k];
    }
    uint32_t inc = s;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d, 64);
        if (lane >= d)
            inc += y;
    }
    if (lane == 63)
        wsum[wid] = inc;
    __syncthreads();
    uint32_t off = 0;
    for (int w = 0; w < wid; w++)
        off += wsum[w];
    uint32_t run = off + inc - s;
    for (int k = 0; k < PER; k++) {
        const uint64_t b = blk0 + threadIdx.x * PER + k;
        if (b < nblk)
            a.blk[b] = run;
        run += v[k];
    }
    if (threadIdx.x == kNT - 1)
        a.wgsum[blockIdx.x] = run;
}

// Step 4b: exclusive prefix of the workgroup totals (one workgroup); the
// predecessor count of L and the split.
__global__ void __launch_bounds__(1024) k_scan_wg(Args a)
{
    __shared__ uint64_t wsum[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint64_t per = (a.nwg + 1023) / 1024;
    const uint64_t k0 = threadIdx.x * per;
    uint64_t s = 0;
    for (uint64_t k = k0; k < k0 + per && k < a.nwg; k++)
        s += a.wgsum[k];
    uint64_t inc = s;
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t y = __shfl_up(inc, d, 64);
        if (lane >= d)
            inc += y;
    }
    if (lane == 63)
        wsum[wid] = inc;
    __syncthreads();
    uint64_t off = 0;
    for (int w = 0; w < wid; w++)
        off += wsum[w];
    uint64_t run = off + inc - s;
    for (uint64_t k = k0; k < k0 + per && k < a.nwg; k++) {
        const uint64_t x = a.wgsum[k];
        a.wgsum[k] = run;
        run += x;
    }
    if (threadIdx.x == 1023) {
        const uint64_t cl = run;  // predecessors of L
        const bool rev = a.ctl[1] != 0;
        const uint64_t split = rev ? a.n - cl : cl;
        a.ctl[2] = cl;
        a.ctl[3] = split;
        if (a.d_split)
            *a.d_split = split;
        if (a.host) {
            a.host[0] = 1;
            a.host[1] = split;
            a.host[2] = a.ctl[0];
            a.host[3] = rev;
        }
    }
}

// Step 5, innermost prefix L[0, m): stable partition in LDS by one workgroup.
template <typename T>
__global__ void __launch_bounds__(1024) k_reorder_base(Args a)
{
    constexpr int CAP = kSmallBytes / sizeof(T);
    constexpr int K = CAP / 1024;
    __shared__ T buf[CAP];
    __shared__ uint32_t sh[K * 16 + 1];
    const bool rev = a.ctl[1] != 0;
    const uint32_t m = (uint32_t)a.m;
    T x[K];
    bool f[K];
    uint32_t rk[K], tot;
    for (int r = 0; r < K; r++) {
        const uint32_t k = r * 1024 + threadIdx.x;
        f[r] = false;
        if (k < m) {
            x[r] = *phys<T>(a, rev, k);
            f[r] = is_pred(x[r], a.pivot) != rev;
        }
    }
    block_rank<1024, K>(f, rk, tot, sh);
    for (int r = 0; r < K; r++) {
        const uint32_t k = r * 1024 + threadIdx.x;
        if (k < m)
            buf[f[r] ? rk[r] : tot + k - rk[r]] = x[r];
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < m; k += 1024)
        *phys<T>(a, rev, k) = buf[k];
}

// Step 5, one tail: blocks [lo_blk, hi_blk) of L.  Each wave owns one block at
// a time: its j-th predecessor (global rank r from the block prefix sums)
// swaps with L[r], a successor in the partitioned prefix.
template <typename T>
__global__ void __launch_bounds__(kNT) k_reorder_tail(Args a)
{
    const bool rev = a.ctl[1] != 0;
    const int lane = threadIdx.x & 63;
    const uint64_t waves = (uint64_t)gridDim.x * (kNT / 64);
    for (uint64_t b = a.lo_blk + (uint64_t)blockIdx.x * (kNT / 64) + (threadIdx.x >> 6); b < a.hi_blk; b += waves) {
        const uint64_t x = b * kBlock + lane;
        bool p = false;
        T v;
        if (x < a.n) {
            v = *phys<T>(a, rev, x);
            p = is_pred(v, a.pivot) != rev;
        }
        const uint64_t m = __ballot(p);
        const uint64_t r = a.wgsum[b / kBlocksPerWg] + a.blk[b] + lanes_below(m);
        if (p) {
            T *dst = phys<T>(a, rev, r);
            const T w = *dst;
            *dst = v;
            *phys<T>(a, rev, x) = w;
        }
    }
}

// ---------------------------------------------------------------------------
// The Medium- and High-Space comparators (Section 5.1): the standard parallel
// partition with an n-sized output array.  The predecessor counts of blocks
// of 64 elements and their prefix sums are formed as above (with the roles
// never swapped); every element is then written to its place in the output
// array -- predecessors to rank, successors to split + (index - rank), a
// stable partition -- and the output is copied back.  Medium-Space keeps only
// the block prefixes (n/64 words); High-Space first writes every element's
// prefix into an explicit n-word array, as the standard algorithm does.

__global__ void k_ps_init(Args a)
{
    if (blockIdx.x == 0 && threadIdx.x < 2)
        a.ctl[threadIdx.x] = 0;  // count unknown, roles not swapped
}

// Predecessors before this lane's element of block b (m: the block's ballot).
__device__ __forceinline__ uint64_t ps_before(const Args &a, uint64_t b, uint64_t m)
{
    return a.wgsum[b / kBlocksPerWg] + a.blk[b] + lanes_below(m);
}

template <typename T>
__global__ void __launch_bounds__(kNT) k_ps_scatter(Args a, T *out)
{
    const T *A = reinterpret_cast<const T *>(a.base);
    const int lane = threadIdx.x & 63;
    const uint64_t nblk = (a.n + kBlock - 1) / kBlock, split = a.ctl[3];
    const uint64_t waves = (uint64_t)gridDim.x * (kNT / 64);
    for (uint64_t b = (uint64_t)blockIdx.x * (kNT / 64) + (threadIdx.x >> 6); b < nblk; b += waves) {
        const uint64_t x = b * kBlock + lane;
        bool p = false;
        T v;
        if (x < a.n) {
            v = A[x];
            p = is_pred(v, a.pivot);
        }
        const uint64_t before = ps_before(a, b, __ballot(p));
        if (x < a.n)
            out[p ? before : split + x - before] = v;
    }
}

template <typename T>
__global__ void __launch_bounds__(kNT) k_ps_elem_prefix(Args a, uint64_t *B)
{
    const T *A = reinterpret_cast<const T *>(a.base);
    const int lane = threadIdx.x & 63;
    const uint64_t nblk = (a.n + kBlock - 1) / kBlock;
    const uint64_t waves = (uint64_t)gridDim.x * (kNT / 64);
    for (uint64_t b = (uint64_t)blockIdx.x * (kNT / 64) + (threadIdx.x >> 6); b < nblk; b += waves) {
        const uint64_t x = b * kBlock + lane;
        const bool p = x < a.n && is_pred(A[x], a.pivot);
        const uint64_t before = ps_before(a, b, __ballot(p));
        if (x < a.n)
            B[x] = before;
    }
}

template <typename T>
__global__ void __launch_bounds__(kNT) k_ps_scatter_explicit(Args a, const uint64_t *B, T *out)
{
    const T *A = reinterpret_cast<const T *>(a.base);
    const uint64_t split = a.ctl[3];
    for (uint64_t x = (uint64_t)blockIdx.x * kNT + threadIdx.x; x < a.n; x += (uint64_t)gridDim.x * kNT) {
        const T v = A[x];
        const uint64_t before = B[x];
        out[is_pred(v, a.pivot) ? before : split + x - before] = v;
    }
}

}  // namespace ls

namespace {

struct LsWork {
    uint64_t *ctl = nullptr;
    uint64_t *wg_part = nullptr;
    uint32_t *blk = nullptr;
    uint64_t *wgsum = nullptr;
    size_t cap_n = 0;
    size_t bytes = 0;
};
std::mutex g_ls_mu;
std::map<std::pair<int, void *>, LsWork> g_ls;

constexpr uint32_t kPartMax = 4096;

}  // namespace

size_t lowspace_aux_bytes(size_t n)
{
    const size_t nblk = (n + ls::kBlock - 1) / ls::kBlock;
    const size_t nwg = (nblk + ls::kBlocksPerWg - 1) / ls::kBlocksPerWg;
    return nblk * sizeof(uint32_t) + nwg * sizeof(uint64_t) + kPartMax * sizeof(uint64_t) + 8 * sizeof(uint64_t);
}

template <typename T>
static int lowspace_run(char *base, size_t n, uint64_t pivot, hipStream_t st, uint64_t *d_split, Workspace *ws,
                        LsWork &w, int cus, uint32_t *launches, bool pre_only)
{
    hipError_t e;
    ls::Args a;
    std::memset(&a, 0, sizeof(a));
    a.base = base;
    a.n = n;
    a.pivot = pivot;
    a.ctl = w.ctl;
    a.wg_part = w.wg_part;
    a.blk = w.blk;
    a.wgsum = w.wgsum;
    const uint64_t nblk = (n + ls::kBlock - 1) / ls::kBlock;
    a.nwg = (nblk + ls::kBlocksPerWg - 1) / ls::kBlocksPerWg;
    a.d_split = d_split;
    a.host = ws->host_dev;
    const uint64_t stream_grid = (uint64_t)cus * 8;
    auto grid_for = [&](uint64_t items) -> uint32_t {
        uint64_t g = (items + ls::kNT - 1) / ls::kNT;
        if (g > stream_grid)
            g = stream_grid;
        return (uint32_t)(g ? g : 1);
    };
    // 1-2. count with the top preprocessing level, decide the roles
    const uint32_t g1 = grid_for(n / 2) < kPartMax ? grid_for(n / 2) : kPartMax;
    a.part_count = g1;
    hipLaunchKernelGGL(ls::k_count_top<T>, dim3(g1), dim3(ls::kNT), 0, st, a);
    hipLaunchKernelGGL(ls::k_decide, dim3(1), dim3(ls::kNT), 0, st, a);
    *launches += 2;
    // 3. the other preprocessing levels
    const uint64_t small = ls::kSmallBytes / sizeof(T);
    uint64_t m = (n + 1) / 2;
    while (m >= 2 && m > small) {
        a.m = m;
        hipLaunchKernelGGL(ls::k_pre_level<T>, dim3(grid_for(m / 2)), dim3(ls::kNT), 0, st, a);
        (*launches)++;
        m = (m + 1) / 2;
    }
    if (m >= 2) {
        a.m = m;
        hipLaunchKernelGGL(ls::k_pre_small<T>, dim3(1), dim3(1024), 0, st, a);
        (*launches)++;
    }
    if (pre_only) {
        if ((e = hipGetLastError()) != hipSuccess)
            return fail_device(e, "Low-Space kernel launch");
        return SS_OK;
    }
    // 4. block counts and prefix sums
    hipLaunchKernelGGL(ls::k_block_counts<T>, dim3((uint32_t)a.nwg), dim3(ls::kNT), 0, st, a);
    hipLaunchKernelGGL(ls::k_scan_wg, dim3(1), dim3(1024), 0, st, a);
    *launches += 2;
    // 5. reorder: prefixes N_0 = n > N_1 > ... > N_K <= one LDS buffer
    std::vector<uint64_t> N{n};
    while (N.back() > small) {
        const uint64_t cur = N.back();
        const uint64_t t = (4 * cur / 5) / ls::kBlock + 1;  // least t with t * B > 4 cur / 5
        N.push_back(t * ls::kBlock);
    }
    a.m = N.back();
    hipLaunchKernelGGL(ls::k_reorder_base<T>, dim3(1), dim3(1024), 0, st, a);
    (*launches)++;
    for (size_t k = N.size() - 1; k-- > 0;) {
        a.lo_blk = N[k + 1] / ls::kBlock;
        a.hi_blk = (N[k] + ls::kBlock - 1) / ls::kBlock;
        const uint64_t waves_needed = a.hi_blk - a.lo_blk;
        uint64_t g = (waves_needed + (ls::kNT / 64) - 1) / (ls::kNT / 64);
        if (g > stream_grid)
            g = stream_grid;
        hipLaunchKernelGGL(ls::k_reorder_tail<T>, dim3((uint32_t)(g ? g : 1)), dim3(ls::kNT), 0, st, a);
        (*launches)++;
    }
    if ((e = hipGetLastError()) != hipSuccess)
        return fail_device(e, "Low-Space kernel launch");
    return SS_OK;
}

// The block-count arrays of a call on n elements, cached per (device, stream).
static int ls_work(int dev, hipStream_t st, size_t n, LsWork **out)
{
    hipError_t e;
    std::lock_guard<std::mutex> lk(g_ls_mu);
    LsWork *w = &g_ls[std::make_pair(dev, (void *)st)];
    if (w->cap_n < n) {
        if (w->ctl)
            (void)hipFree(w->ctl);
        *w = LsWork();
        const size_t nblk = (n + ls::kBlock - 1) / ls::kBlock;
        const size_t nwg = (nblk + ls::kBlocksPerWg - 1) / ls::kBlocksPerWg;
        const size_t bytes = 8 * sizeof(uint64_t) + kPartMax * sizeof(uint64_t) + nwg * sizeof(uint64_t) +
                             nblk * sizeof(uint32_t) + 256;
        char *p = nullptr;
        if ((e = hipMalloc((void **)&p, bytes)) != hipSuccess) {
            (void)hipGetLastError();
            return fail_msg(SS_ENOMEM, std::string("Low-Space aux hipMalloc: ") + hipGetErrorString(e));
        }
        w->ctl = reinterpret_cast<uint64_t *>(p);
        w->wg_part = w->ctl + 8;
        w->wgsum = w->wg_part + kPartMax;
        w->blk = reinterpret_cast<uint32_t *>(w->wgsum + nwg);
        w->cap_n = n;
        w->bytes = bytes;
    }
    *out = w;
    return SS_OK;
}

int lowspace_partition(char *base, size_t n, int dtype, uint64_t pivot, const Resolved &R, hipStream_t st,
                       uint64_t *d_split, size_t *h_split, ss_stats *stats)
{
    if (d_split && ((uintptr_t)d_split % 8))
        return fail_msg(SS_EINVAL, "d_split not 8-byte aligned");
    const bool sync = h_split || stats || (R.flags & SS_FLAG_TIME);
    hipError_t e;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess)
        return fail_device(e, "hipGetDevice");
    int cus = 0, lds = 0;
    int rc = device_info(dev, &cus, &lds);
    if (rc)
        return rc;
    Workspace *ws = nullptr;
    rc = get_workspace(dev, st, &ws);
    if (rc)
        return rc;
    LsWork *w = nullptr;
    if ((rc = ls_work(dev, st, n, &w)))
        return rc;
    RunOut ro;
    std::memset(&ro, 0, sizeof(ro));
    if (n == 0) {
        if (d_split && (e = hipMemsetAsync(d_split, 0, 8, st)) != hipSuccess)
            return fail_device(e, "hipMemsetAsync");
    } else {
        if ((R.flags & SS_FLAG_TIME) && (e = hipEventRecord(ws->ev[0], st)) != hipSuccess)
            return fail_device(e, "hipEventRecord");
        const bool pre_only = (R.flags & SS_FLAG_ONE_LEVEL) != 0;
        switch (dtype) {
        case SS_U32: rc = lowspace_run<uint32_t>(base, n, pivot, st, d_split, ws, *w, cus, &ro.launches, pre_only); break;
        case SS_U64: rc = lowspace_run<uint64_t>(base, n, pivot, st, d_split, ws, *w, cus, &ro.launches, pre_only); break;
        default: rc = lowspace_run<KV>(base, n, pivot, st, d_split, ws, *w, cus, &ro.launches, pre_only); break;
        }
        if (rc)
            return rc;
        if ((R.flags & SS_FLAG_TIME) && (e = hipEventRecord(ws->ev[1], st)) != hipSuccess)
            return fail_device(e, "hipEventRecord");
    }
    if (!sync)
        return SS_OK;
    if ((e = hipStreamSynchronize(st)) != hipSuccess)
        return fail_device(e, "hipStreamSynchronize");
    const volatile uint64_t *hres = ws->host;
    ro.split = n ? hres[1] : 0;
    ro.done = n ? hres[0] != 0 : true;
    const uint64_t pred_count = n ? hres[2] : 0, reversed = n ? hres[3] : 0;
    ro.aux_bytes = ws->bytes + lowspace_aux_bytes(n);
    if (R.flags & SS_FLAG_TIME && n) {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, ws->ev[0], ws->ev[1]);
        ro.first_level_ms = ms;
        ro.total_ms = ms;
    }
    if (h_split)
        *h_split = (size_t)ro.split;
    if (stats) {
        fill_stats(stats, ro, R, dtype);
        // Low-Space has no splitting positions: report the predecessor count
        // and whether the roles were swapped (the array read reversed).
        stats->vmin = pred_count;
        stats->vmax = reversed;
        stats->bytes_moved = 0;
    }
    return SS_OK;
}

}  // namespace ss

namespace ss {

namespace {

// The n-sized output array (and, for High-Space, the n-word prefix array) of
// the explicit-space comparators, cached per (device, stream).
struct PsWork {
    char *buf = nullptr;
    size_t bytes = 0;
};
std::mutex g_ps_mu;
std::map<std::pair<int, void *>, PsWork> g_ps;

template <typename T>
int prefix_run(char *base, size_t n, uint64_t pivot, hipStream_t st, uint64_t *d_split, Workspace *ws, LsWork &w,
               char *outbuf, uint64_t *prefix, int cus, uint32_t *launches)
{
    ls::Args a;
    std::memset(&a, 0, sizeof(a));
    a.base = base;
    a.n = n;
    a.pivot = pivot;
    a.ctl = w.ctl;
    a.blk = w.blk;
    a.wgsum = w.wgsum;
    const uint64_t nblk = (n + ls::kBlock - 1) / ls::kBlock;
    a.nwg = (nblk + ls::kBlocksPerWg - 1) / ls::kBlocksPerWg;
    a.d_split = d_split;
    a.host = ws->host_dev;
    const uint64_t waves_grid = std::min<uint64_t>((nblk + 3) / 4, (uint64_t)cus * 8);
    T *out = reinterpret_cast<T *>(outbuf);
    hipLaunchKernelGGL(ls::k_ps_init, dim3(1), dim3(64), 0, st, a);
    hipLaunchKernelGGL(ls::k_block_counts<T>, dim3((uint32_t)a.nwg), dim3(ls::kNT), 0, st, a);
    hipLaunchKernelGGL(ls::k_scan_wg, dim3(1), dim3(1024), 0, st, a);
    if (prefix) {
        hipLaunchKernelGGL(ls::k_ps_elem_prefix<T>, dim3((uint32_t)waves_grid), dim3(ls::kNT), 0, st, a, prefix);
        hipLaunchKernelGGL(ls::k_ps_scatter_explicit<T>, dim3((uint32_t)std::min<uint64_t>((n + 255) / 256, (uint64_t)cus * 8)),
                           dim3(ls::kNT), 0, st, a, (const uint64_t *)prefix, out);
        *launches += 5;
    } else {
        hipLaunchKernelGGL(ls::k_ps_scatter<T>, dim3((uint32_t)waves_grid), dim3(ls::kNT), 0, st, a, out);
        *launches += 4;
    }
    hipError_t e;
    if ((e = hipGetLastError()) != hipSuccess)
        return fail_device(e, "explicit-space kernel launch");
    if ((e = hipMemcpyAsync(base, outbuf, n * sizeof(T), hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return fail_device(e, "hipMemcpyAsync");
    return SS_OK;
}

}  // namespace

size_t prefix_aux_bytes(size_t n, int dtype, bool explicit_prefix)
{
    return lowspace_aux_bytes(n) + n * (size_t)elem_size(dtype) + (explicit_prefix ? n * sizeof(uint64_t) : 0);
}

// Medium-Space (explicit_prefix false) or High-Space (true) partition.
int prefix_partition(char *base, size_t n, int dtype, uint64_t pivot, const Resolved &R, hipStream_t st,
                     uint64_t *d_split, size_t *h_split, ss_stats *stats, bool explicit_prefix)
{
    if (d_split && ((uintptr_t)d_split % 8))
        return fail_msg(SS_EINVAL, "d_split not 8-byte aligned");
    const bool sync = h_split || stats || (R.flags & SS_FLAG_TIME);
    hipError_t e;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess)
        return fail_device(e, "hipGetDevice");
    int cus = 0, lds = 0;
    int rc = device_info(dev, &cus, &lds);
    if (rc)
        return rc;
    Workspace *ws = nullptr;
    if ((rc = get_workspace(dev, st, &ws)))
        return rc;
    LsWork *w = nullptr;
    if ((rc = ls_work(dev, st, n, &w)))
        return rc;
    const size_t need = n * (size_t)elem_size(dtype) + (explicit_prefix ? n * sizeof(uint64_t) : 0) + 256;
    char *buf = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_ps_mu);
        PsWork &pw = g_ps[std::make_pair(dev, (void *)st)];
        if (pw.bytes < need) {
            if (pw.buf)
                (void)hipFree(pw.buf);
            pw = PsWork();
            if ((e = hipMalloc((void **)&pw.buf, need)) != hipSuccess) {
                (void)hipGetLastError();
                return fail_msg(SS_ENOMEM, std::string("explicit-space output hipMalloc: ") + hipGetErrorString(e));
            }
            pw.bytes = need;
        }
        buf = pw.buf;
    }
    uint64_t *prefix = explicit_prefix
                           ? reinterpret_cast<uint64_t *>(buf + (n * (size_t)elem_size(dtype) + 255) / 256 * 256)
                           : nullptr;
    RunOut ro;
    std::memset(&ro, 0, sizeof(ro));
    if (n == 0) {
        const uint64_t zero = 0;
        if (d_split && (e = hipMemcpy(d_split, &zero, 8, hipMemcpyHostToDevice)) != hipSuccess)
            return fail_device(e, "hipMemcpy");
    } else {
        if ((R.flags & SS_FLAG_TIME) && (e = hipEventRecord(ws->ev[0], st)) != hipSuccess)
            return fail_device(e, "hipEventRecord");
        switch (dtype) {
        case SS_U32: rc = prefix_run<uint32_t>(base, n, pivot, st, d_split, ws, *w, buf, prefix, cus, &ro.launches); break;
        case SS_U64: rc = prefix_run<uint64_t>(base, n, pivot, st, d_split, ws, *w, buf, prefix, cus, &ro.launches); break;
        default: rc = prefix_run<KV>(base, n, pivot, st, d_split, ws, *w, buf, prefix, cus, &ro.launches); break;
        }
        if (rc)
            return rc;
        if ((R.flags & SS_FLAG_TIME) && (e = hipEventRecord(ws->ev[1], st)) != hipSuccess)
            return fail_device(e, "hipEventRecord");
    }
    if (!sync)
        return SS_OK;
    if ((e = hipStreamSynchronize(st)) != hipSuccess)
        return fail_device(e, "hipStreamSynchronize");
    const volatile uint64_t *hres = ws->host;
    ro.split = n ? hres[1] : 0;
    ro.done = true;
    ro.aux_bytes = ws->bytes + prefix_aux_bytes(n, dtype, explicit_prefix);
    if (R.flags & SS_FLAG_TIME && n) {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, ws->ev[0], ws->ev[1]);
        ro.first_level_ms = ms;
        ro.total_ms = ms;
    }
    if (h_split)
        *h_split = (size_t)ro.split;
    if (stats) {
        fill_stats(stats, ro, R, dtype);
        stats->vmin = ro.split;
        stats->vmax = ro.split;
        stats->bytes_moved = 0;
    }
    return SS_OK;
}

}  // namespace ss
