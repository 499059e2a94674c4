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
//   4. Block counts of B = 64 elements and their exclusive prefix sums,
//      stored explicitly (Section 5.1): per-block local prefixes within a
//      workgroup's 1024 blocks plus one prefix per workgroup.  The counts
//      cost no pass of their own: an element is final once the last
//      preprocessing level that touches it is done, so each level's pass
//      counts the part it leaves final, L[ceil(m/2), m) (the top level, run
//      before the roles are known, counts both halves, one for each reading
//      direction), and the LDS tail counts L[0, m).  Section 5.1 overlaps the
//      counting with the preprocessing in the same way.
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
    uint32_t whole;       // store whole vectors and blocks, changed or not (arrays far above the
                          // 256 MiB last-level cache, see kWholeLineBytes)
    uint32_t fuse;        // the preprocessing passes also count each 64-element block's
                          // predecessors (key < pivot) once its elements are final: into blk for
                          // the logical array read forward, into cntr for it read reversed
    uint32_t *cntr;
};

// Above this many bytes an array's passes store whole vectors and blocks, so
// that HBM sees whole lines: the top level at 2^30 u64 took 4.35 ms with only
// the changed vectors stored and 3.7 ms with all of them.  Smaller arrays
// (a Hybrid call's middle region) mostly stay in the 256 MiB Infinity Cache,
// which absorbs partial lines, and there the extra stores only cost time.
constexpr uint64_t kWholeLineBytes = 512ull << 20;

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

// The mirror pass of one preprocessing level on the logical array L[0, m):
// for x < floor(m/2), L[x] and L[m-1-x] swap when the first is a
// predecessor of L and the second a successor.  A thread takes 16-byte
// vectors, kMirrorU at a time (one load each from the front and the back
// before any is used): front vector t holds L[V t, V t + V), its partners
// are L[m - V t - V, m - V t) in reverse order.  Element e of a vector at
// physical element s is at s + e, or at s + V - 1 - e when the vector is
// read reversed.  The last floor(m/2) mod V pairs take a scalar path.
// With `count`, the original predecessors of the whole array are also
// counted (the top level, m = n, runs before the roles are known; its swap
// rule is the same under either role).
constexpr int kMirrorU = 4;

template <typename T>
union Vec16 {
    v4u v;
    T e[16 / sizeof(T)];
};

// Adds to C[b], for the blocks b of 64 logical elements that this wavefront's
// elements fall in, how many of them are predecessors (key < pivot).  Lane
// l holds V elements with block indices bi[e] and predecessor bits pm; the
// wavefront's 64 V elements are consecutive, so they span at most V + 1
// blocks: one ballot per (element, block) and one atomic per block.  Called
// by every lane of the wavefront.
template <int V>
__device__ __forceinline__ void wave_block_add(uint32_t *C, const uint64_t (&bi)[V], uint32_t pm, bool ok)
{
    uint64_t lo = ~0ull;
#pragma unroll
    for (int e = 0; e < V; e++)
        lo = ok && bi[e] < lo ? bi[e] : lo;
    lo = wave_min(lo);
    if (lo == ~0ull)
        return;
    const int lane = threadIdx.x & 63;
    uint32_t mine = 0;
#pragma unroll
    for (int k = 0; k <= V; k++) {
        uint32_t c = 0;
#pragma unroll
        for (int e = 0; e < V; e++)
            c += (uint32_t)__popcll(__ballot(ok && ((pm >> e) & 1u) && bi[e] == lo + (uint64_t)k));
        mine = lane == k ? c : mine;
    }
    if (lane <= V && mine)
        atomicAdd(&C[lo + (uint64_t)lane], mine);
}

template <typename T, bool COUNT>
__device__ __forceinline__ uint64_t mirror_pass(const Args &a, bool rev, uint64_t m)
{
    constexpr int V = 16 / (int)sizeof(T);
    char *base = a.base;
    const uint64_t half = m / 2, nvec = half / V;
    const uint64_t stride = (uint64_t)gridDim.x * kNT;
    const int lane = threadIdx.x & 63;
    uint64_t c = 0;
    // Block counts of the elements this level leaves final: the back part
    // L[ceil(m/2), m) into C; on the top level (roles not yet known, read
    // forward) also the front part, into cntr at the blocks of the array read
    // reversed, whose final part that is.
    uint32_t *C = rev ? a.cntr : a.blk;
    // physical start of front / back vector t (see above)
    auto front_at = [&](uint64_t t) { return rev ? a.n - V * (t + 1) : V * t; };
    auto back_at = [&](uint64_t t) { return rev ? a.n - m + V * t : m - V * (t + 1); };
    // w0: the wavefront's first vector, so every lane runs the same iterations
    for (uint64_t w0 = (uint64_t)blockIdx.x * kNT + (threadIdx.x & ~63u); w0 < nvec; w0 += stride * kMirrorU) {
        const uint64_t t0 = w0 + lane;
        Vec16<T> f[kMirrorU], b[kMirrorU];
#pragma unroll
        for (int u = 0; u < kMirrorU; u++) {
            const uint64_t t = t0 + u * stride;
            if (t < nvec) {
                f[u].v = *reinterpret_cast<const v4u *>(base + front_at(t) * sizeof(T));
                b[u].v = *reinterpret_cast<const v4u *>(base + back_at(t) * sizeof(T));
            }
        }
#pragma unroll
        for (int u = 0; u < kMirrorU; u++) {
            const uint64_t t = t0 + u * stride;
            if (w0 + u * stride >= nvec)
                break;  // uniform: no lane of the wavefront has a vector left
            const bool ok = t < nvec;
            bool any = false;
            uint32_t pmb = 0, pmf = 0;  // predecessor bits after the swaps, by logical offset e
            if (ok) {
#pragma unroll
                for (int e = 0; e < V; e++) {
                    // logical front element V t + e and its partner m - 1 - V t - e
                    T &x = f[u].e[rev ? V - 1 - e : e];
                    T &y = b[u].e[rev ? e : V - 1 - e];
                    const bool px = is_pred(x, a.pivot), py = is_pred(y, a.pivot);
                    if (COUNT)
                        c += (uint64_t)px + (uint64_t)py;
                    const bool sw = (px != rev) && !(py != rev);
                    if (sw) {
                        const T tmp = x;
                        x = y;
                        y = tmp;
                        any = true;
                    }
                    pmb |= (uint32_t)(sw ? px : py) << e;
                    pmf |= (uint32_t)(sw ? py : px) << e;
                }
                if (a.whole || any) {
                    *reinterpret_cast<v4u *>(base + front_at(t) * sizeof(T)) = f[u].v;
                    *reinterpret_cast<v4u *>(base + back_at(t) * sizeof(T)) = b[u].v;
                }
            }
            if (a.fuse) {
                uint64_t bi[V];
#pragma unroll
                for (int e = 0; e < V; e++)
                    bi[e] = (m - 1 - V * t - e) / kBlock;  // logical block of the partner
                wave_block_add<V>(C, bi, pmb, ok);
                if (COUNT) {
#pragma unroll
                    for (int e = 0; e < V; e++)
                        bi[e] = (a.n - 1 - V * t - e) / kBlock;  // front element V t + e, array read reversed
                    wave_block_add<V>(a.cntr, bi, pmf, ok);
                }
            }
        }
    }
    // the last pairs, x in [V nvec, half), one per thread of workgroup 0
    if (blockIdx.x == 0 && threadIdx.x < (uint32_t)(half - V * nvec)) {
        const uint64_t x = V * nvec + threadIdx.x;
        T *pu = phys<T>(a, rev, x), *pv = phys<T>(a, rev, m - 1 - x);
        const T u = *pu, v = *pv;
        const bool pu_ = is_pred(u, a.pivot), pv_ = is_pred(v, a.pivot);
        if (COUNT)
            c += (uint64_t)pu_ + (uint64_t)pv_;
        const bool sw = (pu_ != rev) && !(pv_ != rev);
        if (sw) {
            *pu = v;
            *pv = u;
        }
        if (a.fuse) {
            if (sw ? pu_ : pv_)
                atomicAdd(&C[(m - 1 - x) / kBlock], 1u);
            if (COUNT && (sw ? pv_ : pu_))
                atomicAdd(&a.cntr[(a.n - 1 - x) / kBlock], 1u);
        }
    }
    return c;
}

// Step 1: count predecessors and apply the top preprocessing level.
template <typename T>
__global__ void __launch_bounds__(kNT) k_count_top(Args a)
{
    __shared__ uint64_t red[kNT / 64];
    uint64_t c = mirror_pass<T, true>(a, false, a.n);
    if ((a.n & 1) && blockIdx.x == 0 && threadIdx.x == 0)
        c += is_pred(*reinterpret_cast<const T *>(a.base + (a.n / 2) * sizeof(T)), a.pivot);
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
    (void)mirror_pass<T, false>(a, a.ctl[1] != 0, a.m);
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
    if (a.fuse) {
        // every element of L[0, m0) is final: its blocks' predecessor counts
        uint32_t *C = rev ? a.cntr : a.blk;
        const int lane = threadIdx.x & 63;
        for (uint32_t b = threadIdx.x >> 6; b * kBlock < m0; b += 1024 / 64) {
            const uint32_t x = b * kBlock + lane;
            const uint32_t cb = (uint32_t)__popcll(__ballot(x < m0 && is_pred(buf[x], a.pivot)));
            if (lane == 0 && cb)
                atomicAdd(&C[b], cb);
        }
    }
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

// Step 4a with the counts fused into the preprocessing passes: both count
// arrays start at zero.
__global__ void __launch_bounds__(kNT) k_zero_counts(Args a)
{
    const uint64_t nblk = (a.n + kBlock - 1) / kBlock;
    for (uint64_t b = (uint64_t)blockIdx.x * kNT + threadIdx.x; b < nblk; b += (uint64_t)gridDim.x * kNT) {
        a.blk[b] = 0;
        a.cntr[b] = 0;
    }
}

// Step 4a, fused form: the passes left each block's count of keys below the
// pivot in blk (L read forward) or cntr (L read reversed).  Turn it into the
// block's count of predecessors of L (the complement within the block when
// the roles are swapped) and its exclusive prefix within this workgroup's
// kBlocksPerWg blocks, written over blk; the workgroup total into wgsum.
__global__ void __launch_bounds__(kNT) k_block_prefix(Args a)
{
    __shared__ uint32_t wsum[kNT / 64];
    const bool rev = a.ctl[1] != 0;
    const uint32_t *C = rev ? a.cntr : a.blk;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint64_t blk0 = (uint64_t)blockIdx.x * kBlocksPerWg;
    const uint64_t nblk = (a.n + kBlock - 1) / kBlock;
    constexpr int PER = kBlocksPerWg / kNT;
    uint32_t v[PER], s = 0;
    for (int k = 0; k < PER; k++) {
        const uint64_t b = blk0 + threadIdx.x * PER + k;
        v[k] = 0;
        if (b < nblk) {
            const uint64_t bs = a.n - b * kBlock < (uint64_t)kBlock ? a.n - b * kBlock : (uint64_t)kBlock;
            v[k] = rev ? (uint32_t)bs - C[b] : C[b];
        }
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
    __syncthreads();  // every count of this workgroup is read before blk is written
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

// Step 5, one tail: blocks [lo_blk, hi_blk) of L.  Each wave owns kTailU
// blocks at a time (their elements and prefixes are loaded before any is
// used): a block's j-th predecessor (global rank r from the block prefix
// sums) swaps with L[r], a successor in the partitioned prefix.
constexpr int kTailU = 4;

template <typename T>
__global__ void __launch_bounds__(kNT) k_reorder_tail(Args a)
{
    const bool rev = a.ctl[1] != 0;
    const int lane = threadIdx.x & 63;
    const uint64_t waves = (uint64_t)gridDim.x * (kNT / 64);
    for (uint64_t b0 = a.lo_blk + (uint64_t)blockIdx.x * (kNT / 64) + (threadIdx.x >> 6); b0 < a.hi_blk;
         b0 += waves * kTailU) {
        T v[kTailU];
        bool p[kTailU];
        uint64_t r0[kTailU];
#pragma unroll
        for (int u = 0; u < kTailU; u++) {
            const uint64_t b = b0 + u * waves;
            p[u] = false;
            r0[u] = 0;
            if (b < a.hi_blk) {
                const uint64_t x = b * kBlock + lane;
                if (x < a.n) {
                    v[u] = *phys<T>(a, rev, x);
                    p[u] = is_pred(v[u], a.pivot) != rev;
                }
                r0[u] = a.wgsum[b / kBlocksPerWg] + a.blk[b];
            }
        }
#pragma unroll
        for (int u = 0; u < kTailU; u++) {
            const uint64_t b = b0 + u * waves;
            if (b >= a.hi_blk)
                break;
            const uint64_t m = __ballot(p[u]);
            const uint64_t x = b * kBlock + lane;
            if (p[u]) {
                T *dst = phys<T>(a, rev, r0[u] + lanes_below(m));
                const T w = *dst;
                *dst = v[u];
                v[u] = w;
            }
            if (x < a.n && (a.whole || p[u]))
                *phys<T>(a, rev, x) = v[u];
        }
    }
}

// ---------------------------------------------------------------------------
// The fully implicit Blocked-Prefix-Sum partition (Section 3 as stated, the
// Section 5.1 explicit block counts replaced by values kept in the order of
// the elements themselves).  Steps 1-3 (counting, role swap, preprocessing)
// are the Low-Space ones; then:
//   4'. Blocks of kB = 256 elements (blocks X_0..X_{NB-1}, NB = floor(n/kB),
//       the last one taking the n mod kB elements after it).  A block's first
//       64 pairs (x_2j, x_2j+1) hold a value (Lemma bitstore): pair 0 marks
//       the encoding and pair j >= 1 bit j-1.  Lemma bitstore2 (repeated
//       elements): on the first write the block's 128 pairs are reordered so
//       that its first 64 pairs are all unequal pairs (type 1: the bit is
//       x_2j < x_2j+1, set by ordering the pair) or all equal pairs (type 2:
//       the bit is x_2j != x_2j+1, set by flipping the lowest bit of x_2j+1 --
//       of the payload for key-value records -- and undone when read).
//       Pair 0 is unequal exactly for type 1.  Of 128 pairs at least 64 are of
//       one kind, and 63 bits hold any count up to 2^40.  One wavefront reads
//       or writes a value: one pair per lane, one ballot.
//   4''. The prefix sum over the encoded values is done in place, level by
//       level: level 1 counts every block and leaves in each block the
//       inclusive prefix within its chunk of 256 blocks; level L > 1 scans
//       the last blocks of the level-(L-1) chunks (entries of stride
//       256^(L-1)) the same way, until one chunk remains; then, top down, each
//       chunk adds the value of the entry before it to its other entries.
//       The workgroup of a chunk holds 256 values in LDS at a time: memory
//       per worker, not an array over the input.
//   5'. Reordering as in step 5, with every block's prefix read from its own
//       elements (and type-2 blocks restored) just before the block is used;
//       the innermost prefix restores its blocks in LDS before partitioning.
namespace ip {

constexpr uint64_t kB = 256;     // elements per block
constexpr int kChunk = 256;      // entries per workgroup in a scan level
constexpr int kNT = 256;         // four wavefronts

__device__ __forceinline__ bool el_lt(uint32_t a, uint32_t b) { return a < b; }
__device__ __forceinline__ bool el_lt(uint64_t a, uint64_t b) { return a < b; }
__device__ __forceinline__ bool el_lt(const KV &a, const KV &b)
{
    return a.key < b.key || (a.key == b.key && a.val < b.val);
}
__device__ __forceinline__ bool el_eq(uint32_t a, uint32_t b) { return a == b; }
__device__ __forceinline__ bool el_eq(uint64_t a, uint64_t b) { return a == b; }
__device__ __forceinline__ bool el_eq(const KV &a, const KV &b) { return a.key == b.key && a.val == b.val; }
__device__ __forceinline__ uint32_t el_flip(uint32_t a) { return a ^ 1u; }
__device__ __forceinline__ uint64_t el_flip(uint64_t a) { return a ^ 1ull; }
__device__ __forceinline__ KV el_flip(const KV &a) { return KV{a.key, a.val ^ 1ull}; }

// Lane l's value after exchanging T values across lanes (ds_bpermute per word).
template <typename T>
__device__ __forceinline__ T shfl_el(const T &v, int src)
{
    static_assert(sizeof(T) % 4 == 0, "word-sized elements");
    T out;
    const uint32_t *w = reinterpret_cast<const uint32_t *>(&v);
    uint32_t *o = reinterpret_cast<uint32_t *>(&out);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); k++)
        o[k] = (uint32_t)__shfl((int)w[k], src, 64);
    return out;
}

// Index of the i-th (0-based) set bit of m; m must have more than i set bits.
__device__ __forceinline__ uint32_t nth_set_bit(uint64_t m, uint32_t i)
{
    uint32_t pos = 0;
#pragma unroll
    for (int half = 32; half >= 1; half >>= 1) {
        const uint64_t low = m & ((half == 64 ? ~0ull : (1ull << half) - 1));
        const uint32_t c = (uint32_t)__popcll(low);
        if (i >= c) {
            i -= c;
            m >>= half;
            pos += half;
        } else {
            m = low;
        }
    }
    return pos;
}

// The encode area of a block: pair `lane` = elements 2 lane, 2 lane + 1.
template <typename T>
struct Pair {
    T a, b;
};

// Read the value held by the encode area (one pair per lane); restore type-2
// pairs in registers (p.b = p.a) and report whether the lane's pair changed.
template <typename T>
__device__ __forceinline__ uint64_t decode(Pair<T> &p, int lane, bool &restored)
{
    const bool neq = !el_eq(p.a, p.b);
    const bool type1 = __shfl((int)neq, 0, 64) != 0;
    const uint64_t bits = type1 ? __ballot(el_lt(p.a, p.b)) : __ballot(neq);
    restored = false;
    if (!type1 && lane >= 1 && neq) {
        p.b = p.a;
        restored = true;
    }
    return bits >> 1;
}

// Write value v (< 2^63) into an encode area that already has its type (from
// pair 0).  Returns whether this lane's pair changed; p holds the new pair.
template <typename T>
__device__ __forceinline__ bool encode(Pair<T> &p, int lane, uint64_t v)
{
    const bool type1 = __shfl((int)!el_eq(p.a, p.b), 0, 64) != 0;
    if (lane == 0)
        return false;
    const bool bit = (v >> (lane - 1)) & 1;
    if (type1) {
        if (el_lt(p.a, p.b) != bit) {
            const T t = p.a;
            p.a = p.b;
            p.b = t;
            return true;
        }
        return false;
    }
    // type 2: the pair's two elements hold the same value, kept in p.a
    const T want = bit ? el_flip(p.a) : p.a;
    if (!el_eq(want, p.b)) {
        p.b = want;
        return true;
    }
    return false;
}

struct IpArgs {
    ls::Args a;
    uint64_t nb;        // blocks
    uint64_t stride;    // blocks between entries of this scan level (256^(L-1))
    uint64_t ne;        // entries of this scan level
};

// Block index of entry k of a scan level.
__device__ __forceinline__ uint64_t entry_block(const IpArgs &g, uint64_t k)
{
    const uint64_t e = (k + 1) * g.stride;
    return (e < g.nb ? e : g.nb) - 1;
}

template <typename T>
__device__ __forceinline__ void load_pair(const ls::Args &a, bool rev, uint64_t blk, int lane, Pair<T> &p)
{
    const uint64_t x = blk * kB + 2 * (uint64_t)lane;
    p.a = *ls::phys<T>(a, rev, x);
    p.b = *ls::phys<T>(a, rev, x + 1);
}

template <typename T>
__device__ __forceinline__ void store_pair(const ls::Args &a, bool rev, uint64_t blk, int lane, const Pair<T> &p)
{
    const uint64_t x = blk * kB + 2 * (uint64_t)lane;
    *ls::phys<T>(a, rev, x) = p.a;
    *ls::phys<T>(a, rev, x + 1) = p.b;
}

// Workgroup-inclusive scan of vals[kChunk] in LDS (kNT = kChunk threads).
__device__ __forceinline__ void chunk_scan(uint64_t *vals, uint64_t *wsum)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint64_t x = vals[threadIdx.x];
    uint64_t inc = x;
#pragma unroll
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
    vals[threadIdx.x] = off + inc;
    __syncthreads();
}

// Scan level 1: count every block of L (the last one with its extra
// elements), give its first 64 pairs one kind (first write of Lemma
// bitstore2), and leave the inclusive prefix within the chunk of 256 blocks.
template <typename T>
__global__ void __launch_bounds__(kNT) k_ip_level1(IpArgs g)
{
    __shared__ uint64_t vals[kChunk];
    __shared__ uint64_t wsum[kNT / 64];
    const ls::Args &a = g.a;
    const bool rev = a.ctl[1] != 0;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint64_t c0 = (uint64_t)blockIdx.x * kChunk;
    for (int k = wid; k < kChunk; k += kNT / 64) {
        const uint64_t blk = c0 + k;
        uint64_t cnt = 0;
        if (blk < g.nb) {
            // pairs `lane` (front) and `lane + 64` (back) of the block
            Pair<T> f, bk;
            load_pair(a, rev, blk, lane, f);
            load_pair(a, rev, blk, lane + 64, bk);
            const uint64_t pv = a.pivot;
            auto pred = [&](const T &v) { return ls::is_pred(v, pv) != rev; };
            cnt = (uint64_t)__popcll(__ballot(pred(f.a))) + __popcll(__ballot(pred(f.b))) +
                  __popcll(__ballot(pred(bk.a))) + __popcll(__ballot(pred(bk.b)));
            if (blk == g.nb - 1) {
                // the last block's elements after its first kB
                for (uint64_t x0 = (blk + 1) * kB; x0 < a.n; x0 += 64) {
                    const uint64_t x = x0 + lane;
                    cnt += __popcll(__ballot(x < a.n && pred(*ls::phys<T>(a, rev, x))));
                }
            }
            // Lemma bitstore2, first write: the majority kind of pair to the front 64 slots
            const bool uf = !el_eq(f.a, f.b), ub = !el_eq(bk.a, bk.b);
            const uint64_t mf = __ballot(uf), mb = __ballot(ub);
            const bool type1 = __popcll(mf) + __popcll(mb) >= 64;
            const uint64_t good_f = type1 ? mf : ~mf, good_b = type1 ? mb : ~mb;
            const uint64_t bad_f = ~good_f;
            if (bad_f) {
                // the i-th front pair of the other kind swaps with the i-th back pair of this kind
                const bool fb = (bad_f >> lane) & 1, bg = (good_b >> lane) & 1;
                const uint32_t rf = (uint32_t)__popcll(bad_f & ((1ull << lane) - 1));
                const uint32_t rb = (uint32_t)__popcll(good_b & ((1ull << lane) - 1));
                const int src_for_front = fb ? (int)nth_set_bit(good_b, rf) : lane;
                const int src_for_back = bg && rb < (uint32_t)__popcll(bad_f) ? (int)nth_set_bit(bad_f, rb) : lane;
                const T na = shfl_el(bk.a, src_for_front), nb = shfl_el(bk.b, src_for_front);
                const T ba = shfl_el(f.a, src_for_back), bb = shfl_el(f.b, src_for_back);
                if (fb) {
                    f.a = na;
                    f.b = nb;
                    store_pair(a, rev, blk, lane, f);
                }
                if (bg && rb < (uint32_t)__popcll(bad_f)) {
                    bk.a = ba;
                    bk.b = bb;
                    store_pair(a, rev, blk, lane + 64, bk);
                }
            }
        }
        if (lane == 0)
            vals[k] = cnt;
    }
    __syncthreads();
    chunk_scan(vals, wsum);
    for (int k = wid; k < kChunk; k += kNT / 64) {
        const uint64_t blk = c0 + k;
        if (blk >= g.nb)
            break;
        Pair<T> f;
        load_pair(a, rev, blk, lane, f);
        (void)encode(f, lane, vals[k]);
        store_pair(a, rev, blk, lane, f);  // the whole encode area: whole lines are written
    }
}

// Scan level L > 1 over entries of stride g.stride: decode, scan the chunk,
// encode the inclusive prefixes.
template <typename T>
__global__ void __launch_bounds__(kNT) k_ip_up(IpArgs g)
{
    __shared__ uint64_t vals[kChunk];
    __shared__ uint64_t wsum[kNT / 64];
    const ls::Args &a = g.a;
    const bool rev = a.ctl[1] != 0;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint64_t c0 = (uint64_t)blockIdx.x * kChunk;
    for (int k = wid; k < kChunk; k += kNT / 64) {
        uint64_t v = 0;
        if (c0 + k < g.ne) {
            Pair<T> f;
            load_pair(a, rev, entry_block(g, c0 + k), lane, f);
            bool r;
            v = decode(f, lane, r);
        }
        if (lane == 0)
            vals[k] = v;
    }
    __syncthreads();
    chunk_scan(vals, wsum);
    for (int k = wid; k < kChunk; k += kNT / 64) {
        if (c0 + k >= g.ne)
            break;
        const uint64_t blk = entry_block(g, c0 + k);
        Pair<T> f;
        load_pair(a, rev, blk, lane, f);
        bool r;
        (void)decode(f, lane, r);  // restores type-2 pairs in registers before re-encoding
        (void)encode(f, lane, vals[k]);
        store_pair(a, rev, blk, lane, f);
    }
}

// Down-sweep of level L: chunk c > 0 adds the (global) value of the entry
// before it to its entries except its last one.
template <typename T>
__global__ void __launch_bounds__(kNT) k_ip_down(IpArgs g)
{
    const ls::Args &a = g.a;
    const bool rev = a.ctl[1] != 0;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint64_t c = (uint64_t)blockIdx.x + 1;
    const uint64_t c0 = c * kChunk;
    if (c0 >= g.ne)
        return;
    uint64_t off;
    {
        Pair<T> f;
        load_pair(a, rev, entry_block(g, c0 - 1), lane, f);
        bool r;
        off = decode(f, lane, r);
    }
    const uint64_t last = (c0 + kChunk < g.ne ? c0 + kChunk : g.ne) - 1;
    for (uint64_t k = c0 + wid; k < last; k += kNT / 64) {
        const uint64_t blk = entry_block(g, k);
        Pair<T> f;
        load_pair(a, rev, blk, lane, f);
        bool r;
        const uint64_t v = decode(f, lane, r);
        (void)encode(f, lane, v + off);
        store_pair(a, rev, blk, lane, f);
    }
}

// After the top level: the predecessor count of L is the last block's value.
template <typename T>
__global__ void __launch_bounds__(64) k_ip_total(IpArgs g)
{
    const ls::Args &a = g.a;
    const bool rev = a.ctl[1] != 0;
    const int lane = threadIdx.x;
    Pair<T> f;
    load_pair(a, rev, g.nb - 1, lane, f);
    bool r;
    const uint64_t cl = decode(f, lane, r);
    if (lane == 0) {
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

// Reordering, one tail: blocks [lo_blk, hi_blk) of L, one wavefront per
// block.  The block's inclusive prefix is read from (and type-2 pairs are
// restored in) its encode area; its j-th predecessor then swaps with L[r],
// r = prefix - count + j, a successor in the partitioned prefix.
template <typename T>
__global__ void __launch_bounds__(kNT) k_ip_tail(IpArgs g)
{
    const ls::Args &a = g.a;
    const bool rev = a.ctl[1] != 0;
    const int lane = threadIdx.x & 63;
    const uint64_t waves = (uint64_t)gridDim.x * (kNT / 64);
    const uint64_t pv = a.pivot, lim = a.lo_blk * kB;
    for (uint64_t blk = a.lo_blk + (uint64_t)blockIdx.x * (kNT / 64) + (threadIdx.x >> 6); blk < a.hi_blk;
         blk += waves) {
        Pair<T> f;
        load_pair(a, rev, blk, lane, f);
        bool restored;
        const uint64_t incl = decode(f, lane, restored);
        const uint64_t end = blk == g.nb - 1 ? a.n : (blk + 1) * kB;
        // count the block's predecessors (elements 0..127 are in f, the rest are read)
        uint64_t cnt = (uint64_t)__popcll(__ballot(ls::is_pred(f.a, pv) != rev)) +
                       __popcll(__ballot(ls::is_pred(f.b, pv) != rev));
        for (uint64_t x = blk * kB + 128 + lane; x - lane < end; x += 64) {
            const bool p = x < end && (ls::is_pred(*ls::phys<T>(a, rev, x), pv) != rev);
            cnt += __popcll(__ballot(p));
        }
        uint64_t r = incl - cnt;
        // Every target lies in the partitioned prefix [0, lo_blk kB); the bound
        // is implied by the prefix values and kept as a guard.  With `whole`
        // each part of the block is written back whole (restored pairs
        // included), so that its lines are written whole.
        {
            // the encode area: element 2 lane then 2 lane + 1, in element order
            const bool p0 = ls::is_pred(f.a, pv) != rev, p1 = ls::is_pred(f.b, pv) != rev;
            const uint64_t m0 = __ballot(p0), m1 = __ballot(p1);
            uint64_t rr = r + lanes_below(m0) + lanes_below(m1);
            if (p0 && rr < lim) {
                T *dst = ls::phys<T>(a, rev, rr);
                const T w = *dst;
                *dst = f.a;
                f.a = w;
            }
            rr += p0;
            if (p1 && rr < lim) {
                T *dst = ls::phys<T>(a, rev, rr);
                const T w = *dst;
                *dst = f.b;
                f.b = w;
            }
            if (a.whole || p0 || p1 || restored)
                store_pair(a, rev, blk, lane, f);
            r += __popcll(m0) + __popcll(m1);
        }
        for (uint64_t x0 = blk * kB + 128; x0 < end; x0 += 64) {
            const uint64_t x = x0 + lane;
            bool p = false;
            T v;
            if (x < end) {
                v = *ls::phys<T>(a, rev, x);
                p = ls::is_pred(v, pv) != rev;
            }
            const uint64_t m = __ballot(p);
            if (p && r + lanes_below(m) < lim) {
                T *dst = ls::phys<T>(a, rev, r + lanes_below(m));
                const T w = *dst;
                *dst = v;
                v = w;
            }
            if (x < end && (a.whole || p))
                *ls::phys<T>(a, rev, x) = v;
            r += __popcll(m);
        }
    }
}

// Reordering, innermost prefix L[0, m) (m a multiple of kB, at most one LDS
// buffer): restore the type-2 blocks in LDS, then partition stably.
template <typename T>
__global__ void __launch_bounds__(1024) k_ip_base(IpArgs g)
{
    constexpr int CAP = ls::kSmallBytes / sizeof(T);
    constexpr int K = CAP / 1024;
    __shared__ T buf[CAP];
    __shared__ uint32_t sh[K * 16 + 1];
    const ls::Args &a = g.a;
    const bool rev = a.ctl[1] != 0;
    const uint32_t m = (uint32_t)a.m;
    for (uint32_t k = threadIdx.x; k < m; k += 1024)
        buf[k] = *ls::phys<T>(a, rev, k);
    __syncthreads();
    // type-2 blocks: pair 0 equal; pairs 1..63 restore x_2j+1 = x_2j
    for (uint32_t k = threadIdx.x; k < (m / (uint32_t)kB) * 64; k += 1024) {
        const uint32_t blk = k / 64, j = k % 64;
        if (j >= 1 && el_eq(buf[blk * kB], buf[blk * kB + 1]))
            buf[blk * kB + 2 * j + 1] = buf[blk * kB + 2 * j];
    }
    __syncthreads();
    T x[K];
    bool f[K];
    uint32_t rk[K], tot;
    for (int r = 0; r < K; r++) {
        const uint32_t k = r * 1024 + threadIdx.x;
        f[r] = false;
        if (k < m) {
            x[r] = buf[k];
            f[r] = ls::is_pred(x[r], a.pivot) != rev;
        }
    }
    __syncthreads();
    block_rank<1024, K>(f, rk, tot, sh);
    for (int r = 0; r < K; r++) {
        const uint32_t k = r * 1024 + threadIdx.x;
        if (k < m)
            buf[f[r] ? rk[r] : tot + k - rk[r]] = x[r];
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < m; k += 1024)
        *ls::phys<T>(a, rev, k) = buf[k];
}

}  // namespace ip

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
    uint32_t *cntr = nullptr;   // block counts of the array read reversed (fused counting)
    uint64_t *wgsum = nullptr;
    size_t cap_n = 0;
    size_t bytes = 0;
};
std::mutex g_ls_mu;
std::map<std::pair<int, void *>, LsWork> g_ls;

constexpr uint32_t kPartMax = 4096;

}  // namespace

// Elements for which the implicit variant sizes the Low-Space work arrays.
size_t implicit_work_elems(size_t n, int dtype)
{
    const size_t small = ls::kSmallBytes / (size_t)elem_size(dtype);
    return n < small ? n : small;
}

size_t lowspace_aux_bytes(size_t n)
{
    const size_t nblk = (n + ls::kBlock - 1) / ls::kBlock;
    const size_t nwg = (nblk + ls::kBlocksPerWg - 1) / ls::kBlocksPerWg;
    return 2 * nblk * sizeof(uint32_t) + nwg * sizeof(uint64_t) + kPartMax * sizeof(uint64_t) + 8 * sizeof(uint64_t);
}

// Steps 4'-5' of the implicit variant (after steps 1-3 on n > one LDS buffer).
// With stop_after_sum the call ends once every block holds its prefix.
template <typename T>
static void implicit_steps(const ls::Args &a0, hipStream_t st, uint64_t stream_grid, uint32_t *launches,
                           bool stop_after_sum)
{
    ls::ip::IpArgs g;
    std::memset(&g, 0, sizeof(g));
    g.a = a0;
    g.nb = a0.n / ls::ip::kB;
    auto chunks = [](uint64_t ne) { return (ne + ls::ip::kChunk - 1) / ls::ip::kChunk; };
    // up-sweep: level 1 over every block, then the last blocks of the chunks
    std::vector<std::pair<uint64_t, uint64_t>> lv;  // (stride, entries) per level
    g.stride = 1;
    g.ne = g.nb;
    lv.push_back({g.stride, g.ne});
    hipLaunchKernelGGL(ls::ip::k_ip_level1<T>, dim3((uint32_t)chunks(g.ne)), dim3(ls::ip::kNT), 0, st, g);
    (*launches)++;
    while (g.ne > (uint64_t)ls::ip::kChunk) {
        g.stride *= ls::ip::kChunk;
        g.ne = (g.nb + g.stride - 1) / g.stride;
        lv.push_back({g.stride, g.ne});
        hipLaunchKernelGGL(ls::ip::k_ip_up<T>, dim3((uint32_t)chunks(g.ne)), dim3(ls::ip::kNT), 0, st, g);
        (*launches)++;
    }
    hipLaunchKernelGGL(ls::ip::k_ip_total<T>, dim3(1), dim3(64), 0, st, g);
    (*launches)++;
    // down-sweep, top level first
    for (size_t L = lv.size() - 1; L-- > 0;) {
        g.stride = lv[L].first;
        g.ne = lv[L].second;
        const uint64_t c = chunks(g.ne);
        if (c > 1) {
            hipLaunchKernelGGL(ls::ip::k_ip_down<T>, dim3((uint32_t)(c - 1)), dim3(ls::ip::kNT), 0, st, g);
            (*launches)++;
        }
    }
    if (stop_after_sum)
        return;
    // reorder: prefixes N_0 = n > N_1 > ... > N_K <= one LDS buffer, each a whole number of blocks
    const uint64_t small = ls::kSmallBytes / sizeof(T);
    std::vector<uint64_t> N{a0.n};
    while (N.back() > small) {
        const uint64_t cur = N.back();
        const uint64_t t = (4 * cur / 5) / ls::ip::kB + 1;  // least t with t * kB > 4 cur / 5
        N.push_back(t * ls::ip::kB);
    }
    g.a.m = N.back();
    hipLaunchKernelGGL(ls::ip::k_ip_base<T>, dim3(1), dim3(1024), 0, st, g);
    (*launches)++;
    for (size_t k = N.size() - 1; k-- > 0;) {
        g.a.lo_blk = N[k + 1] / ls::ip::kB;
        g.a.hi_blk = k == 0 ? g.nb : N[k] / ls::ip::kB;
        const uint64_t waves_needed = g.a.hi_blk - g.a.lo_blk;
        uint64_t gr = (waves_needed + (ls::ip::kNT / 64) - 1) / (ls::ip::kNT / 64);
        if (gr > stream_grid)
            gr = stream_grid;
        hipLaunchKernelGGL(ls::ip::k_ip_tail<T>, dim3((uint32_t)(gr ? gr : 1)), dim3(ls::ip::kNT), 0, st, g);
        (*launches)++;
    }
}

template <typename T>
static int lowspace_run(char *base, size_t n, uint64_t pivot, hipStream_t st, uint64_t *d_split, Workspace *ws,
                        LsWork &w, int cus, uint32_t *launches, bool pre_only, bool implicit)
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
    a.cntr = w.cntr;
    a.wgsum = w.wgsum;
    const uint64_t nblk = (n + ls::kBlock - 1) / ls::kBlock;
    a.nwg = (nblk + ls::kBlocksPerWg - 1) / ls::kBlocksPerWg;
    a.d_split = d_split;
    a.host = ws->host_dev;
    a.whole = (uint64_t)n * sizeof(T) > ls::kWholeLineBytes ? 1u : 0u;
    // The explicit path counts its blocks inside the preprocessing passes
    // (Section 5.1 overlaps the counting with preprocessing).
    const uint64_t small = ls::kSmallBytes / sizeof(T);
    a.fuse = !pre_only && !(implicit && n > small) ? 1u : 0u;
    const uint64_t stream_grid = (uint64_t)cus * 8;
    auto grid_for = [&](uint64_t items) -> uint32_t {
        uint64_t g = (items + ls::kNT - 1) / ls::kNT;
        if (g > stream_grid)
            g = stream_grid;
        return (uint32_t)(g ? g : 1);
    };
    // mirror passes: one thread per kMirrorU 16-byte vectors of the front half
    auto mirror_grid = [&](uint64_t m) -> uint32_t {
        const uint64_t vec = (m / 2) / (16 / sizeof(T));
        return grid_for(a.whole ? (vec + ls::kMirrorU - 1) / ls::kMirrorU : vec);
    };
    // 1-2. count with the top preprocessing level, decide the roles
    const uint32_t g1 = mirror_grid(n) < kPartMax ? mirror_grid(n) : kPartMax;
    a.part_count = g1;
    if (a.fuse) {
        hipLaunchKernelGGL(ls::k_zero_counts, dim3(grid_for(nblk)), dim3(ls::kNT), 0, st, a);
        (*launches)++;
    }
    hipLaunchKernelGGL(ls::k_count_top<T>, dim3(g1), dim3(ls::kNT), 0, st, a);
    hipLaunchKernelGGL(ls::k_decide, dim3(1), dim3(ls::kNT), 0, st, a);
    *launches += 2;
    // 3. the other preprocessing levels
    uint64_t m = (n + 1) / 2;
    while (m >= 2 && m > small) {
        a.m = m;
        hipLaunchKernelGGL(ls::k_pre_level<T>, dim3(mirror_grid(m)), dim3(ls::kNT), 0, st, a);
        (*launches)++;
        m = (m + 1) / 2;
    }
    if (m >= 2 || (a.fuse && m == 1)) {  // (m = 1: no level left, but L[0] still needs its count)
        a.m = m;
        hipLaunchKernelGGL(ls::k_pre_small<T>, dim3(1), dim3(1024), 0, st, a);
        (*launches)++;
    }
    if (pre_only && !implicit) {
        if ((e = hipGetLastError()) != hipSuccess)
            return fail_device(e, "Low-Space kernel launch");
        return SS_OK;
    }
    if (implicit && n > small) {
        // 4'-5'. values kept in the blocks' element order (with pre_only: stop after the prefix sum)
        implicit_steps<T>(a, st, stream_grid, launches, pre_only);
        if ((e = hipGetLastError()) != hipSuccess)
            return fail_device(e, "implicit Blocked-Prefix-Sum kernel launch");
        return SS_OK;
    }
    // 4. block counts (left by the passes) and prefix sums
    hipLaunchKernelGGL(ls::k_block_prefix, dim3((uint32_t)a.nwg), dim3(ls::kNT), 0, st, a);
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
        // large arrays: kTailU blocks per wavefront; small ones one, for more waves in flight
        const uint64_t per = a.whole ? ls::kTailU : 1;
        const uint64_t waves_needed = (a.hi_blk - a.lo_blk + per - 1) / per;
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
                             2 * nblk * sizeof(uint32_t) + 256;
        char *p = nullptr;
        if ((e = hipMalloc((void **)&p, bytes)) != hipSuccess) {
            (void)hipGetLastError();
            return fail_msg(SS_ENOMEM, std::string("Low-Space aux hipMalloc: ") + hipGetErrorString(e));
        }
        w->ctl = reinterpret_cast<uint64_t *>(p);
        w->wg_part = w->ctl + 8;
        w->wgsum = w->wg_part + kPartMax;
        w->blk = reinterpret_cast<uint32_t *>(w->wgsum + nwg);
        w->cntr = w->blk + nblk;
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
    // The implicit variant keeps no block arrays: only arrays of at most one
    // LDS buffer, which it partitions with the explicit steps, use them.
    const bool implicit = R.algo == SS_IMPLICIT;
    const size_t nw = implicit ? implicit_work_elems(n, dtype) : n;
    LsWork *w = nullptr;
    if ((rc = ls_work(dev, st, nw, &w)))
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
        case SS_U32: rc = lowspace_run<uint32_t>(base, n, pivot, st, d_split, ws, *w, cus, &ro.launches, pre_only, implicit);
            break;
        case SS_U64: rc = lowspace_run<uint64_t>(base, n, pivot, st, d_split, ws, *w, cus, &ro.launches, pre_only, implicit);
            break;
        default: rc = lowspace_run<KV>(base, n, pivot, st, d_split, ws, *w, cus, &ro.launches, pre_only, implicit);
            break;
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
    ro.aux_bytes = ws->bytes + lowspace_aux_bytes(nw);
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
    a.whole = (uint64_t)n * sizeof(T) > ls::kWholeLineBytes ? 1u : 0u;
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
