// ss_quicksort.hip -- parallel quicksort built on the partition (Section 5.2,
// "Example Application: A Full Quicksort").
//
// The paper's quicksort uses the parallel partition at the upper levels and a
// serial partition once a subproblem is small.  Here every level partitions
// all segments longer than the leaf size at once with the batched Smoothed
// Striding partition, and the short segments are finished by a
// workgroup-local radix sort in LDS.
//
// The segment lists live on the device and a level is a fixed chain of
// launches, so the host never waits for a level before issuing the next one:
//   * k_qprep: the pivot of every segment -- the lower median of 64 keys at
//     equally spaced positions (ss_pivot.h), or the pivot carried over for a
//     second pass (below);
//   * the batched partition (ss_batched.hip) by key < pivot;
//   * k_qchildren: a segment with no key below its pivot p (p is its
//     minimum) goes to the next level with pivot p + 1, i.e. it is
//     partitioned by key <= p and its block of copies of p becomes final, so
//     every level makes progress even when keys repeat; otherwise both parts
//     are strictly smaller than the segment because p itself is on the
//     right.  Children longer than the leaf size are appended to the next
//     level's list, shorter ones (two elements or more) to this level's leaf
//     list (appends use atomic counters; an element's result does not depend
//     on its segment's place in a list);
//   * k_qleaf: every leaf of the level is sorted by one workgroup.
// The host keeps one level in flight ahead of the one it inspects: after
// level L completes it reads the number and the longest length of level
// L + 1's segments from mapped memory, and issues level L + 2 with the
// number of partition levels that the longest segment needs.
// Leaves are sorted by qleaf_sort (ss_leafsort.h).
#include "ss_common.h"
#include "ss_device.h"
#include "ss_internal.h"
#include "ss_leafsort.h"
#include "ss_pivot.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

namespace ss {


template <typename T>
__global__ void __launch_bounds__(256) k_qpivot(const char *base, const uint64_t *start, const uint64_t *len,
                                                uint32_t m, uint64_t *piv_dev, uint64_t *piv_host)
{
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= m)
        return;
    const T *A = reinterpret_cast<const T *>(base) + start[k];
    const uint64_t l = len[k];
    uint64_t a = qkey(A[0]), b = qkey(A[l / 2]), c = qkey(A[l - 1]);
    if (a > b) {
        const uint64_t t = a;
        a = b;
        b = t;
    }
    if (b > c)
        b = c;
    const uint64_t p = a > b ? a : b;  // median of the three
    piv_dev[k] = p;
    if (piv_host)
        piv_host[k] = p;
}

// Leaves are taken by workgroups in turn (leaf b, b + grid, ...); each leaf
// (at most CAP elements) is sorted by key by one workgroup.  The number of
// leaves is *count when count is set, else nleaves.  When pub_dst is set,
// workgroup 0 first writes the quicksort's per-level report to the host.
// Plain keys take the bucket sort (k_qleaf); a leaf with a crowded bucket is
// appended to fb (its index into the leaf list; *fb_count is zero before
// k_qleaf) and sorted by the radix sort in k_qleaf_fb, launched right after.
// Records take the radix sort in k_qleaf itself.
struct QLeafArgs {
    char *base;
    const uint64_t *start, *len;
    const uint32_t *count;
    uint32_t nleaves;
    const uint32_t *pub_count;  // report: pub_dst[0] = *pub_count, pub_dst[1] = *pub_max
    const uint64_t *pub_max;
    uint64_t *pub_dst;
    uint32_t *fb, *fb_count;    // leaves left to the radix sort (plain keys)
};

template <typename T, int CAP, int KEYBITS>
__global__ void __launch_bounds__(leaf_buckets<T>() ? leaf_bucket_nt<T>() : kLeafRadixNT) k_qleaf(QLeafArgs a)
{
    if (a.pub_dst && blockIdx.x == 0 && threadIdx.x == 0) {
        a.pub_dst[0] = *a.pub_count;
        a.pub_dst[1] = *a.pub_max;
    }
    const uint32_t nleaves = a.count ? *a.count : a.nleaves;
    for (uint32_t leaf = blockIdx.x; leaf < nleaves; leaf += gridDim.x) {
        T *A = reinterpret_cast<T *>(a.base) + a.start[leaf];
        if constexpr (leaf_buckets<T>()) {
            if (!qleaf_sort<T, CAP, KEYBITS, leaf_bucket_nt<T>(), false>(A, (uint32_t)a.len[leaf]) &&
                threadIdx.x == 0)
                a.fb[atomicAdd(a.fb_count, 1u)] = leaf;
        } else {
            qleaf_sort<T, CAP, KEYBITS, kLeafRadixNT, true>(A, (uint32_t)a.len[leaf]);
        }
    }
}

template <typename T, int CAP, int KEYBITS>
__global__ void __launch_bounds__(kLeafRadixNT) k_qleaf_fb(QLeafArgs a)
{
    const uint32_t m = *a.fb_count;
    for (uint32_t k = blockIdx.x; k < m; k += gridDim.x) {
        const uint32_t leaf = a.fb[k];
        qleaf_sort<T, CAP, KEYBITS, kLeafRadixNT, true>(reinterpret_cast<T *>(a.base) + a.start[leaf],
                                                        (uint32_t)a.len[leaf]);
    }
}

__global__ void k_leaf_fb_reset(uint32_t *fb_count)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *fb_count = 0;
}


namespace {

struct QsWork {
    uint64_t *dev = nullptr;     // uploaded segment lists
    size_t dev_words = 0;
    uint64_t *host = nullptr;    // mapped: pivots, splits
    uint64_t *host_dev = nullptr;
    size_t host_words = 0;
    uint64_t *stage = nullptr;   // pinned staging for uploads
    size_t stage_words = 0;
};
std::mutex g_q_mu;
std::map<std::pair<int, void *>, QsWork> g_q;

int qs_reserve(int dev, void *stream, size_t dev_words, size_t host_words, size_t stage_words, QsWork **out)
{
    std::lock_guard<std::mutex> lk(g_q_mu);
    QsWork &w = g_q[std::make_pair(dev, stream)];
    hipError_t e;
    if (w.dev_words < dev_words) {
        if (w.dev)
            (void)hipFree(w.dev);
        w.dev = nullptr;
        w.dev_words = 0;
        if ((e = hipMalloc((void **)&w.dev, dev_words * sizeof(uint64_t))) != hipSuccess) {
            (void)hipGetLastError();
            return fail_msg(SS_ENOMEM, std::string("quicksort workspace: ") + hipGetErrorString(e));
        }
        w.dev_words = dev_words;
    }
    if (w.host_words < host_words) {
        if (w.host)
            (void)hipHostFree(w.host);
        w.host = nullptr;
        w.host_words = 0;
        if ((e = hipHostMalloc((void **)&w.host, host_words * sizeof(uint64_t),
                               hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess) {
            (void)hipGetLastError();
            return fail_msg(SS_ENOMEM, std::string("quicksort host buffer: ") + hipGetErrorString(e));
        }
        if ((e = hipHostGetDevicePointer((void **)&w.host_dev, w.host, 0)) != hipSuccess)
            return fail_device(e, "hipHostGetDevicePointer");
        w.host_words = host_words;
    }
    if (w.stage_words < stage_words) {
        if (w.stage)
            (void)hipHostFree(w.stage);
        w.stage = nullptr;
        w.stage_words = 0;
        if ((e = hipHostMalloc((void **)&w.stage, stage_words * sizeof(uint64_t), hipHostMallocDefault)) !=
            hipSuccess) {
            (void)hipGetLastError();
            return fail_msg(SS_ENOMEM, std::string("quicksort staging: ") + hipGetErrorString(e));
        }
        w.stage_words = stage_words;
    }
    *out = &w;
    return SS_OK;
}

template <typename T>
hipError_t launch_qpivot(const char *base, const BatchState &B, uint32_t m, uint64_t *piv_dev, uint64_t *piv_host,
                         hipStream_t st)
{
    hipLaunchKernelGGL(k_qpivot<T>, dim3((m + 255) / 256), dim3(256), 0, st, base, B.start, B.len, m, piv_dev,
                       piv_host);
    return hipGetLastError();
}

template <typename T, int CAP, int KEYBITS>
static int leaf_grids(int *grid, int *grid_fb)
{
    int dev = 0, cus = 0, lds = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess || device_info(dev, &cus, &lds) != SS_OK)
        return SS_EDEVICE;
    const int nt = leaf_buckets<T>() ? leaf_bucket_nt<T>() : kLeafRadixNT;
    if (occupancy(dev, reinterpret_cast<const void *>(&k_qleaf<T, CAP, KEYBITS>), nt, &occ) != SS_OK)
        return SS_EDEVICE;
    *grid = occ * cus;
    if (occupancy(dev, reinterpret_cast<const void *>(&k_qleaf_fb<T, CAP, KEYBITS>), kLeafRadixNT, &occ) != SS_OK)
        return SS_EDEVICE;
    *grid_fb = occ * cus;
    return SS_OK;
}

// Sort the leaves of `a` (plain keys: the bucket kernel, then the radix
// kernel over the leaves it left; a.fb_count must be zero).
template <typename T, int CAP, int KEYBITS>
static hipError_t launch_leaves(const QLeafArgs &a, hipStream_t st, uint32_t *launches)
{
    static int grid = 0, grid_fb = 0;
    if (!grid && leaf_grids<T, CAP, KEYBITS>(&grid, &grid_fb) != SS_OK)
        grid = grid_fb = 256;
    uint32_t g = (uint32_t)grid;
    if (!a.count && a.nleaves < g)
        g = a.nleaves ? a.nleaves : 1u;
    const int nt = leaf_buckets<T>() ? leaf_bucket_nt<T>() : kLeafRadixNT;
    hipLaunchKernelGGL((k_qleaf<T, CAP, KEYBITS>), dim3(g), dim3(nt), 0, st, a);
    (*launches)++;
    if (leaf_buckets<T>()) {
        hipLaunchKernelGGL((k_qleaf_fb<T, CAP, KEYBITS>), dim3((uint32_t)grid_fb), dim3(kLeafRadixNT), 0, st, a);
        (*launches)++;
    }
    return hipGetLastError();
}

hipError_t launch_qleaf(int dtype, const QLeafArgs &a, hipStream_t st, uint32_t *launches)
{
    switch (dtype) {
    case SS_U32: return launch_leaves<uint32_t, 16384, 32>(a, st, launches);
    case SS_U64: return launch_leaves<uint64_t, 16384, 64>(a, st, launches);
    default: return launch_leaves<KV, 8192, 64>(a, st, launches);
    }
}

// ------------------------------------------------------------ device-driven levels

// Segment lists: start, len and carried pivot (0: choose the sample median;
// otherwise the pivot of a key <= p pass, stored as p + 1).
struct SegList {
    uint64_t *start, *len, *pv;
    uint32_t *count;
};

struct QsCtl {
    uint64_t *piv;         // this level's pivots
    uint32_t *leaf_count;  // leaves of this level
    uint64_t *leaf_start, *leaf_len;
    uint64_t *report;      // [0] segments of the next level, [1] the longest of them
    uint32_t *overflow;    // set if a list capacity would be exceeded (never, by the bounds below)
    uint32_t *fb, *fb_count;  // leaves left to the radix sort (k_qleaf_fb)
    uint32_t cap_segs, cap_leaves;
    uint64_t leaf_cap;     // segments up to this length are leaves
};

__global__ void k_qinit(SegList L, QsCtl C, uint64_t n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        L.start[0] = 0;
        L.len[0] = n;
        L.pv[0] = 0;
        *L.count = 1;
        *C.overflow = 0;
        *C.fb_count = 0;
    }
}

// One wavefront per segment (grid: one block of four wavefronts per four
// segments of the list's capacity).
template <typename T>
__global__ void __launch_bounds__(256) k_qprep(const char *base, SegList cur, SegList nxt, QsCtl C)
{
    const uint32_t k = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *nxt.count = 0;
        *C.leaf_count = 0;
        *C.fb_count = 0;
        C.report[1] = 0;
    }
    if (k >= *cur.count)
        return;
    if (cur.pv[k]) {
        if (lane == 0)
            C.piv[k] = cur.pv[k];
        return;
    }
    const uint64_t p = sample_median64(reinterpret_cast<const T *>(base) + cur.start[k], cur.len[k], lane);
    if (lane == 0)
        C.piv[k] = p;
}

__device__ __forceinline__ void q_emit(const SegList &nxt, const QsCtl &C, uint64_t s, uint64_t l, uint64_t pv)
{
    if (l > C.leaf_cap) {
        const uint32_t i = atomicAdd(nxt.count, 1u);
        if (i >= C.cap_segs) {  // cannot happen (disjoint long segments); keep the count within capacity
            atomicSub(nxt.count, 1u);
            atomicOr(C.overflow, 1u);
            return;
        }
        nxt.start[i] = s;
        nxt.len[i] = l;
        nxt.pv[i] = pv;
        atomicMax(reinterpret_cast<unsigned long long *>(&C.report[1]), (unsigned long long)l);
    } else if (l >= 2) {
        const uint32_t i = atomicAdd(C.leaf_count, 1u);
        if (i >= C.cap_leaves) {
            atomicSub(C.leaf_count, 1u);
            atomicOr(C.overflow, 1u);
            return;
        }
        C.leaf_start[i] = s;
        C.leaf_len[i] = l;
    }
}

__global__ void __launch_bounds__(256) k_qchildren(SegList cur, SegList nxt, QsCtl C, const uint64_t *split)
{
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k < *cur.count) {
        const uint64_t s = cur.start[k], l = cur.len[k], rel = split[k] - s, p = C.piv[k];
        if (split[k] < s || rel > l) {  // an unfinished partition (cannot happen: the chain ends with a cleanup)
            atomicOr(C.overflow, 2u);
            return;
        }
        if (!cur.pv[k] && rel == 0) {
            if (p != ~0ull)
                q_emit(nxt, C, s, l, p + 1);  // next level: key <= p
            // p = 2^64 - 1 is the minimum: every key equals it, the segment is sorted
        } else {
            if (!cur.pv[k])
                q_emit(nxt, C, s, rel, 0);
            // after a key <= p pass, [s, s + rel) holds only copies of p and is final
            q_emit(nxt, C, s + rel, l - rel, 0);
        }
    }
}

}  // namespace

uint64_t quicksort_leaf_cap(int dtype) { return dtype == SS_KV16 ? 8192 : 16384; }

// Partition sublevels of one quicksort level whose longest segment has
// max_len elements, for groups of S0 elements.  The first sublevel leaves a
// middle region of about 4.4 / sqrt(S0) of a segment and every later one
// about 0.11 of the region before it (Section 4's bound on the splitting
// positions' spread); sublevels are added until the expected region is at
// most kQsCleanupBytes, which the batched chain's closing one-workgroup
// cleanup then partitions serially.
constexpr uint64_t kQsCleanupBytes = 256 << 10;

static uint32_t qs_sublevels(uint64_t max_len, uint64_t S0, int w)
{
    if (max_len <= S0)
        return 1;
    const double base = (double)kQsCleanupBytes / w;
    double r = (double)max_len * 4.4 / std::sqrt((double)S0);
    uint32_t lv = 1;
    while (r > base && lv < 16) {
        r *= 0.11;
        lv++;
    }
    return lv;
}

namespace {

// Device workspace of the device-driven quicksort, cached per (device,
// stream) and grown on demand.
struct QsDev {
    char *dev = nullptr;
    size_t dev_bytes = 0;
    uint64_t *rep = nullptr;      // mapped host: per level {segments of the next level, longest}
    uint64_t *rep_dev = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};
std::mutex g_qd_mu;
std::map<std::pair<int, void *>, QsDev> g_qd;

constexpr uint32_t kMaxQsLevels = 4096;

int qs_dev_reserve(int dev, void *stream, size_t bytes, QsDev **out)
{
    std::lock_guard<std::mutex> lk(g_qd_mu);
    QsDev &w = g_qd[std::make_pair(dev, stream)];
    hipError_t e;
    if (w.dev_bytes < bytes) {
        if (w.dev)
            (void)hipFree(w.dev);
        w.dev = nullptr;
        w.dev_bytes = 0;
        if ((e = hipMalloc((void **)&w.dev, bytes)) != hipSuccess) {
            (void)hipGetLastError();
            return fail_msg(SS_ENOMEM, std::string("quicksort workspace: ") + hipGetErrorString(e));
        }
        w.dev_bytes = bytes;
    }
    if (!w.rep) {
        if ((e = hipHostMalloc((void **)&w.rep, 2 * kMaxQsLevels * sizeof(uint64_t),
                               hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess) {
            (void)hipGetLastError();
            w.rep = nullptr;
            return fail_msg(SS_ENOMEM, std::string("quicksort report buffer: ") + hipGetErrorString(e));
        }
        if ((e = hipHostGetDevicePointer((void **)&w.rep_dev, w.rep, 0)) != hipSuccess)
            return fail_device(e, "hipHostGetDevicePointer");
        for (auto &ev : w.ev)
            if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
                return fail_device(e, "hipEventCreate");
    }
    *out = &w;
    return SS_OK;
}

template <typename T>
hipError_t launch_qprep(const char *base, const SegList &cur, const SegList &nxt, const QsCtl &C, uint32_t grid,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_qprep<T>, dim3(grid), dim3(256), 0, st, base, cur, nxt, C);  // grid: segments / 4
    return hipGetLastError();
}

}  // namespace

// Quicksort of base[0, n).  Segments longer than the leaf capacity are
// disjoint, so a level holds at most n / (cap + 1) of them and at most twice
// as many leaves; the batched state is sized for that.
int quicksort_run(char *base, size_t n, int dtype, const Resolved &R, hipStream_t st, uint32_t *levels_out,
                  uint32_t *launches)
{
    hipError_t e;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess)
        return fail_device(e, "hipGetDevice");
    *levels_out = 0;
    if (n < 2)
        return SS_OK;
    const uint64_t cap = quicksort_leaf_cap(dtype);
    const uint64_t tile_elems = R.tile / R.w;
    const uint64_t capS = n / (cap + 1) + 2, capL = 2 * capS + 2;
    const uint64_t items = n / tile_elems + 3 * capS + 64;
    // word layout of the workspace
    const size_t words = 2 * 3 * capS + capS /*piv*/ + 2 * capL /*leaves*/ + 3 * capS /*lo, hi, split*/ +
                         (capS + 1) /*first*/ + items /*vout*/ + (capS + 1) / 2 + 1 /*g*/ + (items + 1) / 2 /*imap*/ +
                         capS / 8 + 1 /*cls*/ + 8 /*ctl*/ + 8 /*counts, report, overflow*/ +
                         (capL + 1) / 2 + 1 /*fb*/;
    QsDev *W = nullptr;
    int rc = qs_dev_reserve(dev, st, words * sizeof(uint64_t), &W);
    if (rc)
        return rc;
    uint64_t *p = reinterpret_cast<uint64_t *>(W->dev);
    auto take = [&](size_t nw) {
        uint64_t *q = p;
        p += nw;
        return q;
    };
    // [0] list A, [1] list B, [2] leaves, [3] overflow, [4] leaves for the radix sort
    uint32_t *counts = reinterpret_cast<uint32_t *>(take(3));
    SegList LA{take(capS), take(capS), take(capS), counts + 0};
    SegList LB{take(capS), take(capS), take(capS), counts + 1};
    QsCtl C;
    C.piv = take(capS);
    C.leaf_count = counts + 2;
    C.overflow = counts + 3;
    C.leaf_start = take(capL);
    C.leaf_len = take(capL);
    C.fb = reinterpret_cast<uint32_t *>(take((capL + 1) / 2 + 1));
    C.fb_count = counts + 4;
    C.report = take(2);
    C.cap_segs = (uint32_t)capS;
    C.cap_leaves = (uint32_t)capL;
    C.leaf_cap = cap;
    BatchState B;
    B.pivot = C.piv;
    B.lo = take(capS);
    B.hi = take(capS);
    B.split = take(capS);
    B.first = take(capS + 1);
    B.vout = take(items);
    B.g = reinterpret_cast<uint32_t *>(take((capS + 1) / 2 + 1));
    B.imap = reinterpret_cast<uint32_t *>(take((items + 1) / 2));
    B.cls = reinterpret_cast<uint8_t *>(take(capS / 8 + 1));
    B.ctl = take(8);
    B.num = (uint32_t)capS;
    B.base_lines = 1;  // segments are parts of the array: lines stay aligned to the base

    const BatchClasses BC = batched_default_classes(R);
    hipLaunchKernelGGL(k_qinit, dim3(1), dim3(64), 0, st, LA, C, (uint64_t)n);
    (*launches)++;
    if (n <= cap) {
        // the whole array is one leaf
        QLeafArgs a{base, LA.start, LA.len, nullptr, 1u, nullptr, nullptr, nullptr, C.fb, C.fb_count};
        if ((e = launch_qleaf(dtype, a, st, launches)) != hipSuccess)
            return fail_device(e, "leaf sort launch");
        if ((e = hipStreamSynchronize(st)) != hipSuccess)
            return fail_device(e, "hipStreamSynchronize");
        return SS_OK;
    }
    // A level's segments are at most twice as many as its parent level's
    // (and within the list's capacity): the per-segment grids and the batched
    // state's count bound are sized for that.
    auto enqueue = [&](uint32_t L, uint64_t max_len, uint64_t max_segs) -> int {
        const SegList &cur = (L & 1) ? LB : LA;
        const SegList &nxt = (L & 1) ? LA : LB;
        const uint32_t segs = (uint32_t)std::min<uint64_t>(max_segs, capS);
        const uint32_t grid_s = (segs + 255) / 256, grid_w = (segs + 3) / 4;
        hipError_t e2;
        switch (dtype) {
        case SS_U32: e2 = launch_qprep<uint32_t>(base, cur, nxt, C, grid_w, st); break;
        case SS_U64: e2 = launch_qprep<uint64_t>(base, cur, nxt, C, grid_w, st); break;
        default: e2 = launch_qprep<KV>(base, cur, nxt, C, grid_w, st); break;
        }
        if (e2 != hipSuccess)
            return fail_device(e2, "pivot launch");
        B.start = cur.start;
        B.len = cur.len;
        B.count = cur.count;
        B.num = segs;
        const int rc2 =
            batched_core(base, dtype, R, BC, B, qs_sublevels(max_len, tile_elems, R.w), st, nullptr, launches);
        if (rc2)
            return rc2;
        hipLaunchKernelGGL(k_qchildren, dim3(grid_s), dim3(256), 0, st, cur, nxt, C, (const uint64_t *)B.split);
        QLeafArgs a{base,         C.leaf_start,      C.leaf_len, C.leaf_count, 0u, nxt.count,
                    C.report + 1, W->rep_dev + 2 * L, C.fb,       C.fb_count};
        if ((e2 = launch_qleaf(dtype, a, st, launches)) != hipSuccess)
            return fail_device(e2, "leaf sort launch");
        *launches += 2;
        if ((e2 = hipEventRecord(W->ev[L & 3], st)) != hipSuccess)
            return fail_device(e2, "hipEventRecord");
        return SS_OK;
    };
    // Level L + 2 is issued once level L has completed: its segments are
    // children of level L + 1's, whose count and longest length level L
    // reported.
    if ((rc = enqueue(0, n, 1)) || (rc = enqueue(1, n, 2)))
        return rc;
    uint32_t L = 0;
    for (;;) {
        if ((e = hipEventSynchronize(W->ev[L & 3])) != hipSuccess)
            return fail_device(e, "hipEventSynchronize");
        const volatile uint64_t *rep = W->rep + 2 * L;
        const uint64_t next_segs = rep[0], next_max = rep[1];  // level L + 1
        if (next_segs == 0)
            break;  // level L + 1 (already issued) has nothing to do
        if (L + 2 >= kMaxQsLevels)
            return fail_msg(SS_EDEVICE, "quicksort: no progress");
        if ((rc = enqueue(L + 2, next_max, 2 * next_segs)))
            return rc;
        L++;
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess)
        return fail_device(e, "hipStreamSynchronize");
    uint32_t ovf = 0;
    if ((e = hipMemcpy(&ovf, C.overflow, sizeof(ovf), hipMemcpyDeviceToHost)) != hipSuccess)
        return fail_device(e, "hipMemcpy");
    if (ovf)
        return fail_msg(SS_EDEVICE, ovf & 2u ? "quicksort: unfinished partition" : "quicksort: segment list overflow");
    *levels_out = L + 1;
    return SS_OK;
}

}  // namespace ss

using namespace ss;

extern "C" int ss_quicksort_ex(void *d_ptr, size_t n, int dtype, const ss_params *p, void *stream,
                               ss_stats *stats)
{
    int rc = check_array(d_ptr, n, dtype);
    if (rc)
        return rc;
    Resolved R;
    if ((rc = resolve_params(p, dtype, &R, batched_auto_engine(dtype))))
        return rc;
    if (dtype == SS_U32 && !(p && (p->engine || p->tile_bytes || p->b))) {
        // u32 levels: the LDS body with 64 KiB groups, which hold a whole leaf-sized
        // segment (measured 8.6% faster than the register body on 2^28 keys)
        ss_params q;
        std::memset(&q, 0, sizeof(q));
        if (p)
            q = *p;
        q.engine = SS_ENGINE_LDS;
        q.tile_bytes = 65536;
        if ((rc = resolve_params(&q, dtype, &R)))
            return rc;
    }
    if (R.algo != SS_SMOOTHED)
        return fail_msg(SS_EUNSUPPORTED, "quicksort levels use the batched Smoothed Striding partition");
    if ((rc = check_lines(n, R)))
        return rc;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    const bool timing = (R.flags & SS_FLAG_TIME) != 0;
    if (timing) {
        if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
            return fail_msg(SS_EDEVICE, "hipEventCreate");
        (void)hipEventRecord(t0, st);
    }
    uint32_t levels = 0, launches = 0;
    rc = quicksort_run((char *)d_ptr, n, dtype, R, st, &levels, &launches);
    float ms = 0;
    if (timing) {
        (void)hipEventRecord(t1, st);
        (void)hipEventSynchronize(t1);
        (void)hipEventElapsedTime(&ms, t0, t1);
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
    }
    if (rc)
        return rc;
    if (stats) {
        RunOut ro;
        std::memset(&ro, 0, sizeof(ro));
        ro.launches = launches;
        ro.total_ms = ms;
        fill_stats(stats, ro, R, dtype);
        stats->levels = levels;
    }
    return SS_OK;
}

extern "C" int ss_quicksort(void *d_ptr, size_t n, int dtype)
{
    return ss_quicksort_ex(d_ptr, n, dtype, nullptr, nullptr, nullptr);
}

namespace ss {

// Upload num (start, len) pairs through the quicksort staging buffer into the
// device list area; returns device pointers to the starts and lengths.
static int upload_segments(int dev, hipStream_t st, const uint64_t *h_starts, const uint64_t *h_lens, size_t num,
                           QsWork **wout, uint64_t **d_starts, uint64_t **d_lens)
{
    QsWork *w = nullptr;
    // device words: starts, lengths, then (ss_sort_segments) the leaf sort's
    // radix list, num 32-bit entries and its count
    int rc = qs_reserve(dev, st, 2 * num + (num + 1) / 2 + 16, 16, 2 * num + 16, &w);
    if (rc)
        return rc;
    hipError_t e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess)  // the staging buffer may still be read
        return fail_device(e, "hipStreamSynchronize");
    std::memcpy(w->stage, h_starts, num * sizeof(uint64_t));
    std::memcpy(w->stage + num, h_lens, num * sizeof(uint64_t));
    if ((e = hipMemcpyAsync(w->dev, w->stage, 2 * num * sizeof(uint64_t), hipMemcpyHostToDevice, st)) != hipSuccess)
        return fail_device(e, "hipMemcpyAsync");
    *wout = w;
    *d_starts = w->dev;
    *d_lens = w->dev + num;
    return SS_OK;
}

static int check_segments(void *d_base, const uint64_t *h_starts, const uint64_t *h_lens, size_t num, int dtype,
                          uint64_t max_len)
{
    if (!elem_size(dtype))
        return fail_msg(SS_EINVAL, "unknown dtype");
    if (num && (!h_starts || !h_lens))
        return fail_msg(SS_EINVAL, "null starts or lengths");
    uint64_t end = 0;
    for (size_t k = 0; k < num; k++) {
        if (h_lens[k] == 0 || h_lens[k] > max_len)
            return fail_msg(SS_EINVAL, "segment length out of range");
        if (h_starts[k] + h_lens[k] > end)
            end = h_starts[k] + h_lens[k];
    }
    return check_array(d_base, (size_t)end, dtype);
}

}  // namespace ss

extern "C" size_t ss_sort_segment_cap(int dtype)
{
    return elem_size(dtype) ? (size_t)quicksort_leaf_cap(dtype) : 0;
}

extern "C" int ss_median3_pivots(void *d_base, const uint64_t *h_starts, const uint64_t *h_lens, size_t num,
                                 int dtype, uint64_t *d_pivots, uint64_t *h_pivots, void *stream)
{
    int rc = check_segments(d_base, h_starts, h_lens, num, dtype, ~0ull);
    if (rc)
        return rc;
    if (num == 0)
        return SS_OK;
    if (!d_pivots || ((uintptr_t)d_pivots % 8))
        return fail_msg(SS_EINVAL, "d_pivots must be an 8-byte aligned device array");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess)
        return fail_device(e, "hipGetDevice");
    QsWork *w = nullptr;
    uint64_t *ds = nullptr, *dl = nullptr;
    if ((rc = upload_segments(dev, st, h_starts, h_lens, num, &w, &ds, &dl)))
        return rc;
    BatchState B;
    std::memset(&B, 0, sizeof(B));
    B.start = ds;
    B.len = dl;
    switch (dtype) {
    case SS_U32: e = launch_qpivot<uint32_t>((const char *)d_base, B, (uint32_t)num, d_pivots, nullptr, st); break;
    case SS_U64: e = launch_qpivot<uint64_t>((const char *)d_base, B, (uint32_t)num, d_pivots, nullptr, st); break;
    default: e = launch_qpivot<KV>((const char *)d_base, B, (uint32_t)num, d_pivots, nullptr, st); break;
    }
    if (e != hipSuccess)
        return fail_device(e, "pivot launch");
    if (h_pivots) {
        if ((e = hipMemcpyAsync(h_pivots, d_pivots, num * sizeof(uint64_t), hipMemcpyDeviceToHost, st)) != hipSuccess)
            return fail_device(e, "hipMemcpyAsync");
        if ((e = hipStreamSynchronize(st)) != hipSuccess)
            return fail_device(e, "hipStreamSynchronize");
    }
    return SS_OK;
}

extern "C" int ss_sort_segments(void *d_base, const uint64_t *h_starts, const uint64_t *h_lens, size_t num,
                                int dtype, void *stream)
{
    int rc = check_segments(d_base, h_starts, h_lens, num, dtype, elem_size(dtype) ? quicksort_leaf_cap(dtype) : 0);
    if (rc)
        return rc;
    if (num == 0)
        return SS_OK;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess)
        return fail_device(e, "hipGetDevice");
    QsWork *w = nullptr;
    uint64_t *ds = nullptr, *dl = nullptr;
    if ((rc = upload_segments(dev, st, h_starts, h_lens, num, &w, &ds, &dl)))
        return rc;
    if (num > 0xffffffffull)
        return fail_msg(SS_EINVAL, "too many segments");
    uint32_t *fb = reinterpret_cast<uint32_t *>(w->dev + 2 * num), *fb_count = fb + num;
    hipLaunchKernelGGL(k_leaf_fb_reset, dim3(1), dim3(64), 0, st, fb_count);
    uint32_t launches = 0;
    QLeafArgs a{(char *)d_base, ds, dl, nullptr, (uint32_t)num, nullptr, nullptr, nullptr, fb, fb_count};
    if ((e = launch_qleaf(dtype, a, st, &launches)) != hipSuccess)
        return fail_device(e, "segment sort launch");
    return SS_OK;
}
