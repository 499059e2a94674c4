// ss_serving.hip -- device-resident job state for continuous batching of
// partition and sort jobs (the serving loop built on the batched partition
// of Section 4 and the quicksort of Section 5.2).
//
// Every job occupies a slot.  Its pending work is a set of segments in a
// device list (a whole partition job, or a segment of a sort job) and of
// leaves (short segments of a sort job), and a per-slot counter holds how
// many of them are outstanding.  A tick is a fixed chain of launches on one
// stream with no host decision in between:
//   k_ssubmit  append the jobs submitted since the last tick to the list;
//   k_sprep    pivots: a partition job's own pivot, a sort segment's
//              sample median (ss_pivot.h), or the pivot carried over for a
//              key <= p pass;
//   the batched partition of every listed segment (ss_batched.hip);
//   k_schild   a partition job is done; a sort segment's children go to the
//              next list (longer than the leaf capacity) or to the leaf list,
//              exactly as in the quicksort (a segment whose pivot was its
//              minimum is passed on for a key <= p pass);
//   k_sleaf    every leaf is sorted by one workgroup.
// A slot's counter is raised by the children a segment emits before that
// segment is counted off, so it reaches zero only when the whole job is
// done; the thread that takes it to zero raises the slot's done flag in
// mapped host memory (a partition job's split is written there first).  The
// host reads the flags after the tick's event, so it never waits for a tick
// to issue the next one.
#include "ss_common.h"
#include "ss_device.h"
#include "ss_internal.h"
#include "ss_leafsort.h"
#include "ss_pivot.h"

#include <cstring>
#include <vector>

namespace ss {

namespace {

struct SrvSub {
    uint64_t start, len, pivot;
    uint32_t slot, kind;  // kind 0: partition by key < pivot; 1: sort
};

struct SrvDev {
    uint64_t *start[2], *len[2], *pv[2];
    uint32_t *job[2];
    uint32_t *count;      // [0], [1] list counts, [2] leaves, [3] overflow flags, [4] leaves for the radix sort
    uint32_t *fb;         // leaves the bucket sort left to the radix sort (indices into the leaf list)
    uint64_t *piv;
    uint64_t *leaf_start, *leaf_len;
    uint32_t *leaf_job;
    uint8_t *kind;
    uint64_t *jpivot, *jstart;
    uint32_t *outstanding;
    uint32_t *h_done;     // mapped host memory
    uint64_t *h_split;    // mapped host memory
    uint32_t *h_flags;    // mapped host memory: a copy of the overflow flags (nonzero once any is set)
    uint32_t cap_segs, cap_leaves, max_jobs;
    uint64_t leaf_cap;
};

// Raise overflow flag bits on the device and mirror them into mapped host
// memory, so the host sees a failure at its next wait without synchronizing.
// Concurrent raisers may leave the mirror with a subset of the bits, never
// with none; ss_server_status reads the exact set.
__device__ __forceinline__ void srv_flag(const SrvDev &D, uint32_t bits)
{
    const uint32_t old = atomicOr(&D.count[3], bits);
    *reinterpret_cast<volatile uint32_t *>(D.h_flags) = old | bits;
    __threadfence_system();
}

__device__ __forceinline__ void srv_finish(const SrvDev &D, uint32_t slot)
{
    if (atomicSub(&D.outstanding[slot], 1u) == 1u) {
        __threadfence_system();
        D.h_done[slot] = 1u;
    }
}

__global__ void __launch_bounds__(256) k_ssubmit(SrvDev D, const SrvSub *sub, uint32_t nsub, uint32_t cur)
{
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nsub)
        return;
    const SrvSub x = sub[i];
    D.kind[x.slot] = (uint8_t)x.kind;
    D.jpivot[x.slot] = x.pivot;
    D.jstart[x.slot] = x.start;
    D.outstanding[x.slot] = 1u;
    const uint32_t k = atomicAdd(&D.count[cur], 1u);
    if (k >= D.cap_segs) {  // admission keeps this from happening; keep the count within capacity
        atomicSub(&D.count[cur], 1u);
        srv_flag(D, 1u);
        return;
    }
    D.start[cur][k] = x.start;
    D.len[cur][k] = x.len;
    D.pv[cur][k] = 0;
    D.job[cur][k] = x.slot;
}

// One wavefront per listed segment (grid: one block per four list entries).
template <typename T>
__global__ void __launch_bounds__(256) k_sprep(const char *base, SrvDev D, uint32_t cur)
{
    const uint32_t k = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        D.count[cur ^ 1u] = 0;
        D.count[2] = 0;
        D.count[4] = 0;
    }
    if (k >= D.count[cur])
        return;
    const uint32_t slot = D.job[cur][k];
    uint64_t p;
    if (D.kind[slot] == 0)
        p = D.jpivot[slot];
    else if (D.pv[cur][k])
        p = D.pv[cur][k];
    else
        p = sample_median64(reinterpret_cast<const T *>(base) + D.start[cur][k], D.len[cur][k], lane);
    if (lane == 0)
        D.piv[k] = p;
}

__device__ __forceinline__ uint32_t srv_emit(const SrvDev &D, uint32_t nxt, uint32_t slot, uint64_t s, uint64_t l,
                                             uint64_t pv)
{
    if (l > D.leaf_cap) {
        const uint32_t i = atomicAdd(&D.count[nxt], 1u);
        if (i >= D.cap_segs) {
            atomicSub(&D.count[nxt], 1u);
            srv_flag(D, 1u);
            return 0;
        }
        D.start[nxt][i] = s;
        D.len[nxt][i] = l;
        D.pv[nxt][i] = pv;
        D.job[nxt][i] = slot;
        return 1;
    }
    if (l >= 2) {
        const uint32_t i = atomicAdd(&D.count[2], 1u);
        if (i >= D.cap_leaves) {
            atomicSub(&D.count[2], 1u);
            srv_flag(D, 1u);
            return 0;
        }
        D.leaf_start[i] = s;
        D.leaf_len[i] = l;
        D.leaf_job[i] = slot;
        return 1;
    }
    return 0;
}

__global__ void __launch_bounds__(256) k_schild(SrvDev D, uint32_t cur, const uint64_t *split)
{
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= D.count[cur])
        return;
    const uint32_t slot = D.job[cur][k], nxt = cur ^ 1u;
    const uint64_t s = D.start[cur][k], l = D.len[cur][k], rel = split[k] - s;
    if (split[k] < s || rel > l) {  // an unfinished partition (the batched chain ends with a cleanup)
        srv_flag(D, 2u);
        return;
    }
    if (D.kind[slot] == 0) {
        D.h_split[slot] = rel;
        __threadfence_system();
        srv_finish(D, slot);
        return;
    }
    const uint64_t p = D.piv[k];
    uint32_t e = 0;
    const uint64_t c0 = rel;
    if (!D.pv[cur][k] && rel == 0) {
        if (p != ~0ull)
            e += srv_emit(D, nxt, slot, s, l, p + 1);  // next tick: key <= p
    } else {
        if (!D.pv[cur][k])
            e += srv_emit(D, nxt, slot, s, c0, 0);
        e += srv_emit(D, nxt, slot, s + c0, l - c0, 0);  // after a key <= p pass the left part is final
    }
    if (e)
        atomicAdd(&D.outstanding[slot], e);
    srv_finish(D, slot);
}

// Plain keys take the bucket sort; a leaf with a crowded bucket goes to the
// radix sort in k_sleaf_fb, which finishes it.  Records take the radix sort.
template <typename T, int CAP, int KEYBITS>
__global__ void __launch_bounds__(leaf_buckets<T>() ? leaf_bucket_nt<T>() : kLeafRadixNT) k_sleaf(char *base, SrvDev D)
{
    const uint32_t n = D.count[2] < D.cap_leaves ? D.count[2] : D.cap_leaves;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        T *A = reinterpret_cast<T *>(base) + D.leaf_start[i];
        bool sorted;
        if constexpr (leaf_buckets<T>())
            sorted = qleaf_sort<T, CAP, KEYBITS, leaf_bucket_nt<T>(), false>(A, (uint32_t)D.leaf_len[i]);
        else
            sorted = qleaf_sort<T, CAP, KEYBITS, kLeafRadixNT, true>(A, (uint32_t)D.leaf_len[i]);
        if (threadIdx.x == 0) {
            if (sorted)
                srv_finish(D, D.leaf_job[i]);
            else
                D.fb[atomicAdd(&D.count[4], 1u)] = i;
        }
    }
}

template <typename T, int CAP, int KEYBITS>
__global__ void __launch_bounds__(kLeafRadixNT) k_sleaf_fb(char *base, SrvDev D)
{
    const uint32_t m = D.count[4];
    for (uint32_t k = blockIdx.x; k < m; k += gridDim.x) {
        const uint32_t i = D.fb[k];
        qleaf_sort<T, CAP, KEYBITS, kLeafRadixNT, true>(reinterpret_cast<T *>(base) + D.leaf_start[i],
                                                        (uint32_t)D.leaf_len[i]);
        if (threadIdx.x == 0)
            srv_finish(D, D.leaf_job[i]);
    }
}

}  // namespace

// ------------------------------------------------------------------ host side

struct Server {
    int dev = 0, dtype = 0, w = 0;
    char *base = nullptr;
    uint64_t capacity = 0;
    hipStream_t st = nullptr;
    Resolved R;
    SrvDev D;
    BatchState B;
    char *dmem = nullptr;
    uint32_t *hmem = nullptr;   // mapped: done flags then splits
    SrvSub *stage[2] = {nullptr, nullptr};
    SrvSub *dsub = nullptr;
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    hipEvent_t tick_ev[4] = {};
    uint32_t stage_cap = 0, cur = 0, ticks_issued = 0, ticks_done = 0, leaf_grid = 0, leaf_grid_fb = 0, seg_grid = 0,
             seg_grid_w = 0;
    std::vector<SrvSub> pending;
};

static void server_free(Server *s)
{
    if (!s)
        return;
    if (s->st)
        (void)hipStreamSynchronize(s->st);
    if (s->dmem)
        (void)hipFree(s->dmem);
    if (s->hmem)
        (void)hipHostFree(s->hmem);
    for (auto &p : s->stage)
        if (p)
            (void)hipHostFree(p);
    for (auto &e : s->stage_ev)
        if (e)
            (void)hipEventDestroy(e);
    for (auto &e : s->tick_ev)
        if (e)
            (void)hipEventDestroy(e);
    delete s;
}

uint64_t server_items_cap(uint64_t capacity, uint64_t tile_elems, uint64_t cap_segs)
{
    return capacity / tile_elems + 3 * cap_segs + 64;
}

}  // namespace ss

using namespace ss;

struct ss_server {
    Server *s;
};

extern "C" int ss_server_create(void *d_base, size_t capacity, int dtype, uint32_t max_jobs, uint32_t max_segments,
                                void *stream, ss_server **out)
{
    if (!out)
        return fail_msg(SS_EINVAL, "null output");
    *out = nullptr;
    int rc = check_array(d_base, capacity, dtype);
    if (rc)
        return rc;
    if (max_jobs == 0 || max_segments == 0 || max_jobs > (1u << 24) || max_segments > (1u << 26))
        return fail_msg(SS_EINVAL, "max_jobs / max_segments out of range");
    Server *s = new Server();
    s->dtype = dtype;
    s->w = elem_size(dtype);
    s->base = (char *)d_base;
    s->capacity = capacity;
    s->st = (hipStream_t)stream;
    hipError_t e;
    if ((rc = resolve_params(nullptr, dtype, &s->R, batched_auto_engine(dtype)))) {
        delete s;
        return rc;
    }
    if ((e = hipGetDevice(&s->dev)) != hipSuccess) {
        delete s;
        return fail_device(e, "hipGetDevice");
    }
    const uint64_t cap_segs = max_segments, cap_leaves = 2ull * max_segments + 2;
    const uint64_t tile_elems = s->R.tile / s->R.w;
    const uint64_t items = server_items_cap(capacity, tile_elems, cap_segs);
    const size_t words = 2 * (3 * cap_segs + cap_segs / 2 + 1) /*lists*/ + 3 /*counts*/ + cap_segs /*piv*/ +
                         2 * cap_leaves + 2 * (cap_leaves / 2 + 1) /*leaves, radix list*/ + max_jobs / 8 + 1 /*kind*/ +
                         2 * (size_t)max_jobs /*jpivot, jstart*/ + max_jobs / 2 + 1 /*outstanding*/ +
                         3 * cap_segs /*lo, hi, split*/ + cap_segs + 1 /*first*/ + items /*vout*/ +
                         cap_segs / 2 + 1 /*g*/ + items / 2 + 1 /*imap*/ + cap_segs / 8 + 1 /*cls*/ + 8 /*ctl*/ +
                         64 * 4 /*submission staging on the device*/ + 16;
    if ((e = hipMalloc((void **)&s->dmem, words * sizeof(uint64_t))) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return fail_msg(SS_ENOMEM, std::string("server state: ") + hipGetErrorString(e));
    }
    const size_t hbytes = (size_t)max_jobs * (sizeof(uint32_t) + sizeof(uint64_t)) + 128;
    if ((e = hipHostMalloc((void **)&s->hmem, hbytes, hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess) {
        (void)hipGetLastError();
        server_free(s);
        return fail_msg(SS_ENOMEM, std::string("server host flags: ") + hipGetErrorString(e));
    }
    std::memset(s->hmem, 0, hbytes);
    uint32_t *hdev = nullptr;
    if ((e = hipHostGetDevicePointer((void **)&hdev, s->hmem, 0)) != hipSuccess) {
        server_free(s);
        return fail_device(e, "hipHostGetDevicePointer");
    }
    uint64_t *p = reinterpret_cast<uint64_t *>(s->dmem);
    auto take = [&](size_t nw) {
        uint64_t *q = p;
        p += nw;
        return q;
    };
    SrvDev &D = s->D;
    for (int l = 0; l < 2; l++) {
        D.start[l] = take(cap_segs);
        D.len[l] = take(cap_segs);
        D.pv[l] = take(cap_segs);
        D.job[l] = reinterpret_cast<uint32_t *>(take(cap_segs / 2 + 1));
    }
    D.count = reinterpret_cast<uint32_t *>(take(3));
    D.piv = take(cap_segs);
    D.leaf_start = take(cap_leaves);
    D.leaf_len = take(cap_leaves);
    D.leaf_job = reinterpret_cast<uint32_t *>(take(cap_leaves / 2 + 1));
    D.fb = reinterpret_cast<uint32_t *>(take(cap_leaves / 2 + 1));
    D.kind = reinterpret_cast<uint8_t *>(take(max_jobs / 8 + 1));
    D.jpivot = take(max_jobs);
    D.jstart = take(max_jobs);
    D.outstanding = reinterpret_cast<uint32_t *>(take(max_jobs / 2 + 1));
    D.h_done = hdev;
    D.h_split = reinterpret_cast<uint64_t *>(reinterpret_cast<char *>(hdev) + ((size_t)max_jobs * 4 + 63) / 64 * 64);
    D.h_flags = reinterpret_cast<uint32_t *>(D.h_split + max_jobs);
    D.cap_segs = (uint32_t)cap_segs;
    D.cap_leaves = (uint32_t)cap_leaves;
    D.max_jobs = max_jobs;
    D.leaf_cap = quicksort_leaf_cap(dtype);
    BatchState &B = s->B;
    std::memset(&B, 0, sizeof(B));
    B.pivot = D.piv;
    B.lo = take(cap_segs);
    B.hi = take(cap_segs);
    B.split = take(cap_segs);
    B.first = take(cap_segs + 1);
    B.vout = take(items);
    B.g = reinterpret_cast<uint32_t *>(take(cap_segs / 2 + 1));
    B.imap = reinterpret_cast<uint32_t *>(take(items / 2 + 1));
    B.cls = reinterpret_cast<uint8_t *>(take(cap_segs / 8 + 1));
    B.ctl = take(8);
    B.num = (uint32_t)cap_segs;
    s->stage_cap = 64 * 4 * sizeof(uint64_t) / sizeof(SrvSub);  // submissions per tick staged on the device
    s->dsub = reinterpret_cast<SrvSub *>(take(64 * 4));
    for (int i = 0; i < 2; i++) {
        if ((e = hipHostMalloc((void **)&s->stage[i], s->stage_cap * sizeof(SrvSub), hipHostMallocDefault)) !=
                hipSuccess ||
            (e = hipEventCreateWithFlags(&s->stage_ev[i], hipEventDisableTiming)) != hipSuccess) {
            (void)hipGetLastError();
            server_free(s);
            return fail_msg(SS_ENOMEM, "server staging");
        }
    }
    for (auto &ev : s->tick_ev)
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) {
            server_free(s);
            return fail_device(e, "hipEventCreate");
        }
    // zero the counters (a fill kernel would do as well; this runs once, outside any graph)
    if ((e = hipMemsetAsync(D.count, 0, 6 * sizeof(uint32_t), s->st)) != hipSuccess ||
        (e = hipMemsetAsync(D.outstanding, 0, (size_t)max_jobs * sizeof(uint32_t), s->st)) != hipSuccess) {
        server_free(s);
        return fail_device(e, "hipMemsetAsync");
    }
    s->seg_grid = (uint32_t)((cap_segs + 255) / 256);
    s->seg_grid_w = (uint32_t)((cap_segs + 3) / 4);
    *out = new ss_server{s};
    return SS_OK;
}

extern "C" int ss_server_destroy(ss_server *h)
{
    if (!h)
        return SS_OK;
    server_free(h->s);
    delete h;
    return SS_OK;
}

extern "C" int ss_server_submit(ss_server *h, uint32_t slot, uint64_t start, uint64_t len, int kind, uint64_t pivot)
{
    if (!h)
        return fail_msg(SS_EINVAL, "null server");
    Server *s = h->s;
    if (slot >= s->D.max_jobs)
        return fail_msg(SS_EINVAL, "slot out of range");
    if (kind != 0 && kind != 1)
        return fail_msg(SS_EINVAL, "kind must be 0 (partition) or 1 (sort)");
    if (start > s->capacity || len > s->capacity - start)
        return fail_msg(SS_EINVAL, "job outside the served array");
    if ((kind == 0 && len == 0) || (kind == 1 && len < 2)) {
        // nothing to do: done at once
        reinterpret_cast<volatile uint64_t *>(
            reinterpret_cast<char *>(s->hmem) + ((size_t)s->D.max_jobs * 4 + 63) / 64 * 64)[slot] = 0;
        reinterpret_cast<volatile uint32_t *>(s->hmem)[slot] = 1;
        return SS_OK;
    }
    reinterpret_cast<volatile uint32_t *>(s->hmem)[slot] = 0;
    s->pending.push_back(SrvSub{start, len, pivot, slot, (uint32_t)kind});
    return SS_OK;
}

// The tick's leaf sorts: the bucket kernel for plain keys, then the radix
// kernel over the leaves it left (records: the radix kernel alone).
template <typename T, int CAP, int KEYBITS>
static int launch_sleaves(Server *s, hipStream_t st)
{
    constexpr bool BUCKETS = leaf_buckets<T>();
    constexpr int NT = BUCKETS ? leaf_bucket_nt<T>() : kLeafRadixNT;
    if (!s->leaf_grid) {
        int cus = 0, lds = 0, occ = 0, occ_fb = 0;
        int r2 = device_info(s->dev, &cus, &lds);
        if (!r2)
            r2 = occupancy(s->dev, reinterpret_cast<const void *>(&k_sleaf<T, CAP, KEYBITS>), NT, &occ);
        if (!r2)
            r2 = occupancy(s->dev, reinterpret_cast<const void *>(&k_sleaf_fb<T, CAP, KEYBITS>), kLeafRadixNT, &occ_fb);
        if (r2)
            return r2;
        s->leaf_grid = (uint32_t)(occ * cus);
        s->leaf_grid_fb = (uint32_t)(occ_fb * cus);
    }
    hipLaunchKernelGGL((k_sleaf<T, CAP, KEYBITS>), dim3(s->leaf_grid), dim3(NT), 0, st, s->base, s->D);
    if (BUCKETS)
        hipLaunchKernelGGL((k_sleaf_fb<T, CAP, KEYBITS>), dim3(s->leaf_grid_fb), dim3(kLeafRadixNT), 0, st, s->base,
                           s->D);
    return SS_OK;
}

// Issue one tick; max_len bounds the longest segment it can hold (the longest
// active job), which sets the number of partition levels.
extern "C" int ss_server_tick(ss_server *h, uint64_t max_len)
{
    if (!h)
        return fail_msg(SS_EINVAL, "null server");
    Server *s = h->s;
    hipError_t e;
    const hipStream_t st = s->st;
    const uint32_t cur = s->cur;
    // submissions, in batches that fit the device staging area
    size_t done = 0;
    while (done < s->pending.size()) {
        const uint32_t nb = (uint32_t)std::min<size_t>(s->pending.size() - done, s->stage_cap);
        const int sb = (int)(s->ticks_issued & 1);
        if ((e = hipEventSynchronize(s->stage_ev[sb])) != hipSuccess)  // the previous copy from this buffer
            return fail_device(e, "hipEventSynchronize");
        std::memcpy(s->stage[sb], s->pending.data() + done, nb * sizeof(SrvSub));
        if ((e = hipMemcpyAsync(s->dsub, s->stage[sb], nb * sizeof(SrvSub), hipMemcpyHostToDevice, st)) !=
                hipSuccess ||
            (e = hipEventRecord(s->stage_ev[sb], st)) != hipSuccess)
            return fail_device(e, "submission copy");
        hipLaunchKernelGGL(k_ssubmit, dim3((nb + 255) / 256), dim3(256), 0, st, s->D, (const SrvSub *)s->dsub, nb,
                           cur);
        done += nb;
        if (done < s->pending.size() && (e = hipStreamSynchronize(st)) != hipSuccess)  // the device staging is reused
            return fail_device(e, "hipStreamSynchronize");
    }
    s->pending.clear();
    switch (s->dtype) {
    case SS_U32: hipLaunchKernelGGL(k_sprep<uint32_t>, dim3(s->seg_grid_w), dim3(256), 0, st, s->base, s->D, cur); break;
    case SS_U64: hipLaunchKernelGGL(k_sprep<uint64_t>, dim3(s->seg_grid_w), dim3(256), 0, st, s->base, s->D, cur); break;
    default: hipLaunchKernelGGL(k_sprep<KV>, dim3(s->seg_grid_w), dim3(256), 0, st, s->base, s->D, cur); break;
    }
    BatchState B = s->B;
    B.start = s->D.start[cur];
    B.len = s->D.len[cur];
    B.count = s->D.count + cur;
    uint32_t launches = 0;
    const uint64_t tile_elems = s->R.tile / s->R.w;
    const int rc = batched_core(s->base, s->dtype, s->R, batched_default_classes(s->R), B,
                                batched_levels(max_len ? max_len : 1, tile_elems), st, nullptr, &launches);
    if (rc)
        return rc;
    hipLaunchKernelGGL(k_schild, dim3(s->seg_grid), dim3(256), 0, st, s->D, cur, (const uint64_t *)B.split);
    int rc2;
    switch (s->dtype) {
    case SS_U32: rc2 = launch_sleaves<uint32_t, 16384, 32>(s, st); break;
    case SS_U64: rc2 = launch_sleaves<uint64_t, 16384, 64>(s, st); break;
    default: rc2 = launch_sleaves<KV, 8192, 64>(s, st); break;
    }
    if (rc2)
        return rc2;
    if ((e = hipGetLastError()) != hipSuccess)
        return fail_device(e, "tick launch");
    if ((e = hipEventRecord(s->tick_ev[s->ticks_issued & 3], st)) != hipSuccess)
        return fail_device(e, "hipEventRecord");
    s->ticks_issued++;
    s->cur ^= 1u;
    // keep at most four ticks in flight (the event ring)
    if (s->ticks_issued - s->ticks_done > 3) {
        if ((e = hipEventSynchronize(s->tick_ev[s->ticks_done & 3])) != hipSuccess)
            return fail_device(e, "hipEventSynchronize");
        s->ticks_done++;
    }
    return SS_OK;
}

// Wait until at most `in_flight` issued ticks are still running; *flags
// (nullable) receives the mirrored overflow flags (nonzero: a capacity was
// exceeded, which admission is meant to prevent).
extern "C" int ss_server_wait(ss_server *h, uint32_t in_flight, uint32_t *flags)
{
    if (!h)
        return fail_msg(SS_EINVAL, "null server");
    Server *s = h->s;
    hipError_t e;
    while (s->ticks_issued - s->ticks_done > in_flight) {
        if ((e = hipEventSynchronize(s->tick_ev[s->ticks_done & 3])) != hipSuccess)
            return fail_device(e, "hipEventSynchronize");
        s->ticks_done++;
    }
    if (flags) {
        const size_t off = ((size_t)s->D.max_jobs * 4 + 63) / 64 * 64 + (size_t)s->D.max_jobs * 8;
        *flags = *reinterpret_cast<volatile uint32_t *>(reinterpret_cast<char *>(s->hmem) + off);
    }
    return SS_OK;
}

// 1 if the job in `slot` has finished in a tick that has completed (its split,
// for a partition job, in *split), else 0.
extern "C" int ss_server_done(ss_server *h, uint32_t slot, uint64_t *split)
{
    if (!h || slot >= h->s->D.max_jobs)
        return fail_msg(SS_EINVAL, "null server or slot out of range");
    Server *s = h->s;
    const uint32_t f = reinterpret_cast<volatile uint32_t *>(s->hmem)[slot];
    if (f && split)
        *split = reinterpret_cast<volatile uint64_t *>(reinterpret_cast<char *>(s->hmem) +
                                                       ((size_t)s->D.max_jobs * 4 + 63) / 64 * 64)[slot];
    return f ? 1 : 0;
}

// Overflow flags of the device lists (0 when every capacity held).
extern "C" int ss_server_status(ss_server *h, uint32_t *flags)
{
    if (!h || !flags)
        return fail_msg(SS_EINVAL, "null argument");
    Server *s = h->s;
    hipError_t e;
    if ((e = hipStreamSynchronize(s->st)) != hipSuccess)
        return fail_device(e, "hipStreamSynchronize");
    if ((e = hipMemcpy(flags, s->D.count + 3, sizeof(uint32_t), hipMemcpyDeviceToHost)) != hipSuccess)
        return fail_device(e, "hipMemcpy");
    return SS_OK;
}

// Device bytes the job reserves in the server's lists: one list entry per
// segment that can be pending at once (a sort job of n records has at most
// n / (leaf capacity + 1) + 1 disjoint long segments), two leaf entries per
// segment, and one item per group of those segments.
extern "C" size_t ss_server_job_aux_bytes(int dtype, int kind, uint64_t len)
{
    const int w = elem_size(dtype);
    if (!w)
        return 0;
    const uint64_t segs = kind == 0 ? 1 : len / (quicksort_leaf_cap(dtype) + 1) + 1;
    const uint64_t per_seg = 2 * (3 * 8 + 4) + 8 + 3 * 8 + 8 + 4 + 1 + 2 * (16 + 4) + 3 * 12;
    return (size_t)(segs * per_seg + (len / (kDefaultRegsTile / w)) * 12 + 64);
}
