// ss_quicksort.hip -- parallel quicksort built on the partition (Section 5.2,
// "Example Application: A Full Quicksort").
//
// The paper's quicksort uses the parallel partition at the upper levels and a
// serial partition once a subproblem is small.  Here every level partitions
// all segments longer than the leaf size at once with the batched Smoothed
// Striding partition, and the short segments are finished by a
// workgroup-local radix sort in LDS.
//
// Per level:
//   * k_qpivot: median of the keys at lo, lo + len/2 and hi - 1 of every
//     segment (median-of-3);
//   * batched partition by key < p;
//   * a segment with no key below p (p is its minimum) is partitioned again
//     by key <= p: its equal keys form a block that is final, so every level
//     makes progress even when keys repeat; otherwise both parts are strictly
//     smaller than the segment because p itself is on the right;
//   * children longer than the leaf size become the next level's segments,
//     the others (of two elements or more) leaves.
// Leaves: one workgroup per leaf; least-significant-digit radix sort with
// 8-bit digits over the key (KV16 records move with their key).  Within a
// pass, each wavefront ranks 64 elements at a time: eight ballots give each
// lane the mask of lanes holding the same digit, the lowest lane of that
// mask advances the wavefront's counter for the digit, and a scan over
// (digit, wavefront) turns the counters into destinations.  The sort is
// stable and needs no atomics.
#include "ss_common.h"
#include "ss_device.h"
#include "ss_internal.h"

#include <cstring>
#include <map>
#include <mutex>
#include <vector>

namespace ss {

template <typename T>
__device__ __forceinline__ uint64_t qkey(const T &x)
{
    return key_of(x);
}

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

template <typename T>
struct Digit {
    __device__ static __forceinline__ uint32_t of(const T &x, uint32_t sh) { return (uint32_t)(qkey(x) >> sh) & 255u; }
};

// One workgroup sorts leaf blockIdx.x (at most CAP elements) by key.
template <typename T, int CAP, int KEYBITS>
__global__ void __launch_bounds__(1024) k_qleaf(char *base, const uint64_t *start, const uint64_t *len)
{
    constexpr int NT = 1024, NW = NT / 64;
    constexpr int E = CAP / NT;  // elements per thread
    __shared__ T buf[CAP];
    __shared__ uint32_t cnt[NW][256];
    __shared__ uint32_t dig_base[256];

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    T *A = reinterpret_cast<T *>(base) + start[blockIdx.x];
    const uint32_t n = (uint32_t)len[blockIdx.x];
    const uint64_t lt = (1ull << lane) - 1;

    // Striped arrangement: element r of thread (wid, lane) is at
    // index wid * 64 * E + r * 64 + lane, so element order is (wave, round, lane).
    T x[E];
    bool valid[E];
    for (int r = 0; r < E; r++) {
        const uint32_t idx = wid * 64 * E + r * 64 + lane;
        valid[r] = idx < n;
        if (valid[r])
            x[r] = A[idx];
    }
    for (uint32_t sh = 0; sh < KEYBITS; sh += 8) {
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
}

namespace {

struct QsWork {
    uint64_t *dev = nullptr;     // pivots (second pass), leaf list
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

hipError_t launch_qleaf(int dtype, char *base, const uint64_t *start, const uint64_t *len, uint32_t nleaves,
                        hipStream_t st)
{
    switch (dtype) {
    case SS_U32:
        hipLaunchKernelGGL((k_qleaf<uint32_t, 16384, 32>), dim3(nleaves), dim3(1024), 0, st, base, start, len);
        break;
    case SS_U64:
        hipLaunchKernelGGL((k_qleaf<uint64_t, 16384, 64>), dim3(nleaves), dim3(1024), 0, st, base, start, len);
        break;
    default:
        hipLaunchKernelGGL((k_qleaf<KV, 8192, 64>), dim3(nleaves), dim3(1024), 0, st, base, start, len);
        break;
    }
    return hipGetLastError();
}

}  // namespace

uint64_t quicksort_leaf_cap(int dtype) { return dtype == SS_KV16 ? 8192 : 16384; }

int quicksort_run(char *base, size_t n, int dtype, const Resolved &R, hipStream_t st, uint32_t *levels_out,
                  uint32_t *launches)
{
    hipError_t e;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess)
        return fail_device(e, "hipGetDevice");
    const uint64_t cap = quicksort_leaf_cap(dtype);
    const size_t max_segs = n / cap + 2;
    const size_t max_leaves = 2 * max_segs * 64 + 16;
    QsWork *w = nullptr;
    int rc = qs_reserve(dev, st, max_segs + 2 * max_leaves, 2 * max_segs, 2 * max_leaves + 3 * max_segs, &w);
    if (rc)
        return rc;
    uint64_t *piv2_dev = w->dev;                      // pivots of the second pass
    uint64_t *leaf_dev = w->dev + max_segs;           // leaves: starts then lengths
    uint64_t *piv_host = w->host, *piv_host_dev = w->host_dev;
    uint64_t *split_host = w->host + max_segs, *split_host_dev = w->host_dev + max_segs;

    std::vector<uint64_t> seg_start, seg_len, leaf_start, leaf_len;
    if (n > cap) {
        seg_start.push_back(0);
        seg_len.push_back(n);
    } else if (n >= 2) {
        leaf_start.push_back(0);
        leaf_len.push_back(n);
    }
    uint32_t levels = 0;
    std::vector<uint64_t> nxt_start, nxt_len, eq_idx;
    auto add_child = [&](uint64_t s, uint64_t l) {
        if (l > cap) {
            nxt_start.push_back(s);
            nxt_len.push_back(l);
        } else if (l >= 2) {
            leaf_start.push_back(s);
            leaf_len.push_back(l);
        }
    };
    while (!seg_start.empty()) {
        const uint32_t m = (uint32_t)seg_start.size();
        const uint64_t icap = batched_items_cap(seg_len.data(), m, R.tile / R.w);
        BatchState B;
        uint64_t *bstage = nullptr;
        if ((rc = batched_state(dev, st, m, icap, &B, &bstage)))
            return rc;
        if ((e = hipStreamSynchronize(st)) != hipSuccess)
            return fail_device(e, "hipStreamSynchronize");
        std::memcpy(bstage, seg_start.data(), m * sizeof(uint64_t));
        std::memcpy(bstage + m, seg_len.data(), m * sizeof(uint64_t));
        if ((e = hipMemcpyAsync(B.start, bstage, 2 * (size_t)m * sizeof(uint64_t), hipMemcpyHostToDevice, st)) !=
            hipSuccess)
            return fail_device(e, "hipMemcpyAsync");
        // median-of-3 pivots, on the device and in mapped host memory
        switch (dtype) {
        case SS_U32: e = launch_qpivot<uint32_t>(base, B, m, piv2_dev, piv_host_dev, st); break;
        case SS_U64: e = launch_qpivot<uint64_t>(base, B, m, piv2_dev, piv_host_dev, st); break;
        default: e = launch_qpivot<KV>(base, B, m, piv2_dev, piv_host_dev, st); break;
        }
        if (e != hipSuccess)
            return fail_device(e, "pivot launch");
        (*launches)++;
        B.pivot = piv2_dev;
        uint32_t lv = 0;
        if ((rc = batched_core(base, dtype, R, B, icap, st, split_host_dev, true, launches, &lv)))
            return rc;
        if ((e = hipStreamSynchronize(st)) != hipSuccess)
            return fail_device(e, "hipStreamSynchronize");
        levels++;
        // children; segments whose pivot was their minimum need the <= pass
        nxt_start.clear();
        nxt_len.clear();
        eq_idx.clear();
        std::vector<uint64_t> split1(split_host, split_host + m), piv(piv_host, piv_host + m);
        for (uint32_t k = 0; k < m; k++) {
            const uint64_t s1 = split1[k];
            if (s1 == ~0ull)
                return fail_msg(SS_EDEVICE, "quicksort: unfinished partition");
            if (s1 == 0) {
                eq_idx.push_back(k);
                continue;
            }
            add_child(seg_start[k], s1);
            add_child(seg_start[k] + s1, seg_len[k] - s1);
        }
        if (!eq_idx.empty()) {
            std::vector<uint64_t> es, el, ep;
            for (uint64_t k : eq_idx) {
                if (piv[k] == ~0ull) {
                    continue;  // every key equals the largest possible key: the segment is sorted
                }
                es.push_back(seg_start[k]);
                el.push_back(seg_len[k]);
                ep.push_back(piv[k] + 1);  // key <= p  <=>  key < p + 1
            }
            const uint32_t m2 = (uint32_t)es.size();
            if (m2) {
                const uint64_t icap2 = batched_items_cap(el.data(), m2, R.tile / R.w);
                BatchState B2;
                if ((rc = batched_state(dev, st, m2, icap2, &B2, &bstage)))
                    return rc;
                if ((e = hipStreamSynchronize(st)) != hipSuccess)
                    return fail_device(e, "hipStreamSynchronize");
                std::memcpy(bstage, es.data(), m2 * sizeof(uint64_t));
                std::memcpy(bstage + m2, el.data(), m2 * sizeof(uint64_t));
                std::memcpy(w->stage, ep.data(), m2 * sizeof(uint64_t));
                if ((e = hipMemcpyAsync(B2.start, bstage, 2 * (size_t)m2 * sizeof(uint64_t), hipMemcpyHostToDevice,
                                        st)) != hipSuccess ||
                    (e = hipMemcpyAsync(piv2_dev, w->stage, m2 * sizeof(uint64_t), hipMemcpyHostToDevice, st)) !=
                        hipSuccess)
                    return fail_device(e, "hipMemcpyAsync");
                B2.pivot = piv2_dev;
                if ((rc = batched_core(base, dtype, R, B2, icap2, st, split_host_dev, true, launches, &lv)))
                    return rc;
                if ((e = hipStreamSynchronize(st)) != hipSuccess)
                    return fail_device(e, "hipStreamSynchronize");
                for (uint32_t k = 0; k < m2; k++) {
                    const uint64_t s2 = split_host[k];
                    if (s2 == ~0ull || s2 == 0)
                        return fail_msg(SS_EDEVICE, "quicksort: unfinished equal-key pass");
                    add_child(es[k] + s2, el[k] - s2);  // [start, start + s2) holds only the pivot's key
                }
            }
        }
        seg_start.swap(nxt_start);
        seg_len.swap(nxt_len);
        if (leaf_start.size() > max_leaves)
            return fail_msg(SS_EDEVICE, "quicksort: leaf list overflow");
        if (levels > 4096)
            return fail_msg(SS_EDEVICE, "quicksort: no progress");
    }
    const size_t nl = leaf_start.size();
    if (nl) {
        std::memcpy(w->stage, leaf_start.data(), nl * sizeof(uint64_t));
        std::memcpy(w->stage + nl, leaf_len.data(), nl * sizeof(uint64_t));
        if ((e = hipMemcpyAsync(leaf_dev, w->stage, 2 * nl * sizeof(uint64_t), hipMemcpyHostToDevice, st)) !=
            hipSuccess)
            return fail_device(e, "hipMemcpyAsync");
        for (size_t k0 = 0; k0 < nl; k0 += 65535) {
            const uint32_t cnt = (uint32_t)(nl - k0 < 65535 ? nl - k0 : 65535);
            if ((e = launch_qleaf(dtype, base, leaf_dev + k0, leaf_dev + nl + k0, cnt, st)) != hipSuccess)
                return fail_device(e, "leaf sort launch");
            (*launches)++;
        }
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess)
        return fail_device(e, "hipStreamSynchronize");
    *levels_out = levels;
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
    if ((rc = resolve_params(p, dtype, &R)))
        return rc;
    if (R.algo != SS_SMOOTHED)
        return fail_msg(SS_EUNSUPPORTED, "quicksort levels use the batched Smoothed Striding partition");
    if (R.engine != SS_ENGINE_REGS)
        return fail_msg(SS_EUNSUPPORTED, "quicksort levels use the register engine");
    if (!p || !p->max_levels)
        R.levels = 6;
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
    int rc = qs_reserve(dev, st, 2 * num + 16, 16, 2 * num + 16, &w);
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
    for (size_t k0 = 0; k0 < num; k0 += 65535) {
        const uint32_t cnt = (uint32_t)(num - k0 < 65535 ? num - k0 : 65535);
        if ((e = launch_qleaf(dtype, (char *)d_base, ds + k0, dl + k0, cnt, st)) != hipSuccess)
            return fail_device(e, "segment sort launch");
    }
    return SS_OK;
}
