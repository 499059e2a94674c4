// ss_api.cpp -- host driver and C ABI (include/ss.h).
//
// Responsibilities: argument validation (before any device work), the
// per-(device, stream) workspace, the choice of kernel variant and grid, the
// chain of Partial Partition Step launches of the recursion (Section 4,
// Recursive Smoothed Striding), planned per call from n and closed by the
// one-workgroup serial base case, and the per-call statistics.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "ss.h"
#include "ss_common.h"
#include "ss_internal.h"

namespace ss {

thread_local std::string t_last_error;

int fail_device(hipError_t e, const char *what)
{
    t_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return SS_EDEVICE;
}

int fail_msg(int code, const std::string &msg)
{
    t_last_error = msg;
    return code;
}

namespace {

std::mutex g_mu;

struct DevInfo {
    int cus = 0;
    int lds = 0;
    int major = 0, minor = 0;
    std::map<std::pair<const void *, size_t>, int> occupancy;
};
std::map<int, DevInfo> g_dev;
std::map<std::pair<int, void *>, Workspace> g_ws;

}  // namespace

int device_info(int dev, int *cus, int *lds)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_dev.find(dev);
    if (it == g_dev.end()) {
        hipDeviceProp_t prop;
        hipError_t e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess)
            return fail_device(e, "hipGetDeviceProperties");
        DevInfo d;
        d.cus = prop.multiProcessorCount;
        d.lds = (int)prop.sharedMemPerBlock;
        d.major = prop.major;
        d.minor = prop.minor;
        it = g_dev.emplace(dev, d).first;
    }
    *cus = it->second.cus;
    *lds = it->second.lds;
    return SS_OK;
}

int occupancy(int dev, const void *fn, int nt, int *blocks, size_t shmem)
{
    std::lock_guard<std::mutex> lk(g_mu);
    DevInfo &d = g_dev[dev];
    const auto key = std::make_pair(fn, shmem);
    auto it = d.occupancy.find(key);
    if (it != d.occupancy.end()) {
        *blocks = it->second;
        return SS_OK;
    }
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, nt, shmem);
    if (e != hipSuccess)
        return fail_device(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (nb < 1)
        nb = 1;
    d.occupancy[key] = nb;
    *blocks = nb;
    return SS_OK;
}

int get_workspace(int dev, void *stream, Workspace **out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(dev, stream);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) {
        *out = &it->second;
        return SS_OK;
    }
    Workspace w;
    w.part_words = (size_t)kMaxLevels * 2 * kMaxGrid;
    w.ctl_words = (size_t)kMaxLevels * kCtlWords;
    const size_t words = w.part_words + w.ctl_words + kResultWords;
    hipError_t e = hipMalloc((void **)&w.part, words * sizeof(uint64_t));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail_msg(SS_ENOMEM, std::string("workspace hipMalloc: ") + hipGetErrorString(e));
    }
    w.ctl = w.part + w.part_words;
    w.result = w.ctl + w.ctl_words;
    e = hipHostMalloc((void **)&w.host, (w.ctl_words + kResultWords) * sizeof(uint64_t),
                      hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) {
        (void)hipFree(w.part);
        (void)hipGetLastError();
        return fail_msg(SS_ENOMEM, std::string("workspace hipHostMalloc: ") + hipGetErrorString(e));
    }
    e = hipHostGetDevicePointer((void **)&w.host_dev, w.host, 0);
    if (e != hipSuccess)
        return fail_device(e, "hipHostGetDevicePointer");
    for (int k = 0; k < 4; k++) {
        e = hipEventCreate(&w.ev[k]);
        if (e != hipSuccess)
            return fail_device(e, "hipEventCreate");
    }
    w.bytes = words * sizeof(uint64_t);
    it = g_ws.emplace(key, w).first;
    *out = &it->second;
    return SS_OK;
}

int elem_size(int dtype)
{
    switch (dtype) {
    case SS_U32: return 4;
    case SS_U64: return 8;
    case SS_KV16: return 16;
    default: return 0;
    }
}

int ilog2(uint64_t x)
{
    int r = 0;
    while ((1ull << r) < x)
        r++;
    return r;
}

// Resolve defaults and validate parameters (no device work).
int resolve_params(const ss_params *p, int dtype, Resolved *r, uint32_t auto_engine)
{
    const int w = elem_size(dtype);
    if (!w)
        return fail_msg(SS_EINVAL, "unknown dtype");
    ss_params q;
    std::memset(&q, 0, sizeof(q));
    if (p)
        q = *p;
    if (q.algo < SS_SMOOTHED || q.algo > SS_IMPLICIT)
        return fail_msg(SS_EINVAL, "unknown algo");
    if (q.flags & ~(SS_FLAG_ONE_LEVEL | SS_FLAG_TIME | SS_FLAG_GRAPH | kExchangeFlags | SS_FLAG_STABLE))
        return fail_msg(SS_EINVAL, "unknown flags");
    if (q.engine > SS_ENGINE_STAGED)
        return fail_msg(SS_EINVAL, "unknown engine");
    uint32_t engine = q.engine ? q.engine : auto_engine;
    if (!q.engine && engine == SS_ENGINE_LDS && (q.tile_bytes == 131072u || (q.flags & kExchangeFlags)))
        engine = SS_ENGINE_REGS;  // options only the register engines have
    const uint32_t tile = q.tile_bytes ? q.tile_bytes : engine == SS_ENGINE_LDS ? 32768u : kDefaultRegsTile;
    if (tile != 32768u && tile != 65536u && !(tile == 131072u && (engine == SS_ENGINE_REGS || engine == SS_ENGINE_STAGED)))
        return fail_msg(SS_EINVAL, "tile_bytes must be 32768, 65536 or (register engines) 131072");
    if ((q.flags & kExchangeFlags) && engine == SS_ENGINE_LDS)
        return fail_msg(SS_EINVAL, "the write-minimal exchange applies to the register engine");
    const uint32_t b = q.b ? q.b : kDefaultLineBytes / w;
    const uint64_t line = (uint64_t)b * w;
    if (b == 0 || (b & (b - 1)) || line < 64 || line > 4096 || line > tile)
        return fail_msg(SS_EINVAL, "b * sizeof(element) must be a power of two in [64, 4096] bytes");
    const uint32_t levels = q.max_levels;  // 0: planned per call from n (planned_levels)
    if (levels > (uint32_t)kMaxLevels)
        return fail_msg(SS_EINVAL, "max_levels above 32");
    r->algo = q.algo;
    r->engine = engine;
    r->w = w;
    r->b = b;
    r->log2b = ilog2(b);
    r->tile = tile;
    r->s_max = (uint32_t)(tile / line);
    r->levels = levels;
    r->seed = q.seed ? q.seed : 0x5EEDC0DE2004ull;
    r->flags = q.flags;
    // The automatic first-level choice needs the default geometry and the
    // register engine, and pays only for 8- and 16-byte elements.
    r->auto_xch = !q.engine && !q.tile_bytes && !q.b && w >= 8 &&
                  (engine == SS_ENGINE_REGS || engine == SS_ENGINE_STAGED) &&
                  !(q.flags & (kExchangeFlags | SS_FLAG_STABLE)) &&
                  (q.algo == SS_SMOOTHED || q.algo == SS_STRIDED || q.algo == SS_HYBRID);
    return SS_OK;
}

#define SS_LDS_VARIANT(D, T, NT, TB) \
    {D, SS_ENGINE_LDS, TB, NT, {&launch_level<T, NT, TB>}, {&level_fn<T, NT, TB>}, {0}}
#define SS_RS_FORMS(F, T, NT, NV) {F<T, NT, NV, kFormDirect>, F<T, NT, NV, kFormExchange>, F<T, NT, NV, kFormStaged>}
#define SS_RS_VARIANT(D, T, NT, NV)                                                                        \
    {D,                                                                                                    \
     SS_ENGINE_REGS,                                                                                       \
     NT * NV * 16,                                                                                         \
     NT,                                                                                                   \
     SS_RS_FORMS(&launch_level_rs_t, T, NT, NV),                                                          \
     SS_RS_FORMS(&level_rs_fn_t, T, NT, NV),                                                              \
     {level_form_lds<T, NT, NV, kFormDirect>(), level_form_lds<T, NT, NV, kFormExchange>(),              \
      level_form_lds<T, NT, NV, kFormStaged>()}}
// The automatic choice's exchange kernel: 32 KiB groups over 512 threads
// (four vectors a thread), so each wavefront ranks and swaps half as many
// elements per group as with 256 threads.
#define SS_XCH_VARIANT(D, T, NT, NV)                                                      \
    {D,                                                                                   \
     kEngineAutoExchange,                                                                 \
     NT * NV * 16,                                                                        \
     NT,                                                                                  \
     {nullptr, &launch_level_rs_t<T, NT, NV, kFormExchange>, nullptr},                    \
     {nullptr, &level_rs_fn_t<T, NT, NV, kFormExchange>, nullptr},                        \
     {0, level_form_lds<T, NT, NV, kFormExchange>(), 0}}
#define SS_RS_ALL(NT, NV) \
    SS_RS_VARIANT(SS_U32, uint32_t, NT, NV), SS_RS_VARIANT(SS_U64, uint64_t, NT, NV), SS_RS_VARIANT(SS_KV16, KV, NT, NV)

const Variant *pick_variant(int dtype, uint32_t engine, uint32_t tile)
{
    static const Variant v[] = {
        SS_LDS_VARIANT(SS_U32, uint32_t, 256, 65536), SS_LDS_VARIANT(SS_U64, uint64_t, 256, 65536),
        SS_LDS_VARIANT(SS_KV16, KV, 256, 65536),      SS_LDS_VARIANT(SS_U32, uint32_t, 256, 32768),
        SS_LDS_VARIANT(SS_U64, uint64_t, 256, 32768), SS_LDS_VARIANT(SS_KV16, KV, 256, 32768),
        SS_RS_ALL(256, 8),                            SS_RS_ALL(512, 8),
        SS_RS_ALL(512, 16),
        SS_XCH_VARIANT(SS_U64, uint64_t, 512, 4),     SS_XCH_VARIANT(SS_KV16, KV, 512, 4),
    };
    for (const Variant &x : v)
        if (x.dtype == dtype && x.engine == engine && x.tile == tile)
            return &x;
    return nullptr;
}

int check_array(const void *d_ptr, size_t n, int dtype)
{
    const int w = elem_size(dtype);
    if (!w)
        return fail_msg(SS_EINVAL, "unknown dtype");
    if (n > 0 && !d_ptr)
        return fail_msg(SS_EINVAL, "null array pointer with n > 0");
    const uintptr_t align = w == 16 ? 16 : (uintptr_t)w;
    if ((uintptr_t)d_ptr % align)
        return fail_msg(SS_EINVAL, "array pointer not aligned to its element size");
    if (n > (size_t)1 << 40)
        return fail_msg(SS_EINVAL, "n above 2^40");
    return SS_OK;
}

// Line indices are 32-bit: the first level's line count must fit.
int check_lines(uint64_t n, const Resolved &R)
{
    if ((n + 2ull * R.b) / R.b >= (1ull << 32))
        return fail_msg(SS_EINVAL, "array has 2^32 lines or more for this b; use longer lines");
    return SS_OK;
}

// Partial Partition Steps a call runs before its serial base case.  The
// first level leaves a middle region of about 4.4 / sqrt(S) of the array
// (S elements per group: the groups' predecessor counts spread about 4.4
// standard deviations each way around their mean, times g groups); each
// later level (32 KiB groups of 128-byte lines on a region that is already
// nearly partitioned) leaves about a ninth of its region.  The plan stops
// once the expected region is at most two of the base case's passes; the
// base case partitions whatever is left, so the plan affects only time.
uint32_t planned_levels(uint64_t n, const Resolved &R)
{
    const uint64_t S0 = (uint64_t)R.s_max << R.log2b;
    if (n <= S0)
        return 1;
    const double base = 2.0 * (double)cleanup_pass_elems(R.w);
    double r = (double)n * 4.4 / std::sqrt((double)S0);
    uint32_t lv = 1;
    while (r > base && lv < (uint32_t)kMaxLevels) {
        r *= 0.11;
        lv++;
    }
    return lv;
}

// Run the recursion of Smoothed Striding (or the single Strided step) on
// [lo0, hi0) of the array.  Writes the result record to ws->result and the
// split to d_split.  When `sync` it waits and fills *ro from the host copy.
// `wsx` (nullable) replaces the per-(device, stream) workspace: a workspace
// without host memory or events, for asynchronous calls only.
int run_partition(char *base, size_t n, int dtype, uint64_t pivot, const Resolved &R, hipStream_t st,
                  uint64_t *d_split, bool sync, RunOut *ro, Workspace *wsx)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail_device(e, "hipGetDevice");
    int cus = 0, lds = 0;
    int rc = device_info(dev, &cus, &lds);
    if (rc)
        return rc;
    Workspace *ws = wsx;
    if (!ws && (rc = get_workspace(dev, st, &ws)))
        return rc;
    if (wsx && (sync || (R.flags & SS_FLAG_TIME)))
        return fail_msg(SS_EINVAL, "a caller-supplied workspace serves asynchronous calls only");
    auto grid_of = [&](const void *fn, int nt, size_t shmem, uint32_t *grid) -> int {
        int occ = 0;
        const int r = occupancy(dev, fn, nt, &occ, shmem);
        const uint64_t g = (uint64_t)occ * (uint64_t)cus;
        *grid = (uint32_t)(g < (uint64_t)kMaxGrid ? g : (uint64_t)kMaxGrid);
        return r;
    };
    const bool staged = R.engine == SS_ENGINE_STAGED;
    const uint32_t regs = staged ? (uint32_t)SS_ENGINE_REGS : R.engine;
    const Variant *V = pick_variant(dtype, regs, R.tile);
    if (!V)
        return fail_msg(SS_EUNSUPPORTED, "no kernel variant for dtype/tile");
    // Store forms: the first level's (exchange if forced, else stable from
    // registers or staged in LDS), the second level's and the later levels'.
    const bool xch = (R.flags & kExchangeFlags) != 0;
    const int f0 = xch ? kFormExchange : staged ? kFormStaged : kFormDirect;
    const int f1 = xch ? kFormExchange : kFormDirect;
    const int ft = f1;
    if (!V->launch[f0] || !V->launch[f1])
        return fail_msg(SS_EUNSUPPORTED, "the write-minimal exchange needs a register engine");
    uint32_t P = 0, P1 = 0;
    if ((rc = grid_of(V->fn[f0](true), V->nt, V->lds[f0], &P)))
        return rc;
    if ((rc = grid_of(V->fn[f1](false), V->nt, V->lds[f1], &P1)))
        return rc;
    ro->grid = P;
    // Levels from the third on work on regions a few hundred times smaller
    // than the array; there a group is latency-bound, so they use 32 KiB
    // groups of 128-byte lines (more, shorter groups per level).
    const Variant *Vt = pick_variant(dtype, regs, 32768u);
    if (!Vt || !Vt->launch[ft])
        return fail_msg(SS_EUNSUPPORTED, "no tail kernel variant");
    uint32_t Pt = 0;
    if ((rc = grid_of(Vt->fn[ft](false), Vt->nt, Vt->lds[ft], &Pt)))
        return rc;
    const uint32_t log2b_t = (uint32_t)ilog2(128 / R.w), s_max_t = 32768u / 128u;
    ro->aux_bytes = ws->bytes;
    ro->launches = 0;
    ro->xch_mask = 0;
    ro->written = 0;
    ro->written0 = 0;

    // Automatic choice for large arrays: the first level is launched as a
    // pair, the stable form with the default groups and the exchange form
    // with 32 KiB groups; the stable kernel takes the choice from a sample of
    // the keys and records it, so that exactly one of them runs.
    const bool autox = R.auto_xch && n >= kAutoExchangeMin;
    const Variant *Vx = nullptr;
    const int fx = kFormExchange;
    uint32_t Px = 0;
    if (autox) {
        Vx = pick_variant(dtype, kEngineAutoExchange, 32768u);
        if (!Vx || !Vx->launch[fx])
            return fail_msg(SS_EUNSUPPORTED, "no exchange variant");
        if ((rc = grid_of(Vx->fn[fx](true), Vx->nt, Vx->lds[fx], &Px)))
            return rc;
    }

    const bool timing = (R.flags & SS_FLAG_TIME) != 0;
    const bool strided = R.algo == SS_STRIDED;
    const bool one_level = (R.flags & SS_FLAG_ONE_LEVEL) != 0;
    const uint32_t budget = one_level || strided ? 1u : R.levels ? R.levels : planned_levels(n, R);
    if (budget > ws->levels_cap)
        return fail_msg(SS_EINVAL, "more levels than the workspace holds");
    // An asynchronous call on a region of one group with a register body is
    // a single launch: the group's splitting position is the split, which the
    // first level stores itself (no base case, no host copy).
    const bool single = !sync && !timing && !one_level && !strided && !xch && !autox && d_split &&
                        regs != SS_ENGINE_LDS && n <= ((uint64_t)R.s_max << R.log2b);

    uint64_t lo = 0, hi = n;
    uint32_t level = 0;  // global level index (fresh offsets per level)
    ro->levels_run = 0;
    // Expected region of each level (the model of planned_levels): levels
    // from the third on launch about three workgroups per expected group
    // rather than a full grid, so that a small level dispatches, and the next
    // level reduces, only a few partials (a larger region than expected only
    // gives each workgroup more groups).
    const uint64_t tail_group = (uint64_t)s_max_t << log2b_t;
    double expect = (double)n * 4.4 / std::sqrt((double)((uint64_t)R.s_max << R.log2b));
    for (;;) {
        LevelArgs a;
        std::memset(&a, 0, sizeof(a));
        a.base = base;
        a.n = n;
        a.pivot = pivot;
        a.seed = R.seed;
        a.log2b = R.log2b;
        a.s_max = R.s_max;
        a.strided = strided ? 1u : 0u;
        a.xch_shift = (R.flags & SS_FLAG_EXCHANGE_SKEWED) ? kSkewShift : 0u;
        uint32_t prev_count = 0;
        const uint64_t *prev = nullptr;
        const uint64_t *prev_ctl = nullptr;
        const uint32_t first_level = level;
        // Level k of this round keeps its partials and record in slot k.
        for (uint32_t k = 0; k < budget; k++, level++) {
            const bool first = k == 0;
            const bool tail = level >= 2;
            const bool xl = xch;  // this level in the exchange form
            a.log2b = tail ? log2b_t : R.log2b;
            a.s_max = tail ? s_max_t : R.s_max;
            uint32_t grid = tail ? Pt : level == 0 ? P : P1;
            if (tail) {
                const double want = 3.0 * std::ceil(expect / (double)tail_group) + 8.0;
                if (want < (double)grid)
                    grid = (uint32_t)want;
            }
            if (level >= 1)
                expect *= 0.11;  // the region entering the next level
            if (first) {
                const Geo G = plan_geo(lo, hi, a.log2b, a.s_max);
                grid = G.g < grid ? G.g : grid;
                a.lo = lo;
                a.hi = hi;
            }
            a.level = level;
            a.prev = prev;
            a.prev_ctl = prev_ctl;
            a.prev_count = prev_count;
            a.out = ws->part + (size_t)k * 2 * kMaxGrid;
            a.ctl = ws->ctl + (size_t)k * kCtlWords;
            if (level == 0 && xch) {
                if ((e = launch_xch_prepare(dtype, base, n, pivot, ws->result, xch, st)) != hipSuccess)
                    return fail_device(e, "exchange prepare launch");
                ro->launches++;
            }
            if (timing && level == 0) {
                if ((e = hipEventRecord(ws->ev[0], st)) != hipSuccess)
                    return fail_device(e, "hipEventRecord");
            }
            a.written = xl ? ws->result + (level == 0 ? kResultWrittenFirst : kResultWritten) : nullptr;
            a.split_out = single ? d_split : nullptr;
            // without the sample kernel, the first level clears the count of stored elements
            if (level == 0 && autox) {
                // the pair: stable form (gate 0, which samples the keys and records
                // the choice), then exchange form (gate 1); the exchange form
                // leaves the stable form's partial slots alone
                a.sample_out = ws->result;
                a.gate = nullptr;
                a.gate_want = 0;
                a.gate_keep = 0;
                if ((e = V->launch[f0](first, grid, a, st)) != hipSuccess)
                    return fail_device(e, "level kernel launch");
                LevelArgs ax = a;
                ax.s_max = (uint32_t)(Vx->tile / ((uint64_t)R.b * R.w));
                const Geo Gx = plan_geo(lo, hi, ax.log2b, ax.s_max);
                const uint32_t grid_x = Gx.g < Px ? Gx.g : Px;
                ax.sample_out = nullptr;
                ax.gate = ws->result + kResultGate;
                ax.gate_want = 1;
                ax.gate_keep = grid;
                ax.written = ws->result + kResultWrittenFirst;
                if ((e = Vx->launch[fx](first, grid_x, ax, st)) != hipSuccess)
                    return fail_device(e, "level kernel launch");
                ro->launches += 2;
                a.sample_out = nullptr;
                a.gate = nullptr;
                a.written = nullptr;
                grid = grid_x > grid ? grid_x : grid;
            } else {
                const LevelLaunch L = level == 0 ? V->launch[f0] : tail ? Vt->launch[ft] : V->launch[f1];
                if ((e = L(first, grid, a, st)) != hipSuccess)
                    return fail_device(e, "level kernel launch");
                ro->launches++;
                if (xl && level < 64)
                    ro->xch_mask |= 1ull << level;
            }
            if (timing && level == 0) {
                if ((e = hipEventRecord(ws->ev[1], st)) != hipSuccess)
                    return fail_device(e, "hipEventRecord");
            }
            prev = a.out;
            prev_ctl = a.ctl;
            prev_count = grid;
        }
        uint64_t *host = sync ? ws->host_dev : nullptr;
        if (single) {
            ro->levels_run = level;
            return SS_OK;
        }
        if (!one_level) {
            // The serial base case (Recursive Smoothed Striding) or the Serial
            // Cleanup Step (Strided): one workgroup partitions [v_min, v_max).
            if ((e = launch_cleanup(dtype, base, pivot, prev, prev_count, ws->result, d_split, ws->ctl, budget, host,
                                    st)) != hipSuccess)
                return fail_device(e, "cleanup kernel launch");
            ro->launches++;
        } else {
            if ((e = launch_finish(prev, prev_count, prev_ctl, ws->result, d_split, ws->ctl, budget, host, st)) !=
                hipSuccess)
                return fail_device(e, "finish kernel launch");
            ro->launches++;
        }
        ro->levels_run = level;
        if (!sync)
            return SS_OK;
        if ((e = hipStreamSynchronize(st)) != hipSuccess)
            return fail_device(e, "hipStreamSynchronize");
        const volatile uint64_t *res = ws->host;
        for (uint32_t k = 0; k < budget; k++) {
            const uint32_t l = first_level + k;
            if (l >= (uint32_t)SS_MAX_LEVELS)
                break;
            const volatile uint64_t *c = ws->host + kResultWordsDev + (size_t)k * kCtlWords;
            ro->level_lo[l] = c[0];
            ro->level_hi[l] = c[1];
            ro->level_g[l] = (uint32_t)c[2];
            ro->level_s[l] = (uint32_t)c[3];
        }
        ro->vmin = res[2];
        ro->vmax = res[3];
        if (autox && res[kResultGate]) {
            ro->xch_mask |= 1ull;
            ro->grid = Px;
        }
        if (ro->xch_mask) {
            ro->written = res[kResultWritten] + ((ro->xch_mask & 1) ? res[kResultWrittenFirst] : 0);
            ro->written0 = (ro->xch_mask & 1) ? res[kResultWrittenFirst] : 0;
        }
        if (res[0] || (R.flags & SS_FLAG_ONE_LEVEL)) {
            ro->done = res[0] != 0;
            ro->split = res[1];
            break;
        }
        if (level >= kHostLevelCap)
            return fail_msg(SS_EDEVICE, "recursion did not converge");
        lo = res[2];
        hi = res[3];
    }
    if (timing) {
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, ws->ev[0], ws->ev[1])) != hipSuccess)
            return fail_device(e, "hipEventElapsedTime");
        ro->first_level_ms = ms;
    }
    return SS_OK;
}

void fill_stats(ss_stats *st, const RunOut &ro, const Resolved &R, int dtype)
{
    std::memset(st, 0, sizeof(*st));
    st->split = ro.split;
    st->aux_bytes = ro.aux_bytes;
    st->grid = ro.grid;
    st->b = R.b;
    st->s_max = R.s_max;
    st->launches = ro.launches;
    st->vmin = ro.vmin;
    st->vmax = ro.vmax;
    st->first_level_ms = ro.first_level_ms;
    st->total_ms = ro.total_ms;
    st->lds_bytes = R.tile + R.tile / 64 * 4 + 1024;
    uint64_t moved = 0;
    uint32_t lv = 0, xn = 0, xm = 0;
    for (uint32_t l = 0; l < ro.levels_run && l < (uint32_t)SS_MAX_LEVELS; l++) {
        if (ro.level_hi[l] > ro.level_lo[l]) {
            st->level_lo[lv] = ro.level_lo[l];
            st->level_hi[lv] = ro.level_hi[l];
            st->level_g[lv] = ro.level_g[l];
            st->level_s[lv] = ro.level_s[l];
            // a level in the exchange form reads its region and writes only what it stored
            const bool x = l < 64 && ((ro.xch_mask >> l) & 1);
            moved += (x ? 1ull : 2ull) * elem_size(dtype) * (ro.level_hi[l] - ro.level_lo[l]);
            if (x) {
                xn++;
                xm |= 1u << lv;
            }
            lv++;
        }
    }
    st->levels = lv;
    st->bytes_moved = moved + (uint64_t)elem_size(dtype) * ro.written;
    st->exchange_levels = xn;
    st->exchange_mask = xm;
    if (ro.levels_run && ro.level_hi[0] > ro.level_lo[0])
        st->first_level_bytes = (uint64_t)elem_size(dtype) * ((ro.xch_mask & 1) ? (ro.level_hi[0] - ro.level_lo[0]) + ro.written0
                                                                             : 2 * (ro.level_hi[0] - ro.level_lo[0]));
}

}  // namespace ss

using namespace ss;

extern "C" {

// Hybrid Smoothed Striding (Section 4): one Partial Partition Step, then the
// Blocked-Prefix-Sum partition (the Low-Space implementation) of the middle
// region [v_min, v_max).  The host reads (v_min, v_max) between the phases.
static int hybrid_partition(char *base, size_t n, int dtype, uint64_t pivot, const Resolved &R, hipStream_t st,
                            uint64_t *d_split, size_t *h_split, ss_stats *stats)
{
    Resolved R1 = R;
    R1.algo = SS_SMOOTHED;
    R1.flags = R.flags | SS_FLAG_ONE_LEVEL;  // with SS_FLAG_TIME the first level is timed as usual
    RunOut ro;
    std::memset(&ro, 0, sizeof(ro));
    hipEvent_t t0 = nullptr, t1 = nullptr;
    const bool timing = (R.flags & SS_FLAG_TIME) != 0;
    if (timing) {
        if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
            return fail_msg(SS_EDEVICE, "hipEventCreate");
        (void)hipEventRecord(t0, st);
    }
    int rc = run_partition(base, n, dtype, pivot, R1, st, nullptr, true, &ro, nullptr);
    if (rc)
        return rc;
    uint64_t split = ro.vmin;
    size_t mid_aux = 0;
    if (!(R.flags & SS_FLAG_ONE_LEVEL) && ro.vmax > ro.vmin) {
        Resolved R2 = R;
        R2.algo = SS_LOWSPACE;
        R2.flags = R.flags & ~SS_FLAG_TIME;
        size_t sub = 0;
        ss_stats st2;
        rc = lowspace_partition(base + ro.vmin * (uint64_t)R.w, (size_t)(ro.vmax - ro.vmin), dtype, pivot, R2, st,
                                nullptr, &sub, &st2);
        if (rc)
            return rc;
        split = ro.vmin + sub;
        mid_aux = st2.aux_bytes;
    }
    if (timing) {
        (void)hipEventRecord(t1, st);
        (void)hipEventSynchronize(t1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, t0, t1);
        ro.total_ms = ms;
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
    }
    if (d_split) {
        hipError_t e = hipMemcpy(d_split, &split, sizeof(split), hipMemcpyHostToDevice);
        if (e != hipSuccess)
            return fail_device(e, "hipMemcpy");
    }
    if (h_split)
        *h_split = (size_t)split;
    if (stats) {
        ro.split = split;
        fill_stats(stats, ro, R, dtype);
        stats->split = split;
        stats->aux_bytes = ro.aux_bytes > mid_aux ? ro.aux_bytes : mid_aux;
        if (!(R.flags & SS_FLAG_ONE_LEVEL)) {
            stats->vmin = split;
            stats->vmax = split;
        }
    }
    return SS_OK;
}

int ss_partition_ex(void *d_ptr, size_t n, int dtype, uint64_t pivot, const ss_params *p, void *stream,
                    uint64_t *d_split, size_t *h_split, ss_stats *stats)
{
    int rc = check_array(d_ptr, n, dtype);
    if (rc)
        return rc;
    Resolved R;
    // single-array calls: the first level is staged in LDS (see SS_ENGINE_AUTO)
    rc = resolve_params(p, dtype, &R, SS_ENGINE_STAGED);
    if (rc)
        return rc;
    if (R.algo == SS_LOWSPACE || R.algo == SS_IMPLICIT)
        return lowspace_partition((char *)d_ptr, n, dtype, pivot, R, (hipStream_t)stream, d_split, h_split,
                                  stats);
    if (R.algo == SS_MEDIUMSPACE || R.algo == SS_HIGHSPACE)
        return prefix_partition((char *)d_ptr, n, dtype, pivot, R, (hipStream_t)stream, d_split, h_split, stats,
                                R.algo == SS_HIGHSPACE);
    if ((rc = check_lines(n, R)))
        return rc;
    if (R.algo == SS_HYBRID) {
        if (d_split && ((uintptr_t)d_split % 8))
            return fail_msg(SS_EINVAL, "d_split not 8-byte aligned");
        if (n == 0) {
            if (h_split)
                *h_split = 0;
            const uint64_t zero = 0;
            if (d_split && hipMemcpy(d_split, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess)
                return fail_msg(SS_EDEVICE, "hipMemcpy");
            if (stats) {
                RunOut ro;
                std::memset(&ro, 0, sizeof(ro));
                fill_stats(stats, ro, R, dtype);
            }
            return SS_OK;
        }
        return hybrid_partition((char *)d_ptr, n, dtype, pivot, R, (hipStream_t)stream, d_split, h_split, stats);
    }
    if (d_split && ((uintptr_t)d_split % 8))
        return fail_msg(SS_EINVAL, "d_split not 8-byte aligned");
    const bool sync = h_split || stats;
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {
        if (d_split) {
            hipError_t e = hipMemsetAsync(d_split, 0, sizeof(uint64_t), st);
            if (e != hipSuccess)
                return fail_device(e, "hipMemsetAsync");
        }
        if (sync) {
            hipError_t e = hipStreamSynchronize(st);
            if (e != hipSuccess)
                return fail_device(e, "hipStreamSynchronize");
        }
        if (h_split)
            *h_split = 0;
        if (stats) {
            RunOut ro;
            std::memset(&ro, 0, sizeof(ro));
            fill_stats(stats, ro, R, dtype);
        }
        return SS_OK;
    }
    RunOut ro;
    std::memset(&ro, 0, sizeof(ro));
    hipEvent_t t0 = nullptr, t1 = nullptr;
    const bool timing = (R.flags & SS_FLAG_TIME) != 0;
    if (timing) {
        if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
            return fail_msg(SS_EDEVICE, "hipEventCreate");
        (void)hipEventRecord(t0, st);
    }
    rc = run_partition((char *)d_ptr, n, dtype, pivot, R, st, d_split, sync || timing, &ro, nullptr);
    if (timing) {
        (void)hipEventRecord(t1, st);
        (void)hipEventSynchronize(t1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, t0, t1);
        ro.total_ms = ms;
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
    }
    if (rc)
        return rc;
    if (h_split)
        *h_split = (size_t)ro.split;
    if (stats)
        fill_stats(stats, ro, R, dtype);
    return SS_OK;
}

int ss_partition_each(void *d_base, const uint64_t *h_offsets, size_t num, int dtype, const uint64_t *h_pivots,
                      uint64_t *d_splits, const ss_params *p, void *stream, float *h_ms)
{
    if (num == 0)
        return SS_OK;
    if (!h_offsets || !h_pivots || !d_splits)
        return fail_msg(SS_EINVAL, "null offsets, pivots or splits");
    if ((uintptr_t)d_splits % 8)
        return fail_msg(SS_EINVAL, "d_splits not 8-byte aligned");
    for (size_t k = 0; k < num; k++)
        if (h_offsets[k + 1] < h_offsets[k])
            return fail_msg(SS_EINVAL, "offsets must not decrease");
    int rc = check_array(d_base, (size_t)h_offsets[num], dtype);
    if (rc)
        return rc;
    Resolved R;
    rc = resolve_params(p, dtype, &R, SS_ENGINE_STAGED);
    if (rc)
        return rc;
    if (R.algo != SS_SMOOTHED && R.algo != SS_STRIDED)
        return fail_msg(SS_EINVAL, "ss_partition_each runs Smoothed Striding or Strided");
    if ((rc = check_lines(h_offsets[num], R)))
        return rc;
    R.flags &= ~SS_FLAG_TIME;
    hipStream_t st = (hipStream_t)stream;
    const int w = elem_size(dtype);
    static thread_local std::vector<hipEvent_t> evs;
    if (h_ms) {
        while (evs.size() < num + 1) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess)
                return fail_msg(SS_EDEVICE, "hipEventCreate");
            evs.push_back(e);
        }
        if (hipEventRecord(evs[0], st) != hipSuccess)
            return fail_msg(SS_EDEVICE, "hipEventRecord");
    }
    for (size_t k = 0; k < num; k++) {
        const uint64_t n = h_offsets[k + 1] - h_offsets[k];
        if (n == 0) {
            const hipError_t e = hipMemsetAsync(d_splits + k, 0, sizeof(uint64_t), st);
            if (e != hipSuccess)
                return fail_device(e, "hipMemsetAsync");
        } else {
            RunOut ro;
            std::memset(&ro, 0, sizeof(ro));
            if ((rc = run_partition((char *)d_base + h_offsets[k] * (uint64_t)w, (size_t)n, dtype, h_pivots[k], R, st,
                                    d_splits + k, false, &ro, nullptr)))
                return rc;
        }
        if (h_ms && hipEventRecord(evs[k + 1], st) != hipSuccess)
            return fail_msg(SS_EDEVICE, "hipEventRecord");
    }
    if (h_ms) {
        hipError_t e = hipEventSynchronize(evs[num]);
        if (e != hipSuccess)
            return fail_device(e, "hipEventSynchronize");
        for (size_t k = 0; k < num; k++)
            if ((e = hipEventElapsedTime(&h_ms[k], evs[0], evs[k + 1])) != hipSuccess)
                return fail_device(e, "hipEventElapsedTime");
    }
    return SS_OK;
}

int ss_partition(void *d_ptr, size_t n, int dtype, uint64_t pivot, size_t *split)
{
    if (!split)
        return fail_msg(SS_EINVAL, "split must not be NULL");
    return ss_partition_ex(d_ptr, n, dtype, pivot, nullptr, nullptr, nullptr, split, nullptr);
}

size_t ss_aux_bytes(size_t n, int dtype, int algo)
{
    if (!elem_size(dtype))
        return 0;
    const size_t ws = ((size_t)kMaxLevels * 2 * kMaxGrid + (size_t)kMaxLevels * kCtlWords + kResultWords) *
                      sizeof(uint64_t);
    if (algo == SS_LOWSPACE || algo == SS_HYBRID)  // hybrid: Low-Space arrays for the middle region (< n)
        return ws + lowspace_aux_bytes(n);
    if (algo == SS_IMPLICIT)
        return ws + lowspace_aux_bytes(implicit_work_elems(n, dtype));
    if (algo == SS_MEDIUMSPACE || algo == SS_HIGHSPACE)
        return ws + prefix_aux_bytes(n, dtype, algo == SS_HIGHSPACE);
    return ws;
}

const char *ss_strerror(int code)
{
    switch (code) {
    case SS_OK: return "success";
    case SS_EINVAL: return "invalid argument";
    case SS_ENOMEM: return "device workspace allocation failed";
    case SS_EDEVICE: return "HIP runtime or kernel failure";
    case SS_EUNSUPPORTED: return "unsupported combination";
    case SS_EINCOMPLETE: return "recursion budget exhausted";
    default: return "unknown status";
    }
}

const char *ss_last_error(void) { return t_last_error.c_str(); }

int ss_device_info(int *compute_units, int *lds_per_block, int *arch_major, int *arch_minor)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail_device(e, "hipGetDevice");
    int cus = 0, lds = 0;
    int rc = device_info(dev, &cus, &lds);
    if (rc)
        return rc;
    if (compute_units)
        *compute_units = cus;
    if (lds_per_block)
        *lds_per_block = lds;
    std::lock_guard<std::mutex> lk(g_mu);
    if (arch_major)
        *arch_major = g_dev[dev].major;
    if (arch_minor)
        *arch_minor = g_dev[dev].minor;
    return SS_OK;
}

}  // extern "C"
