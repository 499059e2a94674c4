// ss_level_rs.h -- register-resident Partial Partition Step (kernel template;
// ss_level_rs.hip instantiates the stable form, ss_level_xch.hip the
// write-minimal exchange).
//
// Same step and same result as the LDS-tile kernel (one Partial Partition
// Step of Smoothed Striding, Section 4; stable partition of every group
// U_i's slot sequence, so the arrangement is identical), but the group's
// elements stay in VGPRs and each element is stored directly to its
// destination line: predecessors to slot rank, successors to slot
// c_i + (slot - rank).  Without an LDS tile the number of resident
// workgroups per CU is bounded only by registers, so more of a group's bytes
// are in flight per CU, and groups can be larger (a smaller middle region)
// at the same occupancy.  Stores are 4/8/16-byte scattered writes; a
// wavefront's predecessors (and successors) go to consecutive slots, so each
// store instruction covers a few contiguous runs of lines, which the L2
// merges into whole-line writes.
//
// Per group: (1) load the group's lines into registers (16-byte vectors, 8
// lanes per 128-byte line); (2) evaluate key < pivot and count predecessors
// per (round, wave) with ballots; (3) one wave scans those counts; (4) each
// element's rank is recomputed from the ballots and the element is stored;
// (5) the next group's loads are issued; (6) thread 0 folds v_i into the
// workgroup's (v_min, v_max).
//
// With the write-minimal exchange (SS_FLAG_EXCHANGE) step (4) instead swaps
// the misplaced pairs of the group through a table of slot numbers in LDS
// and writes only those elements: at a skewed pivot most lines are never
// written.  With groups of at most 32 KiB the exchange stages the group in
// an LDS tile and issues the next group's loads before ranking it.
//
// A group whose lines are all real and that fills the whole tile (every
// group of a level except at most the two touching the region's ends, and
// the last partial round of small regions) takes a branch-free path; the
// others take a general path that masks virtual elements (front padding up
// to the line boundary, padding after the region's end).
#pragma once

#include "ss_common.h"
#include "ss_device.h"
#include "ss_internal.h"
#include "ss_levelctx.h"

namespace ss {

// The exchange form with groups of at most 32 KiB stages each group in an
// LDS tile and loads the next group into registers while the current one is
// ranked and swapped (its barriers wait for LDS only), so HBM reads stay in
// flight through the exchange's passes.
template <typename T, int NT, int NV, int FORM>
constexpr bool xch_prefetch()
{
    return FORM == kFormExchange && NT * NV * 16 <= 32768;
}

// Store forms: kForm* in ss_common.h.
template <typename T, int NT, int NV, bool FIRST, int FORM>
__global__ void __launch_bounds__(NT) k_level_rs(const LevelArgs a)
{
    constexpr bool XCH = FORM == kFormExchange;
    constexpr bool STAGED = FORM == kFormStaged;
    constexpr bool PREFETCH = xch_prefetch<T, NT, NV, FORM>();
    using Ctx = LevelCtx<T, NT, NV, PREFETCH>;
    constexpr int W = Ctx::W;
    constexpr int NW = Ctx::NW;
    constexpr int MAXS = Ctx::NVEC * 16 / 64;  // lines of at least 64 bytes
    static_assert(Ctx::E <= 256 && NV * Ctx::V <= 64, "tile shape");

    __shared__ uint32_t xoff[MAXS];
    __shared__ uint32_t cnt[Ctx::E + 2];
    __shared__ uint64_t red[2 * NW];

    const int tid = threadIdx.x;
    const uint32_t bid = blockIdx.x;

    // A first level launched as one of a stable/exchange pair: the kernel the
    // choice does not select only leaves neutral partials behind.  The first
    // kernel of the pair takes the choice from the key sample (every
    // workgroup reads the same 4096 keys) and records it for the second.
    if (FIRST && a.sample_out) {
        __shared__ uint32_t sampled;
        if (tid == 0)
            sampled = 0;
        __syncthreads();
        uint32_t mine = 0;
        const T *const A = reinterpret_cast<const T *>(a.base);
        for (uint32_t k = tid; k < kGateSamples; k += NT) {
            const uint64_t pos = (uint64_t)(k / kGateRunLen) * a.n / kGateRuns + k % kGateRunLen;
            mine += key_of(A[pos < a.n ? pos : a.n - 1]) < a.pivot;
        }
        atomicAdd(&sampled, mine);
        __syncthreads();
        const uint32_t skewed = gate_skewed(sampled, W) ? 1u : 0u;
        if (bid == 0 && tid == 0) {
            a.sample_out[kResultGate] = skewed;
            a.sample_out[kResultWritten] = 0ull;
            a.sample_out[kResultWrittenFirst] = 0ull;
        }
        if (skewed != a.gate_want) {
            if (tid == 0 && bid >= a.gate_keep) {
                a.out[2 * bid] = ~0ull;
                a.out[2 * bid + 1] = 0ull;
            }
            return;
        }
    }
    if (FIRST && a.gate && *a.gate != a.gate_want) {
        if (tid == 0 && bid >= a.gate_keep) {
            a.out[2 * bid] = ~0ull;
            a.out[2 * bid + 1] = 0ull;
        }
        return;
    }

    uint64_t lo, hi;
    if (FIRST) {
        lo = a.lo;
        hi = a.hi;
    } else {
        prev_region<NT>(a.prev, a.prev_count, a.prev_ctl, red, lo, hi);
    }
    if (!(lo < hi)) {
        if (tid == 0) {
            a.out[2 * bid] = bid == 0 ? lo : ~0ull;
            a.out[2 * bid + 1] = bid == 0 ? lo : 0ull;
            if (bid == 0) {
                a.ctl[0] = lo; a.ctl[1] = lo; a.ctl[2] = 0; a.ctl[3] = 0;
            }
        }
        return;
    }

    const Geo G = plan_geo(lo, hi, a.log2b, a.s_max);
    Ctx x;
    x.g = G.g;
    x.s = G.s;
    x.fp = G.fp;
    x.real_end = (uint64_t)G.fp + (hi - lo);
    x.A0 = a.base + lo * W - (uint64_t)G.fp * W;
    x.log2b = a.log2b;
    x.vpl_log2 = a.log2b + Ctx::LOG2W - 4;
    x.nvec = G.s << x.vpl_log2;
    x.pivot = a.pivot;
    x.xoff = xoff;
    x.cnt = cnt;
    x.tid = tid;
    x.lane = tid & 63;
    x.wid = tid >> 6;

    if (bid == 0 && tid == 0) {
        a.ctl[0] = lo; a.ctl[1] = hi; a.ctl[2] = G.g; a.ctl[3] = G.s;
    }
    for (uint32_t j = tid; j < G.s; j += NT)
        xoff[j] = a.strided ? 0u : chunk_offset(a.seed, a.level, j, G.g);
    __syncthreads();

    uint64_t vmin = ~0ull, vmax = 0;
    auto fold = [&](uint32_t c, uint32_t i) {
        if (tid == 0) {
            uint64_t vi;
            if (c >= (G.s << x.log2b)) {
                vi = hi;
            } else {
                const uint64_t vp =
                    ((uint64_t)x.line_of(c >> x.log2b, i) << x.log2b) + (c & ((1u << x.log2b) - 1));
                vi = vp >= x.real_end ? hi : lo + (vp - G.fp);
            }
            vmin = vi < vmin ? vi : vmin;
            vmax = vi > vmax ? vi : vmax;
        }
    };
    using Mask = typename Ctx::Mask;
    auto load_any = [&](v4u (&buf)[NV], uint32_t i, Mask &m) __attribute__((always_inline)) -> bool {
        const bool f = x.fast(i);
        if (f)
            x.template load<true>(buf, i, m);
        else
            x.template load<false>(buf, i, m);
        return f;
    };
    // dynamic LDS: the exchange table (Ctx::XCH_BYTES; with 32 KiB groups two
    // of them, then the group's tile) or the staging tile (NVEC vectors)
    extern __shared__ v4u dyn_lds[];
    uint16_t *const xt = reinterpret_cast<uint16_t *>(dyn_lds);
    uint64_t written = 0;             // exchange form: elements this workgroup stored
    auto part_any = [&](const v4u (&buf)[NV], uint32_t i, bool f, const Mask &m) -> uint32_t {
        if constexpr (XCH)
            return f ? x.template exchange<true>(buf, i, m, xt, a.xch_shift, written)
                     : x.template exchange<false>(buf, i, m, xt, a.xch_shift, written);
        else
            return f ? x.template partition<true>(buf, i, m) : x.template partition<false>(buf, i, m);
    };

    const uint32_t step = gridDim.x;
    uint32_t i = bid;
    if constexpr (PREFETCH) {
        // The group is staged into an LDS tile after the exchange tables (two
        // of S / 2 slots), and the next group's loads are issued into the
        // registers as soon as the tile is written, so that they are in flight
        // while the group is ranked and swapped (its barriers wait for LDS
        // only).  A group that is not wholly real (at most the two at the
        // region's ends) or that may fall back to the stable form takes the
        // register-resident exchange below, then issues the next loads.
        v4u *const tile = dyn_lds + 2 * Ctx::XCH_BYTES / 16;
        v4u buf[NV];
        Mask m;
        bool fast = false;
        if (i < G.g)
            fast = load_any(buf, i, m);
        while (i < G.g) {
            const uint32_t nx = i + step;
            const bool staged = fast && !a.xch_shift;
            uint64_t pb = 0;
            uint32_t c = 0;
            if (staged)
                pb = x.stage_exchange(buf, tile);
            else
                c = fast ? x.template exchange<true>(buf, i, m, xt, a.xch_shift, written)
                         : x.template exchange<false>(buf, i, m, xt, a.xch_shift, written);
            // one place that loads the next group, so the loaded registers are
            // never copied (a copy would wait for the loads)
            bool nfast = false;
            if (nx < G.g)
                nfast = load_any(buf, nx, m);
            if (staged)
                c = x.finish_exchange(pb, i, tile, xt, written);
            fold(c, i);
            x.bar();  // the counts, the tables and the tile are rewritten by the next group
            i = nx;
            fast = nfast;
        }
        if (tid == 0) {
            a.out[2 * bid] = vmin;
            a.out[2 * bid + 1] = vmax;
            if (FIRST && a.split_out && bid == 0 && G.g == 1)
                *a.split_out = vmin;
            if (a.written && written)
                atomicAdd(reinterpret_cast<unsigned long long *>(a.written), (unsigned long long)written);
        }
        return;
    }

    // One register buffer: the next group's loads are issued right after this
    // group's stores (staged form: right after the tile is complete, ahead of
    // the tile's write-back), before the barrier that lets the counts be
    // rewritten.
    v4u buf[NV];
    Mask m;
    bool fast = false;
    if (i < G.g)
        fast = load_any(buf, i, m);
    while (i < G.g) {
        if constexpr (STAGED) {
            const uint32_t c = fast ? x.template stage<true>(buf, m, dyn_lds) : x.template stage<false>(buf, m, dyn_lds);
            fold(c, i);
            __syncthreads();  // the tile is complete
            const bool fast_cur = fast;
            const Mask m_cur = m;
            const uint32_t icur = i;
            i += step;
            if (i < G.g)
                fast = load_any(buf, i, m);
            if (fast_cur)
                x.template write_back<true>(dyn_lds, icur, m_cur);
            else
                x.template write_back<false>(dyn_lds, icur, m_cur);
        } else {
            fold(part_any(buf, i, fast, m), i);
            i += step;
            if (i < G.g)
                fast = load_any(buf, i, m);
        }
        __syncthreads();  // the counts (and the staging tile) are rewritten by the next group
    }
    if (tid == 0) {
        a.out[2 * bid] = vmin;
        a.out[2 * bid + 1] = vmax;
        if (FIRST && a.split_out && bid == 0 && G.g == 1)
            *a.split_out = vmin;  // one group: its splitting position is the split
        if (XCH && a.written && written)
            atomicAdd(reinterpret_cast<unsigned long long *>(a.written), (unsigned long long)written);
    }
}

template <typename T, int NT, int NV, int FORM>
const void *level_rs_fn_t(bool first)
{
    return first ? reinterpret_cast<const void *>(&k_level_rs<T, NT, NV, true, FORM>)
                 : reinterpret_cast<const void *>(&k_level_rs<T, NT, NV, false, FORM>);
}

// Dynamic LDS of a form: the exchange form's table of slot numbers, or the
// staged form's tile of one group.
template <typename T, int NT, int NV, int FORM>
constexpr size_t level_rs_lds()
{
    return FORM == kFormExchange ? (xch_prefetch<T, NT, NV, FORM>()
                                        ? 2 * LevelCtx<T, NT, NV>::XCH_BYTES + (size_t)NT * NV * 16
                                        : LevelCtx<T, NT, NV>::XCH_BYTES)
           : FORM == kFormStaged ? (size_t)LevelCtx<T, NT, NV>::NVEC * 16
                                 : 0;
}

template <typename T, int NT, int NV, int FORM>
size_t level_form_lds()
{
    return level_rs_lds<T, NT, NV, FORM>();
}

template <typename T, int NT, int NV, int FORM>
hipError_t launch_level_rs_t(bool first, uint32_t grid, const LevelArgs &a, hipStream_t st)
{
    constexpr size_t shmem = level_rs_lds<T, NT, NV, FORM>();
    if (shmem > 32768) {
        const hipError_t e = hipFuncSetAttribute(level_rs_fn_t<T, NT, NV, FORM>(first),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess)
            return e;
    }
    if (first)
        hipLaunchKernelGGL((k_level_rs<T, NT, NV, true, FORM>), dim3(grid), dim3(NT), shmem, st, a);
    else
        hipLaunchKernelGGL((k_level_rs<T, NT, NV, false, FORM>), dim3(grid), dim3(NT), shmem, st, a);
    return hipGetLastError();
}

// The register-engine group shapes the host selects from: groups of 32, 64 and
// 128 KiB (threads x 16-byte vectors per thread).  X(T, NT, NV) is applied to each.
#define SS_RS_VARIANTS(X, T) X(T, 256, 8) X(T, 512, 8) X(T, 512, 16)

}  // namespace ss
