// ss_level.hip -- the Partial Partition Step of (Recursive) Smoothed Striding
// on gfx950, and the reduction that ends a recursion.
//
// One launch performs one Partial Partition Step (Section 4): the region is
// cut into s chunks of g lines; group U_i takes line (X_j + i) mod g of chunk
// j; every group is partitioned serially by one workgroup; the splitting
// positions v_i are reduced to (v_min, v_max), which bound the region of the
// next level (Section 4, "Recursive Smoothed Striding").
//
// Workgroup body for one group U_i (s lines, at most one LDS tile):
//   1. every thread loads 16-byte vectors of U_i's lines straight into
//      registers (8 consecutive lanes cover one 128-byte line, so each load
//      instruction reads whole lines);
//   2. the decider key < pivot is evaluated per element, and wavefront
//      ballots with mbcnt give each element its rank among the predecessors
//      of its wave; a scan over the per-wave counts makes the ranks
//      group-wide;
//   3. each element is written into the LDS tile at its destination slot:
//      predecessors to slot rank, successors to slot c_i + (slot - rank),
//      a stable partition of the group's slot sequence;
//   4. the tile is written back to the same lines (coalesced), while the
//      next group's loads are already in flight;
//   5. v_i (array position of slot c_i, or hi when the group holds only
//      predecessors) updates the workgroup's running (min, max), written once
//      as its partial.  The next level reduces all partials redundantly in
//      every workgroup (concurrent reads only), so no atomics touch data or
//      control words: each line is owned by exactly one workgroup per level.
#include "ss_common.h"
#include "ss_device.h"

namespace ss {

template <typename T, int NT, int TILE_BYTES, bool FIRST>
__global__ void __launch_bounds__(NT) k_level(const LevelArgs a)
{
    constexpr int W = sizeof(T);
    constexpr int V = Elem<T>::V;
    constexpr int NVEC = TILE_BYTES / 16;  // 16-byte vectors per tile
    constexpr int NV = NVEC / NT;          // vectors per thread
    constexpr int NW = NT / 64;            // waves
    constexpr int MAXS = TILE_BYTES / 64;  // lines of at least 64 bytes
    static_assert(NV * NT == NVEC && NV * NW <= 64 && NV <= 32, "tile shape");

    __shared__ v4u tile[NVEC];
    __shared__ uint32_t xoff[MAXS];
    __shared__ uint32_t wtot[NV * NW];
    __shared__ uint32_t wpre[NV * NW + 1];
    __shared__ uint64_t red[2 * NW];

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const uint32_t bid = blockIdx.x;

    uint64_t lo, hi;
    if (FIRST) {
        lo = a.lo;
        hi = a.hi;
    } else {
        prev_region<NT>(a.prev, a.prev_count, a.prev_ctl, red, lo, hi);
    }
    if (!(lo < hi)) {
        // Previous level left no middle: the partition is complete, split = lo.
        if (tid == 0) {
            a.out[2 * bid] = bid == 0 ? lo : ~0ull;
            a.out[2 * bid + 1] = bid == 0 ? lo : 0ull;
            if (bid == 0) {
                a.ctl[0] = lo; a.ctl[1] = lo; a.ctl[2] = 0; a.ctl[3] = 0;
            }
        }
        return;
    }

    const uint32_t log2b = a.log2b;
    const uint32_t b = 1u << log2b;
    const Geo G = plan_geo(lo, hi, log2b, a.s_max);
    const uint32_t g = G.g, s = G.s, fp = G.fp;
    const uint64_t real_end = (uint64_t)fp + (hi - lo);  // virtual index past the last real element
    char *const A0 = a.base + lo * W - (uint64_t)fp * W; // line-aligned anchor
    const uint32_t vpl_log2 = log2b + (W == 4 ? 2 : W == 8 ? 3 : 4) - 4;  // log2 vectors per line
    const uint32_t nvec = s << vpl_log2;                                  // vectors of one group

    if (bid == 0 && tid == 0) {
        a.ctl[0] = lo; a.ctl[1] = hi; a.ctl[2] = g; a.ctl[3] = s;
    }
    for (uint32_t j = tid; j < s; j += NT)
        xoff[j] = a.strided ? 0u : chunk_offset(a.seed, a.level, j, g);
    __syncthreads();

    // Virtual element index of the first element of vector q of group i.
    auto vec_start = [&](uint32_t q, uint32_t i) -> uint64_t {
        const uint32_t j = q >> vpl_log2, u = q & ((1u << vpl_log2) - 1);
        uint32_t r = xoff[j] + i;
        r = r >= g ? r - g : r;
        return (((uint64_t)j * g + r) << log2b) + (uint64_t)u * V;
    };

    v4u buf[NV];
    uint32_t partial = 0;  // bit r: vector r is not entirely real
    auto load_group = [&](uint32_t i) {
        partial = 0;
#pragma unroll
        for (int r = 0; r < NV; r++) {
            const uint32_t q = r * NT + tid;
            if (q < nvec) {
                const uint64_t e0 = vec_start(q, i);
                if (e0 >= fp && e0 + V <= real_end) {
                    buf[r] = *reinterpret_cast<const v4u *>(A0 + e0 * W);
                } else {
                    partial |= 1u << r;
                    buf[r] = v4u{0u, 0u, 0u, 0u};
#pragma unroll
                    for (int e = 0; e < V; e++)
                        if (e0 + e >= fp && e0 + e < real_end)
                            Elem<T>::load1(buf[r], e, A0 + (e0 + e) * W);
                }
            }
        }
    };

    uint64_t vmin = ~0ull, vmax = 0;
    uint32_t i = bid;
    if (i < g)
        load_group(i);
    while (i < g) {
        // 2. decider and wave-level ranks
        uint32_t pbits[NV], lex[NV];
#pragma unroll
        for (int r = 0; r < NV; r++) {
            const uint32_t q = r * NT + tid;
            uint32_t bits = 0;
            if (q < nvec) {
                if (!((partial >> r) & 1)) {
#pragma unroll
                    for (int e = 0; e < V; e++)
                        bits |= (uint32_t)(Elem<T>::key(buf[r], e) < a.pivot) << e;
                } else {
                    const uint64_t e0 = vec_start(q, i);
#pragma unroll
                    for (int e = 0; e < V; e++) {
                        const uint64_t vp = e0 + e;
                        const bool real = vp >= fp && vp < real_end;
                        const bool p = real ? Elem<T>::key(buf[r], e) < a.pivot : vp < fp;
                        bits |= (uint32_t)p << e;
                    }
                }
            }
            pbits[r] = bits;
            uint32_t ex = 0, tot = 0;
#pragma unroll
            for (int e = 0; e < V; e++) {
                const uint64_t m = __ballot((bits >> e) & 1);
                ex += lanes_below(m);
                tot += __popcll(m);
            }
            lex[r] = ex;
            if (lane == 0)
                wtot[r * NW + wid] = tot;
        }
        __syncthreads();
        if (wid == 0) {
            const uint32_t x = lane < NV * NW ? wtot[lane] : 0u;
            uint32_t inc = x;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t y = __shfl_up(inc, d, 64);
                if (lane >= d)
                    inc += y;
            }
            if (lane < NV * NW)
                wpre[lane] = inc - x;
            if (lane == 63)
                wpre[NV * NW] = inc;
        }
        __syncthreads();
        const uint32_t c = wpre[NV * NW];  // predecessors in U_i (virtual ones included)

        // 3. stable partition of the group's slots into the LDS tile
#pragma unroll
        for (int r = 0; r < NV; r++) {
            const uint32_t q = r * NT + tid;
            if (q < nvec) {
                uint32_t rp = wpre[r * NW + wid] + lex[r];
                const bool full = !((partial >> r) & 1);
                const uint64_t e0 = full ? 0 : vec_start(q, i);
#pragma unroll
                for (int e = 0; e < V; e++) {
                    const bool p = (pbits[r] >> e) & 1;
                    const uint32_t slot = q * V + e;
                    const uint32_t d = p ? rp : c + slot - rp;
                    if (full || (e0 + e >= fp && e0 + e < real_end))
                        Elem<T>::put(tile, d, buf[r], e);
                    rp += p;
                }
            }
        }
        __syncthreads();

        // 4. next group's loads go out before this group's stores
        const uint32_t inext = i + gridDim.x;
        const uint32_t partial_cur = partial;
        if (inext < g)
            load_group(inext);
#pragma unroll
        for (int r = 0; r < NV; r++) {
            const uint32_t q = r * NT + tid;
            if (q < nvec) {
                const v4u v = tile[q];
                const uint64_t e0 = vec_start(q, i);
                if (!((partial_cur >> r) & 1)) {
                    *reinterpret_cast<v4u *>(A0 + e0 * W) = v;
                } else {
#pragma unroll
                    for (int e = 0; e < V; e++)
                        if (e0 + e >= fp && e0 + e < real_end)
                            Elem<T>::store1(v, e, A0 + (e0 + e) * W);
                }
            }
        }

        // 5. splitting position of U_i
        if (tid == 0) {
            uint64_t vi;
            if (c >= (s << log2b)) {
                vi = hi;
            } else {
                const uint32_t j = c >> log2b, o = c & (b - 1);
                uint32_t r = xoff[j] + i;
                r = r >= g ? r - g : r;
                const uint64_t vp = ((((uint64_t)j * g + r) << log2b)) + o;
                vi = vp >= real_end ? hi : lo + (vp - fp);
            }
            vmin = vi < vmin ? vi : vmin;
            vmax = vi > vmax ? vi : vmax;
        }
        i = inext;
    }
    if (tid == 0) {
        a.out[2 * bid] = vmin;
        a.out[2 * bid + 1] = vmax;
    }
}

// Reduce the last level's partials: result[0] = 1 if the partition is
// complete, result[1] = split (when complete), result[2..3] = (vmin, vmax);
// result[4..] belong to earlier kernels of the call and are only copied.
// d_split (nullable) receives the split or UINT64_MAX.  host (nullable, in
// mapped host memory) receives the result words and then `nctl` level
// records starting at `ctl`, so the host reads them without a copy.
__global__ void __launch_bounds__(256) k_finish(const uint64_t *prev, uint32_t count, const uint64_t *prev_ctl,
                                                uint64_t *result, uint64_t *d_split, const uint64_t *ctl,
                                                uint32_t nctl, uint64_t *host)
{
    __shared__ uint64_t red[8];
    uint64_t lo, hi;
    prev_region<256>(prev, count, prev_ctl, red, lo, hi);
    const bool done = !(lo < hi);
    if (threadIdx.x == 0) {
        result[0] = done;
        result[1] = done ? lo : ~0ull;
        result[2] = lo;
        result[3] = hi;
        if (d_split)
            *d_split = done ? lo : ~0ull;
    }
    if (host) {
        if (threadIdx.x < 4)
            host[threadIdx.x] = threadIdx.x == 0 ? (uint64_t)done : threadIdx.x == 1 ? (done ? lo : ~0ull)
                                                                   : threadIdx.x == 2 ? lo : hi;
        else if (threadIdx.x < kResultWordsDev)
            host[threadIdx.x] = result[threadIdx.x];  // words written by earlier kernels of the call
        for (uint32_t k = threadIdx.x; k < nctl * kCtlWords; k += 256)
            host[kResultWordsDev + k] = ctl[k];
    }
}

// Launch helpers (host side) -------------------------------------------------

template <typename T, int NT, int TB>
hipError_t launch_level(bool first, uint32_t grid, const LevelArgs &a, hipStream_t st)
{
    if (first)
        hipLaunchKernelGGL((k_level<T, NT, TB, true>), dim3(grid), dim3(NT), 0, st, a);
    else
        hipLaunchKernelGGL((k_level<T, NT, TB, false>), dim3(grid), dim3(NT), 0, st, a);
    return hipGetLastError();
}

template <typename T, int NT, int TB>
const void *level_fn(bool first)
{
    return first ? reinterpret_cast<const void *>(&k_level<T, NT, TB, true>)
                 : reinterpret_cast<const void *>(&k_level<T, NT, TB, false>);
}

hipError_t launch_finish(const uint64_t *prev, uint32_t count, const uint64_t *prev_ctl, uint64_t *result,
                         uint64_t *d_split, const uint64_t *ctl, uint32_t nctl, uint64_t *host, hipStream_t st)
{
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, st, prev, count, prev_ctl, result, d_split, ctl, nctl, host);
    return hipGetLastError();
}

#define SS_INSTANTIATE(T, NT, TB)                                                                   \
    template hipError_t launch_level<T, NT, TB>(bool, uint32_t, const LevelArgs &, hipStream_t);    \
    template const void *level_fn<T, NT, TB>(bool);

SS_INSTANTIATE(uint32_t, 256, 65536)
SS_INSTANTIATE(uint64_t, 256, 65536)
SS_INSTANTIATE(KV, 256, 65536)
SS_INSTANTIATE(uint32_t, 256, 32768)
SS_INSTANTIATE(uint64_t, 256, 32768)
SS_INSTANTIATE(KV, 256, 32768)

}  // namespace ss
