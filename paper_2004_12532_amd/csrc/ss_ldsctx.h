// ss_ldsctx.h -- the workgroup body of one group of a Partial Partition Step
// (Section 4) with the group permuted through an LDS tile: load the group's
// lines into registers, rank its predecessors with wavefront ballots and a
// scan of per-wave counts, write every element to its slot of the stable
// partition in the tile (predecessors to slot rank, successors to slot
// c_i + slot - rank), and write the tile back to the group's lines as whole
// 16-byte vectors.  Used by the batched kernel where scattered element
// stores cost more than the staging (4-byte keys).
#pragma once

#include "ss_common.h"
#include "ss_device.h"

namespace ss {

// The same group body with the group permuted through an LDS tile of
// TILE_BYTES: elements are written to their slots in the tile, and the tile
// is written back to the group's lines as whole 16-byte vectors.  Used where
// scattered element stores cost more than the staging (4-byte keys).
template <typename T, int NT, int TILE_BYTES>
struct LdsCtx {
    static constexpr int W = sizeof(T);
    static constexpr int LOG2W = W == 4 ? 2 : W == 8 ? 3 : 4;
    static constexpr int V = Elem<T>::V;
    static constexpr int NVEC = TILE_BYTES / 16;
    static constexpr int NV = NVEC / NT;
    static constexpr int NW = NT / 64;
    static constexpr int E = NV * NW;
    static_assert(NV * NT == NVEC && E <= 64, "tile shape");

    char *A0;
    const uint32_t *xoff;
    v4u *tile;          // NVEC vectors of LDS
    uint32_t *wtot;     // E words of LDS
    uint32_t *wpre;     // E + 1 words of LDS
    uint64_t pivot;
    uint64_t real_end;
    uint32_t fp, g, s;
    uint32_t log2b, vpl_log2, nvec;
    int tid, lane, wid;

    __device__ __forceinline__ uint64_t vec_start(uint32_t q, uint32_t i) const
    {
        const uint32_t j = q >> vpl_log2, u = q & ((1u << vpl_log2) - 1);
        uint32_t r = xoff[j] + i;
        r = r >= g ? r - g : r;
        return (((uint64_t)j * g + r) << log2b) + (uint64_t)u * V;
    }
    __device__ __forceinline__ char *elem_ptr(uint64_t vpos) const { return A0 + (vpos << LOG2W); }

    // bit r of `partial`: vector r is not entirely real
    __device__ __forceinline__ void load(v4u (&buf)[NV], uint32_t i, uint32_t &partial) const
    {
        partial = 0;
#pragma unroll
        for (int r = 0; r < NV; r++) {
            const uint32_t q = r * NT + tid;
            buf[r] = v4u{0u, 0u, 0u, 0u};
            if (q < nvec) {
                const uint64_t e0 = vec_start(q, i);
                if (e0 >= fp && e0 + V <= real_end) {
                    buf[r] = *reinterpret_cast<const v4u *>(elem_ptr(e0));
                } else {
                    partial |= 1u << r;
#pragma unroll
                    for (int e = 0; e < V; e++)
                        if (e0 + e >= fp && e0 + e < real_end)
                            Elem<T>::load1(buf[r], e, elem_ptr(e0 + e));
                }
            }
        }
    }

    // Stable partition of group i into the tile, then the tile back to the
    // group's lines; returns c_i.
    __device__ __forceinline__ uint32_t partition_store(const v4u (&buf)[NV], uint32_t i, uint32_t partial) const
    {
        uint32_t pbits[NV], lex[NV];
#pragma unroll
        for (int r = 0; r < NV; r++) {
            const uint32_t q = r * NT + tid;
            uint32_t bits = 0;
            if (q < nvec) {
                if (!((partial >> r) & 1)) {
#pragma unroll
                    for (int e = 0; e < V; e++)
                        bits |= (uint32_t)(Elem<T>::key(buf[r], e) < pivot) << e;
                } else {
                    const uint64_t e0 = vec_start(q, i);
#pragma unroll
                    for (int e = 0; e < V; e++) {
                        const uint64_t vp = e0 + e;
                        const bool real = vp >= fp && vp < real_end;
                        bits |= (uint32_t)(real ? Elem<T>::key(buf[r], e) < pivot : vp < fp) << e;
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
            const uint32_t x = lane < E ? wtot[lane] : 0u;
            uint32_t inc = x;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t y = __shfl_up(inc, d, 64);
                if (lane >= d)
                    inc += y;
            }
            if (lane < E)
                wpre[lane] = inc - x;
            if (lane == 63)
                wpre[E] = inc;
        }
        __syncthreads();
        const uint32_t c = wpre[E];
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
#pragma unroll
        for (int r = 0; r < NV; r++) {
            const uint32_t q = r * NT + tid;
            if (q < nvec) {
                const v4u v = tile[q];
                const uint64_t e0 = vec_start(q, i);
                if (!((partial >> r) & 1)) {
                    *reinterpret_cast<v4u *>(elem_ptr(e0)) = v;
                } else {
#pragma unroll
                    for (int e = 0; e < V; e++)
                        if (e0 + e >= fp && e0 + e < real_end)
                            Elem<T>::store1(v, e, elem_ptr(e0 + e));
                }
            }
        }
        return c;
    }
};

}  // namespace ss
