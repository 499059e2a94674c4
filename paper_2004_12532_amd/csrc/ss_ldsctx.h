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
    static_assert(NV * NT == NVEC && E <= 64 && NV * V <= 64, "tile shape");

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

    // Every slot of group i is a real element and the group fills the tile.
    __device__ __forceinline__ bool fast(uint32_t i) const
    {
        if (nvec != (uint32_t)NVEC)
            return false;
        uint32_t r0 = xoff[0] + i;
        r0 = r0 >= g ? r0 - g : r0;
        if (fp && r0 == 0)
            return false;
        uint32_t rl = xoff[s - 1] + i;
        rl = rl >= g ? rl - g : rl;
        return ((uint64_t)((s - 1) * g + rl + 1) << log2b) <= real_end;
    }

    // Real elements and virtual front predecessors of this thread's vectors
    // (bit r * V + e), as in LevelCtx.
    struct Mask {
        uint64_t real, front;
    };

    template <bool FAST>
    __device__ __forceinline__ void load(v4u (&buf)[NV], uint32_t i, Mask &m) const
    {
        m.real = 0;
        m.front = 0;
#pragma unroll
        for (int r = 0; r < NV; r++) {
            const uint32_t q = r * NT + tid;
            if (FAST) {
                buf[r] = *reinterpret_cast<const v4u *>(elem_ptr(vec_start(q, i)));
            } else {
                buf[r] = v4u{0u, 0u, 0u, 0u};
                if (q < nvec) {
                    const uint64_t e0 = vec_start(q, i);
                    if (e0 >= fp && e0 + V <= real_end) {
                        buf[r] = *reinterpret_cast<const v4u *>(elem_ptr(e0));
                        m.real |= (uint64_t)((1u << V) - 1) << (r * V);
                    } else {
#pragma unroll
                        for (int e = 0; e < V; e++) {
                            const uint64_t vp = e0 + e;
                            if (vp >= fp && vp < real_end) {
                                Elem<T>::load1(buf[r], e, elem_ptr(vp));
                                m.real |= 1ull << (r * V + e);
                            } else if (vp < fp) {
                                m.front |= 1ull << (r * V + e);
                            }
                        }
                    }
                }
            }
        }
    }

    // Stable partition of group i into the tile, then the tile back to the
    // group's lines; returns c_i.
    template <bool FAST>
    __device__ __forceinline__ uint32_t partition_store(const v4u (&buf)[NV], uint32_t i, const Mask &m) const
    {
        constexpr uint32_t VM = (1u << V) - 1;
        uint64_t pb = 0;
#pragma unroll
        for (int r = 0; r < NV; r++) {
            uint32_t bits = 0;
#pragma unroll
            for (int e = 0; e < V; e++)
                bits |= (uint32_t)(Elem<T>::key(buf[r], e) < pivot) << e;
            if (!FAST)
                bits = (bits & (uint32_t)(m.real >> (r * V)) & VM) | ((uint32_t)(m.front >> (r * V)) & VM);
            pb |= (uint64_t)bits << (r * V);
            uint32_t tot = 0;
#pragma unroll
            for (int e = 0; e < V; e++)
                tot += __popcll(__ballot((bits >> e) & 1));
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
            const uint32_t bits = (uint32_t)(pb >> (r * V)) & VM;
            uint32_t rp = wpre[r * NW + wid];
#pragma unroll
            for (int e = 0; e < V; e++)
                rp += lanes_below(__ballot((bits >> e) & 1));
#pragma unroll
            for (int e = 0; e < V; e++) {
                const bool p = (bits >> e) & 1;
                const uint32_t slot = q * V + e;
                const uint32_t d = p ? rp : c + slot - rp;
                rp += p;
                if (FAST || ((m.real >> (r * V + e)) & 1))
                    Elem<T>::put(tile, d, buf[r], e);
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NV; r++) {
            const uint32_t q = r * NT + tid;
            if (FAST) {
                *reinterpret_cast<v4u *>(elem_ptr(vec_start(q, i))) = tile[q];
            } else if (q < nvec) {
                const uint32_t vm = (uint32_t)(m.real >> (r * V)) & VM;
                if (vm) {
                    const v4u v = tile[q];
                    const uint64_t e0 = vec_start(q, i);
                    if (vm == VM) {
                        *reinterpret_cast<v4u *>(elem_ptr(e0)) = v;
                    } else {
#pragma unroll
                        for (int e = 0; e < V; e++)
                            if ((vm >> e) & 1)
                                Elem<T>::store1(v, e, elem_ptr(e0 + e));
                    }
                }
            }
        }
        return c;
    }
};

}  // namespace ss
