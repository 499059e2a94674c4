// ss_levelctx.h -- the workgroup body of one group of a Partial Partition
// Step (Section 4) with the group held in registers: load the group's lines,
// rank its predecessors with wavefront ballots and a scan of per-wave counts,
// and store every element at its slot of the stable partition of the group
// (predecessors to slot rank, successors to slot c_i + slot - rank), or, in
// the write-minimal form, swap only the misplaced pairs.  Shared by the
// single-array level kernel and the batched kernel.
#pragma once

#include "ss_common.h"
#include "ss_device.h"

namespace ss {

// LDSBAR: the workgroup barriers of the body wait only for LDS accesses, so
// the next group's loads, issued before the staged exchange ranks and swaps
// the current group, stay in flight across them.
template <typename T, int NT, int NV, bool LDSBAR = false>
struct LevelCtx {
    static constexpr int W = sizeof(T);
    static constexpr int LOG2W = W == 4 ? 2 : W == 8 ? 3 : 4;
    static constexpr int V = Elem<T>::V;
    static constexpr int NW = NT / 64;
    static constexpr int NVEC = NT * NV;
    static constexpr int E = NV * NW;  // (round, wave) counts

    char *A0;           // line-aligned anchor of the region
    const uint32_t *xoff;
    uint32_t *cnt;      // E + 1 words of LDS
    uint64_t pivot;
    uint64_t real_end;  // virtual index past the last real element
    uint32_t fp;        // virtual predecessors in front
    uint32_t g, s;
    uint32_t log2b, vpl_log2, nvec;
    int tid, lane, wid;

    __device__ __forceinline__ void bar() const
    {
        if constexpr (LDSBAR)
            lds_barrier();
        else
            __syncthreads();
    }

    __device__ __forceinline__ uint32_t line_of(uint32_t j, uint32_t i) const
    {
        uint32_t r = xoff[j] + i;
        r = r >= g ? r - g : r;
        return j * g + r;
    }
    __device__ __forceinline__ uint64_t vec_start(uint32_t q, uint32_t i) const
    {
        return ((uint64_t)line_of(q >> vpl_log2, i) << log2b) + (q & ((1u << vpl_log2) - 1)) * V;
    }
    __device__ __forceinline__ char *elem_ptr(uint64_t vpos) const { return A0 + (vpos << LOG2W); }

    // Every slot of group i is a real element and the group fills the tile.
    __device__ __forceinline__ bool fast(uint32_t i) const
    {
        if (nvec != (uint32_t)NVEC)
            return false;
        if (fp && line_of(0, i) == 0)
            return false;
        return ((uint64_t)(line_of(s - 1, i) + 1) << log2b) <= real_end;
    }

    // Which slots of this thread's vectors are real elements, and which are
    // virtual predecessors in front of the region (bit r * V + e for element
    // e of vector r).  Slots past the region's end, and vectors past the
    // group's last line, are virtual successors: neither bit is set.
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

    // Decider bits of vector r; virtual front elements count as predecessors.
    template <bool FAST>
    __device__ __forceinline__ uint32_t bits_of(const v4u &v, int r, const Mask &m) const
    {
        uint32_t bits = 0;
#pragma unroll
        for (int e = 0; e < V; e++)
            bits |= (uint32_t)(Elem<T>::key(v, e) < pivot) << e;
        if (!FAST) {
            constexpr uint32_t VM = (1u << V) - 1;
            bits = (bits & (uint32_t)(m.real >> (r * V)) & VM) | ((uint32_t)(m.front >> (r * V)) & VM);
        }
        return bits;
    }

    // Count the group's predecessors: per-(round, wave) counts, scanned by
    // wave 0 into exclusive offsets cnt[0..E) and the total cnt[E] = c_i.
    // Returns the decider bits of this thread's slots (bit r * V + e).
    template <bool FAST>
    __device__ __forceinline__ uint64_t count(const v4u (&buf)[NV], const Mask &m) const
    {
        uint64_t pb = 0;
#pragma unroll
        for (int r = 0; r < NV; r++) {
            const uint32_t bits = bits_of<FAST>(buf[r], r, m);
            pb |= (uint64_t)bits << (r * V);
            uint32_t tot = 0;
#pragma unroll
            for (int e = 0; e < V; e++)
                tot += __popcll(__ballot((bits >> e) & 1));
            if (lane == 0)
                cnt[r * NW + wid] = tot;
        }
        bar();
        if (wid == 0) {
            constexpr int C = (E + 63) / 64;
            uint32_t x[C], sum = 0;
#pragma unroll
            for (int k = 0; k < C; k++) {
                const int idx = lane * C + k;
                x[k] = idx < E ? cnt[idx] : 0u;
                sum += x[k];
            }
            uint32_t inc = sum;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t y = __shfl_up(inc, d, 64);
                if (lane >= d)
                    inc += y;
            }
            uint32_t run = inc - sum;
#pragma unroll
            for (int k = 0; k < C; k++) {
                const int idx = lane * C + k;
                if (idx < E)
                    cnt[idx] = run;
                run += x[k];
            }
            if (lane == 63)
                cnt[E] = inc;
        }
        bar();
        return pb;
    }

    // Visit every slot of this thread in order with its rank among the
    // group's predecessors: f(r, e, slot, is_pred, preds before the slot).
    template <typename F>
    __device__ __forceinline__ void for_ranks(uint64_t pb, F &&f) const
    {
#pragma unroll
        for (int r = 0; r < NV; r++) {
            const uint32_t q = r * NT + tid;
            const uint32_t bits = (uint32_t)(pb >> (r * V)) & ((1u << V) - 1);
            uint32_t rp = cnt[r * NW + wid];
#pragma unroll
            for (int e = 0; e < V; e++)
                rp += lanes_below(__ballot((bits >> e) & 1));
#pragma unroll
            for (int e = 0; e < V; e++) {
                const bool p = (bits >> e) & 1;
                f(r, e, q * V + e, p, rp);
                rp += p;
            }
        }
    }

    __device__ __forceinline__ char *slot_ptr(uint32_t d, uint32_t i) const
    {
        const uint32_t b = 1u << log2b;
        return elem_ptr(((uint64_t)line_of(d >> log2b, i) << log2b) + (d & (b - 1)));
    }

    // Store every real element at its slot of the stable partition.  An
    // element whose slot does not change is not stored: in a region that is
    // already nearly partitioned (the middle region a level leaves behind)
    // the slots before the first misplaced element and after the last one
    // keep their elements, so their lines are only read.
    template <bool FAST>
    __device__ __forceinline__ void store_stable(const v4u (&buf)[NV], uint32_t i, const Mask &m, uint64_t pb,
                                                 uint32_t c) const
    {
        for_ranks(pb, [&](int r, int e, uint32_t slot, bool p, uint32_t rp) {
            const uint32_t d = p ? rp : c + slot - rp;
            if ((FAST || ((m.real >> (r * V + e)) & 1)) && d != slot)
                Elem<T>::store1(buf[r], e, slot_ptr(d, i));
        });
    }

    // Stable partition of group i; returns its predecessor count c_i.
    template <bool FAST>
    __device__ __forceinline__ uint32_t partition(const v4u (&buf)[NV], uint32_t i, const Mask &m) const
    {
        const uint64_t pb = count<FAST>(buf, m);
        const uint32_t c = cnt[E];
        store_stable<FAST>(buf, i, m, pb, c);
        return c;
    }

    // Staged form of the stable partition: every real element goes to its
    // slot of an LDS tile of NVEC vectors (slot order), from which
    // write_back later stores whole lines.  Virtual slots stay unwritten:
    // virtual predecessors are a prefix and virtual successors a suffix of
    // the slot sequence, so the stable partition leaves them in place.
    // Returns c_i.
    template <bool FAST>
    __device__ __forceinline__ uint32_t stage(const v4u (&buf)[NV], const Mask &m, v4u *tile) const
    {
        const uint64_t pb = count<FAST>(buf, m);
        const uint32_t c = cnt[E];
        for_ranks(pb, [&](int r, int e, uint32_t slot, bool p, uint32_t rp) {
            if (FAST || ((m.real >> (r * V + e)) & 1))
                Elem<T>::put(tile, p ? rp : c + slot - rp, buf[r], e);
        });
        return c;
    }

    // Store the staged tile of group i to the group's lines: thread tid
    // stores the vectors it loaded, so every wavefront store covers whole
    // lines.  A vector that is not wholly real (general path only) is
    // stored element by element.
    template <bool FAST>
    __device__ __forceinline__ void write_back(const v4u *tile, uint32_t i, const Mask &m) const
    {
        constexpr uint32_t VM = (1u << V) - 1;
#pragma unroll
        for (int r = 0; r < NV; r++) {
            const uint32_t q = r * NT + tid;
            if (!FAST && q >= nvec)
                continue;
            const v4u v = tile[q];
            char *const p = elem_ptr(vec_start(q, i));
            const uint32_t real = FAST ? VM : (uint32_t)(m.real >> (r * V)) & VM;
            if (real == VM) {
                *reinterpret_cast<v4u *>(p) = v;
            } else {
#pragma unroll
                for (int e = 0; e < V; e++)
                    if ((real >> e) & 1)
                        Elem<T>::store1(v, e, p + e * W);
            }
        }
    }

    // Slots of the exchange table: a group has at most S / 2 misplaced pairs.
    // (A variant with two tables filled in one pass, saving two barriers per
    // group, measured slower: 2.75 against 2.27 ms at 2^30 u64, q = 0.01.)
    static constexpr int XCH_SLOTS = NVEC * V / 2;
    static constexpr size_t XCH_BYTES = XCH_SLOTS * sizeof(uint16_t);

    // The write-minimal exchange of a group whose slots are all real (the fast
    // path), staged through an LDS tile of the group's vectors (vector q at
    // tile[q]), in three phases and three barriers, the last at the end of
    // the group in the caller.
    //  (a) stage_exchange: each thread evaluates its slots and writes its
    //      vectors to the tile; lane 0 of each wavefront posts the predecessor
    //      count of each of its (round, wavefront) blocks, which lie in slot
    //      order.  The caller then issues the next group's loads into the
    //      registers the group leaves free.
    //  (b) finish_exchange: every wavefront scans the block counts itself (c_i
    //      and the blocks' offsets), ranks the misplaced elements of its
    //      blocks and writes two tables: the k-th successor from the front
    //      below c_i at xt[k], the k-th predecessor from the back at or after
    //      c_i at xt[S/2 + k].  Blocks with neither kind are skipped on a
    //      wavefront-uniform test.  The wavefront holding slot c_i posts its
    //      rank, so m_i = c_i - rank.
    //  (c) Thread t < m_i swaps pair t: both values come from the tile, and
    //      each is stored at the other's slot.
    // These are the pairs of the serial two-pointer scan, as in exchange()
    // below.  Slot numbers read back from the tables are clamped to the group,
    // so no store leaves the group's lines whatever the tables hold.  xt holds
    // S 16-bit slot numbers.
    __device__ __forceinline__ uint64_t stage_exchange(const v4u (&buf)[NV], v4u *tile) const
    {
        const Mask all{~0ull, 0ull};
        uint64_t pb = 0;
#pragma unroll
        for (int r = 0; r < NV; r++) {
            const uint32_t bits = bits_of<true>(buf[r], r, all);
            pb |= (uint64_t)bits << (r * V);
            uint32_t tot = 0;
#pragma unroll
            for (int e = 0; e < V; e++)
                tot += __popcll(__ballot((bits >> e) & 1));
            if (lane == 0)
                cnt[r * NW + wid] = tot;
            tile[r * NT + tid] = buf[r];
        }
        return pb;
    }

    // Phases (b) and (c) for the group staged by stage_exchange, whose decider
    // bits are pb.  Returns c_i.
    __device__ __forceinline__ uint32_t finish_exchange(uint64_t pb, uint32_t i, const v4u *tile, uint16_t *xt,
                                                        uint64_t &written) const
    {
        static_assert(E <= 64, "one wavefront scans the block counts");
        constexpr uint32_t VM = (1u << V) - 1;
        constexpr uint32_t S = NVEC * V;
        constexpr uint32_t HALF = S / 2;
        static_assert((HALF & (HALF - 1)) == 0, "table index masks");
        bar();
        // (b)
        const uint32_t bc = lane < E ? cnt[lane] : 0u;
        const uint32_t inc = wave_scan_incl(bc, lane);
        const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
        const uint32_t excl = inc - bc;
        uint16_t *const bt = xt + HALF;
#pragma unroll 1
        for (int r = 0; r < NV; r++) {
            const uint32_t blk = r * NW + wid;
            const uint32_t s_lo = blk * 64 * V;  // the block's first slot
            const uint32_t bits = (uint32_t)(pb >> (r * V)) & VM;
            const uint32_t s0 = s_lo + lane * V;
            uint32_t wf = 0, wb = 0;
#pragma unroll
            for (int e = 0; e < V; e++) {
                const bool p = (bits >> e) & 1, below = s0 + e < c;
                wf |= (uint32_t)(!p && below) << e;
                wb |= (uint32_t)(p && !below) << e;
            }
            const bool holds_c = s_lo <= c && c < s_lo + 64 * V;
            if (!holds_c && __ballot((wf | wb) != 0) == 0)
                continue;
            uint32_t rp = (uint32_t)__builtin_amdgcn_readlane((int)excl, (int)blk);
#pragma unroll
            for (int k = 0; k < V; k++)
                rp += lanes_below(__ballot((bits >> k) & 1));
            if (holds_c && s0 <= c && c < s0 + V)
                cnt[E] = rp + __popc(bits & ((1u << (c - s0)) - 1));
#pragma unroll
            for (int e = 0; e < V; e++) {
                if ((wf >> e) & 1)
                    xt[(s0 + e - rp) & (HALF - 1)] = (uint16_t)(s0 + e);
                if ((wb >> e) & 1)
                    bt[(c - rp - 1) & (HALF - 1)] = (uint16_t)(s0 + e);
                rp += (bits >> e) & 1;
            }
        }
        bar();
        // (c)
        uint32_t m = c < S ? c - cnt[E] : 0u;
        m = m < HALF ? m : HALF;
        written += 2ull * m;
        for (uint32_t t = tid; t < m; t += NT) {
            uint32_t xs = xt[t], ys = bt[t];
            xs = xs < S ? xs : S - 1;
            ys = ys < S ? ys : S - 1;
            Elem<T>::store1(tile[ys / V], (int)(ys % V), slot_ptr(xs, i));
            Elem<T>::store1(tile[xs / V], (int)(xs % V), slot_ptr(ys, i));
        }
        return c;
    }

    // Write-minimal partition of group i (the two-pointer exchange of the
    // serial step, Section 4): the k-th successor from the front of the slot
    // order that lies in [0, c_i) swaps with the k-th predecessor from the
    // back that lies in [c_i, S).  These are exactly the pairs a serial
    // two-pointer scan of the slot sequence swaps, so the group ends in the
    // same arrangement, and only the swapped elements are written.  Every
    // misplaced element is real: virtual front slots are predecessors below
    // c_i and virtual tail slots successors above it.  xt holds XCH_SLOTS
    // 16-bit slot numbers of LDS.
    //
    // The group first counts its misplaced pairs m_i: c_i minus the
    // predecessors below slot c_i, read from the rank of slot c_i (one more
    // word of LDS at cnt[E + 1]).  With shift > 0 it falls back to the stable
    // partition when m_i << shift exceeds its slot count: once a few percent
    // of the elements move, the swapped elements dirty nearly every line
    // anyway and the exchange's extra passes cost more than they save.
    // shift = 0 exchanges every group.  `written` grows by the elements the
    // group stores (2 m_i, or its slot count when stored stably).  Returns c_i.
    // With the group's vectors in an LDS tile (tile not null) the swaps are
    // made by xchg_tile.
    template <bool FAST>
    __device__ __forceinline__ uint32_t exchange(const v4u (&buf)[NV], uint32_t i, const Mask &m,
                                                 uint16_t *xt, uint32_t shift, uint64_t &written) const
    {
        const uint64_t pb = count<FAST>(buf, m);
        const uint32_t c = cnt[E];
        const uint32_t S = nvec * V;
        uint32_t mis = 0;
        if (c < S) {
            // slot c_i is element e of vector q = r * NT + t (r uniform over the workgroup)
            const uint32_t q = c / V, e = c % V, r = q / NT, t = q % NT;
            if ((uint32_t)wid == t / 64) {
                const uint32_t bits = (uint32_t)(pb >> (r * V)) & ((1u << V) - 1);
                uint32_t rp = cnt[r * NW + wid];
#pragma unroll
                for (int k = 0; k < V; k++)
                    rp += lanes_below(__ballot((bits >> k) & 1));
                if ((uint32_t)lane == t % 64)
                    cnt[E + 1] = rp + __popc(bits & ((1u << e) - 1));
            }
            bar();
            mis = c - cnt[E + 1];
        }
        if (shift && (mis << shift) > S) {
            store_stable<FAST>(buf, i, m, pb, c);
            written += S;
            return c;
        }
        written += 2ull * mis;
        if (mis == 0)
            return c;
        // (1) each misplaced successor posts its slot under its front rank
        for_ranks(pb, [&](int, int, uint32_t slot, bool p, uint32_t rp) {
            if (!p && slot < c)
                xt[slot - rp] = (uint16_t)slot;
        });
        bar();
        // (2) each misplaced predecessor takes its partner's slot, stores
        // itself there and posts its own slot in exchange
        for_ranks(pb, [&](int r, int e, uint32_t slot, bool p, uint32_t rp) {
            if (p && slot >= c) {
                const uint32_t k = c - rp - 1;
                Elem<T>::store1(buf[r], e, slot_ptr(xt[k], i));
                xt[k] = (uint16_t)slot;
            }
        });
        bar();
        // (3) each misplaced successor stores itself at its partner's slot
        for_ranks(pb, [&](int r, int e, uint32_t slot, bool p, uint32_t rp) {
            if (!p && slot < c)
                Elem<T>::store1(buf[r], e, slot_ptr(xt[slot - rp], i));
        });
        return c;
    }
};

}  // namespace ss
