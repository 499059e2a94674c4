// ss_common.h -- internal definitions shared by the library's HIP sources.
//
// Geometry of one Partial Partition Step (Section 4, "Formal Algorithm
// Description"): the region [lo, hi) of the array is viewed as lines of b
// elements counted from the array's first element (so an array's result
// depends only on its contents, never on where it sits in memory).  If the
// region does not start on a line boundary, the fp elements between the
// boundary and lo are treated as virtual predecessors (they precede the
// region, where everything is already a predecessor, and are never read or
// written); past hi the padding up to s*g*b elements is made of virtual
// successors (Section 4, footnote on gb not dividing n).  With L lines in
// total, g = ceil(L / s_max) groups and s = ceil(L / g) lines per group, so
// the padding s*g - L is below g lines and lies in the last chunk: in every
// group the virtual predecessors form a prefix of its slots and the virtual
// successors a suffix, so a stable in-group partition never moves them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ss {

struct KV {
    uint64_t key;
    uint64_t val;
};

// SplitMix64 (Steele, Lea & Flood 2014): output number ctr (0-based) of the
// stream whose state starts at seed.
__host__ __device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t ctr)
{
    uint64_t z = seed + (ctr + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Random chunk offset X_j of level `level`, uniform over [0, g) (the paper
// draws X_j uniformly from {1..g}; 0-based it is X_j mod g): counter
// (level << 40 | j) of the stream, top 32 bits scaled by Lemire's
// multiply-shift.
__host__ __device__ __forceinline__ uint32_t chunk_offset(uint64_t seed, uint32_t level, uint32_t j,
                                                          uint32_t g)
{
    const uint64_t r = splitmix64_at(seed, ((uint64_t)level << 40) | j);
    return (uint32_t)(((r >> 32) * (uint64_t)g) >> 32);
}

struct Geo {
    uint64_t nv;  // virtual length: front padding + real elements
    uint64_t L;   // lines
    uint32_t g;   // groups
    uint32_t s;   // lines per group
    uint32_t fp;  // virtual predecessors in front of the region
};

// Geometry of the region [lo, hi) of an array whose lines start at its
// element 0 (lo and hi relative to the array's first element).
__host__ __device__ __forceinline__ Geo plan_geo(uint64_t lo, uint64_t hi, uint32_t log2b, uint32_t s_max)
{
    Geo G;
    G.fp = (uint32_t)(lo & ((1ull << log2b) - 1));
    G.nv = (hi - lo) + G.fp;
    G.L = (G.nv + (1ull << log2b) - 1) >> log2b;
    const uint64_t g = (G.L + s_max - 1) / s_max;
    G.g = (uint32_t)(g ? g : 1);
    G.s = (uint32_t)((G.L + G.g - 1) / G.g);
    return G;
}

// Arguments of one level launch.
struct LevelArgs {
    char *base;             // array base
    uint64_t n;             // array length (elements)
    uint64_t pivot;
    uint64_t seed;
    const uint64_t *prev;   // previous level's partials {vmin, vmax} per workgroup (non-first levels)
    const uint64_t *prev_ctl;  // previous level's record (its g tells whether one partial suffices)
    uint64_t *out;          // this level's partials
    uint64_t *ctl;          // this level's record, written by workgroup 0: lo, hi, g, s
    uint64_t lo, hi;        // region of a first level
    uint32_t prev_count;    // workgroups of the previous level
    uint32_t level;         // recursion depth, selects the offsets' counter block
    uint32_t log2b;         // log2 of elements per line
    uint32_t s_max;         // lines-per-group bound
    uint32_t strided;       // 1: every offset is 0 (the Strided Algorithm)
    uint32_t xch_shift;     // exchange form: a group whose misplaced pairs m satisfy m << xch_shift > slots
                            // is stored stably instead (0: every group by exchange)
    uint32_t gate_want;     // first level: run only if *gate == gate_want, else only neutral partials
    uint32_t gate_keep;     //   from workgroup gate_keep on (the other kernel of the pair wrote the rest)
    const uint64_t *gate;   // null: always run
    uint64_t *written;      // exchange form: elements stored, summed over the workgroups (null: not kept)
    uint64_t *split_out;    // first level of a region of one group: workgroup 0 stores the split here
                            //   (null: a later kernel does)
    uint64_t *sample_out;   // first level of the automatic choice: take the form from the key sample,
                            //   run only if it selects gate_want, and (workgroup 0) store the choice and
                            //   clear the exchange form's counts in these result words (null: no sample)
};

// The automatic choice's key sample: kGateRuns runs of kGateRunLen
// consecutive keys, run c starting at c n / kGateRuns.  The exchange form is
// chosen when at most 1/den of the sample, or at least 1 - 1/den, are
// predecessors (den = 9 for 16-byte records, 16 otherwise: about where the
// exchange stops beating the stable form, q = 0.12 and 0.07).
constexpr uint32_t kGateRuns = 64;
constexpr uint32_t kGateRunLen = 64;
constexpr uint32_t kGateSamples = kGateRuns * kGateRunLen;
__host__ __device__ __forceinline__ bool gate_skewed(uint64_t preds, int w)
{
    const uint64_t den = w >= 16 ? 9 : 16;
    return preds * den <= kGateSamples || preds * den >= (den - 1) * kGateSamples;
}

// Forms of a level kernel's store (ss_level_rs.h): every element stored to
// its slot from registers, the write-minimal exchange, or the stable
// partition staged in an LDS tile and written back as whole lines.
enum { kFormDirect = 0, kFormExchange = 1, kFormStaged = 2, kForms = 3 };

constexpr int kCtlWords = 8;        // words per level record
constexpr int kResultWordsDev = 8;  // result words ahead of the level records in the host copy

}  // namespace ss
