// ss_internal.h -- host-side declarations shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "ss.h"
#include "ss_common.h"

namespace ss {

constexpr int kMaxLevels = 32;      // level records / partial buffers kept per workspace
constexpr int kMaxGrid = 4096;      // upper bound of workgroups in a level launch
constexpr int kResultWords = kResultWordsDev;  // done, split, vmin, vmax, ...
constexpr uint32_t kHostLevelCap = 512;
constexpr uint32_t kDefaultEngine = SS_ENGINE_REGS;
constexpr uint32_t kDefaultRegsTile = 131072;
constexpr uint32_t kDefaultLineBytes = 512;
constexpr uint32_t kExchangeFlags = SS_FLAG_EXCHANGE | SS_FLAG_EXCHANGE_SKEWED;
constexpr uint32_t kSkewShift = 5;  // skewed: misplaced pairs at most 1/32 of a group's slots
constexpr uint64_t kAutoExchangeMin = 1ull << 22;  // automatic exchange choice from this many elements on
// Engine id of the kernel shapes that serve only the exchange form of the
// automatic first-level choice (not a public SS_ENGINE_* value).
constexpr uint32_t kEngineAutoExchange = 0x100;
constexpr int kResultWrittenFirst = 5;  // result word: elements stored by a first level in the exchange form
constexpr int kResultWritten = 6;   // result word: elements stored by later exchange-form levels
constexpr int kResultGate = 7;      // result word: 1 when the exchange form was chosen

struct Workspace {
    uint64_t *part = nullptr;    // kMaxLevels x 2 x kMaxGrid partials (device)
    uint64_t *ctl = nullptr;     // kMaxLevels x kCtlWords level records (device)
    uint64_t *result = nullptr;  // kResultWords (device)
    uint64_t *host = nullptr;    // mapped pinned host memory: result words then level records
    uint64_t *host_dev = nullptr;  // the same memory as seen from the device
    size_t part_words = 0, ctl_words = 0;
    size_t bytes = 0;
    uint32_t levels_cap = kMaxLevels;  // level slots of part and ctl
    hipEvent_t ev[4] = {};
};

struct Resolved {
    int algo;
    uint32_t engine;
    int w;
    uint32_t b, log2b;
    uint32_t tile;
    uint32_t s_max;
    uint32_t levels;
    uint64_t seed;
    uint32_t flags;
    bool auto_xch;  // choose the first level's form from a sample of the keys
};

struct RunOut {
    uint64_t split;
    bool done;
    uint64_t vmin, vmax;
    uint32_t grid;
    uint32_t levels_run;
    uint32_t launches;
    uint64_t aux_bytes;
    float first_level_ms, total_ms;
    uint64_t xch_mask;     // bit l: level l ran in the exchange form
    uint64_t written;      // elements those levels stored
    uint64_t written0;     // of which the first level stored
    uint64_t level_lo[SS_MAX_LEVELS], level_hi[SS_MAX_LEVELS];
    uint32_t level_g[SS_MAX_LEVELS], level_s[SS_MAX_LEVELS];
};

using LevelLaunch = hipError_t (*)(bool first, uint32_t grid, const LevelArgs &a, hipStream_t st);
using LevelFn = const void *(*)(bool first);

// A level kernel shape: its launchers, kernel handles and dynamic LDS per
// store form (kForm*; null where the engine has no such form: the LDS
// engine has only the stable form).
struct Variant {
    int dtype;
    uint32_t engine;
    uint32_t tile;
    int nt;
    LevelLaunch launch[kForms];
    LevelFn fn[kForms];
    size_t lds[kForms];
};

template <typename T, int NT, int TB>
hipError_t launch_level(bool first, uint32_t grid, const LevelArgs &a, hipStream_t st);
template <typename T, int NT, int TB>
const void *level_fn(bool first);
template <typename T, int NT, int NV, int FORM>
hipError_t launch_level_rs_t(bool first, uint32_t grid, const LevelArgs &a, hipStream_t st);
template <typename T, int NT, int NV, int FORM>
const void *level_rs_fn_t(bool first);
template <typename T, int NT, int NV, int FORM>
size_t level_form_lds();
const Variant *pick_variant(int dtype, uint32_t engine, uint32_t tile);
hipError_t launch_xch_prepare(int dtype, const char *base, uint64_t n, uint64_t pivot, uint64_t *result, bool force,
                              hipStream_t st);
hipError_t launch_finish(const uint64_t *prev, uint32_t count, const uint64_t *prev_ctl, uint64_t *result,
                         uint64_t *d_split, const uint64_t *ctl, uint32_t nctl, uint64_t *host, hipStream_t st);
hipError_t launch_cleanup(int dtype, char *base, uint64_t pivot, const uint64_t *prev, uint32_t count,
                          uint64_t *result, uint64_t *d_split, const uint64_t *ctl, uint32_t nctl, uint64_t *host,
                          hipStream_t st);
uint64_t cleanup_pass_elems(int w);  // elements the serial base case partitions in one pass

int fail_device(hipError_t e, const char *what);
int fail_msg(int code, const std::string &msg);
int elem_size(int dtype);
int ilog2(uint64_t x);
int check_array(const void *d_ptr, size_t n, int dtype);
int resolve_params(const ss_params *p, int dtype, Resolved *r, uint32_t auto_engine = kDefaultEngine);
int check_lines(uint64_t n, const Resolved &R);
int device_info(int dev, int *cus, int *lds);
int occupancy(int dev, const void *fn, int nt, int *blocks, size_t shmem = 0);
int get_workspace(int dev, void *stream, Workspace **out);
void fill_stats(ss_stats *st, const RunOut &ro, const Resolved &R, int dtype);
int run_partition(char *base, size_t n, int dtype, uint64_t pivot, const Resolved &R, hipStream_t st,
                  uint64_t *d_split, bool sync, RunOut *ro, Workspace *wsx);
uint32_t planned_levels(uint64_t n, const Resolved &R);

// Size classes of a batched call: arrays of length <= max_len[c] (and above
// the previous class's bound) use lines of 2^log2b[c] elements and groups of
// at most s_max[c] lines.  One class covers every length by default.
constexpr int kMaxClasses = 8;
struct BatchClasses {
    uint32_t n;
    uint64_t max_len[kMaxClasses];
    uint32_t log2b[kMaxClasses];
    uint32_t s_max[kMaxClasses];
};

// Device state of a batched partition: one entry per array (see ss_batched.hip).
struct BatchState {
    uint64_t *start;   // first element of array k (relative to the base)
    uint64_t *len;     // its length
    const uint64_t *pivot;
    uint64_t *lo, *hi; // current region (absolute element indices)
    uint64_t *split;   // absolute split, ~0 while open
    uint32_t *g;       // groups at the current level (0: finished)
    uint64_t *first;   // first item of array k at the current level (num + 1 entries)
    uint32_t *imap;    // item -> array
    uint64_t *vout;    // item -> splitting position
    uint64_t *ctl;     // [0] items of the current level, [1] open arrays
    uint8_t *cls;      // size class of array k
    const uint32_t *count;  // device word holding the number of arrays (nullable: then num)
    uint32_t num;      // number of arrays, or the capacity when count is set (sizes the grids)
    uint32_t base_lines = 0;  // 1: lines are counted from the base's element 0 (the arrays are parts of
                              // one array); 0: from each array's first element (an array gets
                              // the same bytes alone or in any batch)
};
int batched_state(int dev, void *stream, uint32_t num, uint64_t items_cap, BatchState *B, uint64_t **host_stage,
                  hipEvent_t *stage_copied);
uint64_t batched_items_cap(const uint64_t *lens, uint32_t num, uint64_t tile_elems);
uint32_t batched_levels(uint64_t max_len, uint64_t tile_elems);
uint32_t batched_planned_levels(uint64_t max_len, uint64_t S0, int w);
int batched_graph(int dev, char *base, int dtype, const Resolved &R, const BatchClasses &BC, BatchState &B,
                  uint64_t items_cap, uint32_t levels, hipStream_t st, uint64_t *d_splits, uint32_t *launches,
                  const BatchClasses *tailC = nullptr);
void batched_graphs_forget(const void *state);
BatchClasses batched_default_classes(const Resolved &R);
void batched_installed_classes(int dev, int dtype, const Resolved &R, BatchClasses *C);
bool batched_has_tuning(int dev, int dtype);
uint32_t batched_auto_engine(int dtype);
// Group bytes of the tail geometry (levels from the second on, when a caller
// asks for it: batched_tail_classes).
constexpr uint32_t kTailGroupBytes = 32768;
BatchClasses batched_tail_classes(const BatchClasses &BC, int w);
int batched_core(char *base, int dtype, const Resolved &R, const BatchClasses &BC, BatchState &B, uint32_t levels,
                 hipStream_t st, uint64_t *d_splits, uint32_t *launches, const BatchClasses *tailC = nullptr);

uint64_t quicksort_leaf_cap(int dtype);

int lowspace_partition(char *base, size_t n, int dtype, uint64_t pivot, const Resolved &R, hipStream_t st,
                       uint64_t *d_split, size_t *h_split, ss_stats *stats);
size_t lowspace_aux_bytes(size_t n);
size_t implicit_work_elems(size_t n, int dtype);
int prefix_partition(char *base, size_t n, int dtype, uint64_t pivot, const Resolved &R, hipStream_t st,
                     uint64_t *d_split, size_t *h_split, ss_stats *stats, bool explicit_prefix);
size_t prefix_aux_bytes(size_t n, int dtype, bool explicit_prefix);

}  // namespace ss
