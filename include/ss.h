/*
 * ss.h -- C ABI of an in-place parallel partition library for AMD Instinct
 * MI355X (gfx950), after Kuszmaul & Westover, "In-Place Parallel-Partition
 * Algorithms using Exclusive-Read-and-Write Memory" (arXiv 2004.12532).
 *
 * The operation (Section 2, "The Parallel Partition Problem"): a decider
 * splits the elements of an array A[0, n) into predecessors and successors;
 * the array is reordered in place so that every predecessor precedes every
 * successor.  Throughout this library the decider is
 *
 *     predecessor  <=>  key < pivot        (keys and pivot compared unsigned)
 *
 * and indices are 0-based with half-open ranges (the paper is 1-indexed).
 * On success A is a permutation of its input, A[0, split) holds exactly the
 * predecessors and split is their count.  The order inside each side is
 * unspecified but is a deterministic function of the input, the pivot and
 * the parameters (including the seed).
 *
 * Element types (ss_dtype):
 *   SS_U32  : uint32_t keys; the pivot is compared with the zero-extended
 *             key, so any pivot >= 2^32 makes every element a predecessor.
 *   SS_U64  : uint64_t keys.
 *   SS_KV16 : 16-byte records {uint64_t key; uint64_t payload;} stored
 *             array-of-structures; only the key is compared and the payload
 *             moves with its key.
 *
 * Memory and ownership: every pointer named d_* is a device pointer
 * allocated by the caller (hipMalloc, or a PyTorch CUDA tensor); the caller
 * owns it.  The array must be aligned to its element size (16 bytes for
 * SS_KV16).  The library keeps a small per-stream workspace in device memory
 * (allocated on first use, kept until the process ends) whose size is
 * reported by ss_aux_bytes and in ss_stats.aux_bytes; host pointers (h_*,
 * params, stats) are read or written only during the call.
 *
 * Streams: `stream` is a hipStream_t passed as void*; NULL is the default
 * stream.  Calls that return a host value (h_split, stats, the plain
 * ss_partition / ss_quicksort) synchronize that stream before returning.
 * Concurrent calls on different streams are safe; concurrent calls on the
 * same stream are serialized by the stream.
 *
 * Errors: every entry point returns SS_OK (0) or a negative ss_status.
 * Argument errors (SS_EINVAL, SS_EUNSUPPORTED) are detected before any
 * device work, so the array is untouched.  SS_ENOMEM: the workspace could
 * not be allocated (array untouched).  SS_EDEVICE: a HIP call failed; the
 * array may be partly reordered; ss_last_error() describes the failure.
 */
#ifndef SS_H
#define SS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum ss_dtype { SS_U32 = 1, SS_U64 = 2, SS_KV16 = 3 };

/* Partition algorithms.
 * SS_SMOOTHED : Recursive Smoothed Striding (Section 4, "The Smoothed
 *               Striding Algorithm", "Formal Algorithm Description" and the
 *               recursive variant analysed by Theorem groupedPartitionAlg).
 * SS_STRIDED  : the Strided Algorithm (Section 4, "The Strided Algorithm"):
 *               the same Partial Partition Step with every chunk offset 0,
 *               then one serial cleanup of [v_min, v_max) by a single
 *               workgroup.
 * SS_LOWSPACE : the Low-Space implementation of the Blocked-Prefix-Sum
 *               partition (Section 3 with the explicit block-count array of
 *               Section 5.1); its auxiliary memory is two 32-bit words per
 *               block of 64 elements (n/8 bytes): the block counts of the
 *               array read forward and read reversed, both filled by the
 *               preprocessing passes before the roles are known.
 * SS_HYBRID   : the Hybrid Smoothed Striding Algorithm (Section 4): one
 *               Partial Partition Step, then the Blocked-Prefix-Sum partition
 *               (SS_LOWSPACE) of the middle region [v_min, v_max).  The call
 *               synchronizes the stream once between the two phases (the
 *               host needs v_min and v_max), so it is never asynchronous.
 * SS_MEDIUMSPACE, SS_HIGHSPACE : the Medium- and High-Space comparators
 *               (Section 5.1): the standard parallel partition into an
 *               n-element output array, copied back.  Medium-Space keeps the
 *               predecessor prefix only per block of 64 elements (n/64
 *               words); High-Space also writes every element's prefix into an
 *               n-word array first.  Not in place: ss_aux_bytes reports the
 *               extra n elements (and n words).
 * SS_IMPLICIT : the Blocked-Prefix-Sum partition of Section 3 as stated, with
 *               no auxiliary array: the predecessor prefix of every block of
 *               256 elements is kept in the order of the block's first 64
 *               element pairs (Lemma bitstore; with repeated elements
 *               Lemma bitstore2, which may flip the lowest bit of an element
 *               -- of the payload for SS_KV16 -- while the value is stored
 *               and restores it before the element is used).  Counting, role
 *               swap and preprocessing are those of SS_LOWSPACE.  Arrays of at
 *               most 64 KiB are partitioned by one workgroup directly.
 *               Auxiliary memory is a constant 33 KiB plus the workspace.
 *               With SS_FLAG_ONE_LEVEL (arrays above 64 KiB) the call stops
 *               once every block holds its inclusive prefix: the array is
 *               then preprocessed and encoded, not partitioned. */
enum ss_algo {
    SS_SMOOTHED = 0,
    SS_STRIDED = 1,
    SS_LOWSPACE = 2,
    SS_HYBRID = 3,
    SS_MEDIUMSPACE = 4,
    SS_HIGHSPACE = 5,
    SS_IMPLICIT = 6
};

enum ss_status {
    SS_OK = 0,
    SS_EINVAL = -1,        /* bad argument: null pointer with n > 0, misaligned pointer, bad enum or parameter,
                              n above 2^40, or an array of 2^32 lines or more (line indices are 32-bit) */
    SS_ENOMEM = -2,        /* device workspace allocation failed */
    SS_EDEVICE = -3,       /* a HIP runtime call or kernel launch failed */
    SS_EUNSUPPORTED = -4,  /* valid but unsupported combination (e.g. an algorithm not offered for a dtype) */
    SS_EINCOMPLETE = -5    /* reserved: the recursion ended without a result */
};

/* Flags for ss_params.flags. */
#define SS_FLAG_ONE_LEVEL 1u   /* run only the first Partial Partition Step; the array is then only
                                  partially partitioned: [0, v_min) predecessors, [v_max, n)
                                  successors, reported in ss_stats (Section 4).  With SS_LOWSPACE:
                                  stop after the preprocessing phase (Section 3); ss_stats.vmin is
                                  then the predecessor count and ss_stats.vmax is 1 if the roles
                                  were swapped (the array is read reversed).  With SS_IMPLICIT
                                  (above 64 KiB): stop once every block holds its prefix.  For
                                  tests. */
#define SS_FLAG_TIME 2u        /* time the first-level kernel and the whole call with HIP events on
                                  the call's stream; reported in ss_stats (synchronizes). */
/* Flag bits 4 and 8 are reserved (unknown flags are rejected with SS_EINVAL). */
#define SS_FLAG_GRAPH 16u      /* batched calls: issue the level chain as a captured HIP graph, cached per
                                  (stream, buffers, batch shape) and replayed when they recur */
#define SS_FLAG_EXCHANGE 32u   /* single-array Smoothed Striding, Strided and Hybrid calls: partition
                                  each group by the two-pointer exchange of Section 4 (the k-th
                                  successor from the front below c_i swaps with the k-th predecessor
                                  from the back above it) and write only the swapped elements.  Same
                                  split and sides; each group ends as a serial two-pointer partition
                                  of its slot sequence leaves it.  At a skewed pivot most lines are
                                  only read.  Register engines; with SS_ENGINE_AUTO it selects one. */
#define SS_FLAG_EXCHANGE_SKEWED 64u /* as SS_FLAG_EXCHANGE, but only for groups whose misplaced pairs
                                  are at most 1/32 of their slots; the other groups take the stable
                                  partition.  Same split and sides; the arrangement depends on which
                                  groups were skewed. */
#define SS_FLAG_STABLE 128u    /* never use the exchange form (see below) */
/* Without SS_FLAG_EXCHANGE, SS_FLAG_EXCHANGE_SKEWED or SS_FLAG_STABLE, a
 * Smoothed Striding, Strided or Hybrid call on at least 2^22 elements of 8 or
 * 16 bytes, with default engine, b and tile_bytes, chooses the form of its
 * first level from a sample of 4096 keys at fixed positions (64 runs of 64 keys
 * spread evenly over the array).  It takes the exchange form with 32768-byte
 * groups when at most 1/16 (8-byte keys) or 1/9 (16-byte records) of the
 * sample, or at least 15/16 or 8/9, are predecessors; else the stable form.
 * The choice depends only on the input, so a call stays deterministic;
 * ss_stats.exchange_levels reports it. */

/* Tuning parameters; a zero field means "choose automatically". */
typedef struct ss_params {
    int32_t algo;         /* ss_algo */
    uint32_t b;           /* elements per cache line (the paper's b); b * sizeof(element) must be a
                             power of two between 64 and 4096 bytes.  Default: 512-byte lines. */
    uint32_t tile_bytes;  /* bytes of one group (s * b * sizeof(element) at most): 32768, 65536 or
                             131072 (the last only with SS_ENGINE_REGS or SS_ENGINE_STAGED).  Default: chosen per engine. */
    uint32_t max_levels;  /* Partial Partition Steps of the recursion (1..32), after which the
                             serial base case (one workgroup) partitions what is left.  Default:
                             planned from n, so that the region left is expected to take the base
                             case at most two passes. */
    uint64_t seed;        /* seed of the random chunk offsets X_j; 0 selects a fixed default */
    uint32_t flags;       /* SS_FLAG_* */
    uint32_t engine;      /* workgroup body of a Partial Partition Step: SS_ENGINE_* (0 = auto) */
} ss_params;

/* Workgroup bodies of the Partial Partition Step.  All compute the same
 * stable partition of every group, so results are identical.
 * SS_ENGINE_LDS    : the group is permuted through an LDS tile and written
 *                    back as whole lines.
 * SS_ENGINE_REGS   : the group stays in registers and every element is stored
 *                    straight to its destination (no LDS tile, higher
 *                    occupancy).
 * SS_ENGINE_STAGED : the first level holds the group in registers, stages its
 *                    stable partition in an LDS tile of the group's size and
 *                    writes it back as whole lines while the next group's
 *                    loads are in flight; later levels store from registers
 *                    as SS_ENGINE_REGS does.
 * In every stable body an element whose slot does not change is not stored.
 * SS_ENGINE_AUTO   : SS_ENGINE_STAGED with 131072-byte groups in
 *                    ss_partition / ss_partition_ex.  The batched calls and
 *                    the serving engine use the register engine with
 *                    131072-byte groups, and the LDS engine with 32768-byte
 *                    groups for SS_U32 (four 4-byte scattered stores per
 *                    16-byte vector cost more than staging through LDS); the
 *                    quicksort's levels use the LDS engine with 65536-byte
 *                    groups for SS_U32.  An explicit p->engine / tile_bytes
 *                    overrides these; the batched calls take SS_ENGINE_STAGED
 *                    as SS_ENGINE_REGS. */
#define SS_ENGINE_AUTO 0u
#define SS_ENGINE_LDS 1u
#define SS_ENGINE_REGS 2u
#define SS_ENGINE_STAGED 3u

#define SS_MAX_LEVELS 32

/* Filled by the *_ex entry points when stats != NULL (the call then synchronizes). */
typedef struct ss_stats {
    uint64_t split;                      /* the split index */
    uint64_t aux_bytes;                  /* device workspace (HBM) this call used */
    uint32_t lds_bytes;                  /* LDS per workgroup of the level kernel */
    uint32_t grid;                       /* workgroups of a full level launch */
    uint32_t b;                          /* elements per line used */
    uint32_t s_max;                      /* lines per group bound used */
    uint32_t levels;                     /* Partial Partition Steps that had work */
    uint32_t launches;                   /* kernels launched */
    uint64_t level_lo[SS_MAX_LEVELS];    /* region [lo, hi) of each level with work */
    uint64_t level_hi[SS_MAX_LEVELS];
    uint32_t level_g[SS_MAX_LEVELS];     /* groups g and lines per group s of each level */
    uint32_t level_s[SS_MAX_LEVELS];
    uint64_t vmin, vmax;                 /* splitting-position range after the last level run */
    float first_level_ms;                /* SS_FLAG_TIME: duration of the first level kernel */
    float total_ms;                      /* SS_FLAG_TIME: duration of the whole call on the stream */
    uint64_t bytes_moved;                /* algorithmic HBM bytes: 2 * elem_size * sum of level sizes; a
                                            level in the exchange form counts its reads and the elements
                                            it stored */
    uint32_t exchange_levels;            /* levels (of those listed) run in the write-minimal exchange form */
    uint32_t exchange_mask;              /* bit l: listed level l ran in the exchange form (l < 32) */
    uint64_t first_level_bytes;          /* algorithmic HBM bytes of the first level alone (2 * elem_size *
                                            n, or n * elem_size plus the elements it stored in the
                                            exchange form) */
} ss_stats;

/* Partition d_ptr[0, n) in place by key < pivot with Recursive Smoothed
 * Striding and default parameters; *split receives the split index.
 * Blocking (default stream).  n == 0 gives *split = 0.
 * Section 2 (problem), Section 4 (algorithm). */
int ss_partition(void *d_ptr, size_t n, int dtype, uint64_t pivot, size_t *split);

/* The same with explicit parameters (p may be NULL), a stream, and outputs:
 *   d_split (device, nullable): receives the split as uint64_t, written on
 *            the stream (asynchronous when h_split and stats are NULL);
 *   h_split (host, nullable):   receives the split (call synchronizes);
 *   stats   (host, nullable):   per-level record (call synchronizes).
 * If h_split and stats are both NULL the call does not synchronize.  Every
 * call finishes on the device: the recursion's serial base case partitions
 * whatever region the planned levels leave (a larger region takes it
 * longer), so SS_EINCOMPLETE is not returned by partition calls.
 * SS_FLAG_ONE_LEVEL stops after the first level instead (no base case). */
int ss_partition_ex(void *d_ptr, size_t n, int dtype, uint64_t pivot, const ss_params *p,
                    void *stream, uint64_t *d_split, size_t *h_split, ss_stats *stats);

/* Sort d_ptr[0, n) ascending by key in place with a parallel quicksort built
 * on the partition (Section 5.2, "Example Application: A Full Quicksort"):
 * every segment's pivot is the lower median of 64 of its keys at equally
 * spaced positions, the partition runs at every level for all segments
 * longer than 2^14 elements (8192 for SS_KV16), equal keys are gathered in a
 * final middle block, and a workgroup-local sort in LDS finishes the short
 * segments.  SS_KV16 payloads move
 * with their keys; the order of records with equal keys is unspecified.
 * Blocking (default stream). */
int ss_quicksort(void *d_ptr, size_t n, int dtype);

/* The same with parameters (p may be NULL; p->algo selects the partition
 * used at the upper levels), a stream and optional stats (blocking). */
int ss_quicksort_ex(void *d_ptr, size_t n, int dtype, const ss_params *p, void *stream,
                    ss_stats *stats);

/* Partition `num` independent arrays stored back to back in d_base (Section 2
 * problem applied to each, Section 4 algorithm): array k is
 * d_base[h_offsets[k], h_offsets[k+1]) in elements, with its own pivot
 * d_pivots[k] (device); its split, relative to its own start, is written to
 * d_splits[k] (device).  h_offsets is a host array of num+1 non-decreasing
 * element offsets.  All arrays are processed by one persistent kernel per
 * recursion level; an array that fits one group finishes at the first level.
 * The number of levels is planned from the longest array, and an array still
 * open after them is finished by a single-workgroup cleanup, so a call is a
 * fixed launch sequence (with SS_FLAG_GRAPH, replayed from a cached HIP
 * graph).  Calls on the register body (the default except for SS_U32, or
 * p->engine = SS_ENGINE_REGS) take lines and groups from the installed
 * size-class tuning (ss_autotune_batched / ss_set_batched_tuning) unless p sets b or
 * tile_bytes.  The offsets are staged through one of two pinned host buffers
 * used alternately; a call waits only until the copy from its buffer, issued
 * two calls earlier on the stream, has been read, so back-to-back calls queue
 * on the device without waiting for each other.  It returns without waiting
 * unless stats != NULL.  stats may be NULL. */
int ss_partition_batched(void *d_base, const uint64_t *h_offsets, size_t num, int dtype,
                         const uint64_t *d_pivots, uint64_t *d_splits, const ss_params *p,
                         void *stream, ss_stats *stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): the
 * asynchronous form of ss_partition_ex (d_split required, no h_split or
 * stats) that allocates nothing.  Its partials, level records and result
 * words live in one fixed device array per GPU (16 level slots, about
 * 1 MiB; the library holds it until the process ends) instead of the
 * per-stream workspace.  p may be NULL; it accepts Smoothed Striding or
 * Strided, any b, tile_bytes and engine, SS_FLAG_STABLE / SS_FLAG_EXCHANGE*,
 * and max_levels up to 16 (SS_EINVAL above; the default plan stays far
 * below).  SS_FLAG_TIME and SS_FLAG_GRAPH are rejected.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialized by the caller.  The same
 * arrangement and split as ss_partition_ex with the same parameters. */
int ss_partition_noalloc(void *d_ptr, size_t n, int dtype, uint64_t pivot, const ss_params *p, void *stream,
                         uint64_t *d_split);

/* One call per array, the per-array counterpart of ss_partition_batched:
 * array k is d_base[h_offsets[k], h_offsets[k+1]) (elements; host offsets,
 * non-decreasing, num + 1 of them), partitioned by h_pivots[k] (host) with
 * the single-array path of ss_partition_ex (its own level chain, planned
 * from its length, and base case; an array that fits one group is a single
 * launch), issued back to back on the stream.  d_splits[k] (device)
 * receives the split relative to the array's start.  Without h_ms the call
 * does not synchronize.  With h_ms (host, num floats) an event is recorded
 * after every array and the call waits for the last one: h_ms[k] is the time
 * from the call's first launch to array k's completion on the stream.
 * Section 4 (the step), applied once per array. */
int ss_partition_each(void *d_base, const uint64_t *h_offsets, size_t num, int dtype, const uint64_t *h_pivots,
                      uint64_t *d_splits, const ss_params *p, void *stream, float *h_ms);

/* Batched partition of disjoint segments of one array: segment k is
 * d_base[h_starts[k], h_starts[k] + h_lens[k]) in elements (host arrays;
 * segments may appear in any order but must not overlap), with pivot
 * d_pivots[k] (device); d_splits[k] (device) receives its split relative to
 * h_starts[k].  Same algorithm and semantics as ss_partition_batched, which
 * is the case of back-to-back segments.  Used by the serving loop to put
 * the pending work of many jobs into one launch sequence. */
int ss_partition_segments(void *d_base, const uint64_t *h_starts, const uint64_t *h_lens, size_t num, int dtype,
                          const uint64_t *d_pivots, uint64_t *d_splits, const ss_params *p, void *stream,
                          ss_stats *stats);

/* Size classes of the batched calls: arrays of length in
 * (max_len[c-1], max_len[c]] use lines of b[c] elements and groups of
 * group_bytes[c] bytes (s = group_bytes / (b * element size) lines); the
 * last class in use takes every longer array.  group_bytes <= 131072. */
#define SS_MAX_CLASSES 8
typedef struct ss_batched_tuning {
    uint32_t nclass;                      /* classes in use, 1..SS_MAX_CLASSES */
    uint32_t b[SS_MAX_CLASSES];           /* elements per line (b * element size: 64..4096 bytes) */
    uint32_t group_bytes[SS_MAX_CLASSES]; /* bytes per group */
    uint64_t max_len[SS_MAX_CLASSES];     /* upper length bound of each class */
    float ms[SS_MAX_CLASSES];             /* ss_autotune_batched: best time of the class's tuning batch */
} ss_batched_tuning;

/* Autotune the batched partition for dtype on the current device: for each
 * of seven length classes (up to 2^10, 2^12, ..., 2^20 elements, and longer)
 * a synthetic batch of about 2^24 elements (log-uniform lengths in the class,
 * uniform keys, pivots at uniform quantiles) is partitioned with every
 * candidate line size (128..1024 bytes) and group size (32..128 KiB), timed
 * with HIP events on the register body; the fastest candidate of each class
 * (the default geometry unless a candidate is 3% faster) is installed for
 * later batched calls of this dtype on this device and returned in *out
 * (nullable).  Allocates and frees its own device scratch (a few hundred
 * MiB); synchronizes `stream`. */
int ss_autotune_batched(int dtype, void *stream, ss_batched_tuning *out);

/* Install a size-class table (e.g. one saved from ss_autotune_batched) for
 * dtype on the current device; t == NULL restores the single default class
 * (512-byte lines, 128 KiB groups).  SS_EINVAL for an invalid table. */
int ss_set_batched_tuning(int dtype, const ss_batched_tuning *t);

/* The table in use for dtype on the current device (the default class when
 * none is installed). */
int ss_get_batched_tuning(int dtype, ss_batched_tuning *t);

/* Device-resident serving engine: continuous batching of partition and sort
 * jobs over one caller-owned array d_base[0, capacity) of dtype (the job
 * records live there; the caller places each job in a disjoint range).  All
 * job state -- pending segments, leaves, per-job outstanding counters --
 * stays on the device; a tick is a fixed launch sequence (submitted jobs
 * appended; pivots; one batched Smoothed Striding partition of every pending
 * segment of every job, Section 4; children and leaves of sort jobs as in the
 * quicksort, Section 5.2; leaf sorts) issued on `stream` without waiting.
 * Finished jobs raise a flag in mapped host memory, read with
 * ss_server_done once the tick that finished them has completed
 * (ss_server_wait).  max_jobs slots; max_segments bounds the segments
 * pending at once (a sort job of n records can hold n / (leaf capacity + 1)
 * + 1 of them; the caller's admission must keep the sum within it -- see
 * ss_server_job_aux_bytes).  The engine allocates its device state at
 * creation and nothing per tick.  Calls on one engine must not overlap. */
typedef struct ss_server ss_server;
int ss_server_create(void *d_base, size_t capacity, int dtype, uint32_t max_jobs, uint32_t max_segments,
                     void *stream, ss_server **out);
int ss_server_destroy(ss_server *s);
/* Queue a job for the next tick: kind 0 partitions d_base[start, start+len)
 * by key < pivot, kind 1 sorts it ascending by key.  The slot must be free
 * (its previous job reported done). */
int ss_server_submit(ss_server *s, uint32_t slot, uint64_t start, uint64_t len, int kind, uint64_t pivot);
/* Issue one tick; max_len bounds the longest pending segment (the longest
 * active job will do) and sets the number of partition levels.  At most four
 * ticks are kept in flight (the call waits for the oldest beyond that). */
int ss_server_tick(ss_server *s, uint64_t max_len);
/* Wait until at most `in_flight` issued ticks are still running.  *flags
 * (nullable) receives a copy of the overflow flags kept in mapped host memory:
 * nonzero once a device list overflowed or a partition was left unfinished
 * (the bits may be a subset; ss_server_status gives the exact set). */
int ss_server_wait(ss_server *s, uint32_t in_flight, uint32_t *flags);
/* 1 if the job in `slot` finished in a completed tick (a partition job's split,
 * relative to its start, in *split if non-NULL), 0 if not, < 0 on error. */
int ss_server_done(ss_server *s, uint32_t slot, uint64_t *split);
/* Overflow flags of the device lists after synchronizing the stream (0: every
 * capacity held; 1: a list was full; 2: an unfinished partition). */
int ss_server_status(ss_server *s, uint32_t *flags);
/* Device bytes of list, leaf and item state a job reserves in an engine:
 * what admission adds to the job's input bytes. */
size_t ss_server_job_aux_bytes(int dtype, int kind, uint64_t len);

/* Median-of-3 pivot of every segment (a classic quicksort pivot rule for
 * callers that drive their own quicksort levels, Section 5.2; ss_quicksort
 * itself uses a 64-key sample median): the median of the keys at offsets 0,
 * len/2 and len-1, into d_pivots[k]
 * (device) and, if h_pivots != NULL, h_pivots[k] (host, call synchronizes).
 * Segment lengths must be >= 1. */
int ss_median3_pivots(void *d_base, const uint64_t *h_starts, const uint64_t *h_lens, size_t num, int dtype,
                      uint64_t *d_pivots, uint64_t *h_pivots, void *stream);

/* Sort every segment ascending by key in place with the quicksort's
 * workgroup-local LDS sort, one workgroup per segment: SS_U32 and SS_U64
 * keys are bucketed by their offset from the segment's smallest key and the
 * buckets finished by insertion (a radix sort when a bucket is crowded);
 * SS_KV16 records take a stable radix sort, so records with equal keys keep
 * their order.
 * Segment lengths must be in [1, ss_sort_segment_cap(dtype)]. */
int ss_sort_segments(void *d_base, const uint64_t *h_starts, const uint64_t *h_lens, size_t num, int dtype,
                     void *stream);

/* Largest segment ss_sort_segments accepts: 16384 elements (8192 for SS_KV16). */
size_t ss_sort_segment_cap(int dtype);

/* Device workspace bytes a call on n elements of dtype with algo uses (the
 * auxiliary memory of the in-place model, Section 2 "Memory Model"). */
size_t ss_aux_bytes(size_t n, int dtype, int algo);

/* Static description of a status code. */
const char *ss_strerror(int code);

/* Description of the last SS_EDEVICE failure on this thread ("" if none). */
const char *ss_last_error(void);

/* Memory-bandwidth probe over d_ptr[0, bytes) (bytes a multiple of 16), the
 * GPU counterpart of the paper's bandwidth measurements (Section 5.1, "The
 * Memory-Bandwidth Limitation"): mode 0 reads every byte once, mode 1 reads
 * every 16-byte word and immediately overwrites it with the same value
 * (grid-stride), mode 2 does the same with every workgroup walking one
 * contiguous block of the buffer (the attainable in-place read/write rate).
 * *ms receives the kernel duration (blocking). */
int ss_probe_bandwidth(void *d_ptr, size_t bytes, int mode, void *stream, float *ms);

/* Compute units and LDS bytes per workgroup limit of the current device. */
int ss_device_info(int *compute_units, int *lds_per_block, int *arch_major, int *arch_minor);

#ifdef __cplusplus
}
#endif

#endif /* SS_H */
