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
 *               Section 5.1); its auxiliary memory is about n/32 words. */
enum ss_algo { SS_SMOOTHED = 0, SS_STRIDED = 1, SS_LOWSPACE = 2 };

enum ss_status {
    SS_OK = 0,
    SS_EINVAL = -1,        /* bad argument: null pointer with n > 0, misaligned pointer, bad enum or parameter,
                              n above 2^40, or an array of 2^32 lines or more (line indices are 32-bit) */
    SS_ENOMEM = -2,        /* device workspace allocation failed */
    SS_EDEVICE = -3,       /* a HIP runtime call or kernel launch failed */
    SS_EUNSUPPORTED = -4,  /* valid but unsupported combination (e.g. an algorithm not offered for a dtype) */
    SS_EINCOMPLETE = -5    /* asynchronous call: the device-side recursion budget ran out (see ss_partition_ex) */
};

/* Flags for ss_params.flags. */
#define SS_FLAG_ONE_LEVEL 1u   /* run only the first Partial Partition Step; the array is then only
                                  partially partitioned: [0, v_min) predecessors, [v_max, n)
                                  successors, reported in ss_stats (Section 4).  With SS_LOWSPACE:
                                  stop after the preprocessing phase (Section 3); ss_stats.vmin is
                                  then the predecessor count and ss_stats.vmax is 1 if the roles
                                  were swapped (the array is read reversed).  For tests. */
#define SS_FLAG_TIME 2u        /* time the first-level kernel and the whole call with HIP events on
                                  the call's stream; reported in ss_stats (synchronizes). */
#define SS_FLAG_STREAM 4u      /* register engines: non-temporal (streaming) loads and stores */
#define SS_FLAG_XCD_ORDER 8u   /* register engines: consecutive groups on the same XCD */

/* Tuning parameters; a zero field means "choose automatically". */
typedef struct ss_params {
    int32_t algo;         /* ss_algo */
    uint32_t b;           /* elements per cache line (the paper's b); b * sizeof(element) must be a
                             power of two between 64 and 4096 bytes.  Default: 512-byte lines. */
    uint32_t tile_bytes;  /* bytes of one group (s * b * sizeof(element) at most): 32768, 65536 or
                             131072 (the last only with SS_ENGINE_REGS).  Default: chosen per engine. */
    uint32_t max_levels;  /* recursion levels launched before the host looks at the result (1..32).
                             Default 8. */
    uint64_t seed;        /* seed of the random chunk offsets X_j; 0 selects a fixed default */
    uint32_t flags;       /* SS_FLAG_* */
    uint32_t engine;      /* workgroup body of a Partial Partition Step: SS_ENGINE_* (0 = auto) */
} ss_params;

/* Workgroup bodies of the Partial Partition Step.  Both compute the same
 * stable partition of every group, so results are identical.
 * SS_ENGINE_LDS  : the group is permuted through an LDS tile and written back
 *                  as whole lines.
 * SS_ENGINE_REGS : the group stays in registers and every element is stored
 *                  straight to its destination (no LDS tile, higher occupancy).
 * SS_ENGINE_REGS2: as SS_ENGINE_REGS with two register buffers: the next
 *                  group's loads are in flight while the current one is
 *                  partitioned (32768- or 65536-byte groups). */
#define SS_ENGINE_AUTO 0u
#define SS_ENGINE_LDS 1u
#define SS_ENGINE_REGS 2u
#define SS_ENGINE_REGS2 3u

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
    uint64_t bytes_moved;                /* algorithmic HBM bytes: 2 * elem_size * sum of level sizes */
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
 * If h_split and stats are both NULL the call does not synchronize; if the
 * device-side recursion does not finish within max_levels levels (which for
 * the default budget needs a run of improbable random offsets), *d_split is
 * set to UINT64_MAX and the caller must repeat the call.  A synchronizing
 * call never returns SS_EINCOMPLETE: it continues the recursion from the
 * host until it finishes. */
int ss_partition_ex(void *d_ptr, size_t n, int dtype, uint64_t pivot, const ss_params *p,
                    void *stream, uint64_t *d_split, size_t *h_split, ss_stats *stats);

/* Sort d_ptr[0, n) ascending by key in place with a parallel quicksort built
 * on the partition (Section 5.2, "Example Application: A Full Quicksort"):
 * median-of-3 pivots, the partition at every level for all segments longer
 * than 2^14 elements, equal keys gathered in a final middle block, and a
 * workgroup-local sort in LDS for the short segments.  SS_KV16 payloads move
 * with their keys; the order of records with equal keys is unspecified.
 * Blocking (default stream). */
int ss_quicksort(void *d_ptr, size_t n, int dtype);

/* The same with parameters (p may be NULL; p->algo selects the partition
 * used at the upper levels), a stream and optional stats (blocking). */
int ss_quicksort_ex(void *d_ptr, size_t n, int dtype, const ss_params *p, void *stream,
                    ss_stats *stats);

/* Partition `num` independent arrays stored back to back in d_base (Section 2
 * problem applied to each): array k is d_base[h_offsets[k], h_offsets[k+1])
 * in elements, with its own pivot d_pivots[k] (device); its split, relative
 * to its own start, is written to d_splits[k] (device).  h_offsets is a host
 * array of num+1 non-decreasing element offsets.  All arrays are processed
 * by one persistent kernel per recursion level, arrays that fit one LDS tile
 * as a single group.  stats may be NULL.  Asynchronous unless stats != NULL;
 * d_splits[k] = UINT64_MAX marks an array whose recursion did not finish in
 * the device budget (then SS_EINCOMPLETE is returned by a synchronizing
 * call only if it cannot finish it from the host, which does not happen). */
int ss_partition_batched(void *d_base, const uint64_t *h_offsets, size_t num, int dtype,
                         const uint64_t *d_pivots, uint64_t *d_splits, const ss_params *p,
                         void *stream, ss_stats *stats);

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

/* The quicksort's median-of-3 pivot of every segment (Section 5.2 quicksort;
 * the median of the keys at offsets 0, len/2 and len-1): d_pivots[k]
 * (device) and, if h_pivots != NULL, h_pivots[k] (host, call synchronizes).
 * Segment lengths must be >= 1. */
int ss_median3_pivots(void *d_base, const uint64_t *h_starts, const uint64_t *h_lens, size_t num, int dtype,
                      uint64_t *d_pivots, uint64_t *h_pivots, void *stream);

/* Sort every segment ascending by key in place with the quicksort's
 * workgroup-local LDS sort (stable radix sort; one workgroup per segment).
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
 * every 16-byte word and immediately overwrites it with the same value.
 * *ms receives the kernel duration (blocking). */
int ss_probe_bandwidth(void *d_ptr, size_t bytes, int mode, void *stream, float *ms);

/* Compute units and LDS bytes per workgroup limit of the current device. */
int ss_device_info(int *compute_units, int *lds_per_block, int *arch_major, int *arch_minor);

#ifdef __cplusplus
}
#endif

#endif /* SS_H */
