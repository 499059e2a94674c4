/*
 * oracle.c -- plain, slow, obviously correct serial CPU oracle for the
 * in-place parallel partition (Kuszmaul & Westover, "In-Place
 * Parallel-Partition Algorithms using Exclusive-Read-and-Write Memory").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing but the test-suite, the smoke check
 * and the benchmark's CPU-baseline leg may load or call this file.  It
 * shares no source, header, table or helper with the GPU library, and the
 * GPU library never calls it.
 *
 * Contents (0-indexed, half-open ranges throughout; the paper is 1-indexed):
 *   count_less        the plain definition of the split: how many elements
 *                     satisfy the decider key < pivot (Section 2, "The
 *                     Parallel Partition Problem").
 *   partition         serial two-pointer (Hoare) in-place partition with the
 *                     decider key < pivot; the serial baseline of Section 5.1
 *                     is a serial in-place partition of this kind.  Written
 *                     from the textbook scheme (Hoare 1961), not from any
 *                     library's source.
 *   quicksort         serial quicksort: median-of-3 pivot, the two-pointer
 *                     partition above applied twice (key < p, then key <= p
 *                     on the right part) so equal keys end in a middle block,
 *                     insertion sort at 16 elements and below (Section 5.2,
 *                     "Example Application: A Full Quicksort").
 *   is_partitioned    checks that [0,split) satisfy the decider and
 *                     [split,n) do not.
 *   fingerprint       order-independent multiset fingerprint (sums and xor of
 *                     a 64-bit finalizer of each element) for arrays too big
 *                     to sort in a test.
 *   ss_offsets        the random chunk offsets X_j of one Smoothed Striding
 *                     level (Section 4, Formal Algorithm Description), drawn
 *                     from a SplitMix64 counter stream (Steele, Lea & Flood
 *                     2014) and reduced to {0..g-1} by Lemire's
 *                     multiply-shift on the top 32 bits.
 *   ss_partial_step   one Partial Partition Step of Smoothed Striding
 *                     (Section 4): for every group U_i, a serial two-pointer
 *                     partition over the slots of U_i, whose j-th cache line
 *                     is line j*g + ((X_j + i) mod g) of the array; then the
 *                     splitting positions v_i, v_min, v_max.  Lines past the
 *                     end of the array are virtual successors that are never
 *                     touched (Section 4, footnote on gb not dividing n).
 *                     With X_j = 0 for all j this is the Partial Partition
 *                     Step of the Strided Algorithm (Section 4, "The Strided
 *                     Algorithm").
 *
 * Element kinds: u32 (4 B), u64 (8 B), kv (16 B: u64 key then u64 payload;
 * only the key is compared, the payload travels with it).  Keys compare as
 * unsigned 64-bit integers; a u32 key is zero-extended before comparing.
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t key;
    uint64_t val;
} kv16;

#define KEY_u32(x) ((uint64_t)(x))
#define KEY_u64(x) ((uint64_t)(x))
#define KEY_kv(x) ((x).key)

/* SplitMix64: output number ctr (0-based) of the stream whose state starts at
 * seed: the finalizer applied to seed + (ctr + 1) * golden gamma. */
static uint64_t sm64(uint64_t seed, uint64_t ctr)
{
    uint64_t z = seed + (ctr + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t oracle_splitmix64(uint64_t seed, uint64_t ctr) { return sm64(seed, ctr); }

/* MurmurHash3's 64-bit finalizer (Appleby), used only for fingerprints. */
static uint64_t fmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

static uint64_t bits_u32(uint32_t x) { return (uint64_t)x; }
static uint64_t bits_u64(uint64_t x) { return x; }
static uint64_t bits_kv(kv16 x) { return fmix64(x.key) ^ (x.val * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull); }

static uint64_t median3(uint64_t x, uint64_t y, uint64_t z)
{
    if (x > y) {
        uint64_t t = x;
        x = y;
        y = t;
    }
    if (y > z)
        y = z;
    return x > y ? x : y;
}

/* Decider of the partition: 1 = predecessor, 0 = successor.
 * strict != 0 : key <  pivot
 * strict == 0 : key <= pivot   (used by the quicksort for the equal block) */
#define DEFINE_KIND(T, S)                                                                  \
    static int dec_##S(T x, uint64_t p, int strict)                                        \
    {                                                                                      \
        return strict ? (KEY_##S(x) < p) : (KEY_##S(x) <= p);                            \
    }                                                                                      \
                                                                                           \
    size_t oracle_count_less_##S(const T *a, size_t n, uint64_t pivot)                     \
    {                                                                                      \
        size_t c = 0;                                                                      \
        for (size_t k = 0; k < n; k++)                                                     \
            c += (KEY_##S(a[k]) < pivot);                                                  \
        return c;                                                                          \
    }                                                                                      \
                                                                                           \
    /* Two-pointer partition: i scans up over predecessors, j scans down over          */  \
    /* successors; an out-of-place pair is exchanged.  Returns the split.              */  \
    static size_t hoare_##S(T *a, size_t n, uint64_t p, int strict)                        \
    {                                                                                      \
        size_t i = 0, j = n; /* a[0,i) predecessors, a[j,n) successors */                \
        for (;;) {                                                                         \
            while (i < j && dec_##S(a[i], p, strict))                                      \
                i++;                                                                       \
            while (i < j && !dec_##S(a[j - 1], p, strict))                                 \
                j--;                                                                       \
            if (i >= j)                                                                    \
                return i;                                                                  \
            T t = a[i];                                                                    \
            a[i] = a[j - 1];                                                               \
            a[j - 1] = t;                                                                  \
            i++;                                                                           \
            j--;                                                                           \
        }                                                                                  \
    }                                                                                      \
                                                                                           \
    size_t oracle_partition_##S(T *a, size_t n, uint64_t pivot)                            \
    {                                                                                      \
        return hoare_##S(a, n, pivot, 1);                                                  \
    }                                                                                      \
                                                                                           \
    size_t oracle_partition_le_##S(T *a, size_t n, uint64_t pivot)                         \
    {                                                                                      \
        return hoare_##S(a, n, pivot, 0);                                                  \
    }                                                                                      \
                                                                                           \
    static void insertion_##S(T *a, size_t n)                                              \
    {                                                                                      \
        for (size_t k = 1; k < n; k++) {                                                   \
            T x = a[k];                                                                    \
            size_t m = k;                                                                  \
            while (m > 0 && KEY_##S(a[m - 1]) > KEY_##S(x)) {                              \
                a[m] = a[m - 1];                                                           \
                m--;                                                                       \
            }                                                                              \
            a[m] = x;                                                                      \
        }                                                                                  \
    }                                                                                      \
                                                                                           \
    void oracle_quicksort_##S(T *a, size_t n)                                              \
    {                                                                                      \
        while (n > 16) {                                                                   \
            uint64_t p = median3(KEY_##S(a[0]), KEY_##S(a[n / 2]), KEY_##S(a[n - 1]));     \
            size_t m1 = hoare_##S(a, n, p, 1);               /* [0,m1): key <  p */        \
            size_t m2 = m1 + hoare_##S(a + m1, n - m1, p, 0); /* [m1,m2): key == p */      \
            size_t nl = m1, nr = n - m2;                                                   \
            if (nl < nr) {                                                                 \
                oracle_quicksort_##S(a, nl);                                               \
                a += m2;                                                                   \
                n = nr;                                                                    \
            } else {                                                                       \
                oracle_quicksort_##S(a + m2, nr);                                          \
                n = nl;                                                                    \
            }                                                                              \
        }                                                                                  \
        insertion_##S(a, n);                                                               \
    }                                                                                      \
                                                                                           \
    int oracle_is_partitioned_##S(const T *a, size_t n, uint64_t pivot, size_t split)      \
    {                                                                                      \
        if (split > n)                                                                     \
            return 0;                                                                      \
        for (size_t k = 0; k < split; k++)                                                 \
            if (!(KEY_##S(a[k]) < pivot))                                                  \
                return 0;                                                                  \
        for (size_t k = split; k < n; k++)                                                 \
            if (KEY_##S(a[k]) < pivot)                                                     \
                return 0;                                                                  \
        return 1;                                                                          \
    }                                                                                      \
                                                                                           \
    int oracle_is_sorted_##S(const T *a, size_t n)                                         \
    {                                                                                      \
        for (size_t k = 1; k < n; k++)                                                     \
            if (KEY_##S(a[k - 1]) > KEY_##S(a[k]))                                         \
                return 0;                                                                  \
        return 1;                                                                          \
    }                                                                                      \
                                                                                           \
    void oracle_fingerprint_##S(const T *a, size_t n, uint64_t out[4])                     \
    {                                                                                      \
        uint64_t s1 = 0, s2 = 0, x = 0;                                                    \
        for (size_t k = 0; k < n; k++) {                                                   \
            uint64_t h = fmix64(bits_##S(a[k]));                                           \
            s1 += h;                                                                       \
            s2 += h * h;                                                                   \
            x ^= fmix64(h + 0x2545F4914F6CDD1Dull);                                        \
        }                                                                                  \
        out[0] = (uint64_t)n;                                                              \
        out[1] = s1;                                                                       \
        out[2] = s2;                                                                       \
        out[3] = x;                                                                        \
    }                                                                                      \
                                                                                           \
    /* One Partial Partition Step over a[0,n): g groups of s lines of b elements.      */  \
    /* Slot t of U_i (0 <= t < s*b) is element t mod b of U_i's line j = t div b,      */  \
    /* i.e. array position (j*g + (X_j + i) mod g) * b + t mod b.  Positions >= n are  */  \
    /* virtual successors.  c[i] receives the predecessor count of U_i and v[i] its    */  \
    /* splitting position (first successor, or n); either may be NULL.                 */  \
    int oracle_ss_partial_step_##S(T *a, size_t n, uint32_t b, uint32_t g, uint32_t s,     \
                                   const uint32_t *X, uint64_t pivot, uint64_t *vmin,      \
                                   uint64_t *vmax, uint64_t *c, uint64_t *v)               \
    {                                                                                      \
        if (b == 0 || g == 0 || s == 0)                                                    \
            return -1;                                                                     \
        uint64_t gb = (uint64_t)g * b, slots = (uint64_t)s * b;                            \
        if (n == 0 || (uint64_t)s * gb < n || (uint64_t)(s - 1) * gb >= n)                 \
            return -1; /* the virtual padding must stay inside the last chunk */           \
        for (uint32_t j = 0; j < s; j++)                                                   \
            if (X[j] >= g)                                                                 \
                return -1;                                                                 \
        uint64_t lo_all = n, hi_all = 0;                                                   \
        for (uint32_t i = 0; i < g; i++) {                                                 \
            uint64_t lo = 0, hi = slots; /* slots [0,lo) preds, [hi,slots) succs */        \
            for (;;) {                                                                     \
                while (lo < hi) {                                                          \
                    uint64_t j = lo / b, r = (X[j] + i) % g;                               \
                    uint64_t pos = (j * g + r) * b + lo % b;                               \
                    if (pos >= n || !(KEY_##S(a[pos]) < pivot))                            \
                        break;                                                             \
                    lo++;                                                                  \
                }                                                                          \
                while (lo < hi) {                                                          \
                    uint64_t t = hi - 1, j = t / b, r = (X[j] + i) % g;                    \
                    uint64_t pos = (j * g + r) * b + t % b;                                \
                    if (pos < n && KEY_##S(a[pos]) < pivot)                                \
                        break;                                                             \
                    hi--;                                                                  \
                }                                                                          \
                if (lo >= hi)                                                              \
                    break;                                                                 \
                uint64_t jl = lo / b, jh = (hi - 1) / b;                                   \
                uint64_t pl = (jl * g + (X[jl] + i) % g) * b + lo % b;                     \
                uint64_t ph = (jh * g + (X[jh] + i) % g) * b + (hi - 1) % b;               \
                T tmp = a[pl];                                                             \
                a[pl] = a[ph];                                                             \
                a[ph] = tmp;                                                               \
                lo++;                                                                      \
                hi--;                                                                      \
            }                                                                              \
            uint64_t vi;                                                                   \
            if (lo >= slots) {                                                             \
                vi = n;                                                                    \
            } else {                                                                       \
                uint64_t j = lo / b;                                                       \
                vi = (j * g + (X[j] + i) % g) * b + lo % b;                                \
                if (vi > n)                                                                \
                    vi = n;                                                                \
            }                                                                              \
            if (c)                                                                         \
                c[i] = lo;                                                                 \
            if (v)                                                                         \
                v[i] = vi;                                                                 \
            if (vi < lo_all)                                                               \
                lo_all = vi;                                                               \
            if (vi > hi_all)                                                               \
                hi_all = vi;                                                               \
        }                                                                                  \
        *vmin = lo_all;                                                                    \
        *vmax = hi_all;                                                                    \
        return 0;                                                                          \
    }

DEFINE_KIND(uint32_t, u32)
DEFINE_KIND(uint64_t, u64)
DEFINE_KIND(kv16, kv)

/* X_j for j < s at recursion level `level`: counter (level << 40 | j) of the
 * SplitMix64 stream at seed, top 32 bits scaled to [0, g). */
void oracle_ss_offsets(uint64_t seed, uint32_t level, uint32_t g, uint32_t s, uint32_t *X)
{
    for (uint32_t j = 0; j < s; j++) {
        uint64_t r = sm64(seed, ((uint64_t)level << 40) | j);
        X[j] = (uint32_t)(((r >> 32) * (uint64_t)g) >> 32);
    }
}
