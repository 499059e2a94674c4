// ss_batched.hip -- batched partition of many arrays (placeholder until its
// kernels land: reports SS_EUNSUPPORTED).
#include "ss_internal.h"

using namespace ss;

extern "C" int ss_partition_batched(void *d_base, const uint64_t *h_offsets, size_t num, int dtype,
                                    const uint64_t *d_pivots, uint64_t *d_splits, const ss_params *p,
                                    void *stream, ss_stats *stats)
{
    (void)d_base; (void)h_offsets; (void)num; (void)dtype; (void)d_pivots; (void)d_splits; (void)p;
    (void)stream; (void)stats;
    return fail_msg(SS_EUNSUPPORTED, "batched partition not available");
}
