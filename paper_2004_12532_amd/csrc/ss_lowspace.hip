// ss_lowspace.hip -- Low-Space Blocked-Prefix-Sum partition (placeholder
// until its kernels land: reports SS_EUNSUPPORTED).
#include "ss_internal.h"

namespace ss {

size_t lowspace_aux_bytes(size_t n) { return (n / 32 + 64) * sizeof(uint64_t); }

int lowspace_partition(char *, size_t, int, uint64_t, const Resolved &, hipStream_t, uint64_t *, size_t *,
                       ss_stats *)
{
    return fail_msg(SS_EUNSUPPORTED, "Low-Space partition not available");
}

}  // namespace ss
