// ss_quicksort.hip -- parallel quicksort on the partition (placeholder until
// its kernels land: reports SS_EUNSUPPORTED).
#include "ss_internal.h"

using namespace ss;

extern "C" int ss_quicksort_ex(void *d_ptr, size_t n, int dtype, const ss_params *p, void *stream,
                               ss_stats *stats)
{
    int rc = check_array(d_ptr, n, dtype);
    if (rc)
        return rc;
    (void)p; (void)stream; (void)stats;
    return fail_msg(SS_EUNSUPPORTED, "quicksort not available");
}

extern "C" int ss_quicksort(void *d_ptr, size_t n, int dtype)
{
    return ss_quicksort_ex(d_ptr, n, dtype, nullptr, nullptr, nullptr);
}
