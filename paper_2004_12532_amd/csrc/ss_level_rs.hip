// ss_level_rs.hip -- instantiations of the register-resident Partial
// Partition Step in its stable forms: every element stored to its slot of
// the stable partition of its group from registers, or staged in an LDS tile
// and written back as whole lines.
#include "ss_level_rs.h"

namespace ss {

#define SS_INSTANTIATE_FORM(T, NT, NV, FORM)                                                                  \
    template hipError_t launch_level_rs_t<T, NT, NV, FORM>(bool, uint32_t, const LevelArgs &, hipStream_t); \
    template const void *level_rs_fn_t<T, NT, NV, FORM>(bool);                                              \
    template size_t level_form_lds<T, NT, NV, FORM>();
#define SS_INSTANTIATE_STABLE(T, NT, NV)        \
    SS_INSTANTIATE_FORM(T, NT, NV, kFormDirect) \
    SS_INSTANTIATE_FORM(T, NT, NV, kFormStaged)

SS_RS_VARIANTS(SS_INSTANTIATE_STABLE, uint32_t)
SS_RS_VARIANTS(SS_INSTANTIATE_STABLE, uint64_t)
SS_RS_VARIANTS(SS_INSTANTIATE_STABLE, KV)

}  // namespace ss
