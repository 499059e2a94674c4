// ss_level_rs.hip -- instantiations of the register-resident Partial
// Partition Step in its stable forms: every element stored to its slot of
// the stable partition of its group from registers, or staged in an LDS tile
// and written back as whole lines.
#include "ss_level_rs.h"

namespace ss {

template <typename T, int NT, int NV>
hipError_t launch_level_rs(bool first, uint32_t grid, const LevelArgs &a, hipStream_t st)
{
    return launch_level_rs_t<T, NT, NV, kFormDirect>(first, grid, a, st);
}

template <typename T, int NT, int NV>
const void *level_rs_fn(bool first)
{
    return level_rs_fn_t<T, NT, NV, kFormDirect>(first);
}

template <typename T, int NT, int NV>
hipError_t launch_level_staged(bool first, uint32_t grid, const LevelArgs &a, hipStream_t st)
{
    return launch_level_rs_t<T, NT, NV, kFormStaged>(first, grid, a, st);
}

template <typename T, int NT, int NV>
const void *level_staged_fn(bool first)
{
    return level_rs_fn_t<T, NT, NV, kFormStaged>(first);
}

#define SS_INSTANTIATE_RS(T, NT, NV)                                                                  \
    template hipError_t launch_level_rs<T, NT, NV>(bool, uint32_t, const LevelArgs &, hipStream_t);     \
    template const void *level_rs_fn<T, NT, NV>(bool);                                                  \
    template hipError_t launch_level_staged<T, NT, NV>(bool, uint32_t, const LevelArgs &, hipStream_t); \
    template const void *level_staged_fn<T, NT, NV>(bool);

SS_RS_VARIANTS(SS_INSTANTIATE_RS, uint32_t)
SS_RS_VARIANTS(SS_INSTANTIATE_RS, uint64_t)
SS_RS_VARIANTS(SS_INSTANTIATE_RS, KV)

}  // namespace ss
