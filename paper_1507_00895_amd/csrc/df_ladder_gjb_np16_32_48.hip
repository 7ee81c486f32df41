// FP64 certified ladder builds for n_nu padded to 16, 32, 48.
#include "df_ladder_gjb.hpp"

namespace df {

DF_GJB_INSTANTIATE(16)
DF_GJB_INSTANTIATE(32)
DF_GJB_INSTANTIATE(48)

}  // namespace df
