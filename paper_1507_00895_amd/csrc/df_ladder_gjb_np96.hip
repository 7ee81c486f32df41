// FP64 certified ladder builds for n_nu padded to 96.
#include "df_ladder_gjb.hpp"

namespace df {

DF_GJB_INSTANTIATE(96)

}  // namespace df
