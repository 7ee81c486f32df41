// FP32 ladder builds for n_nu padded to 128.
#include "df_ladder_mixed.hpp"

namespace df {

DF_FP32_INSTANTIATE(128)

}  // namespace df
