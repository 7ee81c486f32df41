// FP32 ladder builds for n_nu padded to 16, 32, 48.
#include "df_ladder_mixed.hpp"

namespace df {

DF_FP32_INSTANTIATE(16)
DF_FP32_INSTANTIATE(32)
DF_FP32_INSTANTIATE(48)

}  // namespace df
