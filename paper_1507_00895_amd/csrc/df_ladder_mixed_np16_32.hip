// Refined (FP32 + FP64 residual) ladder builds for n_nu padded to 16, 32.
#include "df_ladder_mixed.hpp"

namespace df {

DF_MIXED_INSTANTIATE(16)
DF_MIXED_INSTANTIATE(32)

}  // namespace df
