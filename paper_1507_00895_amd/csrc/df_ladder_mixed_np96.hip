// Refined (FP32 + FP64 residual) ladder builds for n_nu padded to 96.
#include "df_ladder_mixed.hpp"

namespace df {

DF_MIXED_INSTANTIATE(96)

}  // namespace df
