// FP64 certified ladder: sizes, dispatch to the per-size builds.
#include "df_ladder_gjb.hpp"

namespace df {

int ladder_gjb_padded_size(int n_nu) {
    if (n_nu <= 0) return 0;
    if (n_nu <= 16) return 16;
    if (n_nu <= 32) return 32;
    if (n_nu <= 48) return 48;
    if (n_nu <= 64) return 64;
    if (n_nu <= 96) return 96;
    if (n_nu <= 128) return 128;   // 8 waves; spills a little (one work-group per CU)
    return 0;
}

bool ladder_gjb_has_occ3(int n_nu) {
    const int np = ladder_gjb_padded_size(n_nu);
    return np != 0 && np <= 64;
}

hipError_t launch_ladder_gjb_f64(const LadderArgs &a, int occ, int grid, hipStream_t s) {
    if ((occ == 3 || occ == 4) && !ladder_gjb_has_occ3(a.n_nu)) return hipErrorInvalidValue;
    if (grid <= 0) return hipErrorInvalidValue;
    // queue launches and persistent grids run the item-loop builds
    const bool loop = a.in_queue != nullptr || a.claim != nullptr;
    switch (ladder_gjb_padded_size(a.n_nu)) {
        case 16: return launch_gjb_16(a, occ, grid, loop, s);
        case 32: return launch_gjb_32(a, occ, grid, loop, s);
        case 48: return launch_gjb_48(a, occ, grid, loop, s);
        case 64: return launch_gjb_64(a, occ, grid, loop, s);
        case 96: return launch_gjb_96(a, 0, grid, loop, s);
        case 128: return launch_gjb_128(a, 0, grid, loop, s);
        default: return hipErrorInvalidValue;
    }
}

int ladder_gjb_occupancy(int n_nu, int occ) {
    switch (ladder_gjb_padded_size(n_nu)) {
        case 16: return occupancy_gjb_16(occ);
        case 32: return occupancy_gjb_32(occ);
        case 48: return occupancy_gjb_48(occ);
        case 64: return occupancy_gjb_64(occ);
        case 96: return occupancy_gjb_96(0);
        case 128: return occupancy_gjb_128(0);
        default: return 0;
    }
}

}  // namespace df
