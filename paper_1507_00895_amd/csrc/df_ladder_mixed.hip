// Mixed-precision and FP32 ladders: sizes, dispatch to the per-size builds.
#include "df_ladder_mixed.hpp"

namespace df {

// The refined and the FP32 kernels serve every size up to 128.
int ladder_mixed_padded_size(int n_nu) {
    if (n_nu <= 0) return 0;
    if (n_nu <= 16) return 16;
    if (n_nu <= 32) return 32;
    if (n_nu <= 48) return 48;
    if (n_nu <= 64) return 64;
    if (n_nu <= 96) return 96;
    if (n_nu <= 128) return 128;
    return 0;
}

int ladder_fp32_padded_size(int n_nu) { return ladder_mixed_padded_size(n_nu); }

bool ladder_mixed_has_occ(int n_nu, int occ) {
    const int np = ladder_mixed_padded_size(n_nu);
    return np != 0 && (occ == 0 || (occ == 3 && np <= 96) || (occ == 4 && np <= 64));
}

bool ladder_fp32_has_occ(int n_nu, int occ) {
    const int np = ladder_fp32_padded_size(n_nu);
    return np != 0 && (occ == 0 || ((occ == 4 || occ == 5) && np <= 64));
}

static int mixed_dispatch(int n_nu, const LadderArgs *a, int occ, int grid, hipStream_t s) {
    switch (ladder_mixed_padded_size(n_nu)) {
        case 16: return mixed_build_16(a, occ, grid, s);
        case 32: return mixed_build_32(a, occ, grid, s);
        case 48: return mixed_build_48(a, occ, grid, s);
        case 64: return mixed_build_64(a, occ, grid, s);
        case 96: return mixed_build_96(a, occ, grid, s);
        case 128: return mixed_build_128(a, occ, grid, s);
        default: return -1;
    }
}

static int fp32_dispatch(int n_nu, const LadderArgs *a, int occ, int grid, hipStream_t s) {
    switch (ladder_fp32_padded_size(n_nu)) {
        case 16: return fp32_build_16(a, occ, grid, s);
        case 32: return fp32_build_32(a, occ, grid, s);
        case 48: return fp32_build_48(a, occ, grid, s);
        case 64: return fp32_build_64(a, occ, grid, s);
        case 96: return fp32_build_96(a, occ, grid, s);
        case 128: return fp32_build_128(a, occ, grid, s);
        default: return -1;
    }
}

hipError_t launch_ladder_mixed(const LadderArgs &a, int occ, int grid, hipStream_t s) {
    if (grid <= 0 || !ladder_mixed_has_occ(a.n_nu, occ)) return hipErrorInvalidValue;
    return mixed_dispatch(a.n_nu, &a, occ, grid, s) == 0 ? hipSuccess : hipErrorLaunchFailure;
}

hipError_t launch_ladder_fp32(const LadderArgs &a, int occ, int grid, hipStream_t s) {
    if (grid <= 0 || !ladder_fp32_has_occ(a.n_nu, occ)) return hipErrorInvalidValue;
    return fp32_dispatch(a.n_nu, &a, occ, grid, s) == 0 ? hipSuccess : hipErrorLaunchFailure;
}

int ladder_mixed_occupancy(int n_nu, int occ) {
    return ladder_mixed_has_occ(n_nu, occ) ? mixed_dispatch(n_nu, nullptr, occ, 0, nullptr) : 0;
}

int ladder_fp32_occupancy(int n_nu, int occ) {
    return ladder_fp32_has_occ(n_nu, occ) ? fp32_dispatch(n_nu, nullptr, occ, 0, nullptr) : 0;
}

}  // namespace df
