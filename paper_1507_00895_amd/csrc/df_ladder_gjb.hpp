// Batched Bethe-Salpeter ladder, FP64 (kernel templates; instantiated per size
// in df_ladder_gjb_np*.hip): certified pivot-free blocked
// Gauss-Jordan inversion on the FP64 matrix cores (df_gj_core.hpp), for the
// quantities of eqs. (dual_ladder), (lin_alg_inv), the radius rule and the
// second-order term Gamma^(2) = gamma chi gamma of eq. (sd).
//
// One work-group of NP/16 waves per (channel, Om_m, q).  Items whose
// Collatz-Wielandt certificate fails (near or outside the convergence radius)
// are appended to a queue that the partial-pivoting kernel processes next, so
// every item gets a stable elimination.  A certified item has rho(M) < 1,
// i.e. it is inside the radius.
#pragma once

#include "df_gj_core.hpp"

namespace df {

constexpr int CERT_ITERS = 6;
constexpr double CERT_MAX_F64 = 0.999;

// LOOP: the work-group may run several items in turn (a queue or a
// persistent grid, for_each_item).  FULL: n_nu equals the padded size NP, so
// no index is clamped and no padding is masked (measured 2-3 % faster than
// the general path on the same items).
// LDS of one item, one allocation per size (shared by the FULL and the
// general item function)
template <int NP> struct GjbLds {
    GjShared<double, NP> sh;
    cd yv[NP];
    cd tv[NP];
    int s_flag;
};
template <int NP> __device__ __forceinline__ GjbLds<NP> &gjb_lds() {
    __shared__ GjbLds<NP> lds;
    return lds;
}

template <int NP, bool LOOP, bool FULL>
__device__ __forceinline__ void gjb_item(LadderArgs a0, int gitem) {
    constexpr int NT = NP / 16;
    typedef MT<double>::v4 d4;
    GjbLds<NP> &L = gjb_lds<NP>();
    GjShared<double, NP> &sh = L.sh;
    cd *yv = L.yv;
    cd *tv = L.tv;
    int &s_flag = L.s_flag;

    // in an item loop, an opaque copy of the thread index per item (see
    // df_gj_core.hpp)
    int tid = threadIdx.x;
    if constexpr (LOOP) asm volatile("" : "+v"(tid));
    const int w = tid >> 6;
    const int l = tid & 63;
    const int lj = l & 15;
    const int lg = l >> 4;
    LadderArgs a = a0;
    const int item = resolve_item(a, gitem);   // gitem: global item (fused launches)
    const int n_nu = FULL ? NP : a.n_nu, N = a.N;
    int q, cm;
    item_coords(a, item, &cm, &q);
    const int im = __builtin_amdgcn_readfirstlane(cm % a.n_om);
    const size_t nn = (size_t)n_nu * n_nu;
    const double *gam = a.gdm + 2 * (size_t)cm * nn;
    const double *pm = a.pdm + 2 * (size_t)cm * nn;
    const double *gtr = a.gtr + 2 * (size_t)cm * nn;

    // ---- t_i = (gamma chi gamma)_ii = sum_j (gamma_ij gamma_ji) chi_j, on its own
    // before the D tiles exist, so its loads do not sit beside them.  Per tile
    // column all loads first and without branches (indices clamped into the
    // matrix, the padding masked afterwards), so that they are in flight together.
    const int nm1 = n_nu - 1;
    {
        cd tp[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) tp[r] = {0.0, 0.0};
#pragma unroll
        for (int tc = 0; tc < NT; ++tc) {
            const int j = 16 * tc + lj;
            const cd xj = ld(a.chi, ((size_t)im * n_nu + clamp_nu<FULL>(j, nm1)) * N + q);
            cd pv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                pv[r] = ld(pm, (size_t)clamp_nu<FULL>(16 * w + MT<double>::row(lg, r), nm1) * n_nu + clamp_nu<FULL>(j, nm1));
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * w + MT<double>::row(lg, r);
                const bool in = FULL || ((i < n_nu) && (j < n_nu));
                tp[r] = fma_c(tp[r], in ? pv[r] : cd{0.0, 0.0}, xj);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) tp[r] = row16_sum(tp[r]);
        if (lj == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) tv[16 * w + MT<double>::row(lg, r)] = tp[r];
        }
    }

    // ---- D = 1 - gamma diag(chi) in accumulator tiles (opaque column index:
    // the chi loads are not shared with the loop above)
    d4 Cr[NT], Ci[NT];
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) {
        int j = 16 * tc + lj;
        asm volatile("" : "+v"(j));
        const cd xj = ld(a.chi, ((size_t)im * n_nu + clamp_nu<FULL>(j, nm1)) * N + q);
        cd gv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            gv[r] = ld(gam, (size_t)clamp_nu<FULL>(16 * w + MT<double>::row(lg, r), nm1) * n_nu + clamp_nu<FULL>(j, nm1));
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * w + MT<double>::row(lg, r);
            const bool in = FULL || ((i < n_nu) && (j < n_nu));
            const cd x = gv[r] * xj;
            Cr[tc][r] = (((i == j) ? 1.0 : 0.0) - (in ? x.re : 0.0));
            Ci[tc][r] = (in ? -x.im : 0.0);
        }
    }

    const double cw = gj_certify<double, NP>(Cr, Ci, sh, CERT_ITERS, CERT_MAX_F64, tid);
    if (!(cw < CERT_MAX_F64)) {
        if (tid == 0 && a.queue) a.queue[atomicAdd(a.queue_count, 1)] = gitem;
        return;   // uniform: every thread of the work-group leaves here
    }

    // look-ahead inversion up to NP = 96: at 96 it removes the spills (7.14 ->
    // 6.76 ms per instance), at 32 / 48 / 64 the fastest builds gain 2 / 3 / 1 %
    // now that t is formed before the D tiles; at 128 it measured even
    gj_sweep<double, NP, (NP != 128)>(Cr, Ci, sh, tid);

    if (w == 0) {
        cd ldv;
        const int stt = gj_logdet<NP>(sh.pivv, &ldv, tid);
        if (l == 0) {
            s_flag = stt;
            const size_t o = (size_t)cm * N + q;
            if (a.logdet) st(a.logdet, o, ldv);
            if (a.status) a.status[o] = (int8_t)stt;
            if (stt != 0 && a.fallback_count) atomicAdd(a.fallback_count, 1);
        }
    }
    __syncthreads();
    const int stt = s_flag;

    // ---- Gamma_nn = sum_l (D^-1)_nl gamma_ln  (gamma^T read row-wise); loads
    // per tile column without branches (clamped indices, padding masked)
    if (stt == 0) {
        const int nm1 = n_nu - 1;
        // an opaque copy of the row base keeps the compiler from sharing these
        // indices with the identical ones of the D build, which would hold them
        // in registers across the sweep
        int row0 = 16 * w, col0 = lj;
        asm volatile("" : "+v"(row0), "+v"(col0));
        cd yp[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) yp[r] = {0.0, 0.0};
#pragma unroll
        for (int tc = 0; tc < NT; ++tc) {
            const int j = 16 * tc + col0;
            cd gv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                gv[r] = ld(gtr, (size_t)clamp_nu<FULL>(row0 + MT<double>::row(lg, r), nm1) * n_nu + clamp_nu<FULL>(j, nm1));
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const bool in = FULL || ((row0 + MT<double>::row(lg, r) < n_nu) && (j < n_nu));
                yp[r] = fma_c(yp[r], cd{Cr[tc][r], Ci[tc][r]}, in ? gv[r] : cd{0.0, 0.0});
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) yp[r] = row16_sum(yp[r]);
        if (lj == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) yv[16 * w + MT<double>::row(lg, r)] = yp[r];
        }
    }
    __syncthreads();
    for (int n = tid; n < n_nu; n += NP * 4) {
        const cd tt = tv[n];
        cd wv;
        if (stt == 0) {
            const cd y = yv[n];
            wv = {y.re - 0.5 * tt.re, y.im - 0.5 * tt.im};
        } else {
            const cd gnn = ld(gam, (size_t)n * n_nu + n);
            wv = {gnn.re + 0.5 * tt.re, gnn.im + 0.5 * tt.im};
        }
        st(a.w, ((size_t)cm * n_nu + n) * N + q, wv);
    }
}

// Items of an item-loop (LOOP) build: a queue's, or a persistent grid's
// (the general path only: both paths in one loop body held more registers).
template <int NP>
__device__ __forceinline__ void gjb_loop(const LadderArgs &a0) {
    for_each_item(a0, [&](int gitem) __attribute__((always_inline)) {
        gjb_item<NP, true, false>(a0, gitem);
    });
}

// One work-group per item (dealt to the XCDs in contiguous ranges), or the
// item loop.  (The one-item kernels call the item function with their argument
// block directly: through a reference and a copy the compiler allocated more
// registers and spilled.)
#define DF_GJB_BODY(NP, LOOP)                                                   \
    if constexpr (LOOP) gjb_loop<NP>(a0);                                       \
    else {                                                                      \
        const int gi = a0.item0 + xcd_item(blockIdx.x, gridDim.x);              \
        if (item_n_nu(a0, gi) == NP) gjb_item<NP, false, true>(a0, gi);         \
        else gjb_item<NP, false, false>(a0, gi);                                \
    }

// Register budgets of the same kernel: the compiler's own (two work-groups
// per CU at NP = 48, 64) and builds capped for three and four waves per SIMD
// (NP <= 64; the four-wave build spills).  (At NP = 96 the capped build
// spills and measured 25 % slower: not built.)  LOOP builds (the compiler's
// budget and the three-wave cap) serve queue launches and persistent grids.
template <int NP, bool LOOP>
__global__ __launch_bounds__(NP * 4) void k_ladder_gjb_f64(LadderArgs a0) {
    DF_GJB_BODY(NP, LOOP)
}
template <int NP, bool LOOP>
__global__ __launch_bounds__(NP * 4) __attribute__((amdgpu_waves_per_eu(3, 3)))
void k_ladder_gjb_f64_o3(LadderArgs a0) {
    DF_GJB_BODY(NP, LOOP)
}
template <int NP>
__global__ __launch_bounds__(NP * 4) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_ladder_gjb_f64_o4(LadderArgs a0) {
    // the general path only: the mask-free one spills more under this cap
    // (measured slower)
    gjb_item<NP, false, false>(a0, a0.item0 + xcd_item(blockIdx.x, gridDim.x));
}

// grid: work-groups of the launch; loop: a queue launch or a persistent grid
// (LOOP build), else one work-group per item
template <int NP>
static hipError_t launch_gjb(const LadderArgs &a, int occ, int grid, bool loop, hipStream_t s) {
    if constexpr (NP <= 64) {
        if (occ == 3) {
            if (loop) hipLaunchKernelGGL((k_ladder_gjb_f64_o3<NP, true>), dim3(grid), dim3(NP * 4), 0, s, a);
            else hipLaunchKernelGGL((k_ladder_gjb_f64_o3<NP, false>), dim3(grid), dim3(NP * 4), 0, s, a);
            return hipGetLastError();
        }
        if (occ == 4) {
            if (loop) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_ladder_gjb_f64_o4<NP>), dim3(grid), dim3(NP * 4), 0, s, a);
            return hipGetLastError();
        }
    }
    if (loop) hipLaunchKernelGGL((k_ladder_gjb_f64<NP, true>), dim3(grid), dim3(NP * 4), 0, s, a);
    else hipLaunchKernelGGL((k_ladder_gjb_f64<NP, false>), dim3(grid), dim3(NP * 4), 0, s, a);
    return hipGetLastError();
}

// resident work-groups per CU of a LOOP build, for persistent grids
template <int NP>
static int occupancy_gjb(int occ) {
    int nb = 0;
    hipError_t e;
    if constexpr (NP <= 64) {
        if (occ == 3) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ladder_gjb_f64_o3<NP, true>, NP * 4, 0);
        else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ladder_gjb_f64<NP, true>, NP * 4, 0);
    } else {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ladder_gjb_f64<NP, true>, NP * 4, 0);
    }
    return e == hipSuccess ? nb : 0;
}

// per-size builds (df_ladder_gjb_np*.hip)
#define DF_GJB_DECLARE(NP)                                                            \
    hipError_t launch_gjb_##NP(const LadderArgs &a, int occ, int grid, bool loop, hipStream_t s); \
    int occupancy_gjb_##NP(int occ);
DF_GJB_DECLARE(16)
DF_GJB_DECLARE(32)
DF_GJB_DECLARE(48)
DF_GJB_DECLARE(64)
DF_GJB_DECLARE(96)
DF_GJB_DECLARE(128)

#define DF_GJB_INSTANTIATE(NP)                                                                    \
    hipError_t launch_gjb_##NP(const LadderArgs &a, int occ, int grid, bool loop, hipStream_t s) { \
        return launch_gjb<NP>(a, occ, grid, loop, s);                                             \
    }                                                                                             \
    int occupancy_gjb_##NP(int occ) { return occupancy_gjb<NP>(occ); }

}  // namespace df
