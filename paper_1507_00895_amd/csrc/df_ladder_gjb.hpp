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
// the general path on the same items).  ITEMS > 1: the work-group holds
// several items, one per slot of NP / 16 waves (k_ladder_gjb_f64_xk); all
// slots take every barrier, so an uncertified item is not left early but
// carried through with its results discarded, and `dummy` marks a slot
// without an item of its own (the last work-group of the launch), which
// computes a copy of the last item and writes nothing.
template <int NP, bool LOOP, bool FULL, int ITEMS = 1>
__device__ __forceinline__ void gjb_item(LadderArgs a0, int gitem, bool dummy = false) {
    constexpr int NT = NP / 16;
    typedef MT<double>::v4 d4;
    __shared__ GjShared<double, NP> shv[ITEMS];
    __shared__ cd yvv[ITEMS][NP];
    __shared__ cd tvv[ITEMS][NP];
    __shared__ int s_flagv[ITEMS];
    const int slot = ITEMS > 1 ? (int)threadIdx.x / (NP * 4) : 0;
    GjShared<double, NP> &sh = shv[slot];
    cd *yv = yvv[slot];
    cd *tv = tvv[slot];
    int &s_flag = s_flagv[slot];

    // in an item loop, an opaque copy of the thread index per item (see
    // df_gj_core.hpp)
    int tid = threadIdx.x - slot * (NP * 4);
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
        rows16_sum<ITEMS == 1>(tp, sh.Xw[w], tv + 16 * w, tid);
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

    const double cw = gj_certify<double, NP, (NP <= 64)>(Cr, Ci, sh, CERT_ITERS, CERT_MAX_F64, tid,
                                             ITEMS > 1 ? shv : nullptr, ITEMS > 1 ? ITEMS : 0);
    bool skip = dummy;   // no results of this half are written
    if (!(cw < CERT_MAX_F64)) {
        if (tid == 0 && a.queue && !dummy) a.queue[atomicAdd(a.queue_count, 1)] = gitem;
        if constexpr (ITEMS == 1) return;   // uniform: every thread of the work-group leaves here
        else skip = true;
    }

    // look-ahead inversion up to NP = 96: at 96 it removes the spills (7.14 ->
    // 6.76 ms per instance), at 32 / 48 / 64 the fastest builds gain 2 / 3 / 1 %
    // now that t is formed before the D tiles; at 128 the persistent (LOOP)
    // build gains 1.7 % with it and the one-item build loses 1.2 %
    gj_sweep<double, NP, (NP != 128) || LOOP>(Cr, Ci, sh, tid);

    if (w == 0) {
        cd ldv;
        const int stt = gj_logdet<NP>(sh.pivv, &ldv, tid);
        if (l == 0) {
            s_flag = stt;
            const size_t o = (size_t)cm * N + q;
            if (!skip) {
                if (a.logdet) st(a.logdet, o, ldv);
                if (a.status) a.status[o] = (int8_t)stt;
                if (stt != 0 && a.fallback_count) atomicAdd(a.fallback_count, 1);
            }
        }
    }
    // ---- Gamma_nn = sum_l (D^-1)_nl gamma_ln  (gamma^T read row-wise); loads
    // per tile column without branches (clamped indices, padding masked).
    // Formed by every wave before the radius test is known (the result is
    // used only inside the radius), so that waves 1.. form it while wave 0
    // forms log det, with one barrier fewer
    {
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
        rows16_sum<ITEMS == 1>(yp, sh.Xw[w], yv + 16 * w, tid);
    }
    __syncthreads();
    const int stt = s_flag;
    if (!skip)
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

// Items of an item-loop (LOOP) build: a queue's, or a persistent grid's.
template <int NP, bool FULL>
__device__ __forceinline__ void gjb_loop(const LadderArgs &a0) {
    for_each_item(a0, [&](int gitem) __attribute__((always_inline)) {
        gjb_item<NP, true, FULL>(a0, gitem);
    });
}

// One work-group per item (dealt to the XCDs in contiguous ranges), or the
// item loop.  (The one-item kernels call the item function with their argument
// block directly: through a reference and a copy the compiler allocated more
// registers and spilled.)  FULL selects the mask-free build, for launches
// whose instances all have n_nu equal to NP (LadderArgs::full); each kernel
// holds one of the two paths, as one holding both needed more registers.
#define DF_GJB_BODY(NP, LOOP, FULL)                                             \
    if constexpr (LOOP) gjb_loop<NP, FULL>(a0);                                 \
    else gjb_item<NP, false, FULL>(a0, a0.item0 + xcd_item(blockIdx.x, gridDim.x));

// Register budgets of the same kernel: the compiler's own (two work-groups
// per CU at NP = 48, 64) and builds capped for three and four waves per SIMD
// (NP <= 64).  (At NP = 96 the capped build spills and measured 6-25 %
// slower: not built.)  LOOP builds (the compiler's budget and the three-wave
// cap) serve queue launches and persistent grids.
template <int NP, bool LOOP, bool FULL>
__global__ __launch_bounds__(NP * 4) void k_ladder_gjb_f64(LadderArgs a0) {
    DF_GJB_BODY(NP, LOOP, FULL)
}
template <int NP, bool LOOP, bool FULL>
__global__ __launch_bounds__(NP * 4) __attribute__((amdgpu_waves_per_eu(3, 3)))
void k_ladder_gjb_f64_o3(LadderArgs a0) {
    DF_GJB_BODY(NP, LOOP, FULL)
}
template <int NP, bool FULL>
__global__ __launch_bounds__(NP * 4) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_ladder_gjb_f64_o4(LadderArgs a0) {
    DF_GJB_BODY(NP, false, FULL)
}

// K items per work-group: an item is NP / 16 waves, and with six-wave
// work-groups (NP = 96) a CU held one work-group even where the registers
// allowed three waves per SIMD (1.5 waves per SIMD measured); a twelve-wave
// work-group of two items fills three per SIMD.  Items K p .. K p + K - 1
// of the launch, p the XCD-mapped work-group index.
template <int NP, bool FULL, int K>
__global__ __launch_bounds__(NP * 4 * K) void k_ladder_gjb_f64_xk(LadderArgs a0) {
    const int slot = (int)threadIdx.x / (NP * 4);
    const int k = K * xcd_item(blockIdx.x, gridDim.x) + slot;
    const bool dummy = k >= a0.n_items;
    gjb_item<NP, false, FULL, K>(a0, a0.item0 + (dummy ? a0.n_items - 1 : k), dummy);
}
// items per work-group of the FP64 build with the compiler's register budget
// (mask-free launches only).  At NP = 32 and 48 four items per work-group
// measured 7-20 % slower than one: only the six-wave items gain.
template <int NP> constexpr int gjb_items_per_group() { return NP == 96 ? 2 : 1; }

// the launch of one build with the launch's FULL choice
#define DF_LAUNCH_FULL(KERN, ...)                                                       \
    do {                                                                                \
        if (a.full) hipLaunchKernelGGL((KERN<__VA_ARGS__, true>), dim3(grid), dim3(NP * 4), 0, s, a); \
        else hipLaunchKernelGGL((KERN<__VA_ARGS__, false>), dim3(grid), dim3(NP * 4), 0, s, a);      \
    } while (0)

// grid: work-groups of the launch; loop: a queue launch or a persistent grid
// (LOOP build), else one work-group per item
template <int NP>
static hipError_t launch_gjb(const LadderArgs &a, int occ, int grid, bool loop, hipStream_t s) {
    if constexpr (NP <= 64) {
        if (occ == 3) {
            if (loop) DF_LAUNCH_FULL(k_ladder_gjb_f64_o3, NP, true);
            else DF_LAUNCH_FULL(k_ladder_gjb_f64_o3, NP, false);
            return hipGetLastError();
        }
        if (occ == 4) {
            if (loop) return hipErrorInvalidValue;
            DF_LAUNCH_FULL(k_ladder_gjb_f64_o4, NP);
            return hipGetLastError();
        }
    }
    if (loop) DF_LAUNCH_FULL(k_ladder_gjb_f64, NP, true);
    else if constexpr (gjb_items_per_group<NP>() > 1) {
        constexpr int K = gjb_items_per_group<NP>();
        // (the general path needs more registers: one item per work-group)
        if (a.full)
            hipLaunchKernelGGL((k_ladder_gjb_f64_xk<NP, true, K>), dim3((grid + K - 1) / K),
                               dim3(NP * 4 * K), 0, s, a);
        else DF_LAUNCH_FULL(k_ladder_gjb_f64, NP, false);
    } else DF_LAUNCH_FULL(k_ladder_gjb_f64, NP, false);
    return hipGetLastError();
}

// resident work-groups per CU of a LOOP build, for persistent grids
template <int NP>
static int occupancy_gjb(int occ) {
    int nb = 0;
    hipError_t e;
    if constexpr (NP <= 64) {
        if (occ == 3) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ladder_gjb_f64_o3<NP, true, false>, NP * 4, 0);
        else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ladder_gjb_f64<NP, true, false>, NP * 4, 0);
    } else {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ladder_gjb_f64<NP, true, false>, NP * 4, 0);
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
