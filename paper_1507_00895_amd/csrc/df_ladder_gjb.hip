// Batched Bethe-Salpeter ladder, FP64: certified pivot-free blocked
// Gauss-Jordan inversion on the FP64 matrix cores (df_gj_core.hpp), for the
// quantities of eqs. (dual_ladder), (lin_alg_inv), the radius rule and the
// second-order term Gamma^(2) = gamma chi gamma of eq. (sd).
//
// One work-group of NP/16 waves per (channel, Om_m, q).  Items whose
// Collatz-Wielandt certificate fails (near or outside the convergence radius)
// are appended to a queue that the partial-pivoting kernel processes next, so
// every item gets a stable elimination.  A certified item has rho(M) < 1,
// i.e. it is inside the radius.
#include "df_gj_core.hpp"

namespace df {

constexpr int CERT_ITERS = 6;
constexpr double CERT_MAX_F64 = 0.999;

template <int NP>
__device__ __forceinline__ void gjb_body(LadderArgs a0) {
    constexpr int NT = NP / 16;
    typedef MT<double>::v4 d4;
    __shared__ GjShared<double, NP> sh;
    __shared__ cd yv[NP];
    __shared__ cd tv[NP];
    __shared__ int s_flag;

    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int l = tid & 63;
    const int lj = l & 15;
    const int lg = l >> 4;
    LadderArgs a = a0;
    const int gitem = a0.item0 + xcd_item(blockIdx.x, gridDim.x);   // global item (fused launches)
    const int item = resolve_item(a, gitem);
    const int n_nu = a.n_nu, N = a.N;
    int q, cm;
    item_coords(a, item, &cm, &q);
    const int im = cm % a.n_om;
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
            const cd xj = ld(a.chi, ((size_t)im * n_nu + min(j, nm1)) * N + q);
            cd pv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                pv[r] = ld(pm, (size_t)min(16 * w + MT<double>::row(lg, r), nm1) * n_nu + min(j, nm1));
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * w + MT<double>::row(lg, r);
                const bool in = (i < n_nu) && (j < n_nu);
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
        const cd xj = ld(a.chi, ((size_t)im * n_nu + min(j, nm1)) * N + q);
        cd gv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            gv[r] = ld(gam, (size_t)min(16 * w + MT<double>::row(lg, r), nm1) * n_nu + min(j, nm1));
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * w + MT<double>::row(lg, r);
            const bool in = (i < n_nu) && (j < n_nu);
            const cd x = gv[r] * xj;
            Cr[tc][r] = (((i == j) ? 1.0 : 0.0) - (in ? x.re : 0.0));
            Ci[tc][r] = (in ? -x.im : 0.0);
        }
    }

    const double cw = gj_certify<double, NP>(Cr, Ci, sh, CERT_ITERS, CERT_MAX_F64);
    if (!(cw < CERT_MAX_F64)) {
        if (tid == 0 && a.queue) a.queue[atomicAdd(a.queue_count, 1)] = gitem;
        return;   // uniform: every thread of the work-group leaves here
    }

    // look-ahead inversion up to NP = 96: at 96 it removes the spills (7.14 ->
    // 6.76 ms per instance), at 32 / 48 / 64 the fastest builds gain 2 / 3 / 1 %
    // now that t is formed before the D tiles; at 128 it measured even
    gj_sweep<double, NP, (NP != 128)>(Cr, Ci, sh);

    if (w == 0) {
        cd ldv;
        const int stt = gj_logdet<NP>(sh.pivv, &ldv);
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
                gv[r] = ld(gtr, (size_t)min(row0 + MT<double>::row(lg, r), nm1) * n_nu + min(j, nm1));
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const bool in = (row0 + MT<double>::row(lg, r) < n_nu) && (j < n_nu);
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

// Two register budgets of the same kernel: the compiler's own (two
// work-groups per CU at NP = 48, 64) and one capped for three waves per SIMD.
// A build capped for four waves (it spills) is a further tuner candidate.
// (At NP = 96 the capped build spills and measured 25 % slower: not built.)
template <int NP>
__global__ __launch_bounds__(NP * 4) void k_ladder_gjb_f64(LadderArgs a0) {
    gjb_body<NP>(a0);
}
template <int NP>
__global__ __launch_bounds__(NP * 4) __attribute__((amdgpu_waves_per_eu(3, 3)))
void k_ladder_gjb_f64_o3(LadderArgs a0) {
    gjb_body<NP>(a0);
}
template <int NP>
__global__ __launch_bounds__(NP * 4) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_ladder_gjb_f64_o4(LadderArgs a0) {
    gjb_body<NP>(a0);
}

template <int NP>
static hipError_t launch_gjb(const LadderArgs &a, int occ, hipStream_t s) {
    if constexpr (NP <= 64) {
        if (occ == 3) {
            hipLaunchKernelGGL((k_ladder_gjb_f64_o3<NP>), dim3(a.n_items), dim3(NP * 4), 0, s, a);
            return hipGetLastError();
        }
        if (occ == 4) {
            hipLaunchKernelGGL((k_ladder_gjb_f64_o4<NP>), dim3(a.n_items), dim3(NP * 4), 0, s, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_ladder_gjb_f64<NP>), dim3(a.n_items), dim3(NP * 4), 0, s, a);
    return hipGetLastError();
}

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

hipError_t launch_ladder_gjb_f64(const LadderArgs &a, int occ, hipStream_t s) {
    if ((occ == 3 || occ == 4) && !ladder_gjb_has_occ3(a.n_nu)) return hipErrorInvalidValue;
    switch (ladder_gjb_padded_size(a.n_nu)) {
        case 16: return launch_gjb<16>(a, occ, s);
        case 32: return launch_gjb<32>(a, occ, s);
        case 48: return launch_gjb<48>(a, occ, s);
        case 64: return launch_gjb<64>(a, occ, s);
        case 96: return launch_gjb<96>(a, 0, s);
        case 128: return launch_gjb<128>(a, 0, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace df
