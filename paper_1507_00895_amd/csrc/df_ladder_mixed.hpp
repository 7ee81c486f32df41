// Batched Bethe-Salpeter ladder, mixed precision (kernel templates; built per
// size in df_ladder_mixed_np*.hip and df_ladder_fp32_np*.hip): FP32 inversion on the FP32
// matrix cores, one FP64 residual correction.  Same outputs as the FP64 path
// (eqs. dual_ladder, lin_alg_inv, the radius rule, Gamma^(2) of eq. sd).
//
// Per (channel, Om_m, q) work-group:
//   1. D = 1 - gamma diag(chi) rounded to FP32 tiles; certificate (bound 0.99)
//      as in the FP64 kernel, uncertified items are queued to the FP64
//      partial-pivoting kernel;
//   2. X ~ D^-1 by the certified blocked Gauss-Jordan sweep in FP32;
//   3. Z0 = X gamma                               (FP32 MFMA)
//      E  = gamma - D Z0 = gamma - Z0 + (gamma diag chi) Z0   (FP64 MFMA, exact Z0)
//      Gamma_nn = (Z0)_nn + (X E)_nn              (FP64 accumulation)
//   Both matrix products take three real products per complex one.
//   This is one step of iterative refinement of the solve D Z = gamma,
//   restricted to the diagonal that the Schwinger-Dyson step needs.  The
//   remaining error is of order (kappa eps32)^2 relative, with kappa the
//   condition number of D after diagonal scaling, which the certificate
//   bounds by 1 / (1 - 0.99): about 4e-11 at eps32 = 6e-8.
//   log det D is the sum of the logs of the FP32 pivots, accumulated in FP64
//   (accuracy about kappa * n * eps32 with kappa <= 20 from the bound); items
//   near the instability (bound >= 0.95, among them every item with an
//   eigenvalue of modulus >= 0.95) are queued to the FP64 kernel, whose
//   determinant and Gamma are exact to FP64 rounding.
#pragma once

#include <type_traits>

#include "df_gj_core.hpp"

namespace df {

constexpr int MIX_CERT_ITERS = 6;
constexpr double CERT_MAX_MIXED = 0.99;
// Refined kernel: items with a bound at or above this go to the FP64 kernel,
// so that every item near the instability gets an FP64 determinant and the
// FP32 sweep meets condition numbers of at most 1 / (1 - 0.95) = 20.
constexpr double CERT_NEAR_MIXED = 0.95;

template <int NP> struct MixedShared {
    union {
        GjShared<float, NP> gj;          // during the FP32 sweep
        struct {
            cf Tw[NP / 16][16][17];      // per-wave exchange of X tiles
            cf Gs[2][16][NP];            // gamma rows of the current / next 16-row block
        } z0;                            // during Z0 = X gamma
        cf Zs[NP][NP];                   // then Z0 (FP32), all rows; later E
    };
};
// Column slot of element (i, j) in Zs: odd rows swap the 16-column halves
// of each 32-column block (NP a multiple of 32), so that the two rows read
// by one half-wave fall in different LDS banks.
template <int NP> __device__ __forceinline__ int zs_col(int i, int j) {
    if constexpr (NP % 32 == 0) return j ^ ((i & 1) << 4);
    else return j;
}
// Without refinement only the sweep's state is needed.
template <int NP> struct PlainShared {
    GjShared<float, NP> gj;
};

// REFINE = false: the FP32 ladder alone, from FP32 copies of the vertex
// arrays: D, t and Gamma_nn = sum_l X_nl gamma_ln with X = D^-1 from the FP32
// sweep, all in FP32.  Relative error of order kappa n eps32, about 1e-6 for
// certified items.  FULL: n_nu equals the padded size NP (no clamped index,
// no masked padding).  ITEMS = 2 (FP32 ladder alone): two items per
// work-group, as in the FP64 kernel's two-item build (gjb_item).
template <int NP, bool REFINE, bool FULL, int ITEMS = 1>
__device__ __forceinline__ void mixed_item(LadderArgs a0, int gitem, bool dummy = false) {
    static_assert(ITEMS == 1 || !REFINE, "two items per work-group: FP32 ladder only");
    constexpr int NT = NP / 16;
    typedef MT<float>::v4 f4;
    typedef MT<double>::v4 d4;
    typedef typename std::conditional<REFINE, MixedShared<NP>, PlainShared<NP>>::type Shared;
    __shared__ Shared shv[ITEMS];
    __shared__ cd ypartv[ITEMS][NP];
    __shared__ cd tvv[ITEMS][NP];
    __shared__ int s_flagv[ITEMS];
    const int half = (ITEMS == 2 && threadIdx.x >= NP * 4) ? 1 : 0;
    Shared &sh = shv[half];
    cd *ypart = ypartv[half];
    cd *tv = tvv[half];
    int &s_flag = s_flagv[half];

    const int tid = threadIdx.x - half * (NP * 4);
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
    const double *chi = a.chi + 2 * ((size_t)im * n_nu) * N;   // chi[j] at chi + 2 (j N + q)

    // ---- D in FP32 tiles (FP32 accumulator layout), t_i in FP64.  Per tile
    // column, all loads first and without branches (indices clamped, the
    // padding masked afterwards).
    f4 Cr[NT], Ci[NT];
    cd tp[4];
    const int nm1 = n_nu - 1;
#pragma unroll
    for (int r = 0; r < 4; ++r) tp[r] = {0.0, 0.0};
    if constexpr (!REFINE) {
        // FP32 ladder: vertex and gamma_ij gamma_ji as FP32 pairs, one load each
        const float *gp = a.gp32 + 4 * (size_t)cm * nn;
        cf tf[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) tf[r] = {0.f, 0.f};
#pragma unroll
        for (int tc = 0; tc < NT; ++tc) {
            const int j = 16 * tc + lj;
            const cd xd = ld(chi, (size_t)clamp_nu<FULL>(j, nm1) * N + q);
            const cf xj = {(float)xd.re, (float)xd.im};
            fv4 gv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                gv[r] = ld4f(gp, (size_t)clamp_nu<FULL>(16 * w + MT<float>::row(lg, r), nm1) * n_nu + clamp_nu<FULL>(j, nm1));
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * w + MT<float>::row(lg, r);
                const bool in = FULL || ((i < n_nu) && (j < n_nu));
                const cf x = cf{gv[r].x, gv[r].y} * xj;
                Cr[tc][r] = ((i == j) ? 1.f : 0.f) - (in ? x.re : 0.f);
                Ci[tc][r] = in ? -x.im : 0.f;
                tf[r] = fma_c(tf[r], in ? cf{gv[r].z, gv[r].w} : cf{0.f, 0.f}, xj);
            }
        }
        // the row sums in FP32 too (the FP32 ladder's own error is far larger),
        // through the wave's LDS block (free before the sweep) in the one-item builds
        rows16_sum<ITEMS == 1>(tf, sh.gj.Xw[w], tv + 16 * w, tid);
    } else {
    // t first, on its own, so that its loads do not sit beside the D tiles
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) {
        const int j = 16 * tc + lj;
        const cd xj = ld(chi, (size_t)clamp_nu<FULL>(j, nm1) * N + q);
        cd pv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            pv[r] = ld(pm, (size_t)clamp_nu<FULL>(16 * w + MT<float>::row(lg, r), nm1) * n_nu + clamp_nu<FULL>(j, nm1));
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * w + MT<float>::row(lg, r);
            const bool in = FULL || ((i < n_nu) && (j < n_nu));
            tp[r] = fma_c(tp[r], in ? pv[r] : cd{0.0, 0.0}, xj);
        }
    }
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) {
        int j = 16 * tc + lj;
        asm volatile("" : "+v"(j));   // keeps each tile column's loads in place
        const cd xj = ld(chi, (size_t)clamp_nu<FULL>(j, nm1) * N + q);
        cd gv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            gv[r] = ld(gam, (size_t)clamp_nu<FULL>(16 * w + MT<float>::row(lg, r), nm1) * n_nu + clamp_nu<FULL>(j, nm1));
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * w + MT<float>::row(lg, r);
            const bool in = FULL || ((i < n_nu) && (j < n_nu));
            const cd x = gv[r] * xj;
            Cr[tc][r] = (float)(((i == j) ? 1.0 : 0.0) - (in ? x.re : 0.0));
            Ci[tc][r] = (float)(in ? -x.im : 0.0);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) tp[r] = row16_sum(tp[r]);
    if (lj == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) tv[16 * w + MT<float>::row(lg, r)] = tp[r];
    }
    }

    // The refined kernel keeps items whose bound is below CERT_NEAR_MIXED; the
    // rest (near the instability, where the determinant decides the radius
    // test) go to the FP64 kernel, which re-certifies them and hands its own
    // uncertified items to the pivoting kernel.
    constexpr double accept = REFINE ? CERT_NEAR_MIXED : CERT_MAX_MIXED;
    const double cw = gj_certify<float, NP>(Cr, Ci, sh.gj, MIX_CERT_ITERS, accept, tid,
                                            ITEMS == 2 ? &shv[ITEMS - 1 - half].gj : nullptr,
                                            ITEMS == 2 ? 1 : 0);
    bool skip = dummy;   // no results of this half are written
    if (!(cw < accept)) {
        if (tid == 0 && !dummy) {
            if (REFINE && a.near_queue) a.near_queue[atomicAdd(a.near_count, 1)] = gitem;
            else if (a.queue) a.queue[atomicAdd(a.queue_count, 1)] = gitem;
        }
        if constexpr (ITEMS == 1) return;   // uniform: every thread of the work-group leaves here
        else skip = true;
    }

    gj_sweep<float, NP, true>(Cr, Ci, sh.gj, tid);   // look-ahead inversion

    if (w == 0) {
        cd ldv;
        const int stt = gj_logdet<NP>(sh.gj.pivv, &ldv, tid);
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

    if constexpr (!REFINE) {
        // Gamma_nn formed by every wave before the radius test is known (used
        // only inside the radius), while wave 0 forms log det, with one
        // barrier fewer
        {
            // ---- Gamma_nn = sum_l X_nl gamma_ln  (gamma^T read row-wise); loads
            // per tile column without branches.  Opaque copies of the row and
            // column bases keep the compiler from sharing these indices with
            // those of the D build (which would hold them across the sweep).
            const float *gtr = a.gtr32 + 2 * (size_t)cm * nn;
            const int nm1 = n_nu - 1;
            int row0 = 16 * w, col0 = lj;
            asm volatile("" : "+v"(row0), "+v"(col0));
            cf yf[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) yf[r] = {0.f, 0.f};
#pragma unroll
            for (int tc = 0; tc < NT; ++tc) {
                const int j = 16 * tc + col0;
                fv2 gv[4];
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    gv[r] = ld2f(gtr, (size_t)clamp_nu<FULL>(row0 + MT<float>::row(lg, r), nm1) * n_nu + clamp_nu<FULL>(j, nm1));
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const bool in = FULL || ((row0 + MT<float>::row(lg, r) < n_nu) && (j < n_nu));
                    yf[r] = fma_c(yf[r], cf{Cr[tc][r], Ci[tc][r]},
                                  in ? cf{gv[r].x, gv[r].y} : cf{0.f, 0.f});
                }
            }
            // row sums through the wave's LDS block (the sweep is over) in the
            // one-item builds
            rows16_sum<ITEMS == 1>(yf, sh.gj.Xw[w], ypart + 16 * w, tid);
        }
        __syncthreads();
        const int stt = s_flag;
        if (!skip)
            for (int n = tid; n < n_nu; n += NP * 4) {
                const cd tt = tv[n];
                cd wv;
                if (stt == 0) {
                    const cd y = ypart[n];
                    wv = {y.re - 0.5 * tt.re, y.im - 0.5 * tt.im};
                } else {
                    const cd gnn = ld(gam, (size_t)n * n_nu + n);
                    wv = {gnn.re + 0.5 * tt.re, gnn.im + 0.5 * tt.im};
                }
                st(a.w, ((size_t)cm * n_nu + n) * N + q, wv);
            }
    } else {
    __syncthreads();   // also ends every use of sh.gj
    const int stt = s_flag;
    // Refinement on this wave's block-row.  The FP32 accumulator layout puts
    // row 4 lg + r of a tile in lane group lg, register r; the FP64 products
    // below feed their A-operand rows in the order perm(i) = 4 (i & 3) + (i >> 2),
    // so that their output sits in the same lanes and registers as the FP32 one.
    if (stt == 0) {
        const float *gp = a.gp32 + 4 * (size_t)cm * nn;   // (gamma, gamma_ij gamma_ji) in FP32
        // ---- Z0 = X gamma on the FP32 matrix cores; the wave's X tiles reach the
        // operand layout through its own LDS slot
        // three real products per complex one: P1 = X_re g_re, P2 = X_im g_im,
        // P3 = (X_re + X_im)(g_re + g_im); Z0 = (P1 - P2, P3 - P1 - P2)
        f4 P1[NT], P2[NT], P3[NT];
#pragma unroll
        for (int tc = 0; tc < NT; ++tc) {
            P1[tc] = f4{0, 0, 0, 0};
            P2[tc] = f4{0, 0, 0, 0};
            P3[tc] = f4{0, 0, 0, 0};
        }
        // gamma goes through LDS one 16-row block at a time, loaded once for
        // the four waves (FP32 pairs of the vertex copy, padding zeroed); the
        // next block is in flight while this one's products run
        fv4 gpre[4];
        auto load_block = [&](int kt) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int e = tid + i * NP * 4, r = e / NP, c = e % NP;
                gpre[i] = ld4f(gp, (size_t)clamp_nu<FULL>(16 * kt + r, nm1) * n_nu + clamp_nu<FULL>(c, nm1));
            }
        };
        auto store_block = [&](int kt) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int e = tid + i * NP * 4, r = e / NP, c = e % NP;
                const bool in = FULL || ((16 * kt + r < n_nu) && (c < n_nu));
                sh.z0.Gs[kt & 1][r][c] = in ? cf{gpre[i].x, gpre[i].y} : cf{0.f, 0.f};
            }
        };
        load_block(0);
        store_block(0);
        __syncthreads();
#pragma unroll
        for (int kt = 0; kt < NT; ++kt) {
            if (kt + 1 < NT) load_block(kt + 1);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                sh.z0.Tw[w][MT<float>::row(lg, r)][lj] = cf{Cr[kt][r], Ci[kt][r]};
            wave_sync_lds();
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                const cf xa = sh.z0.Tw[w][lj][4 * k4 + lg];
                const float xs = xa.re + xa.im;
#pragma unroll
                for (int tc = 0; tc < NT; ++tc) {
                    const cf b = sh.z0.Gs[kt & 1][4 * k4 + lg][16 * tc + lj];
                    P1[tc] = MT<float>::mma(xa.re, b.re, P1[tc]);
                    P2[tc] = MT<float>::mma(xa.im, b.im, P2[tc]);
                    P3[tc] = MT<float>::mma(xs, b.re + b.im, P3[tc]);
                }
            }
            if (kt + 1 < NT) store_block(kt + 1);
            __syncthreads();   // the next block is in place; this one and the slot are free
        }
        __syncthreads();   // Zs overlays the exchange slots
        // ---- share Z0 (the registers are free again once it is in LDS)
#pragma unroll
        for (int tc = 0; tc < NT; ++tc)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * w + MT<float>::row(lg, r);
                sh.Zs[i][zs_col<NP>(i, 16 * tc + lj)] =
                    cf{P1[tc][r] - P2[tc][r], P3[tc][r] - P1[tc][r] - P2[tc][r]};
            }
        __syncthreads();
        // the diagonal of Z0 on this wave's rows, before E replaces Z0
        cd zd[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = 16 * w + MT<float>::row(lg, r);
            const cf z = sh.Zs[n][zs_col<NP>(n, n)];
            zd[r] = {(double)z.re, (double)z.im};
        }

        // ---- E = gamma - Z0 + (gamma diag chi) Z0 on the FP64 matrix cores, on
        // the wave's rows, in passes of two tile columns.  Three real products
        // per complex one, with the start value folded in: A1 = E0_re + sum
        // M_re Z_re, A2 = sum M_im Z_im, A3 = E0_re + E0_im + sum (M_re + M_im)
        // (Z_re + Z_im) give E = (A1 - A2, A3 - A1 - A2).  A pass's E goes to
        // LDS, in FP32, over the Z0 columns that no wave reads after it: E is
        // of order kappa eps32 |gamma|, so its own FP32 rounding adds about
        // 6e-8 of that to Gamma.
        constexpr int PW = 2;
        const int lp = 4 * (lj & 3) + (lj >> 2);   // perm(lj)
        const int ia = 16 * w + lp;
        const size_t rowa = (size_t)clamp_nu<FULL>(ia, nm1) * n_nu;
#pragma unroll
        for (int p0 = 0; p0 < NT; p0 += PW) {
            d4 A1[PW], A2[PW], A3[PW];
#pragma unroll
            for (int u = 0; u < PW; ++u) {
                if (p0 + u >= NT) continue;
                int j = 16 * (p0 + u) + lj;
                asm volatile("" : "+v"(j));
                cd gv[4];
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    gv[r] = ld(gam, (size_t)clamp_nu<FULL>(16 * w + MT<float>::row(lg, r), nm1) * n_nu + clamp_nu<FULL>(j, nm1));
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 16 * w + MT<float>::row(lg, r);
                    const bool in = FULL || ((i < n_nu) && (j < n_nu));
                    const cf z = sh.Zs[i][zs_col<NP>(i, j)];
                    const double er = (in ? gv[r].re : 0.0) - (double)z.re;
                    const double ei = (in ? gv[r].im : 0.0) - (double)z.im;
                    A1[u][r] = er;
                    A2[u][r] = 0.0;
                    A3[u][r] = er + ei;
                }
            }
            // k = 4 s + lg.  The operands of step s + 1 are requested once those
            // of step s have arrived, so their latency hides behind step s's
            // products (scheduling barriers keep the compiler from sinking the
            // requests to their use).
            cd g_nx, x_nx;
            {
                int k = lg;
                asm volatile("" : "+v"(k));
                g_nx = ld(gam, rowa + clamp_nu<FULL>(k, nm1));
                x_nx = ld(chi, (size_t)clamp_nu<FULL>(k, nm1) * N + q);
            }
#pragma unroll
            for (int st_ = 0; st_ < 4 * NT; ++st_) {
                const int k = 4 * st_ + lg;
                const cd g0 = g_nx, xk = x_nx;
                __builtin_amdgcn_sched_barrier(0);
                if (st_ + 1 < 4 * NT) {
                    int kn = k + 4;
                    asm volatile("" : "+v"(kn) : "v"(g0.re), "v"(xk.re));
                    g_nx = ld(gam, rowa + clamp_nu<FULL>(kn, nm1));
                    x_nx = ld(chi, (size_t)clamp_nu<FULL>(kn, nm1) * N + q);
                }
                __builtin_amdgcn_sched_barrier(0);   // the requests stay ahead of the products
                // A operand M_ik = gamma_ik chi_k (FP64), B operand Z0_kj.  No mask:
                // rows k >= n_nu of Z0 are exactly zero (X is the identity there
                // and gamma was masked in Z0), and rows ia >= n_nu of E only ever
                // meet the exact zeros of X off its n_nu x n_nu block
                const cd ga = g0 * xk;
                const double gs = ga.re + ga.im;
                cf z[PW];
#pragma unroll
                for (int u = 0; u < PW; ++u)
                    if (p0 + u < NT) z[u] = sh.Zs[k][zs_col<NP>(k, 16 * (p0 + u) + lj)];
#pragma unroll
                for (int u = 0; u < PW; ++u) {
                    if (p0 + u >= NT) continue;
                    const double br = (double)z[u].re, bi = (double)z[u].im;
                    A1[u] = MT<double>::mma(ga.re, br, A1[u]);
                    A2[u] = MT<double>::mma(ga.im, bi, A2[u]);
                    A3[u] = MT<double>::mma(gs, br + bi, A3[u]);
                }
            }
            __syncthreads();   // every wave is done with these columns of Z0
#pragma unroll
            for (int u = 0; u < PW; ++u) {
                if (p0 + u >= NT) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 16 * w + MT<float>::row(lg, r);
                    const double er = A1[u][r] - A2[u][r];
                    const double ei = A3[u][r] - A1[u][r] - A2[u][r];
                    sh.Zs[i][zs_col<NP>(i, 16 * (p0 + u) + lj)] = cf{(float)er, (float)ei};
                }
            }
        }
        __syncthreads();
        // ---- (X E)_nn for the wave's rows n: lane lj takes k = 16 tc + lj
        cd acc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = {0.0, 0.0};
#pragma unroll
        for (int tc = 0; tc < NT; ++tc)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = 16 * w + MT<float>::row(lg, r);
                const int k = 16 * tc + lj;
                const cf e = sh.Zs[k][zs_col<NP>(k, n)];
                acc[r] = fma_c(acc[r], cd{(double)Cr[tc][r], (double)Ci[tc][r]},
                               cd{(double)e.re, (double)e.im});
            }
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = row16_sum(acc[r]);
        if (lj == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) ypart[16 * w + MT<float>::row(lg, r)] = zd[r] + acc[r];
        }
    }
    __syncthreads();
    for (int n = tid; n < n_nu; n += NP * 4) {
        const cd tt = tv[n];
        cd wv;
        if (stt == 0) {
            const cd y = ypart[n];
            wv = {y.re - 0.5 * tt.re, y.im - 0.5 * tt.im};
        } else {
            const cd gnn = ld(gam, (size_t)n * n_nu + n);
            wv = {gnn.re + 0.5 * tt.re, gnn.im + 0.5 * tt.im};
        }
        st(a.w, ((size_t)cm * n_nu + n) * N + q, wv);
    }
    }   // REFINE
}

// One work-group per item, dealt to the XCDs in contiguous ranges.  (The
// kernels call the item function with their argument block directly: through
// a reference and a copy the compiler allocated more registers and spilled.)
//
// Register budgets: the refined kernel at two (the compiler's budget), three
// and four waves per SIMD; the FP32 one at the compiler's budget, four and
// five.  Builds that cannot hold their work-groups' LDS at that occupancy
// are not made: the refined kernel's Z0 / E buffer is NP^2 complex floats
// (72 KB at NP = 96: two work-groups per CU; 128 KB at 128: one).
template <int NP, bool FULL>
__global__ __launch_bounds__(NP * 4) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_ladder_mixed(LadderArgs a0) {
    mixed_item<NP, true, FULL>(a0, a0.item0 + xcd_item(blockIdx.x, gridDim.x));
}
template <int NP, bool FULL>
__global__ __launch_bounds__(NP * 4) __attribute__((amdgpu_waves_per_eu(3, 3)))
void k_ladder_mixed_o3(LadderArgs a0) {
    mixed_item<NP, true, FULL>(a0, a0.item0 + xcd_item(blockIdx.x, gridDim.x));
}
template <int NP, bool FULL>
__global__ __launch_bounds__(NP * 4) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_ladder_mixed_o4(LadderArgs a0) {
    mixed_item<NP, true, FULL>(a0, a0.item0 + xcd_item(blockIdx.x, gridDim.x));
}
template <int NP, bool FULL>
__global__ __launch_bounds__(NP * 4) void k_ladder_fp32(LadderArgs a0) {
    mixed_item<NP, false, FULL>(a0, a0.item0 + xcd_item(blockIdx.x, gridDim.x));
}
template <int NP, bool FULL>
__global__ __launch_bounds__(NP * 4) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_ladder_fp32_o4(LadderArgs a0) {
    mixed_item<NP, false, FULL>(a0, a0.item0 + xcd_item(blockIdx.x, gridDim.x));
}
template <int NP, bool FULL>
__global__ __launch_bounds__(NP * 4) __attribute__((amdgpu_waves_per_eu(5, 5)))
void k_ladder_fp32_o5(LadderArgs a0) {
    mixed_item<NP, false, FULL>(a0, a0.item0 + xcd_item(blockIdx.x, gridDim.x));
}

// FP32 ladder, two items per work-group (NP = 96; see k_ladder_gjb_f64_x2)
template <int NP, bool FULL>
__global__ __launch_bounds__(NP * 8) void k_ladder_fp32_x2(LadderArgs a0) {
    const int half = threadIdx.x >= NP * 4 ? 1 : 0;
    const int k = 2 * xcd_item(blockIdx.x, gridDim.x) + half;
    const bool dummy = k >= a0.n_items;
    mixed_item<NP, false, FULL, 2>(a0, a0.item0 + (dummy ? a0.n_items - 1 : k), dummy);
}

// builds made for each size
template <int NP> constexpr bool has_mixed_occ(int occ) {
    return occ == 0 || (occ == 3 && NP <= 96) || (occ == 4 && NP <= 64);
}
template <int NP> constexpr bool has_fp32_occ(int occ) {
    return occ == 0 || ((occ == 4 || occ == 5) && NP <= 64);
}

// the launch of one build with the launch's mask-free choice (LadderArgs::full)
#define DF_LAUNCH_FULL_M(KERN)                                                          \
    do {                                                                                \
        if (a->full) hipLaunchKernelGGL((KERN<NP, true>), dim3(grid), dim3(NP * 4), 0, s, *a); \
        else hipLaunchKernelGGL((KERN<NP, false>), dim3(grid), dim3(NP * 4), 0, s, *a);        \
    } while (0)

template <typename K>
static int occupancy_of(K kern, int threads) {
    int nb = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, threads, 0) == hipSuccess ? nb : 0;
}

// grid: work-groups of the launch (one per item unless persistent or a queue);
// with query set, only the resident work-groups per CU are returned
template <int NP>
static int mixed_build(const LadderArgs *a, int occ, int grid, hipStream_t s, bool query) {
    if (!has_mixed_occ<NP>(occ)) return -1;
    if (occ == 3) {
        if constexpr (NP <= 96) {
            if (query) return occupancy_of(k_ladder_mixed_o3<NP, false>, NP * 4);
            DF_LAUNCH_FULL_M(k_ladder_mixed_o3);
            return hipGetLastError() == hipSuccess ? 0 : -1;
        }
    } else if (occ == 4) {
        if constexpr (NP <= 64) {
            if (query) return occupancy_of(k_ladder_mixed_o4<NP, false>, NP * 4);
            DF_LAUNCH_FULL_M(k_ladder_mixed_o4);
            return hipGetLastError() == hipSuccess ? 0 : -1;
        }
    } else {
        if (query) return occupancy_of(k_ladder_mixed<NP, false>, NP * 4);
        DF_LAUNCH_FULL_M(k_ladder_mixed);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    return -1;
}

template <int NP>
static int fp32_build(const LadderArgs *a, int occ, int grid, hipStream_t s, bool query) {
    if (!has_fp32_occ<NP>(occ)) return -1;
    if (occ == 4 || occ == 5) {
        if constexpr (NP <= 64) {
            if (occ == 4) {
                if (query) return occupancy_of(k_ladder_fp32_o4<NP, false>, NP * 4);
                DF_LAUNCH_FULL_M(k_ladder_fp32_o4);
            } else {
                if (query) return occupancy_of(k_ladder_fp32_o5<NP, false>, NP * 4);
                DF_LAUNCH_FULL_M(k_ladder_fp32_o5);
            }
            return hipGetLastError() == hipSuccess ? 0 : -1;
        }
        return -1;
    }
    if (query) return occupancy_of(k_ladder_fp32<NP, false>, NP * 4);
    if (NP == 96 && grid == a->n_items && a->full && !a->in_queue && !a->claim)
        hipLaunchKernelGGL((k_ladder_fp32_x2<NP, true>), dim3((grid + 1) / 2), dim3(NP * 8), 0, s, *a);
    else DF_LAUNCH_FULL_M(k_ladder_fp32);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// per-size builds: launch (a non-null) or occupancy query (a null)
#define DF_MIXED_DECLARE(NP)                                                        \
    int mixed_build_##NP(const LadderArgs *a, int occ, int grid, hipStream_t s);    \
    int fp32_build_##NP(const LadderArgs *a, int occ, int grid, hipStream_t s);
DF_MIXED_DECLARE(16)
DF_MIXED_DECLARE(32)
DF_MIXED_DECLARE(48)
DF_MIXED_DECLARE(64)
DF_MIXED_DECLARE(96)
DF_MIXED_DECLARE(128)

#define DF_MIXED_INSTANTIATE(NP)                                                    \
    int mixed_build_##NP(const LadderArgs *a, int occ, int grid, hipStream_t s) {   \
        return mixed_build<NP>(a, occ, grid, s, a == nullptr);                      \
    }
#define DF_FP32_INSTANTIATE(NP)                                                     \
    int fp32_build_##NP(const LadderArgs *a, int occ, int grid, hipStream_t s) {    \
        return fp32_build<NP>(a, occ, grid, s, a == nullptr);                       \
    }

}  // namespace df
