// Batched Bethe-Salpeter ladder, eqs. (dual_ladder) and (lin_alg_inv), with
// the convergence-radius rule that follows them and the second-order term
// Gamma^(2) = gamma chi gamma of eq. (sd).
//
// One work-group per (channel c, bosonic Om_m, momentum q).  The matrix
// D = 1 - gamma^c_m diag(chi_m(q)) (n_nu x n_nu complex, zero-padded to NP
// with an identity block) lives in registers: thread (tr, tc) of a TR x TC
// grid owns rows tr + TR*a and columns tc + TC*b (cyclic).  D is inverted in
// place by Gauss-Jordan elimination with partial pivoting; rows are never
// moved, the pivot rows are recorded instead.  Each step needs two barriers:
//   1. every wave finds the pivot of column k (held in LDS) by a
//      wave-level arg-max; the owners of the pivot row copy their rows to LDS;
//   2. every thread reads the pivot-row values of its columns and the
//      column-k values of its rows and applies the rank-1 update; the owners
//      of column k+1 publish it for the next step.
// With R the in-place result and sigma(k) the pivot row of step k,
// D^-1[k][sigma(j)] = R[sigma(k)][j], so
//   Gamma_nn = (D^-1 gamma)_nn = sum_j R[sigma(n)][j] gamma[sigma(j)][n].
// log det D = sum_k log(pivot_k) + i pi * parity(sigma).
#include "df_internal.hpp"

extern "C" __device__ __attribute__((const)) unsigned int __ockl_wfred_max_u32(unsigned int);

namespace df {

// Pivot-search key: the magnitude rounded to FP32 (whose bit pattern orders
// like the value for non-negative numbers) with its low 8 bits replaced by
// 255 - row, so that the unsigned maximum picks the largest magnitude and,
// among equal magnitudes, the lowest row.  Rows already pivoted get key 0.
__device__ __forceinline__ unsigned pivot_key(double mag, int row) {
    const unsigned bits = __float_as_uint((float)mag);
    return (bits & 0xFFFFFF00u) | (unsigned)(255 - row);
}

template <int NP, int TR, int TC>
__global__ __launch_bounds__(TR *TC) void k_ladder_fp64(LadderArgs a0) {
    constexpr int NT = TR * TC;
    constexpr int BR = NP / TR;
    constexpr int BC = NP / TC;
    static_assert(BR * TR == NP && BC * TC == NP, "tile");
    static_assert(NP <= 128, "pivot search covers 128 rows");
    static_assert(TC <= 64 && (64 % TC) == 0, "row groups within a wave");

    __shared__ cd colbuf[2][NP];
    __shared__ cd rowblk[BR][NP];
    __shared__ cd pivv[NP];
    __shared__ int prow[NP];
    __shared__ int rowstep[NP];
    __shared__ cd yv[NP];
    __shared__ cd tv[NP];
    __shared__ int s_status;

    const int tid = threadIdx.x;
    const int tr = tid / TC, tc = tid % TC;
    const int lane = tid & 63;
    const int n_work = a0.in_queue ? *a0.in_count : 1;
    for (int wi = a0.in_queue ? (int)blockIdx.x : 0; wi < n_work;
         wi += (a0.in_queue ? (int)gridDim.x : 1)) {
    LadderArgs a = a0;
    const int item = resolve_item(a, a0.in_queue ? a0.in_queue[wi]
                                                  : a0.item0 + xcd_item(blockIdx.x, gridDim.x));
    const int n_nu = a.n_nu, N = a.N;
    int q, cm;
    item_coords(a, item, &cm, &q);
    const int im = cm % a.n_om;
    const size_t nn = (size_t)n_nu * n_nu;
    const double *gam = a.gdm + 2 * (size_t)cm * nn;
    const double *pm = a.pdm + 2 * (size_t)cm * nn;

    // ---- build D = 1 - gamma diag(chi) and t_i = sum_j gamma_ij chi_j gamma_ji
    cd chi_j[BC];
#pragma unroll
    for (int b = 0; b < BC; ++b) {
        const int j = tc + TC * b;
        chi_j[b] = (j < n_nu) ? ld(a.chi, ((size_t)im * n_nu + j) * N + q) : cd{0.0, 0.0};
    }
    cd A[BR][BC];
    cd tpart[BR];
#pragma unroll
    for (int ai = 0; ai < BR; ++ai) {
        const int i = tr + TR * ai;
        tpart[ai] = {0.0, 0.0};
#pragma unroll
        for (int b = 0; b < BC; ++b) {
            const int j = tc + TC * b;
            const double d = (i == j) ? 1.0 : 0.0;
            if (i < n_nu && j < n_nu) {
                const cd gij = ld(gam, (size_t)i * n_nu + j);
                const cd x = gij * chi_j[b];
                A[ai][b] = {d - x.re, -x.im};
                tpart[ai] = fma_c(tpart[ai], ld(pm, (size_t)i * n_nu + j), chi_j[b]);
            } else {
                A[ai][b] = {d, 0.0};
            }
        }
    }
    // t_i: reduce over the TC consecutive lanes that share row i
#pragma unroll
    for (int off = TC / 2; off >= 1; off >>= 1) {
#pragma unroll
        for (int ai = 0; ai < BR; ++ai) {
            tpart[ai].re += __shfl_xor(tpart[ai].re, off, 64);
            tpart[ai].im += __shfl_xor(tpart[ai].im, off, 64);
        }
    }
    if (tc == 0) {
#pragma unroll
        for (int ai = 0; ai < BR; ++ai) {
            colbuf[0][tr + TR * ai] = A[ai][0];
            tv[tr + TR * ai] = tpart[ai];
        }
    }
    __syncthreads();

    // ---- Gauss-Jordan with partial pivoting
    bool used0 = false, used1 = false;
#pragma unroll
    for (int kk = 0; kk < BC; ++kk) {
        for (int tcol = 0; tcol < TC; ++tcol) {
            const int k = kk * TC + tcol;
            const cd *col = colbuf[k & 1];
            // arg-max of |re| + |im| over rows not yet pivoted (lowest index on
            // ties), as one wave-wide unsigned max of packed (magnitude, index) keys
            unsigned key = 0u;
            if (lane < NP && !used0) key = pivot_key(cabs1(col[lane]), lane);
            if (NP > 64 && lane + 64 < NP && !used1) {
                const unsigned k2 = pivot_key(cabs1(col[lane + 64]), lane + 64);
                key = k2 > key ? k2 : key;
            }
            const int p = 255 - (int)(__ockl_wfred_max_u32(key) & 255u);
            if (p == lane) used0 = true;
            if (p == lane + 64) used1 = true;
            const cd piv = col[p];
            // 1/piv with one division (|piv|^2 cannot overflow for these matrices)
            const double inv2 = 1.0 / fma(piv.re, piv.re, piv.im * piv.im);
            const cd ip = {piv.re * inv2, -piv.im * inv2};
            const int trp = p % TR;
            const int ap = p / TR;
            if (tr == trp) {
#pragma unroll
                for (int ai = 0; ai < BR; ++ai)
#pragma unroll
                    for (int b = 0; b < BC; ++b) rowblk[ai][tc + TC * b] = A[ai][b];
            }
            if (tid == 0) {
                prow[k] = p;
                rowstep[p] = k;
                pivv[k] = piv;
            }
            __syncthreads();

            cd r[BC];
#pragma unroll
            for (int b = 0; b < BC; ++b) r[b] = rowblk[ap][tc + TC * b];
            cd f[BR];
#pragma unroll
            for (int ai = 0; ai < BR; ++ai) {
                const int i = tr + TR * ai;
                const cd cv = col[i];
                f[ai] = (i == p) ? cd{1.0 - ip.re, -ip.im} : cv * ip;
            }
#pragma unroll
            for (int ai = 0; ai < BR; ++ai)
#pragma unroll
                for (int b = 0; b < BC; ++b) A[ai][b] = fms(A[ai][b], f[ai], r[b]);
            if (tc == tcol) {
#pragma unroll
                for (int ai = 0; ai < BR; ++ai) {
                    const int i = tr + TR * ai;
                    A[ai][kk] = (i == p) ? ip : cd{-f[ai].re, -f[ai].im};
                }
            }
            if (k + 1 < NP) {
                cd *nxt = colbuf[(k + 1) & 1];
                if (tcol + 1 < TC) {
                    if (tc == tcol + 1) {
#pragma unroll
                        for (int ai = 0; ai < BR; ++ai) nxt[tr + TR * ai] = A[ai][kk];
                    }
                } else if (kk + 1 < BC) {
                    if (tc == 0) {
#pragma unroll
                        for (int ai = 0; ai < BR; ++ai) nxt[tr + TR * ai] = A[ai][kk + 1 < BC ? kk + 1 : kk];
                    }
                }
            }
            __syncthreads();
        }
    }

    // ---- log det and the convergence-radius test (wave 0)
    if (tid < 64) {
        double lre = 0.0, lim = 0.0;
        int inv = 0;
        for (int k = lane; k < NP; k += 64) {
            const cd pv = pivv[k];
            lre += log(hypot(pv.re, pv.im));
            lim += atan2(pv.im, pv.re);
            const int pk = prow[k];
            for (int j = 0; j < k; ++j) inv += (prow[j] > pk) ? 1 : 0;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            lre += __shfl_xor(lre, off, 64);
            lim += __shfl_xor(lim, off, 64);
            inv += __shfl_xor(inv, off, 64);
        }
        if (lane == 0) {
            double ph = lim + ((inv & 1) ? M_PI : 0.0);
            ph = remainder(ph, 2.0 * M_PI);
            if (ph <= -M_PI) ph += 2.0 * M_PI;
            int stt;
            if (!isfinite(lre) || !isfinite(ph)) stt = 2;
            else stt = (cos(ph) > 0.0) ? 0 : 1;
            s_status = stt;
            const size_t o = (size_t)cm * N + q;
            if (a.logdet) st(a.logdet, o, cd{lre, ph});
            if (a.status) a.status[o] = (int8_t)stt;
            if (stt != 0 && a.fallback_count) atomicAdd(a.fallback_count, 1);
        }
    }
    __syncthreads();
    const int stt = s_status;

    // ---- Gamma_nn: partial sums over this thread's columns, then a
    //      reduction over the TC consecutive lanes sharing the rows
    cd ypart[BR];
#pragma unroll
    for (int ai = 0; ai < BR; ++ai) {
        ypart[ai] = {0.0, 0.0};
        if (stt == 0) {
            const int i = tr + TR * ai;
            const int n = rowstep[i];
            if (n < n_nu) {
#pragma unroll
                for (int b = 0; b < BC; ++b) {
                    const int l = prow[tc + TC * b];
                    if (l < n_nu) ypart[ai] = fma_c(ypart[ai], A[ai][b], ld(gam, (size_t)l * n_nu + n));
                }
            }
        }
    }
#pragma unroll
    for (int off = TC / 2; off >= 1; off >>= 1) {
#pragma unroll
        for (int ai = 0; ai < BR; ++ai) {
            ypart[ai].re += __shfl_xor(ypart[ai].re, off, 64);
            ypart[ai].im += __shfl_xor(ypart[ai].im, off, 64);
        }
    }
    if (tc == 0) {
#pragma unroll
        for (int ai = 0; ai < BR; ++ai) {
            const int i = tr + TR * ai;
            yv[rowstep[i]] = ypart[ai];
        }
    }
    __syncthreads();
    for (int n = tid; n < n_nu; n += NT) {
        const cd t = tv[n];
        cd w;
        if (stt == 0) {
            const cd y = yv[n];
            w = {y.re - 0.5 * t.re, y.im - 0.5 * t.im};
        } else {
            const cd gnn = ld(gam, (size_t)n * n_nu + n);
            w = {gnn.re + 0.5 * t.re, gnn.im + 0.5 * t.im};
        }
        st(a.w, ((size_t)cm * n_nu + n) * N + q, w);
    }
    __syncthreads();   // LDS is reused by the next queued item
    }
}

int ladder_padded_size(int n_nu) {
    if (n_nu <= 0) return 0;
    if (n_nu <= 16) return 16;
    if (n_nu <= 32) return 32;
    if (n_nu <= 48) return 48;
    if (n_nu <= 64) return 64;
    if (n_nu <= 96) return 96;
    if (n_nu <= 128) return 128;
    return 0;
}

template <int NP, int TR, int TC>
static hipError_t launch_one(const LadderArgs &a, hipStream_t s) {
    // split huge batches so gridDim.x stays well inside its limit
    const int chunk = 1 << 30;
    for (int off = 0; off < a.n_items; off += chunk) {
        LadderArgs b = a;
        b.item0 = a.item0 + off;
        const int cnt = (a.n_items - off < chunk) ? a.n_items - off : chunk;
        hipLaunchKernelGGL((k_ladder_fp64<NP, TR, TC>), dim3(cnt), dim3(TR * TC), 0, s, b);
    }
    return hipGetLastError();
}

template <int NP, int TR, int TC>
static hipError_t launch_queue(const LadderArgs &a, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_ladder_fp64<NP, TR, TC>), dim3(blocks), dim3(TR * TC), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ladder_fp64_queue(const LadderArgs &a, int blocks, hipStream_t s) {
    switch (ladder_padded_size(a.n_nu)) {
        case 16: return launch_queue<16, 8, 8>(a, blocks, s);
        case 32: return launch_queue<32, 8, 8>(a, blocks, s);
        case 48: return launch_queue<48, 16, 16>(a, blocks, s);
        case 64: return launch_queue<64, 16, 16>(a, blocks, s);
        case 96: return launch_queue<96, 32, 16>(a, blocks, s);
        case 128: return launch_queue<128, 32, 16>(a, blocks, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ladder_fp64(const LadderArgs &a, hipStream_t s) {
    switch (ladder_padded_size(a.n_nu)) {
        case 16: return launch_one<16, 8, 8>(a, s);
        case 32: return launch_one<32, 8, 8>(a, s);
        case 48: return launch_one<48, 16, 16>(a, s);
        case 64: return launch_one<64, 16, 16>(a, s);
        case 96: return launch_one<96, 32, 16>(a, s);
        case 128: return launch_one<128, 32, 16>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace df
