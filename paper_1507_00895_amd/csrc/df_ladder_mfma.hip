// Batched Bethe-Salpeter ladder on the FP64 matrix cores (MFMA), blocked
// Gauss-Jordan inversion; same mathematics as k_ladder_fp64 (eqs. dual_ladder,
// lin_alg_inv, the radius rule, Gamma^(2) of eq. sd), different schedule.
//
// One work-group of W = NP/16 waves per (channel, Om_m, q).  Wave w keeps the
// 16 x NP block-row w of D in MFMA accumulator tiles (16 x 16 complex = two
// real tiles, 4 doubles per lane).  The inversion proceeds in NP/16 panels
// of 16 columns:
//   1. the waves publish tile (w, t) of the panel column to LDS;
//   2. wave 0 runs the 16 Gauss-Jordan steps with partial pivoting on the
//      NP x 16 panel, one row per lane (arg-max by a DPP wave reduction, the
//      pivot row broadcast through LDS), and records the pivots;
//   3. the owners of the 16 pivot rows publish their rows (old values);
//   4. every wave applies the rank-16 update  D += G R  to its other tiles
//      with v_mfma_f64_16x16x4f64 (complex product as four real products),
//      where G = panel result - E_P (E_P has a 1 at (pivot row, step)) and
//      R = the old pivot rows; the panel tile takes the panel result.
// This is the right-looking block form of the in-place Gauss-Jordan sweep:
// after the 16 steps of a panel every other column has been multiplied by
// T = I + G S_P, where S_P selects the pivot rows, and column t of G equals
// T e_p - e_p, which is exactly what the in-place sweep leaves in the panel.
//
// FP64 16x16x4 MFMA lane layout (measured on gfx950):
//   A[i][k] : lane i + 16 k          B[k][j] : lane j + 16 k
//   C[i][j] : lane j + 16 (i % 4), register i / 4
#include "df_internal.hpp"

extern "C" __device__ __attribute__((const)) unsigned int __ockl_wfred_max_u32(unsigned int);

namespace df {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned pkey(double mag, int row) {
    const unsigned bits = __float_as_uint((float)mag);
    return (bits & 0xFFFFFF00u) | (unsigned)(255 - row);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int NP>
__global__ __launch_bounds__(NP * 4) void k_ladder_mfma_f64(LadderArgs a0) {
    constexpr int NT = NP / 16;      // tiles per row / column, = waves
    static_assert(NP % 16 == 0 && NP <= 64, "one panel row per lane");

    __shared__ cd Pn[NP][16];        // panel (NP rows x 16 columns)
    __shared__ cd Rr[16][NP];        // old pivot rows of the current panel
    __shared__ cd bcast[2][16];      // pivot-row broadcast inside wave 0
    __shared__ cd pivv[NP];
    __shared__ int prow[NP];
    __shared__ int rowstep[NP];
    __shared__ cd yv[NP];
    __shared__ cd tv[NP];
    __shared__ int s_status;

    const int tid = threadIdx.x;
    const int w = tid >> 6;          // wave = block-row
    const int l = tid & 63;
    const int lj = l & 15;           // column inside a tile
    const int lg = l >> 4;           // row group: rows lg + 4 r, r = 0..3
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

    // ---- D = 1 - gamma diag(chi) in accumulator tiles; t_i partial sums
    d4 Cr[NT], Ci[NT];
    cd tp[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) tp[r] = {0.0, 0.0};
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) {
        const int j = 16 * tc + lj;
        const cd xj = (j < n_nu) ? ld(a.chi, ((size_t)im * n_nu + j) * N + q) : cd{0.0, 0.0};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * w + lg + 4 * r;
            double dr = (i == j) ? 1.0 : 0.0, di = 0.0;
            if (i < n_nu && j < n_nu) {
                const cd x = ld(gam, (size_t)i * n_nu + j) * xj;
                dr -= x.re;
                di = -x.im;
                tp[r] = fma_c(tp[r], ld(pm, (size_t)i * n_nu + j), xj);
            }
            Cr[tc][r] = dr;
            Ci[tc][r] = di;
        }
    }
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            tp[r].re += __shfl_xor(tp[r].re, off, 64);
            tp[r].im += __shfl_xor(tp[r].im, off, 64);
        }
    }
    if (lj == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) tv[16 * w + lg + 4 * r] = tp[r];
    }

    bool used = false;               // wave 0: row l already pivoted
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        // 1. publish panel tile (w, t)
#pragma unroll
        for (int r = 0; r < 4; ++r) Pn[16 * w + lg + 4 * r][lj] = cd{Cr[t][r], Ci[t][r]};
        __syncthreads();

        // 2. wave 0: 16 Gauss-Jordan steps on the panel, lane = row
        if (w == 0) {
            cd P[16];
            const bool live = l < NP;
#pragma unroll
            for (int j = 0; j < 16; ++j) P[j] = live ? Pn[l][j] : cd{0.0, 0.0};
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const int kk = 16 * t + s;
                const unsigned key = (live && !used) ? pkey(cabs1(P[s]), l) : 0u;
                const int p = 255 - (int)(__ockl_wfred_max_u32(key) & 255u);
                const cd piv = {readlane_d(P[s].re, p), readlane_d(P[s].im, p)};
                const double inv2 = 1.0 / fma(piv.re, piv.re, piv.im * piv.im);
                const cd ip = {piv.re * inv2, -piv.im * inv2};
                cd *bc = bcast[s & 1];
                if (l == p) {
#pragma unroll
                    for (int j = 0; j < 16; ++j) bc[j] = P[j];
                    used = true;
                }
                if (l == 0) {
                    prow[kk] = p;
                    rowstep[p] = kk;
                    pivv[kk] = piv;
                }
                wave_lds_sync();
                const bool me = (l == p);
                const cd f = me ? cd{1.0 - ip.re, -ip.im} : P[s] * ip;
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    if (j == s) continue;
                    P[j] = fms(P[j], f, bc[j]);
                }
                P[s] = me ? ip : cd{-f.re, -f.im};
            }
            if (live) {
#pragma unroll
                for (int j = 0; j < 16; ++j) Pn[l][j] = P[j];
            }
        }
        __syncthreads();

        // 3. owners publish the old pivot rows
        for (int s = 0; s < 16; ++s) {
            const int p = prow[16 * t + s];
            if ((p >> 4) != w) continue;
            const int pl = p & 15;
            if (lg != (pl & 3)) continue;
            const int rp = pl >> 2;
#pragma unroll
            for (int tc = 0; tc < NT; ++tc) {
                double vr, vi;
                switch (rp) {
                    case 0: vr = Cr[tc][0]; vi = Ci[tc][0]; break;
                    case 1: vr = Cr[tc][1]; vi = Ci[tc][1]; break;
                    case 2: vr = Cr[tc][2]; vi = Ci[tc][2]; break;
                    default: vr = Cr[tc][3]; vi = Ci[tc][3]; break;
                }
                Rr[s][16 * tc + lj] = cd{vr, vi};
            }
        }
        __syncthreads();

        // 4. rank-16 update of the other tiles on the matrix cores
        double gr[4], gi[4], gn[4];
#pragma unroll
        for (int k4 = 0; k4 < 4; ++k4) {
            const int k = 4 * k4 + lg;
            const int row = 16 * w + lj;
            cd g = Pn[row][k];
            if (prow[16 * t + k] == row) g.re -= 1.0;
            gr[k4] = g.re;
            gi[k4] = g.im;
            gn[k4] = -g.im;
        }
#pragma unroll
        for (int tc = 0; tc < NT; ++tc) {
            if (tc == t) continue;
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                const cd b = Rr[4 * k4 + lg][16 * tc + lj];
                Cr[tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(gr[k4], b.re, Cr[tc], 0, 0, 0);
                Cr[tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(gn[k4], b.im, Cr[tc], 0, 0, 0);
                Ci[tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(gr[k4], b.im, Ci[tc], 0, 0, 0);
                Ci[tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(gi[k4], b.re, Ci[tc], 0, 0, 0);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const cd v = Pn[16 * w + lg + 4 * r][lj];
            Cr[t][r] = v.re;
            Ci[t][r] = v.im;
        }
        __syncthreads();
    }

    // ---- log det and the radius test (wave 0)
    if (w == 0) {
        double lre = 0.0, lim = 0.0;
        int inv = 0;
        if (l < NP) {
            const cd pv = pivv[l];
            lre = log(hypot(pv.re, pv.im));
            lim = atan2(pv.im, pv.re);
            const int pk = prow[l];
            for (int j = 0; j < l; ++j) inv += (prow[j] > pk) ? 1 : 0;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            lre += __shfl_xor(lre, off, 64);
            lim += __shfl_xor(lim, off, 64);
            inv += __shfl_xor(inv, off, 64);
        }
        if (l == 0) {
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

    // ---- Gamma_nn = sum_j R[sigma(n)][j] gamma[sigma(j)][n]
    if (stt == 0) {
        cd yp[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            yp[r] = {0.0, 0.0};
            const int i = 16 * w + lg + 4 * r;
            const int n = rowstep[i];
            if (n < n_nu) {
#pragma unroll
                for (int tc = 0; tc < NT; ++tc) {
                    const int lcol = prow[16 * tc + lj];
                    if (lcol < n_nu)
                        yp[r] = fma_c(yp[r], cd{Cr[tc][r], Ci[tc][r]},
                                      ld(gam, (size_t)lcol * n_nu + n));
                }
            }
        }
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                yp[r].re += __shfl_xor(yp[r].re, off, 64);
                yp[r].im += __shfl_xor(yp[r].im, off, 64);
            }
        }
        if (lj == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) yv[rowstep[16 * w + lg + 4 * r]] = yp[r];
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

template <int NP>
static hipError_t launch_mfma(const LadderArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_ladder_mfma_f64<NP>), dim3(a.n_items), dim3(NP * 4), 0, s, a);
    return hipGetLastError();
}

int ladder_mfma_padded_size(int n_nu) {
    if (n_nu <= 0) return 0;
    if (n_nu <= 16) return 16;
    if (n_nu <= 32) return 32;
    if (n_nu <= 48) return 48;
    if (n_nu <= 64) return 64;
    return 0;
}

hipError_t launch_ladder_mfma_f64(const LadderArgs &a, hipStream_t s) {
    switch (ladder_mfma_padded_size(a.n_nu)) {
        case 16: return launch_mfma<16>(a, s);
        case 32: return launch_mfma<32>(a, s);
        case 48: return launch_mfma<48>(a, s);
        case 64: return launch_mfma<64>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace df
