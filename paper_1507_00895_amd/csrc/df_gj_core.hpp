// Certified pivot-free blocked Gauss-Jordan inversion of one NP x NP complex
// matrix per work-group on the matrix cores, for FP64 and FP32 tiles.
//
// Layout: W = NP/16 waves; wave w holds block-row w as NT = NP/16 complex
// 16 x 16 accumulator tiles (a real and an imaginary tile, 4 values per lane).
// 16x16x4 MFMA lane layouts on gfx950 (measured):
//   A[i][k] : lane i + 16 k          B[k][j] : lane j + 16 k
//   C[i][j] : lane j + 16 (i % 4), register i / 4   (FP64)
//             lane j + 16 (i / 4), register i % 4   (FP32)
//
// Certificate.  For D = 1 - M, a spectral radius of |M| below one makes D an
// H-matrix: its leading blocks are nonsingular and elimination without
// pivoting is stable.  gj_certify bounds rho(|M|) from above by the
// Collatz-Wielandt quotient max_i (B v)_i / v_i after power steps on
// B = cabs1(M) + eps I (cabs1 = |re| + |im| >= |.|).  The bound also limits the
// condition number of D after diagonal scaling: ||D'^-1|| <= 1 / (1 - rho).
//
// Sweep.  For each tile column t: wave t inverts the diagonal tile A_tt by 16
// scalar Gauss-Jordan steps held in registers (pivot by readlane, pivot-column
// values within a quad by DPP, pivot-row values by bpermute) and publishes it
// with its old block-row; every other wave forms G_w = -A_wt A_tt^-1; every
// wave applies A_w,c += G_w A_t,c (c != t) with G_t = A_tt^-1 - 1 and sets
// tile (w, t) to G_w (A_tt^-1 for w = t).  This is the block form of the
// in-place sweep: afterwards the tiles hold D^-1, and the scalar pivots
// (stored in FP64) multiply to det D.
#pragma once

#include "df_internal.hpp"

extern "C" __device__ __attribute__((const)) unsigned int __ockl_wfred_max_u32(unsigned int);

namespace df {

template <typename T> struct MT;
template <> struct MT<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lg, int r) { return lg + 4 * r; }
};
template <> struct MT<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lg, int r) { return 4 * lg + r; }
};

// ---------------------------------------------------------------- lane ops
__device__ __forceinline__ double readlane_v(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float readlane_v(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

template <int K> __device__ __forceinline__ int quad_bcast_i(int v) {
    return __builtin_amdgcn_mov_dpp(v, K | (K << 2) | (K << 4) | (K << 6), 0xf, 0xf, false);
}
__device__ __forceinline__ int quad_bcast_rt(int v, int k) {
    switch (k) {
        case 0: return quad_bcast_i<0>(v);
        case 1: return quad_bcast_i<1>(v);
        case 2: return quad_bcast_i<2>(v);
        default: return quad_bcast_i<3>(v);
    }
}
// value of quad lane k (k resolves statically once the caller's loop unrolls)
__device__ __forceinline__ double quad_bcast_v(double v, int k) {
    const long long b = __double_as_longlong(v);
    const int lo = quad_bcast_rt((int)(b & 0xffffffffLL), k);
    const int hi = quad_bcast_rt((int)(b >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float quad_bcast_v(float v, int k) {
    return __int_as_float(quad_bcast_rt(__float_as_int(v), k));
}

// value held by the lane at byte address addr (= 4 * lane)
__device__ __forceinline__ double bperm_v(int addr, double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float bperm_v(int addr, float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}

// 1 / z through the hardware reciprocal of |z|^2 refined by Newton steps
// (each step squares the relative error of the estimate)
__device__ __forceinline__ cd recip_fast(cd z) {
    const double m = fma(z.re, z.re, z.im * z.im);
    double y = __builtin_amdgcn_rcp(m);
    double e = fma(-m, y, 1.0);
    y = fma(y, e, y);
    e = fma(-m, y, 1.0);
    y = fma(y, e, y);
    return {z.re * y, -z.im * y};
}
__device__ __forceinline__ cf recip_fast(cf z) {
    const float m = fmaf(z.re, z.re, z.im * z.im);
    float y = __builtin_amdgcn_rcpf(m);
    const float e = fmaf(-m, y, 1.0f);
    y = fmaf(y, e, y);
    return {z.re * y, -z.im * y};
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// wave maximum of a non-negative double (its bit pattern orders like its value)
__device__ __forceinline__ double wave_max_pos(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned hi = __ockl_wfred_max_u32((unsigned)(b >> 32));
    const unsigned lo = __ockl_wfred_max_u32((b >> 32) == hi ? (unsigned)b : 0u);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// ---------------------------------------------------------------- shared state
template <typename T, int NP> struct GjShared {
    static constexpr int NT = NP / 16;
    cplx<T> Tt[16][17];          // diagonal tile, then its inverse
    cplx<T> Rb[16][NP];          // old block-row of the current tile column
    cplx<T> Xw[NT][16][17];      // per-wave layout exchange (accumulator -> operand)
    cd pivv[NP];                 // scalar pivots, FP64
    double vbuf[2][NP];          // power-iteration vectors
    double wmax[NT];
};

// Collatz-Wielandt bound of rho(cabs1(M) + eps I) for M = 1 - D; uniform
// result across the work-group.  Contains barriers: every thread must call.
template <typename T, int NP>
__device__ __forceinline__ double gj_certify(const typename MT<T>::v4 (&Cr)[NP / 16],
                                             const typename MT<T>::v4 (&Ci)[NP / 16],
                                             GjShared<T, NP> &sh, int iters) {
    constexpr int NT = NP / 16;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, lj = l & 15, lg = l >> 4;
    for (int i = tid; i < NP; i += NP * 4) sh.vbuf[0][i] = 1.0;
    __syncthreads();
    for (int it = 0; it < iters; ++it) {
        const double *v = sh.vbuf[it & 1];
        double u[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int tc = 0; tc < NT; ++tc) {
            const int j = 16 * tc + lj;
            const double vj = v[j];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * w + MT<T>::row(lg, r);
                const double mr = ((i == j) ? 1.0 : 0.0) - (double)Cr[tc][r];
                const double b = fabs(mr) + fabs((double)Ci[tc][r]) + ((i == j) ? 1e-12 : 0.0);
                u[r] = fma(b, vj, u[r]);
            }
        }
        // rows live in the 16 lanes of one row group (FP64) or one quarter (FP32)
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r) u[r] += __shfl_xor(u[r], off, 64);
        }
        if (it == iters - 1) {
            double ratio = 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double rr = u[r] / v[16 * w + MT<T>::row(lg, r)];
                ratio = rr > ratio ? rr : ratio;
            }
            const double m = wave_max_pos(ratio);
            if (l == 0) sh.wmax[w] = m;
        } else if (lj == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) sh.vbuf[(it + 1) & 1][16 * w + MT<T>::row(lg, r)] = u[r];
        }
        __syncthreads();
    }
    double cw = 0.0;
    for (int x = 0; x < NT; ++x) cw = sh.wmax[x] > cw ? sh.wmax[x] : cw;
    return cw;
}

// In-place blocked Gauss-Jordan sweep without pivoting.  Contains barriers.
template <typename T, int NP>
__device__ __forceinline__ void gj_sweep(typename MT<T>::v4 (&Cr)[NP / 16],
                                         typename MT<T>::v4 (&Ci)[NP / 16], GjShared<T, NP> &sh) {
    constexpr int NT = NP / 16;
    typedef cplx<T> ct;
    typedef typename MT<T>::v4 v4;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, lj = l & 15, lg = l >> 4;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (w == t) {
#pragma unroll
            for (int tc = 0; tc < NT; ++tc) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const ct v = {Cr[tc][r], Ci[tc][r]};
                    const int i = MT<T>::row(lg, r);
                    if (tc == t) sh.Tt[i][lj] = v;
                    else sh.Rb[i][16 * tc + lj] = v;
                }
            }
            wave_sync_lds();
            // 16 scalar steps: lane holds row l/4, columns 4 (l % 4) + e
            const int gi = l >> 2;
            const int gq = (l & 3) * 4;
            ct x[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) x[e] = sh.Tt[gi][gq + e];
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const int src = 4 * s + (s >> 2);
                const ct piv = {readlane_v(x[s & 3].re, src), readlane_v(x[s & 3].im, src)};
                const ct ip = recip_fast(piv);
                const ct cvl = {quad_bcast_v(x[s & 3].re, s >> 2), quad_bcast_v(x[s & 3].im, s >> 2)};
                const int from = (4 * s + (l & 3)) << 2;
                ct rr[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) rr[e] = {bperm_v(from, x[e].re), bperm_v(from, x[e].im)};
                const bool me = (gi == s);
                const ct f = me ? ct{T(1) - ip.re, -ip.im} : cvl * ip;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    x[e] = fms(x[e], f, rr[e]);
                    if (gq + e == s) x[e] = me ? ip : ct{-f.re, -f.im};
                }
                if (l == 0) sh.pivv[16 * t + s] = cd{(double)piv.re, (double)piv.im};
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) sh.Tt[gi][gq + e] = x[e];
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) sh.Xw[w][MT<T>::row(lg, r)][lj] = ct{Cr[t][r], Ci[t][r]};
        }
        __syncthreads();

        T gr[4], gim[4], gn[4];
        if (w == t) {
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                ct g = sh.Tt[lj][4 * k4 + lg];
                if (lj == 4 * k4 + lg) g.re -= T(1);
                gr[k4] = g.re;
                gim[k4] = g.im;
                gn[k4] = -g.im;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const ct v = sh.Tt[MT<T>::row(lg, r)][lj];
                Cr[t][r] = v.re;
                Ci[t][r] = v.im;
            }
        } else {
            v4 Gr = {0, 0, 0, 0}, Gi = {0, 0, 0, 0};
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                const ct xa = sh.Xw[w][lj][4 * k4 + lg];
                const ct b = sh.Tt[4 * k4 + lg][lj];
                const T nxr = -xa.re, nxi = -xa.im;
                Gr = MT<T>::mma(nxr, b.re, Gr);
                Gr = MT<T>::mma(xa.im, b.im, Gr);
                Gi = MT<T>::mma(nxr, b.im, Gi);
                Gi = MT<T>::mma(nxi, b.re, Gi);
            }
            Cr[t] = Gr;
            Ci[t] = Gi;
            wave_sync_lds();
#pragma unroll
            for (int r = 0; r < 4; ++r) sh.Xw[w][MT<T>::row(lg, r)][lj] = ct{Gr[r], Gi[r]};
            wave_sync_lds();
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                const ct g = sh.Xw[w][lj][4 * k4 + lg];
                gr[k4] = g.re;
                gim[k4] = g.im;
                gn[k4] = -g.im;
            }
        }
#pragma unroll
        for (int tc = 0; tc < NT; ++tc) {
            if (tc == t) continue;
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                const ct b = sh.Rb[4 * k4 + lg][16 * tc + lj];
                Cr[tc] = MT<T>::mma(gr[k4], b.re, Cr[tc]);
                Cr[tc] = MT<T>::mma(gn[k4], b.im, Cr[tc]);
                Ci[tc] = MT<T>::mma(gr[k4], b.im, Ci[tc]);
                Ci[tc] = MT<T>::mma(gim[k4], b.re, Ci[tc]);
            }
        }
        __syncthreads();
    }
}

// log det from the scalar pivots (no row exchanges), by wave 0; returns the
// status code (0 inside, 1 outside, 2 non-finite) to lane 0 of wave 0.
template <int NP>
__device__ __forceinline__ int gj_logdet(const cd *pivv, cd *out_logdet) {
    const int l = threadIdx.x & 63;
    double lre = 0.0, lim = 0.0;
    for (int k = l; k < NP; k += 64) {
        const cd pv = pivv[k];
        lre += log(hypot(pv.re, pv.im));
        lim += atan2(pv.im, pv.re);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        lre += __shfl_xor(lre, off, 64);
        lim += __shfl_xor(lim, off, 64);
    }
    double ph = remainder(lim, 2.0 * M_PI);
    if (ph <= -M_PI) ph += 2.0 * M_PI;
    *out_logdet = cd{lre, ph};
    if (!isfinite(lre) || !isfinite(ph)) return 2;
    return (cos(ph) > 0.0) ? 0 : 1;
}

}  // namespace df
