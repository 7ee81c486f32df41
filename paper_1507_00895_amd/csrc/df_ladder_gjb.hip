// Batched Bethe-Salpeter ladder: certified pivot-free blocked Gauss-Jordan
// inversion on the FP64 matrix cores.  Same quantities as k_ladder_fp64
// (eqs. dual_ladder, lin_alg_inv, the radius rule, Gamma^(2) of eq. sd).
//
// Certificate.  D = 1 - M with M = gamma diag(chi).  If the spectral radius of
// |M| (entrywise modulus) is below one, D is an H-matrix: every leading
// principal block is nonsingular and elimination without pivoting is stable
// (its Schur complements stay H-matrices).  The kernel bounds rho(|M|) from
// above by the Collatz-Wielandt quotient max_i (B v)_i / v_i after a few power
// steps v <- B v on B = cabs1(M) + eps I >= |M| (cabs1 = |re| + |im|); a bound
// below CERT_MAX certifies the item.  Uncertified items (near or outside the
// convergence radius) are appended to a queue that the partial-pivoting
// kernel processes afterwards, so every item gets a stable elimination.
// rho(|M|) < 1 also implies rho(M) < 1: certified items are inside the radius.
//
// Schedule (one work-group of W = NP/16 waves per (channel, Om_m, q); wave w
// holds block-row w of D in MFMA accumulator tiles).  For each tile column t:
//   wave t inverts the diagonal tile A_tt (16 x 16, Gauss-Jordan in LDS) and
//   publishes it with its old block-row; every other wave w forms
//   G_w = -A_wt A_tt^-1 on the matrix cores; then every wave applies
//   A_w,c += G_w A_t,c (c != t) with G_t = A_tt^-1 - 1, and tile (w, t) <- G_w
//   (A_tt^-1 for w = t).  This is the block form of the in-place sweep; after
//   the last tile column the tiles hold D^-1 and the product of the scalar
//   pivots is det D.
//
// FP64 16x16x4 MFMA lane layout (gfx950): A[i][k] at lane i + 16k,
// B[k][j] at lane j + 16k, C[i][j] at lane j + 16 (i % 4), register i / 4.
#include "df_internal.hpp"

extern "C" __device__ __attribute__((const)) unsigned int __ockl_wfred_max_u32(unsigned int);

namespace df {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int CERT_ITERS = 6;
constexpr double CERT_MAX = 0.999;
constexpr double CERT_EPS = 1e-12;

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// value of lane K of this lane's quad (DPP quad permutation)
template <int K>
__device__ __forceinline__ double quad_bcast_d(double v) {
    constexpr int ctrl = K | (K << 2) | (K << 4) | (K << 6);
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), ctrl, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctrl, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// quad broadcast with the quad lane given at run time (resolved statically
// once the caller's loop is unrolled)
__device__ __forceinline__ double quad_bcast_rt(double v, int k) {
    switch (k) {
        case 0: return quad_bcast_d<0>(v);
        case 1: return quad_bcast_d<1>(v);
        case 2: return quad_bcast_d<2>(v);
        default: return quad_bcast_d<3>(v);
    }
}

// value held by the lane whose byte address is addr (= 4 * lane)
__device__ __forceinline__ double bperm_d(int addr, double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// 1 / z: reciprocal of |z|^2 by v_rcp_f64 and two Newton steps (the error of
// the hardware estimate squares at each step, well below double rounding)
__device__ __forceinline__ cd recip_fast(cd z) {
    const double m = fma(z.re, z.re, z.im * z.im);
    double y = __builtin_amdgcn_rcp(m);
    double e = fma(-m, y, 1.0);
    y = fma(y, e, y);
    e = fma(-m, y, 1.0);
    y = fma(y, e, y);
    return {z.re * y, -z.im * y};
}

__device__ __forceinline__ double wave_max_pos(double x) {
    // x >= 0: the bit pattern of a non-negative double orders like its value
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned hi = __ockl_wfred_max_u32((unsigned)(b >> 32));
    const unsigned lo = __ockl_wfred_max_u32((b >> 32) == hi ? (unsigned)b : 0u);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int NP>
__global__ __launch_bounds__(NP * 4) void k_ladder_gjb_f64(LadderArgs a) {
    constexpr int NT = NP / 16;
    static_assert(NP % 16 == 0 && NP >= 16 && NP <= 128, "tiles of 16");

    __shared__ cd Tt[16][17];            // diagonal tile / its inverse (padded rows)
    __shared__ cd Rb[16][NP];            // old block-row t
    __shared__ cd Xw[NT][16][17];        // per-wave layout exchange
    __shared__ cd xrow[2][16], xcol[2][16];
    __shared__ cd pivv[NP];
    __shared__ double vbuf[2][NP];
    __shared__ double wmax[NT];
    __shared__ cd yv[NP];
    __shared__ cd tv[NP];
    __shared__ int s_flag;

    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int l = tid & 63;
    const int lj = l & 15;
    const int lg = l >> 4;
    const int n_nu = a.n_nu, N = a.N;

    const int item = a.item0 + blockIdx.x;
    const int q = item % N;
    const int cm = item / N;
    const int im = cm % a.n_om;
    const size_t nn = (size_t)n_nu * n_nu;
    const double *gam = a.gdm + 2 * (size_t)cm * nn;
    const double *pm = a.pdm + 2 * (size_t)cm * nn;
    const double *gtr = a.gtr + 2 * (size_t)cm * nn;

    // ---- D = 1 - gamma diag(chi) in accumulator tiles, t_i = (gamma chi gamma)_ii
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

    // ---- certificate: Collatz-Wielandt bound of B = cabs1(M) + eps I
    for (int i = tid; i < NP; i += NP * 4) vbuf[0][i] = 1.0;
    __syncthreads();
    double cw = 0.0;
    for (int it = 0; it < CERT_ITERS; ++it) {
        const double *v = vbuf[it & 1];
        double u[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int tc = 0; tc < NT; ++tc) {
            const int j = 16 * tc + lj;
            const double vj = v[j];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * w + lg + 4 * r;
                const double mr = ((i == j) ? 1.0 : 0.0) - Cr[tc][r];
                const double b = fabs(mr) + fabs(Ci[tc][r]) + ((i == j) ? CERT_EPS : 0.0);
                u[r] = fma(b, vj, u[r]);
            }
        }
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r) u[r] += __shfl_xor(u[r], off, 64);
        }
        if (it == CERT_ITERS - 1) {
            double ratio = 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * w + lg + 4 * r;
                const double rr = u[r] / v[i];
                ratio = rr > ratio ? rr : ratio;
            }
            const double m = wave_max_pos(ratio);
            if (l == 0) wmax[w] = m;
        } else if (lj == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) vbuf[(it + 1) & 1][16 * w + lg + 4 * r] = u[r];
        }
        __syncthreads();
    }
    for (int x = 0; x < NT; ++x) cw = wmax[x] > cw ? wmax[x] : cw;
    if (!(cw < CERT_MAX)) {
        if (tid == 0 && a.queue) a.queue[atomicAdd(a.queue_count, 1)] = item;
        return;   // uniform: every thread of the work-group leaves here
    }

    // ---- blocked Gauss-Jordan, tile column by tile column
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (w == t) {
            // publish the old block-row and the diagonal tile
#pragma unroll
            for (int tc = 0; tc < NT; ++tc) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const cd v = {Cr[tc][r], Ci[tc][r]};
                    if (tc == t) Tt[lg + 4 * r][lj] = v;
                    else Rb[lg + 4 * r][16 * tc + lj] = v;
                }
            }
            wave_sync_lds();
            // Gauss-Jordan on the 16 x 16 tile: lane holds row l/4, columns 4 (l%4) + e.
            // The pivot comes by readlane, the pivot-column value of a row from its
            // quad by DPP, the pivot-row values by bpermute: no LDS round trip.
            const int gi = l >> 2;
            const int gq = (l & 3) * 4;
            cd x[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) x[e] = Tt[gi][gq + e];
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const int src = 4 * s + (s >> 2);
                const cd piv = {readlane_d(x[s & 3].re, src), readlane_d(x[s & 3].im, src)};
                const cd ip = recip_fast(piv);
                const cd cvl = {quad_bcast_rt(x[s & 3].re, s >> 2), quad_bcast_rt(x[s & 3].im, s >> 2)};
                const int from = (4 * s + (l & 3)) << 2;
                cd r[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) r[e] = {bperm_d(from, x[e].re), bperm_d(from, x[e].im)};
                const bool me = (gi == s);
                const cd f = me ? cd{1.0 - ip.re, -ip.im} : cvl * ip;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    x[e] = fms(x[e], f, r[e]);
                    if (gq + e == s) x[e] = me ? ip : cd{-f.re, -f.im};
                }
                if (l == 0) pivv[16 * t + s] = piv;
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) Tt[gi][gq + e] = x[e];
        } else {
            // move tile (w, t) from accumulator layout to operand layout
#pragma unroll
            for (int r = 0; r < 4; ++r) Xw[w][lg + 4 * r][lj] = cd{Cr[t][r], Ci[t][r]};
        }
        __syncthreads();

        double gr[4], gi_[4], gn[4];
        if (w == t) {
            // G_t = A_tt^-1 - 1 (operand layout); tile (t, t) <- A_tt^-1
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                cd g = Tt[lj][4 * k4 + lg];
                if (lj == 4 * k4 + lg) g.re -= 1.0;
                gr[k4] = g.re;
                gi_[k4] = g.im;
                gn[k4] = -g.im;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const cd v = Tt[lg + 4 * r][lj];
                Cr[t][r] = v.re;
                Ci[t][r] = v.im;
            }
        } else {
            // G_w = -A_wt A_tt^-1 on the matrix cores
            d4 Gr = {0.0, 0.0, 0.0, 0.0}, Gi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                const cd xa = Xw[w][lj][4 * k4 + lg];
                const cd b = Tt[4 * k4 + lg][lj];
                const double nxr = -xa.re, nxi = -xa.im;
                Gr = __builtin_amdgcn_mfma_f64_16x16x4f64(nxr, b.re, Gr, 0, 0, 0);
                Gr = __builtin_amdgcn_mfma_f64_16x16x4f64(xa.im, b.im, Gr, 0, 0, 0);
                Gi = __builtin_amdgcn_mfma_f64_16x16x4f64(nxr, b.im, Gi, 0, 0, 0);
                Gi = __builtin_amdgcn_mfma_f64_16x16x4f64(nxi, b.re, Gi, 0, 0, 0);
            }
            Cr[t] = Gr;
            Ci[t] = Gi;
            // G_w to operand layout through the wave's own LDS slot
            wave_sync_lds();
#pragma unroll
            for (int r = 0; r < 4; ++r) Xw[w][lg + 4 * r][lj] = cd{Gr[r], Gi[r]};
            wave_sync_lds();
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                const cd g = Xw[w][lj][4 * k4 + lg];
                gr[k4] = g.re;
                gi_[k4] = g.im;
                gn[k4] = -g.im;
            }
        }
        // A_w,c += G_w A_t,c for every other tile column
#pragma unroll
        for (int tc = 0; tc < NT; ++tc) {
            if (tc == t) continue;
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                const cd b = Rb[4 * k4 + lg][16 * tc + lj];
                Cr[tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(gr[k4], b.re, Cr[tc], 0, 0, 0);
                Cr[tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(gn[k4], b.im, Cr[tc], 0, 0, 0);
                Ci[tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(gr[k4], b.im, Ci[tc], 0, 0, 0);
                Ci[tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(gi_[k4], b.re, Ci[tc], 0, 0, 0);
            }
        }
        __syncthreads();
    }

    // ---- log det (no row exchanges) and the radius test
    if (w == 0) {
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
        if (l == 0) {
            double ph = remainder(lim, 2.0 * M_PI);
            if (ph <= -M_PI) ph += 2.0 * M_PI;
            int stt;
            if (!isfinite(lre) || !isfinite(ph)) stt = 2;
            else stt = (cos(ph) > 0.0) ? 0 : 1;
            s_flag = stt;
            const size_t o = (size_t)cm * N + q;
            if (a.logdet) st(a.logdet, o, cd{lre, ph});
            if (a.status) a.status[o] = (int8_t)stt;
            if (stt != 0 && a.fallback_count) atomicAdd(a.fallback_count, 1);
        }
    }
    __syncthreads();
    const int stt = s_flag;

    // ---- Gamma_nn = sum_l (D^-1)_nl gamma_ln  (gamma^T read row-wise)
    if (stt == 0) {
        cd yp[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            yp[r] = {0.0, 0.0};
            const int i = 16 * w + lg + 4 * r;
            if (i < n_nu) {
#pragma unroll
                for (int tc = 0; tc < NT; ++tc) {
                    const int j = 16 * tc + lj;
                    if (j < n_nu)
                        yp[r] = fma_c(yp[r], cd{Cr[tc][r], Ci[tc][r]},
                                      ld(gtr, (size_t)i * n_nu + j));
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
            for (int r = 0; r < 4; ++r) yv[16 * w + lg + 4 * r] = yp[r];
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
static hipError_t launch_gjb(const LadderArgs &a, hipStream_t s) {
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
    return 0;   // n_nu = 128 exceeds the register budget of one block-row per wave
}

hipError_t launch_ladder_gjb_f64(const LadderArgs &a, hipStream_t s) {
    switch (ladder_gjb_padded_size(a.n_nu)) {
        case 16: return launch_gjb<16>(a, s);
        case 32: return launch_gjb<32>(a, s);
        case 48: return launch_gjb<48>(a, s);
        case 64: return launch_gjb<64>(a, s);
        case 96: return launch_gjb<96>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace df
