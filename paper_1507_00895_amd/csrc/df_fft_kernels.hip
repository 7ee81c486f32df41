// Bandwidth-bound steps of the ladder dual-fermion iteration:
//   eq. (gd0) + eq. (dyson)     k_dual_gf      (fused with the inverse FFT of G~)
//   eq. (dual_bubble)           k_bubble       (pair product + forward FFT in LDS)
//   eq. (sd)                    k_sigma_part   (inverse FFT of V, reflected product,
//                                               accumulation over a chunk of Om,
//                                               forward FFT)
//   reduction over Om chunks, linear mixing, Frobenius norms (deterministic order)
//   eq. (spin_symm)             k_gamma_prep   (gamma^{d,m} and gamma_ij gamma_ji)
//
// Every FFT works on one N-point array (N = nk^D <= 4096) resident in LDS;
// the flat index has one bit field per axis (see df_device.hpp).
#include "df_internal.hpp"

namespace df {

// ------------------------------------------------------------------------
// G~ = G~0 / (1 - G~0 Sigma~),  G~0 = 1 / (1/g + Delta - eps) - g.
// One block per fermionic frequency n.  Writes gd[n][k] (if gd_out) and
// the inverse FFT gr[n][r] = (1/N) sum_k e^{ikr} G~(k) (if gr_out).
// With from_gd set, G~ is read from gd instead of being computed.
// ------------------------------------------------------------------------
template <int NTH>
__global__ __launch_bounds__(NTH) void k_dual_gf(DualGfArgs a) {
    extern __shared__ cd lds[];
    cd *X = lds;
    cd *tw = lds + a.grid.N;
    const Grid g = a.grid;
    const int n = blockIdx.x;
    make_twiddles(tw, g);
    cd ginv = {0, 0}, gn = {0, 0}, dn = {0, 0};
    if (!a.from_gd) {
        gn = ld(a.g, n);
        dn = ld(a.delta, n);
        ginv = recip(gn);
    }
    for (int k = threadIdx.x; k < g.N; k += blockDim.x) {
        cd G;
        if (a.from_gd) {
            G = ld(a.gd_in, (size_t)n * g.N + k);
        } else {
            const cd den = {ginv.re + dn.re - a.eps[k], ginv.im + dn.im};
            const cd G0 = recip(den) - gn;
            if (a.sigma) {
                const cd S = ld(a.sigma, (size_t)n * g.N + k);
                const cd one_m = {1.0, 0.0};
                G = cdiv(G0, fms(one_m, G0, S));
            } else {
                G = G0;
            }
            if (a.gd_out) st(a.gd_out, (size_t)n * g.N + k, G);
        }
        X[bitrev_fields(k, g)] = G;
    }
    if (!a.gr_out) return;
    __syncthreads();
    fft_inplace<true>(X, tw, g);
    const double invN = 1.0 / (double)g.N;
    for (int r = threadIdx.x; r < g.N; r += blockDim.x)
        st(a.gr_out, (size_t)n * g.N + r, scale(X[r], invN));
}

// ------------------------------------------------------------------------
// chi_{m,n}(q) = -T FFT_r[ gr_n(-r) gr_{n+m}(r) ](q); zero when n+m leaves
// the window.  One block per (n, m).
// ------------------------------------------------------------------------
template <int NTH>
__global__ __launch_bounds__(NTH) void k_bubble(BubbleArgs a) {
    extern __shared__ cd lds[];
    cd *X = lds;
    cd *tw = lds + a.grid.N;
    const Grid g = a.grid;
    const int n = blockIdx.x, im = blockIdx.y;
    const int m = im - (a.n_om - 1) / 2;
    const int n2 = n + m;
    double *out = a.chi + 2 * ((size_t)im * a.n_nu + n) * g.N;
    if (n2 < 0 || n2 >= a.n_nu) {
        for (int q = threadIdx.x; q < g.N; q += blockDim.x) st(out, q, cd{0.0, 0.0});
        return;
    }
    make_twiddles(tw, g);
    const double *ga = a.gr + 2 * (size_t)n * g.N;
    const double *gb = a.gr + 2 * (size_t)n2 * g.N;
    for (int r = threadIdx.x; r < g.N; r += blockDim.x) {
        const cd x = ld(ga, reflect_fields(r, g)) * ld(gb, r);
        X[bitrev_fields(r, g)] = x;
    }
    __syncthreads();
    fft_inplace<false>(X, tw, g);
    const double mT = -1.0 / a.beta;
    for (int q = threadIdx.x; q < g.N; q += blockDim.x) st(out, q, scale(X[q], mT));
}

// ------------------------------------------------------------------------
// Partial dual self-energy over one chunk of bosonic frequencies:
//   part[chunk][n][k] = (T/2) FFT_r[ sum_{m in chunk} v_{m,n}(-r) gr_{n+m}(r) ](k),
//   v_{m,n} = IFFT_q[ 3 W^m_{m,n} + W^d_{m,n} ].
// One block per (n, chunk); the accumulator lives in registers.
// ------------------------------------------------------------------------
// (1024 threads: capped at 64 registers, so that two work-groups fit a CU)
template <int NTH>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(NTH == 1024 ? 8 : 1)))
void k_sigma_part(SigmaArgs a) {
    constexpr int SIGMA_MAX_PER_THREAD = 4096 / NTH;   // N <= 4096
    extern __shared__ cd lds[];
    cd *X = lds;
    cd *tw = lds + a.grid.N;
    const Grid g = a.grid;
    const int n = blockIdx.x, chunk = blockIdx.y;
    const int nth = blockDim.x;
    const int per = g.N / nth;                   // N is a power of two: N % nth == 0 or N < nth
    const int cnt = per > 0 ? per : (threadIdx.x < g.N ? 1 : 0);
    make_twiddles(tw, g);
    cd acc[SIGMA_MAX_PER_THREAD];
#pragma unroll
    for (int i = 0; i < SIGMA_MAX_PER_THREAD; ++i) acc[i] = {0.0, 0.0};
    const double invN = 1.0 / (double)g.N;
    const int h = (a.n_om - 1) / 2;
    const int m_lo = chunk * a.chunk_len;
    const int m_hi = min(a.n_om, m_lo + a.chunk_len);
    const size_t plane = (size_t)a.n_om * a.n_nu * g.N;   // one channel of W
    for (int im = m_lo; im < m_hi; ++im) {
        const int n2 = n + im - h;
        if (n2 < 0 || n2 >= a.n_nu) continue;
        const size_t off = ((size_t)im * a.n_nu + n) * g.N;
        __syncthreads();
        for (int q = threadIdx.x; q < g.N; q += nth) {
            const cd wd = ld(a.w, off + q);
            const cd wm = ld(a.w, plane + off + q);
            X[bitrev_fields(q, g)] = {3.0 * wm.re + wd.re, 3.0 * wm.im + wd.im};
        }
        __syncthreads();
        fft_inplace<true>(X, tw, g);
        const double *gb = a.gr + 2 * (size_t)n2 * g.N;
#pragma unroll
        for (int i = 0; i < SIGMA_MAX_PER_THREAD; ++i) {
            if (i < cnt) {
                const int r = threadIdx.x + i * nth;
                const cd v = scale(X[reflect_fields(r, g)], invN);
                acc[i] = fma_c(acc[i], v, ld(gb, r));
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SIGMA_MAX_PER_THREAD; ++i) {
        if (i < cnt) {
            const int r = threadIdx.x + i * nth;
            X[bitrev_fields(r, g)] = acc[i];
        }
    }
    __syncthreads();
    fft_inplace<false>(X, tw, g);
    const double hT = 0.5 / a.beta;
    double *out = a.part + 2 * ((size_t)chunk * a.n_nu + n) * g.N;
    for (int k = threadIdx.x; k < g.N; k += nth) st(out, k, scale(X[k], hT));
}

// ------------------------------------------------------------------------
// sigma_calc = sum over chunks of part (fixed order); optionally
// sigma <- (1 - alpha) sigma + alpha sigma_calc with per-block partial sums of
// |sigma_new - sigma_old|^2 and |sigma_new|^2.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce_mix(ReduceMixArgs a) {
    __shared__ double red[2][256];
    double dn = 0.0, nn = 0.0;
    const size_t M = a.count;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < M;
         e += (size_t)gridDim.x * blockDim.x) {
        cd s = ld(a.part, e);
        for (int c = 1; c < a.n_chunks; ++c) s = s + ld(a.part, (size_t)c * M + e);
        if (a.sigma_calc) st(a.sigma_calc, e, s);
        if (a.sigma) {
            const cd old = ld(a.sigma, e);
            const cd nw = {(1.0 - a.alpha) * old.re + a.alpha * s.re,
                           (1.0 - a.alpha) * old.im + a.alpha * s.im};
            st(a.sigma, e, nw);
            const double dr = nw.re - old.re, di = nw.im - old.im;
            dn += dr * dr + di * di;
            nn += nw.re * nw.re + nw.im * nw.im;
        }
    }
    if (!a.sigma) return;
    red[0][threadIdx.x] = dn;
    red[1][threadIdx.x] = nn;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.norm_part[2 * blockIdx.x] = red[0][0];
        a.norm_part[2 * blockIdx.x + 1] = red[1][0];
    }
}

// diff = sqrt(sum dn / sum nn), summed over n_part block partials in order;
// writes diff to out[0]; out[1] = 1 if a partial is not finite.
__global__ __launch_bounds__(256) void k_norm_final(const double *part, int n_part, double *out) {
    __shared__ double red[2][256];
    double dn = 0.0, nn = 0.0;
    for (int i = threadIdx.x; i < n_part; i += blockDim.x) {
        dn += part[2 * i];
        nn += part[2 * i + 1];
    }
    red[0][threadIdx.x] = dn;
    red[1][threadIdx.x] = nn;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double d = red[0][0], m = red[1][0];
        double diff;
        if (m == 0.0) diff = (d == 0.0) ? 0.0 : INFINITY;
        else diff = sqrt(d / m);
        out[0] = diff;
        out[1] = (isfinite(d) && isfinite(m)) ? 0.0 : 1.0;
    }
}

// ------------------------------------------------------------------------
// gamma^{d/m} = gamma^uu +- gamma^ud  and  P^c[i][j] = gamma^c_ij gamma^c_ji.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gamma_prep(GammaPrepArgs a) {
    const size_t nn = (size_t)a.n_nu * a.n_nu;
    const size_t tot = (size_t)a.n_om * nn;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t mb = e / nn;
        const int i = (int)((e % nn) / a.n_nu), j = (int)(e % a.n_nu);
        const size_t et = mb * nn + (size_t)j * a.n_nu + i;
        const cd uu = ld(a.guu, e), ud = ld(a.gud, e);
        const cd uut = ld(a.guu, et), udt = ld(a.gud, et);
        const cd gd = uu + ud, gm = uu - ud;
        const cd gdt = uut + udt, gmt = uut - udt;
        st(a.gdm, e, gd);
        st(a.gdm, tot + e, gm);
        st(a.pdm, e, gd * gdt);
        st(a.pdm, tot + e, gm * gmt);
        if (a.gtr) {
            st(a.gtr, e, gdt);
            st(a.gtr, tot + e, gmt);
        }
        if (a.gp32) {
            const cd pd = gd * gdt, pmm = gm * gmt;
            st4f(a.gp32, e, (float)gd.re, (float)gd.im, (float)pd.re, (float)pd.im);
            st4f(a.gp32, tot + e, (float)gm.re, (float)gm.im, (float)pmm.re, (float)pmm.im);
        }
        if (a.gtr32) {
            st2f(a.gtr32, e, (float)gdt.re, (float)gdt.im);
            st2f(a.gtr32, tot + e, (float)gmt.re, (float)gmt.im);
        }
    }
}

__global__ void k_zero_ints(int *p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
static size_t fft_lds_bytes(const Grid &g) { return (size_t)(g.N + g.nk) * sizeof(cd); }

// Threads per FFT work-group.  The FFT kernels keep N + nk complex doubles in
// LDS, 66.5 KiB at N = 4096, so two work-groups fit a CU: 1024 threads each
// then give 32 waves per CU (256 threads gave 8, and the LDS passes waited
// on their latency).  Smaller grids keep 256 threads and more work-groups.
static int fft_threads(const Grid &g) { return g.N >= 4096 ? 1024 : 256; }

// The FFT kernels keep N + nk complex doubles in LDS: up to 66.5 KiB at
// N = 4096, above the default 64 KiB limit of a launch.
hipError_t set_fft_lds_limits() {
    const int bytes = (4096 + 64) * (int)sizeof(cd);
    const void *kernels[] = {(const void *)k_dual_gf<256>, (const void *)k_dual_gf<1024>,
                             (const void *)k_bubble<256>, (const void *)k_bubble<1024>,
                             (const void *)k_sigma_part<256>, (const void *)k_sigma_part<1024>};
    hipError_t e = hipSuccess;
    for (const void *k : kernels)
        if (e == hipSuccess) e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return e;
}

hipError_t launch_dual_gf(const DualGfArgs &a, hipStream_t s) {
    if (fft_threads(a.grid) == 1024)
        hipLaunchKernelGGL(k_dual_gf<1024>, dim3(a.n_nu), dim3(1024), fft_lds_bytes(a.grid), s, a);
    else
        hipLaunchKernelGGL(k_dual_gf<256>, dim3(a.n_nu), dim3(256), fft_lds_bytes(a.grid), s, a);
    return hipGetLastError();
}

hipError_t launch_bubble(const BubbleArgs &a, hipStream_t s) {
    if (fft_threads(a.grid) == 1024)
        hipLaunchKernelGGL(k_bubble<1024>, dim3(a.n_nu, a.n_om), dim3(1024), fft_lds_bytes(a.grid), s, a);
    else
        hipLaunchKernelGGL(k_bubble<256>, dim3(a.n_nu, a.n_om), dim3(256), fft_lds_bytes(a.grid), s, a);
    return hipGetLastError();
}

hipError_t launch_sigma_part(const SigmaArgs &a, hipStream_t s) {
    if (fft_threads(a.grid) == 1024)
        hipLaunchKernelGGL(k_sigma_part<1024>, dim3(a.n_nu, a.n_chunks), dim3(1024),
                           fft_lds_bytes(a.grid), s, a);
    else
        hipLaunchKernelGGL(k_sigma_part<256>, dim3(a.n_nu, a.n_chunks), dim3(256),
                           fft_lds_bytes(a.grid), s, a);
    return hipGetLastError();
}

hipError_t launch_reduce_mix(const ReduceMixArgs &a, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_mix, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_norm_final(const double *part, int n_part, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(256), 0, s, part, n_part, out);
    return hipGetLastError();
}

hipError_t launch_zero_ints(int *p, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_gamma_prep(const GammaPrepArgs &a, hipStream_t s) {
    const size_t tot = (size_t)a.n_om * a.n_nu * a.n_nu;
    int blocks = (int)((tot + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_gamma_prep, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace df
