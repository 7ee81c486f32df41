// Lattice observables of a dual solution (Sec. 2.3, "Resulting observables").
//
//   k_lattice_fields      per (nu, k): G~0, G~ (eqs. gd0, dyson), Sigma_lat (eq. sigma_lat,
//                         denominator 1 + g Sigma~), G_lat (eq. glat, in a form free of
//                         cancellation), frak G = G~ (G~0 + g) / G~0
//   (k_dual_gf / k_bubble of df_fft_kernels.hip turn frak G, G_lat and G~ into
//    L_nu(q), the per-nu lattice bubble and chi~ at Omega = 0)
//   k_lattice_chi_ladder  per (channel, q): sum_{nu nu'} L_nu Gamma_{nu nu'} L_nu' with
//                         Gamma = [1 - gamma chi~]^-1 gamma at Omega = 0, by Gaussian
//                         elimination with partial pivoting of [D | gamma L] (FP64)
//   k_lattice_chi_sum     chi^{ch/sp}(q) = sum_nu bubble_nu(q) + ladder term
//
// These run once per converged solution, outside the iteration: plain FP64
// kernels sized for clarity, not for the roofline.
#include "df_internal.hpp"

namespace df {

// ------------------------------------------------------------------------
// One block per fermionic frequency n (nu_n = (2n + 1 - n_nu) pi / beta).
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_lattice_fields(LatticeFieldArgs a) {
    const int n = blockIdx.x;
    const cd gn = ld(a.g, n), dn = ld(a.delta, n);
    const cd ginv = recip(gn);
    const double nu = (double)(2 * n + 1 - a.n_nu) * M_PI / a.beta;
    // Sigma^DMFT = i nu + mu - Delta - 1/g
    const cd sdmft = {a.mu - dn.re - ginv.re, nu - dn.im - ginv.im};
    const cd one = {1.0, 0.0};
    for (int k = threadIdx.x; k < a.N; k += blockDim.x) {
        const size_t e = (size_t)n * a.N + k;
        const cd dme = {dn.re - a.eps[k], dn.im};        // Delta - eps
        const cd G0 = recip(ginv + dme) - gn;
        const cd S = a.sigma ? ld(a.sigma, e) : cd{0.0, 0.0};
        const cd G = cdiv(G0, fms(one, G0, S));
        // eq. (glat) with G~ from eqs. (gd0), (dyson) is g (1 + g S) / (1 + g (Delta - eps)(1 + g S)):
        // the same value without the cancellation of its two terms where Delta - eps is small
        const cd h = fma_c(one, gn, S);                   // 1 + g S
        const cd Gl = cdiv(gn * h, fma_c(one, gn * dme, h));
        if (a.sigma_lat) st(a.sigma_lat, e, cdiv(S, fma_c(one, gn, S)) + sdmft);
        if (a.g_lat) st(a.g_lat, e, Gl);
        st(a.gl, e, Gl);
        st(a.gd, e, G);
        st(a.fg, e, cdiv(G * (G0 + gn), G0));
    }
}

// ------------------------------------------------------------------------
// One block (256 threads) per item (channel c, q) of the chunk.  The
// augmented matrix [D | y], D = 1 - gamma diag(chi~(q)), y = gamma L(q), lives in
// this item's slice of the work buffer (row-major, n x (n + 1) complex); the
// waves of the block share it through the CU's cache, ordered by barriers.
// ------------------------------------------------------------------------
__device__ __forceinline__ void argmax_pair(double &v, int &i) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int oi = __shfl_xor(i, off, 64);
        if (ov > v || (ov == v && oi < i)) {
            v = ov;
            i = oi;
        }
    }
}

__device__ __forceinline__ cd wave_sum_c(cd x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        x.re += __shfl_xor(x.re, off, 64);
        x.im += __shfl_xor(x.im, off, 64);
    }
    return x;
}

__global__ __launch_bounds__(256) void k_lattice_chi_ladder(LatticeChiArgs a) {
    const int n = a.n_nu, N = a.N, ldm = n + 1;
    const int item = a.item0 + blockIdx.x;
    const int c = item / N, q = item % N;
    const int tid = threadIdx.x, lane = tid & 63;
    double *M = a.work + 2 * (size_t)blockIdx.x * n * ldm;
    __shared__ cd Lv[128], xv[128], zv[128];
    __shared__ int s_piv;
    for (int i = tid; i < n; i += blockDim.x) {
        Lv[i] = ld(a.L, (size_t)i * N + q);
        xv[i] = ld(a.chi0, (size_t)i * N + q);
    }
    __syncthreads();
    // gamma^{d/m} at Omega = 0 = gamma_uu +- gamma_ud
    const double sgn = (c == 0) ? 1.0 : -1.0;
    const size_t v0 = (size_t)a.i0 * n * n;
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        const cd gu = ld(a.guu, v0 + e), gd = ld(a.gud, v0 + e);
        const cd gm = {gu.re + sgn * gd.re, gu.im + sgn * gd.im};
        const cd x = gm * xv[j];
        st(M, (size_t)i * ldm + j, cd{(i == j ? 1.0 : 0.0) - x.re, -x.im});
    }
    for (int i = tid; i < n; i += blockDim.x) {
        cd y = {0.0, 0.0};
        for (int j = 0; j < n; ++j) {
            const cd gu = ld(a.guu, v0 + (size_t)i * n + j), gd = ld(a.gud, v0 + (size_t)i * n + j);
            y = fma_c(y, cd{gu.re + sgn * gd.re, gu.im + sgn * gd.im}, Lv[j]);
        }
        st(M, (size_t)i * ldm + n, y);
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (tid < 64) {   // partial pivoting: largest |M_ik|, i >= k (lowest index on ties)
            double bv = -1.0;
            int bi = k;
            for (int i = k + lane; i < n; i += 64) {
                const cd x = ld(M, (size_t)i * ldm + k);
                const double v = x.re * x.re + x.im * x.im;
                if (v > bv) {
                    bv = v;
                    bi = i;
                }
            }
            argmax_pair(bv, bi);
            if (lane == 0) s_piv = bi;
        }
        __syncthreads();
        const int p = s_piv;
        if (p != k) {
            for (int j = k + tid; j <= n; j += blockDim.x) {
                const cd x = ld(M, (size_t)k * ldm + j), y = ld(M, (size_t)p * ldm + j);
                st(M, (size_t)k * ldm + j, y);
                st(M, (size_t)p * ldm + j, x);
            }
            __syncthreads();
        }
        const cd inv = recip(ld(M, (size_t)k * ldm + k));
        const int rows = n - 1 - k, cols = n - k;   // rows k+1.., columns k+1..n
        for (int e = tid; e < rows * cols; e += blockDim.x) {
            const int i = k + 1 + e / cols, j = k + 1 + e % cols;
            const cd l = ld(M, (size_t)i * ldm + k) * inv;
            st(M, (size_t)i * ldm + j, fms(ld(M, (size_t)i * ldm + j), l, ld(M, (size_t)k * ldm + j)));
        }
        __syncthreads();
    }
    // back substitution by wave 0, then sum_i L_i z_i
    if (tid < 64) {
        for (int i = n - 1; i >= 0; --i) {
            cd s = {0.0, 0.0};
            for (int j = i + 1 + lane; j < n; j += 64) s = fma_c(s, ld(M, (size_t)i * ldm + j), zv[j]);
            s = wave_sum_c(s);
            if (lane == 0) zv[i] = cdiv(ld(M, (size_t)i * ldm + n) - s, ld(M, (size_t)i * ldm + i));
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        cd r = {0.0, 0.0};
        for (int i = lane; i < n; i += 64) r = fma_c(r, Lv[i], zv[i]);
        r = wave_sum_c(r);
        if (lane == 0) st(a.lad, (size_t)c * N + q, r);
    }
}

// chi_c(q) = sum_nu bubble[nu][q] + lad[c][q], fixed order over nu.
__global__ __launch_bounds__(256) void k_lattice_chi_sum(LatticeSumArgs a) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.N) return;
    cd s = {0.0, 0.0};
    for (int n = 0; n < a.n_nu; ++n) s = s + ld(a.bub, (size_t)n * a.N + q);
    if (a.chi_ch) st(a.chi_ch, q, s + ld(a.lad, q));
    if (a.chi_sp) st(a.chi_sp, q, s + ld(a.lad, (size_t)a.N + q));
}

hipError_t launch_lattice_fields(const LatticeFieldArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_lattice_fields, dim3(a.n_nu), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_lattice_chi_ladder(const LatticeChiArgs &a, int items, hipStream_t s) {
    if (a.n_nu > 128 || items < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_lattice_chi_ladder, dim3(items), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_lattice_chi_sum(const LatticeSumArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_lattice_chi_sum, dim3((a.N + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace df
