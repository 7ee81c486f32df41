// Device helpers shared by the dual-fermion kernels: complex arithmetic and
// an LDS-resident radix-4/2 FFT over the D-dimensional k-grid.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace df {

// ----------------------------------------------------------------- complex
template <typename T> struct alignas(2 * sizeof(T)) cplx {
    T re, im;
};
using cd = cplx<double>;
using cf = cplx<float>;

template <typename T> __device__ __forceinline__ cplx<T> mk(T r, T i) { return {r, i}; }
template <typename T> __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) {
    return {a.re + b.re, a.im + b.im};
}
template <typename T> __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) {
    return {a.re - b.re, a.im - b.im};
}
template <typename T> __device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
    return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
template <typename T> __device__ __forceinline__ cplx<T> scale(cplx<T> a, T s) {
    return {a.re * s, a.im * s};
}
template <typename T> __device__ __forceinline__ cplx<T> conj(cplx<T> a) { return {a.re, -a.im}; }
// c - a*b
template <typename T> __device__ __forceinline__ cplx<T> fms(cplx<T> c, cplx<T> a, cplx<T> b) {
    T r = fma(-a.re, b.re, c.re);
    r = fma(a.im, b.im, r);
    T i = fma(-a.re, b.im, c.im);
    i = fma(-a.im, b.re, i);
    return {r, i};
}
// c + a*b
template <typename T> __device__ __forceinline__ cplx<T> fma_c(cplx<T> c, cplx<T> a, cplx<T> b) {
    T r = fma(a.re, b.re, c.re);
    r = fma(-a.im, b.im, r);
    T i = fma(a.re, b.im, c.im);
    i = fma(a.im, b.re, i);
    return {r, i};
}
// 1 / a (Smith's algorithm)
template <typename T> __device__ __forceinline__ cplx<T> recip(cplx<T> a) {
    if (fabs(a.re) >= fabs(a.im)) {
        T r = a.im / a.re;
        T d = a.re + a.im * r;
        T inv = T(1) / d;
        return {inv, -r * inv};
    } else {
        T r = a.re / a.im;
        T d = a.re * r + a.im;
        T inv = T(1) / d;
        return {r * inv, -inv};
    }
}
template <typename T> __device__ __forceinline__ cplx<T> cdiv(cplx<T> a, cplx<T> b) {
    return a * recip(b);
}
template <typename T> __device__ __forceinline__ T cabs1(cplx<T> a) { return fabs(a.re) + fabs(a.im); }

// Every array these kernels read or write through ld/st lives in device
// global memory: say so, so that the compiler emits global (not flat) loads
// and stores, which do not share a wait counter with LDS traffic.
typedef double dv2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cd ld(const double *p, size_t i) {
    const dv2 v = *(__attribute__((address_space(1))) const dv2 *)(const void *)(p + 2 * i);
    return {v.x, v.y};
}
__device__ __forceinline__ void st(double *p, size_t i, cd v) {
    *(__attribute__((address_space(1))) dv2 *)(void *)(p + 2 * i) = dv2{v.re, v.im};
}
// FP32 pairs and quadruples (element i of an array of them)
typedef float fv2 __attribute__((ext_vector_type(2)));
typedef float fv4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ fv2 ld2f(const float *p, size_t i) {
    return *(__attribute__((address_space(1))) const fv2 *)(const void *)(p + 2 * i);
}
__device__ __forceinline__ fv4 ld4f(const float *p, size_t i) {
    return *(__attribute__((address_space(1))) const fv4 *)(const void *)(p + 4 * i);
}
__device__ __forceinline__ void st2f(float *p, size_t i, float a, float b) {
    *(__attribute__((address_space(1))) fv2 *)(void *)(p + 2 * i) = fv2{a, b};
}
__device__ __forceinline__ void st4f(float *p, size_t i, float a, float b, float c, float d) {
    *(__attribute__((address_space(1))) fv4 *)(void *)(p + 4 * i) = fv4{a, b, c, d};
}

// ----------------------------------------------------------------- k-grid
// Flat index in C order over D axes of nk = 2^lognk points; every axis is a
// field of lognk bits.  Bit reversal and reflection act field by field.
struct Grid {
    int D, lognk, nk, N;
};

__device__ __forceinline__ int bitrev_fields(int r, const Grid &g) {
    int out = 0;
    for (int a = 0; a < g.D; ++a) {
        int c = (r >> (a * g.lognk)) & (g.nk - 1);
        int rc = (int)(__brev((unsigned)c) >> (32 - g.lognk));
        out |= rc << (a * g.lognk);
    }
    return out;
}

__device__ __forceinline__ int reflect_fields(int r, const Grid &g) {
    int out = 0;
    for (int a = 0; a < g.D; ++a) {
        int c = (r >> (a * g.lognk)) & (g.nk - 1);
        out |= ((g.nk - c) & (g.nk - 1)) << (a * g.lognk);
    }
    return out;
}

// tw[t] = exp(-2 pi i t / nk), t < nk, into LDS.
__device__ __forceinline__ void make_twiddles(cd *tw, const Grid &g) {
    for (int t = threadIdx.x; t < g.nk; t += blockDim.x) {
        double s, c;
        sincospi(-2.0 * (double)t / (double)g.nk, &s, &c);
        tw[t] = {c, s};
    }
}

// In-place FFT over every axis of the N-point array X held in LDS, which
// must already be in bit-reversed order on every axis (decimation in time).
// Forward: X(q) = sum_r e^{-i q r} x(r).  INV: the + sign, no 1/N factor.
// Barriers: one after every pass; the caller synchronises before the call.
template <bool INV>
__device__ void fft_inplace(cd *X, const cd *tw, const Grid &g) {
    const int tid = threadIdx.x, nth = blockDim.x;
    const int lognk = g.lognk, nk = g.nk, N = g.N;
    for (int a = 0; a < g.D; ++a) {
        const int sh = a * lognk;
        const int S = 1 << sh;
        int s = 1;
        if (lognk & 1) {
            // radix-2 pass, half length 1, twiddle 1
            for (int u = tid; u < (N >> 1); u += nth) {
                const int lo = u & (S - 1);
                const int rest = u >> sh;
                const int b = rest & ((nk >> 1) - 1);
                const int hi = rest >> (lognk - 1);
                const int p0 = (hi << (sh + lognk)) + ((2 * b) << sh) + lo;
                const cd x0 = X[p0], x1 = X[p0 + S];
                X[p0] = x0 + x1;
                X[p0 + S] = x0 - x1;
            }
            __syncthreads();
            s = 2;
        }
        for (; s < lognk; s += 2) {
            // two radix-2 stages (half lengths h and 2h) fused into one pass
            const int h = 1 << (s - 1);
            for (int u = tid; u < (N >> 2); u += nth) {
                const int lo = u & (S - 1);
                const int rest = u >> sh;
                const int j = rest & (h - 1);
                const int b = (rest >> (s - 1)) & ((nk >> (s + 1)) - 1);
                const int hi = rest >> (lognk - 2);
                const int c0 = (b << (s + 1)) + j;
                const int p0 = (hi << (sh + lognk)) + (c0 << sh) + lo;
                const int hs = h << sh;
                const cd x0 = X[p0], x1 = X[p0 + hs], x2 = X[p0 + 2 * hs], x3 = X[p0 + 3 * hs];
                cd w1 = tw[j << (lognk - s)];
                cd w2 = tw[j << (lognk - s - 1)];
                if (INV) {
                    w1 = conj(w1);
                    w2 = conj(w2);
                }
                // w3 = w2 * exp(-+ i pi / 2)
                const cd w3 = INV ? cd{-w2.im, w2.re} : cd{w2.im, -w2.re};
                const cd t1 = w1 * x1, t3 = w1 * x3;
                const cd y0 = x0 + t1, y1 = x0 - t1, y2 = x2 + t3, y3 = x2 - t3;
                const cd u2 = w2 * y2, u3 = w3 * y3;
                X[p0] = y0 + u2;
                X[p0 + 2 * hs] = y0 - u2;
                X[p0 + hs] = y1 + u3;
                X[p0 + 3 * hs] = y1 - u3;
            }
            __syncthreads();
        }
    }
}

}  // namespace df
