// Anderson acceleration of the dual self-energy iteration (an alternative to
// the linear mixing of the self-consistency loop, Sec. 2.2): both converge to
// the same fixed point Sigma~ = F(Sigma~), where F is one pass of the ladder
// approximation; the accelerated iteration needs fewer passes.
//
// Per instance, a ring of the last m + 1 iterates x_j and residuals
// r_j = F(x_j) - x_j lives in the workspace.  Each iteration:
//   k_acc_record   stores x_k and r_k into ring slot s and forms block
//                  partials of Re <r_j, r_k> for every slot j (FP64);
//   k_acc_dots     reduces them in a fixed order (bit-reproducible);
//   (host)         least squares over the residual differences with real
//                  coefficients, which keep Sigma~(-nu) = Sigma~(nu)* and
//                  the lattice symmetries that every iterate has;
//   k_acc_combine  x_{k+1} = sum_j c_j (x_j + alpha r_j), with the partial
//                  norms of x_{k+1} - x_k and x_{k+1} for the convergence test.
#include "df_internal.hpp"

namespace df {

__global__ __launch_bounds__(256) void k_acc_record(AccRecordArgs a) {
    __shared__ double red[kAccMaxSlots][256];
    double acc[kAccMaxSlots];
#pragma unroll
    for (int j = 0; j < kAccMaxSlots; ++j) acc[j] = 0.0;
    const size_t M = a.count;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < M;
         e += (size_t)gridDim.x * blockDim.x) {
        const cd x = ld(a.x, e);
        const cd f = ld(a.fx, e);
        const cd r = {f.re - x.re, f.im - x.im};
        st(a.xh + 2 * (size_t)a.slot * M, e, x);
        st(a.rh + 2 * (size_t)a.slot * M, e, r);
#pragma unroll
        for (int j = 0; j < kAccMaxSlots; ++j) {
            if (j >= a.n_slots) break;
            const cd rj = (j == a.slot) ? r : ld(a.rh + 2 * (size_t)j * M, e);
            acc[j] = fma(rj.re, r.re, fma(rj.im, r.im, acc[j]));   // Re conj(rj) r
        }
    }
    for (int j = 0; j < a.n_slots; ++j) {
        red[j][threadIdx.x] = acc[j];
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int j = 0; j < a.n_slots; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + s];
        __syncthreads();
    }
    if ((int)threadIdx.x < a.n_slots)
        a.part[(size_t)blockIdx.x * kAccMaxSlots + threadIdx.x] = red[threadIdx.x][0];
}

// dots[j] = sum over blocks of part[b][j], in block order
__global__ __launch_bounds__(64) void k_acc_dots(const double *part, int n_part, int n_slots,
                                                 double *dots) {
    const int j = threadIdx.x;
    if (j >= n_slots) return;
    double s = 0.0;
    for (int b = 0; b < n_part; ++b) s += part[(size_t)b * kAccMaxSlots + j];
    dots[j] = s;
}

__global__ __launch_bounds__(256) void k_acc_combine(AccCombineArgs a) {
    __shared__ double red[2][256];
    double dn = 0.0, nn = 0.0;
    const size_t M = a.count;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < M;
         e += (size_t)gridDim.x * blockDim.x) {
        cd nw = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < kAccMaxSlots; ++j) {
            if (j >= a.n_slots) break;
            const double c = a.coef[j];
            if (c == 0.0) continue;
            const cd xj = ld(a.xh + 2 * (size_t)j * M, e);
            const cd rj = ld(a.rh + 2 * (size_t)j * M, e);
            nw.re = fma(c, fma(a.alpha, rj.re, xj.re), nw.re);
            nw.im = fma(c, fma(a.alpha, rj.im, xj.im), nw.im);
        }
        const cd old = ld(a.x, e);
        st(a.x, e, nw);
        const double dr = nw.re - old.re, di = nw.im - old.im;
        dn += dr * dr + di * di;
        nn += nw.re * nw.re + nw.im * nw.im;
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
        a.norm_part[2 * blockIdx.x] = red[0][0];
        a.norm_part[2 * blockIdx.x + 1] = red[1][0];
    }
}

hipError_t launch_acc_record(const AccRecordArgs &a, int blocks, hipStream_t s) {
    if (a.n_slots < 1 || a.n_slots > kAccMaxSlots || a.slot < 0 || a.slot >= a.n_slots)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_acc_record, dim3(blocks), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_acc_dots, dim3(1), dim3(64), 0, s, a.part, blocks, a.n_slots, a.dots);
    return hipGetLastError();
}

hipError_t launch_acc_combine(const AccCombineArgs &a, int blocks, hipStream_t s) {
    if (a.n_slots < 1 || a.n_slots > kAccMaxSlots) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_acc_combine, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace df
