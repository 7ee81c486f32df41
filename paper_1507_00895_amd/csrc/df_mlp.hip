// Learned warm start: forward, backward and Adam kernels of a small MLP on the
// FP32 matrix cores, behind the C ABI of include/df_mlp.h.
//
// GEMM: C[M x N] = op(A)[M x K] op(B)[K x N], one 64 x 64 tile per work-group
// of four waves (each a 32 x 32 quadrant = 2 x 2 tiles of
// v_mfma_f32_16x16x4f32), K staged through LDS in chunks of 16.  Fused
// epilogues: bias, SiLU with the pre-activation saved, multiplication by
// SiLU'(Z) of the previous layer (backward), split-K partial sums reduced in
// a fixed order by a second kernel.
//
// FP32 16x16x4 lane layout (gfx950): A[i][k] at lane i + 16k, B[k][j] at lane
// j + 16k, C[i][j] at lane j + 16 (i / 4), register i % 4.
#include <math.h>

#include "../../include/df_mlp.h"
#include "df_internal.hpp"

namespace df {

typedef float f4 __attribute__((ext_vector_type(4)));

struct GemmArgs {
    int M, N, K;
    const float *A;
    int lda, transA;          // A(m, k) = transA ? A[k lda + m] : A[m lda + k]
    const float *B;
    int ldb, transB;          // B(k, n) = transB ? B[n ldb + k] : B[k ldb + n]
    float *C;
    int ldc;
    const float *bias;        // [N] or null
    float *Zout;              // pre-activation store (ldc layout) or null
    int act;                  // 1: SiLU
    const float *dz;          // backward: multiply by SiLU'(dz[m ldc + n]) or null
    float *part;              // split-K: partial sums [gridDim.z][M][N]
    int kchunk;               // K range per split (multiple of 16)
};

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = sigm(z);
    return s * (1.0f + z * (1.0f - s));
}

__global__ __launch_bounds__(256) void k_gemm_f32(GemmArgs g) {
    __shared__ float As[16][68];
    __shared__ float Bs[16][68];
    const int tid = threadIdx.x;
    const int w = tid >> 6, l = tid & 63, lj = l & 15, lg = l >> 4;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int kbeg = blockIdx.z * g.kchunk;
    const int kend = min(g.K, kbeg + g.kchunk);
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = kbeg; k0 < kend; k0 += 16) {
#pragma unroll
        for (int e4 = 0; e4 < 4; ++e4) {
            const int e = tid * 4 + e4;                 // 0 .. 1023
            int ml, kl;
            if (g.transA) { ml = e & 63; kl = e >> 6; } else { ml = e >> 4; kl = e & 15; }
            const int m = m0 + ml, k = k0 + kl;
            float va = 0.f;
            if (m < g.M && k < kend)
                va = g.transA ? g.A[(size_t)k * g.lda + m] : g.A[(size_t)m * g.lda + k];
            As[kl][ml] = va;
            int nl, kb;
            if (g.transB) { nl = e >> 4; kb = e & 15; } else { nl = e & 63; kb = e >> 6; }
            const int n = n0 + nl, kk = k0 + kb;
            float vb = 0.f;
            if (n < g.N && kk < kend)
                vb = g.transB ? g.B[(size_t)n * g.ldb + kk] : g.B[(size_t)kk * g.ldb + n];
            Bs[kb][nl] = vb;
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < 4; ++k4) {
            float av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = As[4 * k4 + lg][wm * 32 + 16 * i + lj];
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = Bs[4 * k4 + lg][wn * 32 + 16 * j + lj];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm * 32 + 16 * i + 4 * lg + r;
                const int n = n0 + wn * 32 + 16 * j + lj;
                if (m >= g.M || n >= g.N) continue;
                float v = acc[i][j][r];
                if (gridDim.z > 1) {
                    g.part[((size_t)blockIdx.z * g.M + m) * g.N + n] = v;
                    continue;
                }
                const size_t o = (size_t)m * g.ldc + n;
                if (g.bias) v += g.bias[n];
                if (g.dz) v *= dsilu(g.dz[o]);
                if (g.Zout) g.Zout[o] = v;
                if (g.act) v = silu(v);
                g.C[o] = v;
            }
}

// C[m][n] = sum over splits of part[s][m][n], in split order
__global__ __launch_bounds__(256) void k_sum_splits(const float *part, int splits, int M, int N,
                                                    float *C, int ldc) {
    const size_t tot = (size_t)M * N;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
         e += (size_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int z = 0; z < splits; ++z) s += part[(size_t)z * tot + e];
        C[(e / N) * ldc + e % N] = s;
    }
}

// db[n] = sum_m dZ[m][n]; 64 columns per block, 4 row phases, fixed order
__global__ __launch_bounds__(256) void k_colsum(const float *dZ, int M, int N, float *db) {
    __shared__ float red[4][64];
    const int c = threadIdx.x & 63, p = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + c;
    float s = 0.f;
    if (n < N)
        for (int m = p; m < M; m += 4) s += dZ[(size_t)m * N + n];
    red[p][c] = s;
    __syncthreads();
    if (p == 0 && n < N) db[n] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
}

// dY = 2 (Y - T) / count; per-block partial sums of (Y - T)^2
__global__ __launch_bounds__(256) void k_mse(const float *Y, const float *T, size_t count, float *dY,
                                             float *part) {
    __shared__ float red[256];
    const float sc = 2.0f / (float)count;
    float s = 0.f;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (size_t)gridDim.x * blockDim.x) {
        const float d = Y[e] - T[e];
        dY[e] = sc * d;
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_mse_final(const float *part, int n, size_t count, float *loss) {
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) *loss = red[0] / (float)count;
}

__global__ __launch_bounds__(256) void k_adam(size_t count, float *p, const float *g, float *m, float *v,
                                              float lr, float c1, float c2) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (size_t)gridDim.x * blockDim.x) {
        const float gg = g[e];
        const float mm = 0.9f * m[e] + 0.1f * gg;
        const float vv = 0.999f * v[e] + 0.001f * gg * gg;
        m[e] = mm;
        v[e] = vv;
        p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
    }
}

}  // namespace df

using namespace df;

namespace {

constexpr size_t kAl = 256;
size_t alup(size_t x) { return (x + kAl - 1) & ~(kAl - 1); }
constexpr int kMseBlocks = 256;

int check_net(int32_t n_layers, const int32_t *dims) {
    if (n_layers < 1 || n_layers > DF_MLP_MAX_LAYERS || !dims) return DF_E_INVAL;
    for (int i = 0; i <= n_layers; ++i)
        if (dims[i] < 1 || dims[i] > DF_MLP_MAX_WIDTH) return DF_E_INVAL;
    return DF_OK;
}

size_t n_params(int32_t L, const int32_t *d) {
    size_t c = 0;
    for (int l = 0; l < L; ++l) c += (size_t)d[l + 1] * d[l] + d[l + 1];
    return c;
}

int max_width(int32_t L, const int32_t *d) {
    int m = 0;
    for (int l = 0; l <= L; ++l) m = d[l] > m ? d[l] : m;
    return m;
}

int splits_for(int K) {
    int s = (K + 255) / 256;
    return s < 1 ? 1 : (s > 64 ? 64 : s);
}

// workspace: Z[l], Y[l] for l = 1..L (batch x d_l), dZ ping-pong, split partials, loss partials
struct MlpWs {
    size_t z[DF_MLP_MAX_LAYERS + 1], y[DF_MLP_MAX_LAYERS + 1], dz[2], part, lpart, total;
};

MlpWs mlp_ws(int32_t L, const int32_t *d, int32_t batch) {
    MlpWs w{};
    size_t o = 0;
    for (int l = 1; l <= L; ++l) {
        w.z[l] = o;
        o = alup(o + (size_t)batch * d[l] * sizeof(float));
        w.y[l] = o;
        o = alup(o + (size_t)batch * d[l] * sizeof(float));
    }
    const int mw = max_width(L, d);
    for (int k = 0; k < 2; ++k) {
        w.dz[k] = o;
        o = alup(o + (size_t)batch * mw * sizeof(float));
    }
    w.part = o;
    o = alup(o + (size_t)splits_for(batch) * mw * mw * sizeof(float));
    w.lpart = o;
    o = alup(o + kMseBlocks * sizeof(float));
    w.total = o;
    return w;
}

template <typename T> T *wsp(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

hipError_t gemm(GemmArgs g, hipStream_t st, int splits = 1) {
    g.kchunk = ((g.K + splits - 1) / splits + 15) / 16 * 16;
    if (g.kchunk < 16) g.kchunk = 16;
    splits = (g.K + g.kchunk - 1) / g.kchunk;
    if (splits < 1) splits = 1;
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, splits);
    hipLaunchKernelGGL(k_gemm_f32, grid, dim3(256), 0, st, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || splits == 1) return e;
    const size_t tot = (size_t)g.M * g.N;
    int blocks = (int)((tot + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_sum_splits, dim3(blocks), dim3(256), 0, st, g.part, splits, g.M, g.N, g.C,
                       g.ldc);
    return hipGetLastError();
}

int forward_impl(int32_t L, const int32_t *d, const float *params, const float *X, int32_t batch,
                 float *Yout, void *ws, const MlpWs &w, hipStream_t st) {
    const float *in = X;
    size_t po = 0;
    for (int l = 0; l < L; ++l) {
        const float *W = params + po;
        const float *b = W + (size_t)d[l + 1] * d[l];
        po += (size_t)d[l + 1] * d[l] + d[l + 1];
        const bool last = (l == L - 1);
        GemmArgs g{};
        g.M = batch;
        g.N = d[l + 1];
        g.K = d[l];
        g.A = in;
        g.lda = d[l];
        g.transA = 0;
        g.B = W;
        g.ldb = d[l];
        g.transB = 1;
        g.ldc = d[l + 1];
        g.bias = b;
        g.Zout = wsp<float>(ws, w.z[l + 1]);
        g.act = last ? 0 : 1;
        g.C = (last && Yout) ? Yout : wsp<float>(ws, w.y[l + 1]);
        if (gemm(g, st) != hipSuccess) return DF_E_HIP;
        in = g.C;
    }
    return DF_OK;
}

}  // namespace

extern "C" {

int df_mlp_param_count(int32_t n_layers, const int32_t *dims, size_t *count) {
    if (!count) return DF_E_INVAL;
    const int rc = check_net(n_layers, dims);
    if (rc != DF_OK) return rc;
    *count = n_params(n_layers, dims);
    return DF_OK;
}

int df_mlp_workspace_size(int32_t n_layers, const int32_t *dims, int32_t batch, size_t *bytes) {
    if (!bytes || batch < 1) return DF_E_INVAL;
    const int rc = check_net(n_layers, dims);
    if (rc != DF_OK) return rc;
    *bytes = mlp_ws(n_layers, dims, batch).total;
    return DF_OK;
}

int df_mlp_forward(int32_t n_layers, const int32_t *dims, const float *params, const float *X,
                   int32_t batch, float *Y, void *ws, size_t ws_bytes, df_stream_t stream) {
    int rc = check_net(n_layers, dims);
    if (rc != DF_OK) return rc;
    if (!params || !X || !Y || batch < 1) return DF_E_INVAL;
    const MlpWs w = mlp_ws(n_layers, dims, batch);
    if (!ws || ((uintptr_t)ws & (kAl - 1)) || ws_bytes < w.total) return DF_E_WORKSPACE;
    return forward_impl(n_layers, dims, params, X, batch, Y, ws, w, (hipStream_t)stream);
}

int df_mlp_loss_grad(int32_t n_layers, const int32_t *dims, const float *params, const float *X,
                     const float *T, int32_t batch, float *grads, float *loss, void *ws,
                     size_t ws_bytes, df_stream_t stream) {
    int rc = check_net(n_layers, dims);
    if (rc != DF_OK) return rc;
    if (!params || !X || !T || !grads || batch < 1) return DF_E_INVAL;
    const int32_t L = n_layers;
    const int32_t *d = dims;
    const MlpWs w = mlp_ws(L, d, batch);
    if (!ws || ((uintptr_t)ws & (kAl - 1)) || ws_bytes < w.total) return DF_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    rc = forward_impl(L, d, params, X, batch, nullptr, ws, w, st);
    if (rc != DF_OK) return rc;

    // dZ_L = 2 (Y - T) / count (last layer has no activation)
    const size_t count = (size_t)batch * d[L];
    float *dzc = wsp<float>(ws, w.dz[L & 1]);
    hipLaunchKernelGGL(k_mse, dim3(kMseBlocks), dim3(256), 0, st, wsp<float>(ws, w.y[L]), T, count,
                       dzc, wsp<float>(ws, w.lpart));
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(256), 0, st, wsp<float>(ws, w.lpart), kMseBlocks,
                       count, loss);
    if (hipGetLastError() != hipSuccess) return DF_E_HIP;

    // parameter offsets
    size_t off[DF_MLP_MAX_LAYERS + 1];
    off[0] = 0;
    for (int l = 0; l < L; ++l) off[l + 1] = off[l] + (size_t)d[l + 1] * d[l] + d[l + 1];

    for (int l = L - 1; l >= 0; --l) {
        const float *Xl = (l == 0) ? X : wsp<float>(ws, w.y[l]);
        float *dW = grads + off[l];
        float *db = dW + (size_t)d[l + 1] * d[l];
        const float *dZ = wsp<float>(ws, w.dz[(l + 1) & 1]);
        // dW_l = dZ^T X_l (split over the batch), db_l = column sums of dZ
        GemmArgs g{};
        g.M = d[l + 1];
        g.N = d[l];
        g.K = batch;
        g.A = dZ;
        g.lda = d[l + 1];
        g.transA = 1;
        g.B = Xl;
        g.ldb = d[l];
        g.transB = 0;
        g.C = dW;
        g.ldc = d[l];
        g.part = wsp<float>(ws, w.part);
        if (gemm(g, st, splits_for(batch)) != hipSuccess) return DF_E_HIP;
        hipLaunchKernelGGL(k_colsum, dim3((d[l + 1] + 63) / 64), dim3(256), 0, st, dZ, batch, d[l + 1],
                           db);
        if (hipGetLastError() != hipSuccess) return DF_E_HIP;
        if (l == 0) break;
        // dZ_l = (dZ_{l+1} W_l) * SiLU'(Z_l)
        GemmArgs h{};
        h.M = batch;
        h.N = d[l];
        h.K = d[l + 1];
        h.A = dZ;
        h.lda = d[l + 1];
        h.transA = 0;
        h.B = params + off[l];
        h.ldb = d[l];
        h.transB = 0;
        h.C = wsp<float>(ws, w.dz[l & 1]);
        h.ldc = d[l];
        h.dz = wsp<float>(ws, w.z[l]);
        if (gemm(h, st) != hipSuccess) return DF_E_HIP;
    }
    return DF_OK;
}

int df_mlp_adam(size_t count, float *params, const float *grads, float *m, float *v, int32_t step,
                float lr, df_stream_t stream) {
    if (!params || !grads || !m || !v || step < 1 || count == 0 || !(lr > 0.f)) return DF_E_INVAL;
    const float c1 = 1.0f - powf(0.9f, (float)step);
    const float c2 = 1.0f - powf(0.999f, (float)step);
    int blocks = (int)((count + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_adam, dim3(blocks), dim3(256), 0, (hipStream_t)stream, count, params, grads,
                       m, v, lr, c1, c2);
    return hipGetLastError() == hipSuccess ? DF_OK : DF_E_HIP;
}

}  // extern "C"
