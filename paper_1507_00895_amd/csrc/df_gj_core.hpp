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
// B = cabs1(M) + eps I (cabs1 = |re| + |im| >= |.|), stopping at the first
// step whose bound already passes.  The bound also limits the
// condition number of D after diagonal scaling: ||D'^-1|| <= 1 / (1 - rho).
//
// Sweep.  For each tile column t: wave t inverts the diagonal tile A_tt by 16
// scalar Gauss-Jordan steps on its accumulator registers (pivot by readlane,
// pivot-column values within a 16-lane row by DPP, the pivot-row value of a
// lane's column by bpermute) and publishes it with its old block-row; every other wave forms G_w = -A_wt A_tt^-1; every
// wave applies A_w,c += G_w A_t,c (c != t) with G_t = A_tt^-1 - 1 and sets
// tile (w, t) to G_w (A_tt^-1 for w = t).  This is the block form of the
// in-place sweep: afterwards the tiles hold D^-1, and the scalar pivots
// (stored in the tiles' precision; their product is formed in FP64)
// multiply to det D.
//
// Every function takes the thread index as an argument: the kernels pass an
// opaque copy made per item, so that nothing derived from it is hoisted out
// of a persistent work-group's item loop and held across the whole item.
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
    // c - a b: on the FP64 matrix instruction the last field negates the A
    // operand (bit 0), so no register holds -a
    static __device__ __forceinline__ v4 mma_na(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 1);
    }
    static __device__ __forceinline__ int row(int lg, int r) { return lg + 4 * r; }
    // row s of a tile sits in row group lg_of(s), register r_of(s)
    static __device__ __forceinline__ int lg_of(int s) { return s & 3; }
    static __device__ __forceinline__ int r_of(int s) { return s >> 2; }
};
template <> struct MT<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // c - a b (the FP32 instruction's last field is a broadcast control)
    static __device__ __forceinline__ v4 mma_na(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(-a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lg, int r) { return 4 * lg + r; }
    static __device__ __forceinline__ int lg_of(int s) { return s >> 2; }
    static __device__ __forceinline__ int r_of(int s) { return s & 3; }
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

// value of lane n of the caller's own 16-lane row (DPP row_newbcast; n resolves
// statically once the caller's loop unrolls)
template <int N> __device__ __forceinline__ int row_bcast_i(int v) {
    return __builtin_amdgcn_mov_dpp(v, 0x150 + N, 0xf, 0xf, true);
}
__device__ __forceinline__ int row_bcast_rt(int v, int n) {
    switch (n) {
        case 0: return row_bcast_i<0>(v);
        case 1: return row_bcast_i<1>(v);
        case 2: return row_bcast_i<2>(v);
        case 3: return row_bcast_i<3>(v);
        case 4: return row_bcast_i<4>(v);
        case 5: return row_bcast_i<5>(v);
        case 6: return row_bcast_i<6>(v);
        case 7: return row_bcast_i<7>(v);
        case 8: return row_bcast_i<8>(v);
        case 9: return row_bcast_i<9>(v);
        case 10: return row_bcast_i<10>(v);
        case 11: return row_bcast_i<11>(v);
        case 12: return row_bcast_i<12>(v);
        case 13: return row_bcast_i<13>(v);
        case 14: return row_bcast_i<14>(v);
        default: return row_bcast_i<15>(v);
    }
}
template <int N> __device__ __forceinline__ double row_bcast_d(double v) {
    const long long b = __double_as_longlong(v);
    return __longlong_as_double(__builtin_amdgcn_mov_dpp(b, 0x150 + N, 0xf, 0xf, true));
}
__device__ __forceinline__ double row_bcast_v(double v, int n) {
    switch (n) {   // one 64-bit DPP move (DPP64 supports row_newbcast)
        case 0: return row_bcast_d<0>(v);
        case 1: return row_bcast_d<1>(v);
        case 2: return row_bcast_d<2>(v);
        case 3: return row_bcast_d<3>(v);
        case 4: return row_bcast_d<4>(v);
        case 5: return row_bcast_d<5>(v);
        case 6: return row_bcast_d<6>(v);
        case 7: return row_bcast_d<7>(v);
        case 8: return row_bcast_d<8>(v);
        case 9: return row_bcast_d<9>(v);
        case 10: return row_bcast_d<10>(v);
        case 11: return row_bcast_d<11>(v);
        case 12: return row_bcast_d<12>(v);
        case 13: return row_bcast_d<13>(v);
        case 14: return row_bcast_d<14>(v);
        default: return row_bcast_d<15>(v);
    }
}
__device__ __forceinline__ float row_bcast_v(float v, int n) {
    return __int_as_float(row_bcast_rt(__float_as_int(v), n));
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
// (FP32: the hardware reciprocal is within 2 ulp, measured, enough for the
// FP32 ladder whose own error is of order kappa * n * 2^-24)
__device__ __forceinline__ cf recip_fast(cf z) {
    const float m = fmaf(z.re, z.re, z.im * z.im);
    const float y = __builtin_amdgcn_rcpf(m);
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
// The inverted diagonal tile of step t is published in Xw[t]: the wave that
// inverts it has no layout exchange of its own at that step.
// Store a complex value to LDS as two separate stores of its parts: a
// 16-byte (FP64) or 8-byte (FP32) store of the pair needs the parts in
// adjacent registers, and the parts of a tile element sit in two different
// accumulator tiles, so each such store cost register copies (two per value
// in FP64).  The volatile store (to the LDS address space: d is in LDS)
// keeps the two from being merged back.
template <typename T> __device__ __forceinline__ void put_split(cplx<T> &d, T re, T im) {
    d.re = re;
    *(volatile __attribute__((address_space(3))) T *)(&d.im) = im;
}

template <typename T, int NP> struct GjShared {
    static constexpr int NT = NP / 16;
    // vbuf seen as complex entries, where the tile inversions' lanes without
    // the pivot put their element (vbuf is used by the certificate alone,
    // before the sweep, and written there before it is read)
    static constexpr int DUMP_N = NP >= 64 ? 64 : (NP >= 32 ? 32 : 16);
    __device__ __forceinline__ cplx<T> *dump() {
        static_assert(offsetof(GjShared, vbuf) % alignof(cplx<T>) == 0, "vbuf holds complex entries");
        static_assert(sizeof(vbuf) >= DUMP_N * sizeof(cplx<T>), "vbuf holds DUMP_N complex entries");
        return reinterpret_cast<cplx<T> *>(&vbuf[0][0]);
    }
    cplx<T> Rb[16][NP];          // old block-row of the current tile column
    cplx<T> Xw[NT][16][17];      // per-wave layout exchange (accumulator -> operand)
    cplx<T> pivv[NP];            // scalar pivots, in the tiles' precision
    double vbuf[2][NP];          // power-iteration vectors
    double wmax[2][NT];          // double-buffered: a wave may start the next step early
};

// Sum over the 16 lanes of the caller's DPP row, returned to all of them
// (pairs by quad_perm, then rotations by 4 and 8 within the row).
template <int CTRL> __device__ __forceinline__ float dpp_f(float v) {
    // every lane has a source for these controls; bound_ctrl lets the move
    // fold into the add that consumes it
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}
__device__ __forceinline__ cf row16_sum(cf x);
template <int CTRL> __device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float row16_sum(float x) {
    x += dpp_f<0xB1>(x);    // quad_perm [1,0,3,2]
    x += dpp_f<0x4E>(x);    // quad_perm [2,3,0,1]
    x += dpp_f<0x124>(x);   // row_ror:4
    x += dpp_f<0x128>(x);   // row_ror:8
    return x;
}
__device__ __forceinline__ double row16_sum(double x) {
    x += dpp_d<0xB1>(x);
    x += dpp_d<0x4E>(x);
    x += dpp_d<0x124>(x);
    x += dpp_d<0x128>(x);
    return x;
}
__device__ __forceinline__ cd row16_sum(cd x) { return {row16_sum(x.re), row16_sum(x.im)}; }
__device__ __forceinline__ cf row16_sum(cf x) { return {row16_sum(x.re), row16_sum(x.im)}; }
// Row sums of a 16-row block held one column per lane: v[r] is the lane's
// partial sum of row MT<T>::row(lg, r) (its column lj); the 16 sums go to
// out[0..15] (FP64).  The partials pass through the wave's own LDS block
// buf (16 x 17, free outside the sweep) and each pair of lanes adds one part
// of one row, so the reduction takes about a dozen vector instructions per
// lane where reducing the eight values by DPP across the 16 lanes took 96
// (FP64) or 32 (FP32).  Wave-local: no barrier; out is read after the
// caller's next barrier.
template <typename T>
__device__ __forceinline__ void rows16_sum_lds(const cplx<T> (&v)[4], cplx<T> (*buf)[17], cd *out,
                                               int tid) {
    const int l = tid & 63, lj = l & 15, lg = l >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) put_split<T>(buf[MT<T>::row(lg, r)][lj], v[r].re, v[r].im);
    wave_sync_lds();
    // lane l: row i = l >> 2, part (l >> 1) & 1 (re, im), columns 8 h .. 8 h + 7
    const int h = l & 1, part = (l >> 1) & 1, i = l >> 2;
    const T *src = &buf[i][8 * h].re + part;
    T acc = src[0];
#pragma unroll
    for (int k = 1; k < 8; ++k) acc += src[2 * k];
    // quad_perm [1,0,3,2]: the other half of the row
    if constexpr (sizeof(T) == 8) acc += dpp_d<0xB1>(acc);
    else acc += dpp_f<0xB1>(acc);
    if (h == 0) (&out[i].re)[part] = (double)acc;
    // (this wave's later writes to buf follow its reads: LDS operations of
    // one wave complete in order)
}
// The same sums, through LDS (LDS_SUMS) or by DPP across the lanes (fewer
// registers: the two-item builds at NP = 96, held to 168 VGPRs, spilled more
// with the LDS path, and the FP64 one measured 0.7 % slower).
template <bool LDS_SUMS, typename T>
__device__ __forceinline__ void rows16_sum(cplx<T> (&v)[4], cplx<T> (*buf)[17], cd *out, int tid) {
    if constexpr (LDS_SUMS) {
        rows16_sum_lds<T>(v, buf, out, tid);
    } else {
        const int l = tid & 63, lj = l & 15, lg = l >> 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = row16_sum(v[r]);
        if (lj == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) out[MT<T>::row(lg, r)] = cd{(double)v[r].re, (double)v[r].im};
        }
    }
}

// Sum over the wave, returned uniform: row sums, then the four row leaders.
__device__ __forceinline__ double wave_sum(double x) {
    x = row16_sum(x);
    return (readlane_v(x, 0) + readlane_v(x, 16)) + (readlane_v(x, 32) + readlane_v(x, 48));
}

// Step 0 of the power steps (v = 1): the row sums of B over the wave's
// block-row, each element |re| + |im| in the tiles' own precision (|.| is an
// operand modifier there), accumulated in FP32.
// DW, the wave's diagonal tile, is a compile-time constant here (the caller
// dispatches on the wave-uniform block-row index), so only the four elements
// per lane of that tile choose between the diagonal and off-diagonal forms.
template <typename T, int NP, int DW>
__device__ __forceinline__ void cert_rowsums0(const typename MT<T>::v4 (&Cr)[NP / 16],
                                              const typename MT<T>::v4 (&Ci)[NP / 16], int lj,
                                              int lg, float (&u)[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) u[r] = 0.f;
#pragma unroll
    for (int tc = 0; tc < NP / 16; ++tc)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            T a = fabs(Cr[tc][r]);
            if (tc == DW && lj == MT<T>::row(lg, r)) a = fabs(T(1) - Cr[tc][r]) + T(1e-6);
            u[r] += (float)(a + fabs(Ci[tc][r]));
        }
}
template <typename T, int NP, int K = 0>
__device__ __forceinline__ void cert_rowsums0_at(int wu, const typename MT<T>::v4 (&Cr)[NP / 16],
                                                 const typename MT<T>::v4 (&Ci)[NP / 16], int lj,
                                                 int lg, float (&u)[4]) {
    if constexpr (K + 1 < NP / 16) {
        if (wu == K) cert_rowsums0<T, NP, K>(Cr, Ci, lj, lg, u);
        else cert_rowsums0_at<T, NP, K + 1>(wu, Cr, Ci, lj, lg, u);
    } else {
        cert_rowsums0<T, NP, K>(Cr, Ci, lj, lg, u);
    }
}

// Collatz-Wielandt bound of rho(cabs1(M) + eps I), eps = 1e-6 (it keeps every
// component of v positive and normal in FP32 over the steps taken, and
// raises the bound by eps at most), for M = 1 - D; uniform result across the
// work-group.  Power steps from v = 1; after each step the bound
// max_i (B v)_i / v_i is formed and the loop stops as soon as it is below
// `accept` (any positive v gives a valid bound).  The sums are FP32 (step 0
// forms each element in the tiles' precision): every term is non-negative,
// so the computed sums are within (n + 1) 2^-24 relative of the exact ones,
// and the bound is inflated by (1 + 1e-5) to stay an upper bound.
// Contains barriers: every thread must call.
//
// peers, n_peers: the states of all items of the work-group when it holds
// several (one per slot of waves), else null.  Then the loop stops only when
// every item's bound passes, so that all items take the same barriers; the
// bound of an item that passed earlier keeps shrinking (the quotient of a
// power step never rises).
template <typename T, int NP, bool FAST0 = true>
__device__ __forceinline__ double gj_certify(const typename MT<T>::v4 (&Cr)[NP / 16],
                                             const typename MT<T>::v4 (&Ci)[NP / 16],
                                             GjShared<T, NP> &sh, int iters, double accept,
                                             int tid, const GjShared<T, NP> *peers = nullptr,
                                             int n_peers = 0) {
    constexpr int NT = NP / 16;
    const int w = tid >> 6, l = tid & 63, lj = l & 15, lg = l >> 4;
    double cw = INFINITY;
    if constexpr (!FAST0) {
        // step 0 starts from v = 1 without reading it (no barrier before it)
        for (int it = 0; it < iters; ++it) {
            const double *v = sh.vbuf[it & 1];
            float u[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int tc = 0; tc < NT; ++tc) {
                const int j = 16 * tc + lj;
                const float vj = (it == 0) ? 1.0f : (float)v[j];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 16 * w + MT<T>::row(lg, r);
                    const float mr = (float)(((i == j) ? T(1) : T(0)) - Cr[tc][r]);
                    const float b = fabsf(mr) + fabsf((float)Ci[tc][r]) + ((i == j) ? 1e-6f : 0.0f);
                    u[r] = fmaf(b, vj, u[r]);
                }
            }
            // rows live in the 16 lanes of one DPP row (FP64 layout) or of one
            // quarter (FP32 layout): either way one row of 16 lanes
#pragma unroll
            for (int r = 0; r < 4; ++r) u[r] = row16_sum(u[r]);
            // from v = 1 the first bound is the largest row sum of B
            float ratio = 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float vi = (it == 0) ? 1.0f : (float)v[16 * w + MT<T>::row(lg, r)];
                const float rr = u[r] * __builtin_amdgcn_rcpf(vi);
                ratio = rr > ratio ? rr : ratio;
            }
            const double m = wave_max_pos((double)ratio);
            if (l == 0) sh.wmax[it & 1][w] = m;
            if (lj == 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) sh.vbuf[(it + 1) & 1][16 * w + MT<T>::row(lg, r)] = u[r];
            }
            __syncthreads();
            double c = 0.0, co = 0.0;
            for (int x = 0; x < NT; ++x) c = sh.wmax[it & 1][x] > c ? sh.wmax[it & 1][x] : c;
            for (int k = 0; k < n_peers; ++k)
                for (int x = 0; x < NT; ++x)
                    co = peers[k].wmax[it & 1][x] > co ? peers[k].wmax[it & 1][x] : co;
            // rcpf is within 1 ulp; the factor covers it and the sums' rounding
            cw = c * (1.0 + 1e-5);
            // uniform: every thread of the work-group read the same wmax
            if (cw < accept && co * (1.0 + 1e-5) < accept) break;
        }
        return cw;
    } else {
        // u = B v over the wave's rows (row sums across the 16 lanes of a row),
        // the wave's largest quotient u_i / v_i, the next v; then the block's bound
        // after a barrier.  Returns true when the bound (and every peer's) passes.
        auto finish = [&](int it, float (&u)[4], const double *v) __attribute__((always_inline)) {
            // rows live in the 16 lanes of one DPP row (FP64 layout) or of one
            // quarter (FP32 layout): either way one row of 16 lanes
#pragma unroll
            for (int r = 0; r < 4; ++r) u[r] = row16_sum(u[r]);
            float ratio = 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // from v = 1 the first bound is the largest row sum of B
                const float rr = v ? u[r] * __builtin_amdgcn_rcpf((float)v[16 * w + MT<T>::row(lg, r)]) : u[r];
                ratio = rr > ratio ? rr : ratio;
            }
            const double m = wave_max_pos((double)ratio);
            if (l == 0) sh.wmax[it & 1][w] = m;
            if (lj == 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) sh.vbuf[(it + 1) & 1][16 * w + MT<T>::row(lg, r)] = u[r];
            }
            __syncthreads();
            double c = 0.0, co = 0.0;
            for (int x = 0; x < NT; ++x) c = sh.wmax[it & 1][x] > c ? sh.wmax[it & 1][x] : c;
            for (int k = 0; k < n_peers; ++k)
                for (int x = 0; x < NT; ++x)
                    co = peers[k].wmax[it & 1][x] > co ? peers[k].wmax[it & 1][x] : co;
            // rcpf is within 1 ulp; the factor covers it and the sums' rounding
            cw = c * (1.0 + 1e-5);
            // uniform: every thread of the work-group read the same wmax
            return cw < accept && co * (1.0 + 1e-5) < accept;
        };
        // step 0 from v = 1, without reading it (no barrier before it), by
        // cert_rowsums0
        {
            float u[4];
            cert_rowsums0_at<T, NP>(__builtin_amdgcn_readfirstlane(w), Cr, Ci, lj, lg, u);
            if (finish(0, u, nullptr)) return cw;
        }
        for (int it = 1; it < iters; ++it) {
            const double *v = sh.vbuf[it & 1];
            float u[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int tc = 0; tc < NT; ++tc) {
                const int j = 16 * tc + lj;
                const float vj = (float)v[j];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 16 * w + MT<T>::row(lg, r);
                    const float mr = (float)(((i == j) ? T(1) : T(0)) - Cr[tc][r]);
                    const float b = fabsf(mr) + fabsf((float)Ci[tc][r]) + ((i == j) ? 1e-6f : 0.0f);
                    u[r] = fmaf(b, vj, u[r]);
                }
            }
            if (finish(it, u, v)) break;
        }
        return cw;
    }
}

// Invert one 16 x 16 complex tile in place, held by one wave in the MFMA
// accumulator layout (lane: column lj, rows MT<T>::row(lg, r)), by 16 scalar
// Gauss-Jordan steps without pivoting: pivot by readlane, pivot column within
// the lane's 16-lane row by DPP row_newbcast, pivot-row value of the lane's
// column by one bpermute.  The 16 pivots go to pivrow[0..15] (LDS).
//
// Step s as one update of every element, x <- x - c'_i r'_j, with
//   r'_j = r_j / p (j != s), r'_s = 1 + 1/p,   c'_i = c_i (i != s), c'_s = p - 1,
// where p is the pivot, r_j = x_sj and c_i = x_is: this yields x_ij - c_i r_j / p
// off the pivot row and column, r_j / p on the pivot row, -c_i / p on the
// pivot column and 1/p at the pivot, i.e. the in-place Gauss-Jordan step.
template <typename T, int DUMP_N>
__device__ __forceinline__ void gj_tile_invert(typename MT<T>::v4 &Xr, typename MT<T>::v4 &Xi,
                                               cplx<T> *pivrow, cplx<T> *dump, int tid) {
    static_assert((DUMP_N & (DUMP_N - 1)) == 0, "dump entries: a power of two");
    typedef cplx<T> ct;
    const int l = tid & 63, lj = l & 15, lg = l >> 4;
    // the high word of 1 on the lanes of the pivot column (lj == s), else 0;
    // rotated one lane along the row after each step (row_ror:1: lane lj
    // takes the value of lane lj - 1 mod 16), instead of a compare and select
    // per step
    constexpr int ONE_HI = sizeof(T) == 8 ? 0x3ff00000 : 0x3f800000;
    int one_hi = (lj == 0) ? ONE_HI : 0;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int ls = MT<T>::lg_of(s), rs = MT<T>::r_of(s);
        const int src = s + 16 * ls;
        const ct piv = {readlane_v(Xr[rs], src), readlane_v(Xi[rs], src)};
        // every lane stores its element of row rs per step, the lane that
        // holds the pivot into pivrow[s] and the others into dump (free
        // during the sweep): no branch per step, and no gathering of the
        // pivots from the scalar registers into lanes (a select reads one
        // scalar register at most, so that took four copies and four selects
        // per step)
        {
            cplx<T> *dst = (l == src) ? pivrow + s : dump + (l & (DUMP_N - 1));
            put_split<T>(*dst, Xr[rs], Xi[rs]);
        }
        const int from = (lj + 16 * ls) << 2;
        const ct rr = {bperm_v(from, Xr[rs]), bperm_v(from, Xi[rs])};
        ct c[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) c[r] = {row_bcast_v(Xr[r], s), row_bcast_v(Xi[r], s)};
        const ct ip = recip_fast(piv);
        // r'_j = r_j / p; on the pivot column r_s = p, and (r_s + 1) / p = 1 + 1/p
        T one_s;
        if constexpr (sizeof(T) == 8) one_s = __hiloint2double(one_hi, 0);
        else one_s = __int_as_float(one_hi);
        const ct rp = ct{rr.re + one_s, rr.im} * ip;
        one_hi = __builtin_amdgcn_mov_dpp(one_hi, 0x121, 0xf, 0xf, false);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            ct cf = c[r];
            if (r == rs) cf.re -= (lg == ls) ? T(1) : T(0);
            const ct x = fms(ct{Xr[r], Xi[r]}, cf, rp);
            Xr[r] = x.re;
            Xi[r] = x.im;
        }
    }
}

// Wave priority around a tile inversion, FP32 sweeps only: the inverting
// wave is the item's critical path, and raising its issue priority over the
// other waves of the SIMD (other items' updates) measured 3-5 % faster for
// the FP32 and refined builds; in the FP64 builds it measured slower (and
// the four-wave build spilled more around the priority changes).
template <typename T, bool HIGH> __device__ __forceinline__ void inversion_priority() {
    if constexpr (sizeof(T) == 4) __builtin_amdgcn_s_setprio(HIGH ? 2 : 0);
}

// Scheduling pattern for the current scheduling region: NM times one matrix
// instruction followed by up to NO vector-ALU, scalar-ALU, LDS or
// transcendental instructions, so that a wave's matrix products issue between
// the steps of an independent scalar chain instead of all before or after it.
template <int NM, int NO> __device__ __forceinline__ void interleave_mfma() {
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);    // MFMA
        __builtin_amdgcn_sched_group_barrier(0x486, NO, 0);   // VALU | SALU | DS | TRANS
    }
}

// In-place blocked Gauss-Jordan sweep without pivoting.  Contains barriers.
//
// The tiles rotate: at step t, Cr[p] holds tile column (p + t) mod NT and the
// current column t is always Cr[0].  With the loop unrolled the rotation is
// register renaming; it keeps the loop body free of run-time register
// indexing should the loop ever be rolled to save instruction cache.
template <typename T, int NP>
__device__ __forceinline__ void gj_sweep_plain(typename MT<T>::v4 (&Cr)[NP / 16],
                                         typename MT<T>::v4 (&Ci)[NP / 16], GjShared<T, NP> &sh,
                                         int tid) {
    constexpr int NT = NP / 16;
    typedef cplx<T> ct;
    typedef typename MT<T>::v4 v4;
    const int w = tid >> 6, l = tid & 63, lj = l & 15, lg = l >> 4;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (w == t) {
#pragma unroll
            for (int p = 1; p < NT; ++p) {
                const int c = (p + t) % NT;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    put_split<T>(sh.Rb[MT<T>::row(lg, r)][16 * c + lj], Cr[p][r], Ci[p][r]);
            }
            v4 &Xr = Cr[0];
            v4 &Xi = Ci[0];
            gj_tile_invert<T, GjShared<T, NP>::DUMP_N>(Xr, Xi, sh.pivv + 16 * t, sh.dump(), tid);
#pragma unroll
            for (int r = 0; r < 4; ++r) put_split<T>(sh.Xw[t][MT<T>::row(lg, r)][lj], Xr[r], Xi[r]);
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) put_split<T>(sh.Xw[w][MT<T>::row(lg, r)][lj], Cr[0][r], Ci[0][r]);
        }
        __syncthreads();

        if constexpr (sizeof(T) == 4) {
            T gr[4], gim[4];
            if (w == t) {
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    ct g = sh.Xw[t][lj][4 * k4 + lg];
                    if (lj == 4 * k4 + lg) g.re -= T(1);
                    gr[k4] = g.re;
                    gim[k4] = g.im;
                }
            } else {
                // G = -A_wt A_tt^-1 in the 3M form: T1 = a_re b_re, T2 = a_im b_im,
                // P3 = (a_re + a_im)(b_re + b_im); G = (T2 - T1, T1 + T2 - P3)
                v4 T1 = {0, 0, 0, 0}, T2 = {0, 0, 0, 0}, P3 = {0, 0, 0, 0};
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    const ct xa = sh.Xw[w][lj][4 * k4 + lg];
                    const ct b = sh.Xw[t][4 * k4 + lg][lj];
                    T1 = MT<T>::mma(xa.re, b.re, T1);
                    T2 = MT<T>::mma(xa.im, b.im, T2);
                    P3 = MT<T>::mma(xa.re + xa.im, b.re + b.im, P3);
                }
                const v4 Gr = T2 - T1, Gi = T1 + T2 - P3;
                Cr[0] = Gr;
                Ci[0] = Gi;
                wave_sync_lds();
#pragma unroll
                for (int r = 0; r < 4; ++r) put_split<T>(sh.Xw[w][MT<T>::row(lg, r)][lj], Gr[r], Gi[r]);
                wave_sync_lds();
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    const ct g = sh.Xw[w][lj][4 * k4 + lg];
                    gr[k4] = g.re;
                    gim[k4] = g.im;
                }
            }
#pragma unroll
            for (int p = 1; p < NT; ++p) {
                const int c = (p + t) % NT;
                // three real products per complex one (3M form): T1 = G_re B_re,
                // T2 = G_im B_im, Ci += (G_re + G_im)(B_re + B_im) - T1 - T2.
                // In FP32 the extra accumulators fit the register budget and
                // save a quarter of the matrix products (measured 6 % faster);
                // in FP64 they spill and the four-product form is faster.
                v4 T1 = {0, 0, 0, 0}, T2 = {0, 0, 0, 0};
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    const ct b = sh.Rb[4 * k4 + lg][16 * c + lj];
                    T1 = MT<T>::mma(gr[k4], b.re, T1);
                    T2 = MT<T>::mma(gim[k4], b.im, T2);
                    Ci[p] = MT<T>::mma(gr[k4] + gim[k4], b.re + b.im, Ci[p]);
                }
                Cr[p] += T1 - T2;
                Ci[p] -= T1 + T2;
            }
        } else {
            // G_w in LDS (this wave's exchange slot): the inverse for w = t (its
            // diagonal minus one below), -A_wt A_tt^-1 formed here for the others
            if (w != t) {
                // G = -A_wt A_tt^-1 in the 3M form: T1 = a_re b_re, T2 = a_im b_im,
                // P3 = (a_re + a_im)(b_re + b_im); G = (T2 - T1, T1 + T2 - P3)
                v4 T1 = {0, 0, 0, 0}, T2 = {0, 0, 0, 0}, P3 = {0, 0, 0, 0};
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    const ct xa = sh.Xw[w][lj][4 * k4 + lg];
                    const ct b = sh.Xw[t][4 * k4 + lg][lj];
                    T1 = MT<T>::mma(xa.re, b.re, T1);
                    T2 = MT<T>::mma(xa.im, b.im, T2);
                    P3 = MT<T>::mma(xa.re + xa.im, b.re + b.im, P3);
                }
                const v4 Gr = T2 - T1, Gi = T1 + T2 - P3;
                Cr[0] = Gr;
                Ci[0] = Gi;
                wave_sync_lds();
#pragma unroll
                for (int r = 0; r < 4; ++r) put_split<T>(sh.Xw[w][MT<T>::row(lg, r)][lj], Gr[r], Gi[r]);
                wave_sync_lds();
            }
            // FP64: the A operand comes from LDS one k-slice at a time, used
            // across the tiles, so no copy of G is held through the update
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                ct g = sh.Xw[w][lj][4 * k4 + lg];
                if (w == t && lj == 4 * k4 + lg) g.re -= T(1);
#pragma unroll
                for (int p = 1; p < NT; ++p) {
                    const int c = (p + t) % NT;
                    const ct b = sh.Rb[4 * k4 + lg][16 * c + lj];
                    Cr[p] = MT<T>::mma(g.re, b.re, Cr[p]);
                    Cr[p] = MT<T>::mma_na(g.im, b.im, Cr[p]);
                    Ci[p] = MT<T>::mma(g.re, b.im, Ci[p]);
                    Ci[p] = MT<T>::mma(g.im, b.re, Ci[p]);
                }
            }
        }
        __syncthreads();
        // rotate: the next tile column moves to Cr[0]
        const v4 r0 = Cr[0], i0 = Ci[0];
#pragma unroll
        for (int p = 0; p + 1 < NT; ++p) {
            Cr[p] = Cr[p + 1];
            Ci[p] = Ci[p + 1];
        }
        Cr[NT - 1] = r0;
        Ci[NT - 1] = i0;
    }
}

// The same sweep with look-ahead: the diagonal tile of step t + 1 belongs to
// wave t + 1, which updates that tile first during step t and then inverts it
// while the rest of its update is still in the matrix pipe, so the scalar
// inversion (vector ALU and lane exchanges) overlaps matrix work instead of
// running alone between two barriers; only the first tile is inverted before
// the loop.  The look-ahead wave holds the inversion's temporaries next to its
// update operands, so it pays only where that fits the register budget.
template <typename T, int NP>
__device__ __forceinline__ void gj_sweep_lookahead(typename MT<T>::v4 (&Cr)[NP / 16],
                                         typename MT<T>::v4 (&Ci)[NP / 16], GjShared<T, NP> &sh,
                                         int tid) {
    constexpr int NT = NP / 16;
    typedef cplx<T> ct;
    typedef typename MT<T>::v4 v4;
    const int w = tid >> 6, l = tid & 63, lj = l & 15, lg = l >> 4;
    if (w == 0) {
        inversion_priority<T, true>();
        gj_tile_invert<T, GjShared<T, NP>::DUMP_N>(Cr[0], Ci[0], sh.pivv, sh.dump(), tid);
        inversion_priority<T, false>();
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (w == t) {
#pragma unroll
            for (int p = 1; p < NT; ++p) {
                const int c = (p + t) % NT;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    put_split<T>(sh.Rb[MT<T>::row(lg, r)][16 * c + lj], Cr[p][r], Ci[p][r]);
            }
        }
        // every wave publishes its tile of column t: the inverse for w = t
#pragma unroll
        for (int r = 0; r < 4; ++r) put_split<T>(sh.Xw[w][MT<T>::row(lg, r)][lj], Cr[0][r], Ci[0][r]);
        __syncthreads();
        // wave t + 1 inverts its next diagonal tile inside this step
        const bool ahead = (t + 1 < NT) && (w == t + 1);

        if constexpr (sizeof(T) == 4) {
            T gr[4], gim[4];
            if (w == t) {
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    ct g = sh.Xw[t][lj][4 * k4 + lg];
                    if (lj == 4 * k4 + lg) g.re -= T(1);
                    gr[k4] = g.re;
                    gim[k4] = g.im;
                }
            } else {
                // G = -A_wt A_tt^-1 in the 3M form: T1 = a_re b_re, T2 = a_im b_im,
                // P3 = (a_re + a_im)(b_re + b_im); G = (T2 - T1, T1 + T2 - P3)
                v4 T1 = {0, 0, 0, 0}, T2 = {0, 0, 0, 0}, P3 = {0, 0, 0, 0};
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    const ct xa = sh.Xw[w][lj][4 * k4 + lg];
                    const ct b = sh.Xw[t][4 * k4 + lg][lj];
                    T1 = MT<T>::mma(xa.re, b.re, T1);
                    T2 = MT<T>::mma(xa.im, b.im, T2);
                    P3 = MT<T>::mma(xa.re + xa.im, b.re + b.im, P3);
                }
                const v4 Gr = T2 - T1, Gi = T1 + T2 - P3;
                Cr[0] = Gr;
                Ci[0] = Gi;
                wave_sync_lds();
#pragma unroll
                for (int r = 0; r < 4; ++r) put_split<T>(sh.Xw[w][MT<T>::row(lg, r)][lj], Gr[r], Gi[r]);
                wave_sync_lds();
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    const ct g = sh.Xw[w][lj][4 * k4 + lg];
                    gr[k4] = g.re;
                    gim[k4] = g.im;
                }
            }
            // three real products per complex one (3M form): T1 = G_re B_re,
            // T2 = G_im B_im, Ci += (G_re + G_im)(B_re + B_im) - T1 - T2.
            // In FP32 the extra accumulators fit the register budget and
            // save a quarter of the matrix products (measured 6 % faster);
            // in FP64 they spill and the four-product form is faster.
            auto update = [&](int p_lo, int p_hi) __attribute__((always_inline)) {
#pragma unroll
                for (int p = 1; p < NT; ++p) {
                    if (p < p_lo || p >= p_hi) continue;
                    const int c = (p + t) % NT;
                    v4 T1 = {0, 0, 0, 0}, T2 = {0, 0, 0, 0};
#pragma unroll
                    for (int k4 = 0; k4 < 4; ++k4) {
                        const ct b = sh.Rb[4 * k4 + lg][16 * c + lj];
                        T1 = MT<T>::mma(gr[k4], b.re, T1);
                        T2 = MT<T>::mma(gim[k4], b.im, T2);
                        Ci[p] = MT<T>::mma(gr[k4] + gim[k4], b.re + b.im, Ci[p]);
                    }
                    Cr[p] += T1 - T2;
                    Ci[p] -= T1 + T2;
                }
            };
            if constexpr (NT > 1) {
                if (ahead) {
                    update(1, 2);
                    __builtin_amdgcn_sched_barrier(0);
                    inversion_priority<T, true>();
                    gj_tile_invert<T, GjShared<T, NP>::DUMP_N>(Cr[1], Ci[1], sh.pivv + 16 * (t + 1), sh.dump(), tid);
                    inversion_priority<T, false>();
                    update(2, NT);
                    interleave_mfma<12 * (NT - 2), 20>();
                } else {
                    update(1, NT);
                }
            }
        } else {
            // G_w in LDS (this wave's exchange slot): the inverse for w = t (its
            // diagonal minus one below), -A_wt A_tt^-1 formed here for the others
            if (w != t) {
                // G = -A_wt A_tt^-1 in the 3M form: T1 = a_re b_re, T2 = a_im b_im,
                // P3 = (a_re + a_im)(b_re + b_im); G = (T2 - T1, T1 + T2 - P3)
                v4 T1 = {0, 0, 0, 0}, T2 = {0, 0, 0, 0}, P3 = {0, 0, 0, 0};
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    const ct xa = sh.Xw[w][lj][4 * k4 + lg];
                    const ct b = sh.Xw[t][4 * k4 + lg][lj];
                    T1 = MT<T>::mma(xa.re, b.re, T1);
                    T2 = MT<T>::mma(xa.im, b.im, T2);
                    P3 = MT<T>::mma(xa.re + xa.im, b.re + b.im, P3);
                }
                const v4 Gr = T2 - T1, Gi = T1 + T2 - P3;
                Cr[0] = Gr;
                Ci[0] = Gi;
                wave_sync_lds();
#pragma unroll
                for (int r = 0; r < 4; ++r) put_split<T>(sh.Xw[w][MT<T>::row(lg, r)][lj], Gr[r], Gi[r]);
                wave_sync_lds();
            }
            // FP64: the A operand comes from LDS one k-slice at a time, used
            // across the tiles, so no copy of G is held through the update
            auto update = [&](int p_lo, int p_hi) __attribute__((always_inline)) {
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    ct g = sh.Xw[w][lj][4 * k4 + lg];
                    if (w == t && lj == 4 * k4 + lg) g.re -= T(1);
#pragma unroll
                    for (int p = 1; p < NT; ++p) {
                        if (p < p_lo || p >= p_hi) continue;
                        const int c = (p + t) % NT;
                        const ct b = sh.Rb[4 * k4 + lg][16 * c + lj];
                        Cr[p] = MT<T>::mma(g.re, b.re, Cr[p]);
                        Cr[p] = MT<T>::mma_na(g.im, b.im, Cr[p]);
                        Ci[p] = MT<T>::mma(g.re, b.im, Ci[p]);
                        Ci[p] = MT<T>::mma(g.im, b.re, Ci[p]);
                    }
                }
            };
            if constexpr (NT > 1) {
                if (ahead) {
                    update(1, 2);
                    __builtin_amdgcn_sched_barrier(0);
                    inversion_priority<T, true>();
                    gj_tile_invert<T, GjShared<T, NP>::DUMP_N>(Cr[1], Ci[1], sh.pivv + 16 * (t + 1), sh.dump(), tid);
                    inversion_priority<T, false>();
                    update(2, NT);
                    interleave_mfma<16 * (NT - 2), 28>();
                } else {
                    update(1, NT);
                }
            }
        }
        __syncthreads();
        // rotate: the next tile column moves to Cr[0]
        const v4 r0 = Cr[0], i0 = Ci[0];
#pragma unroll
        for (int p = 0; p + 1 < NT; ++p) {
            Cr[p] = Cr[p + 1];
            Ci[p] = Ci[p + 1];
        }
        Cr[NT - 1] = r0;
        Ci[NT - 1] = i0;
    }
}

// Dispatch: LA selects the look-ahead sweep (measured per build).
template <typename T, int NP, bool LA>
__device__ __forceinline__ void gj_sweep(typename MT<T>::v4 (&Cr)[NP / 16],
                                         typename MT<T>::v4 (&Ci)[NP / 16], GjShared<T, NP> &sh,
                                         int tid) {
    if constexpr (LA) gj_sweep_lookahead<T, NP>(Cr, Ci, sh, tid);
    else gj_sweep_plain<T, NP>(Cr, Ci, sh, tid);
}

// log det from the scalar pivots (no row exchanges), by one wave.  det D is
// the product of the pivots: each lane multiplies its pivots (two at NP > 64)
// and scales the product by a power of two to max(|re|, |im|) in [0.5, 1)
// (so |p| in [0.5, sqrt 2): 64 such factors neither overflow nor underflow),
// the lanes' factors are multiplied by a tree (DPP within each 16-lane row,
// then the four row products) and their exponents summed; one complex
// logarithm follows, log |det| = log |P| + E ln 2 with ln 2 split in a high
// part exact in products with small integers and a low part (Cody and
// Waite), arg det = arg P.  The status is decided by the sign of Re det =
// 2^E Re P: 0 inside (Re det > 0), 1 outside, 2 non-finite.  Uniform result.
template <int CTRL> __device__ __forceinline__ cd dpp_c(cd v) {
    return {dpp_d<CTRL>(v.re), dpp_d<CTRL>(v.im)};
}
__device__ __forceinline__ cd readlane_c(cd v, int lane) {
    return {readlane_v(v.re, lane), readlane_v(v.im, lane)};
}
template <int NP, typename T>
__device__ __forceinline__ int gj_logdet(const cplx<T> *pivv, cd *out_logdet, int tid) {
    const int l = tid & 63;
    auto piv = [&](int k) { return cd{(double)pivv[k].re, (double)pivv[k].im}; };
    cd p = (l < NP) ? piv(l) : cd{1.0, 0.0};
    if constexpr (NP > 64) {
        if (l + 64 < NP) p = p * piv(l + 64);
    }
    int e = 0;
    (void)frexp(fmax(fabs(p.re), fabs(p.im)), &e);   // 0 for 0, inf and NaN: kept as they are
    p = {ldexp(p.re, -e), ldexp(p.im, -e)};
    p = p * dpp_c<0xB1>(p);    // quad_perm [1,0,3,2]
    p = p * dpp_c<0x4E>(p);    // quad_perm [2,3,0,1]
    p = p * dpp_c<0x124>(p);   // row_ror:4
    p = p * dpp_c<0x128>(p);   // row_ror:8
    const cd P = (readlane_c(p, 0) * readlane_c(p, 16)) * (readlane_c(p, 32) * readlane_c(p, 48));
    const double E = wave_sum((double)e);            // exact: integers below 2^53
    constexpr double LN2_HI = 0x1.62e42fefa3800p-1;  // ln 2 to 42 bits: E * LN2_HI exact for |E| < 2^11
    constexpr double LN2_LO = 0x1.ef35793c76730p-45; // ln 2 - LN2_HI
    const double lre = fma(E, LN2_HI, fma(E, LN2_LO, log(hypot(P.re, P.im))));
    const double ph = atan2(P.im, P.re);
    *out_logdet = cd{lre, ph};
    if (!isfinite(lre) || !isfinite(ph)) return 2;
    return (P.re > 0.0) ? 0 : 1;
}

}  // namespace df
