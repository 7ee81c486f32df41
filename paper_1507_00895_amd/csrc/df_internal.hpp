// Kernel argument blocks and launcher declarations of libdf (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "df_device.hpp"

namespace df {

// fermionic index into the vertex and bubble arrays; FULL: n_nu equals the
// padded size and no index leaves the window
template <bool FULL> __device__ __forceinline__ int clamp_nu(int j, int nm1) {
    if constexpr (FULL) return j;
    else return j < nm1 ? j : nm1;
}

struct DualGfArgs {
    Grid grid;
    int n_nu;
    const double *g, *delta, *eps;   // inputs (unused with from_gd)
    const double *sigma;             // may be null (Sigma~ = 0)
    const double *gd_in;             // with from_gd: G~ to transform
    double *gd_out;                  // may be null
    double *gr_out;                  // may be null: [n_nu][N] inverse FFT of G~
    int from_gd;
};

struct BubbleArgs {
    Grid grid;
    int n_nu, n_om;
    double beta;
    const double *gr;                // [n_nu][N]
    double *chi;                     // [n_om][n_nu][N]
};

struct SigmaArgs {
    Grid grid;
    int n_nu, n_om;
    int chunk_len, n_chunks;
    double beta;
    const double *w;                 // [2][n_om][n_nu][N]
    const double *gr;                // [n_nu][N]
    double *part;                    // [n_chunks][n_nu][N]
};

struct ReduceMixArgs {
    size_t count;                    // n_nu * N complex elements
    int n_chunks;
    double alpha;
    const double *part;
    double *sigma_calc;              // may be null
    double *sigma;                   // may be null: no mixing
    double *norm_part;               // [gridDim][2]
};

// Anderson acceleration (df_accel.hip): ring of up to kAccMaxSlots iterates
constexpr int kAccMaxSlots = 9;

struct AccRecordArgs {
    size_t count;                    // n_nu * N complex elements
    const double *x, *fx;            // current iterate, F(iterate)
    double *xh, *rh;                 // rings [kAccMaxSlots][count]
    int slot, n_slots;               // slot written now; slots in use (incl. it)
    double *part;                    // [blocks][kAccMaxSlots] partial dots
    double *dots;                    // [kAccMaxSlots]: Re <r_j, r_slot>
};

struct AccCombineArgs {
    size_t count;
    const double *xh, *rh;
    int n_slots;
    double coef[kAccMaxSlots];       // real weights, summing to one
    double alpha;
    double *x;                       // in: x_k, out: x_{k+1}
    double *norm_part;               // [blocks][2]
};

struct GammaPrepArgs {
    int n_nu, n_om;
    const double *guu, *gud;
    double *gdm;                     // [2][n_om][n_nu][n_nu]
    double *pdm;                     // [2][n_om][n_nu][n_nu]
    double *gtr;                     // [2][n_om][n_nu][n_nu] (may be null)
    float *gp32;                     // [2][n_om][n_nu][n_nu] (gamma, gamma_ij gamma_ji) in FP32, or null
    float *gtr32;                    // [2][n_om][n_nu][n_nu] gamma transposed in FP32, or null
};

// One instance of a fused multi-instance ladder launch (device-side table).
struct LadderInst {
    const double *gdm, *pdm, *gtr, *chi;
    const float *gp32, *gtr32;
    double *w, *logdet;
    int8_t *status;
    int *count;                      // ladders outside the radius (atomic)
    int n_nu, n_om, N;
    int item0;                       // first global item of this instance
    const int *qlist;                // symmetry-reduced launch (else null): solved q
    int n_q, im0;                    // their count; first solved bosonic index
};

struct LadderArgs {
    const double *gdm;               // [2][n_om][n_nu][n_nu]
    const double *pdm;               // [2][n_om][n_nu][n_nu]
    const double *chi;               // [n_om][n_nu][N]
    double *w;                       // [2][n_om][n_nu][N]
    double *logdet;                  // [2][n_om][N] or null
    int8_t *status;                  // [2][n_om][N] or null
    int n_nu, n_om, N;
    int item0, n_items;              // items are (c, m, q), q fastest
    int *fallback_count;             // may be null: atomically counts status != 0
    const double *gtr;               // [2][n_om][n_nu][n_nu] gamma transposed (gjb kernel)
    int *queue;                      // certified kernels: uncertified items are appended here
    int *queue_count;                // its length (zeroed before the launch)
    int *near_queue;                 // refined kernel: items whose certificate bound is
    int *near_count;                 // >= CERT_NEAR_MIXED go here for the FP64 kernel
    const int *in_queue;             // queue launches: process these items ...
    const int *in_count;             // ... (count on the device) instead of item0 + block
    int *claim;                      // persistent launches: per-XCD item counters [kXcd]
                                     // (zeroed before the launch); null: static mapping
    const LadderInst *insts;         // non-null: fused launch over n_insts instances,
    int n_insts;                     // items are global; the fields above are resolved per item
    const float *gp32;               // FP32 ladder: (gamma, gamma_ij gamma_ji) pairs, FP32
    const float *gtr32;              // FP32 ladder: gamma transposed, FP32
    const int *qlist;                // non-null: symmetry-reduced items (see item_coords)
    int n_q, im0;
    int full;                        // 1: every instance of the launch has n_nu equal to the
                                     // padded size (the mask-free build runs)
};

// Fused launches: find the instance of a global item, fill the per-instance
// fields of a, return the item's index within its instance.  The item is
// uniform over the work-group and the table is read only: it is read through
// the constant address space, so that the instance's fields arrive in scalar
// registers (vector loads would hold them, and the item coordinates built
// from them, in vector registers for the whole item).
typedef __attribute__((address_space(4))) const LadderInst *ConstLadderInstPtr;
__device__ __forceinline__ int resolve_item(LadderArgs &a, int item) {
    if (!a.insts) return item;
    const ConstLadderInstPtr tab = (ConstLadderInstPtr)(const void *)a.insts;
    int k = 0;
    while (k + 1 < a.n_insts && tab[k + 1].item0 <= item) ++k;
    const auto &d = tab[k];
    a.gdm = d.gdm;
    a.pdm = d.pdm;
    a.gtr = d.gtr;
    a.gp32 = d.gp32;
    a.gtr32 = d.gtr32;
    a.chi = d.chi;
    a.w = d.w;
    a.logdet = d.logdet;
    a.status = d.status;
    a.fallback_count = d.count;
    a.n_nu = d.n_nu;
    a.n_om = d.n_om;
    a.N = d.N;
    a.qlist = d.qlist;
    a.n_q = d.n_q;
    a.im0 = d.im0;
    return item - d.item0;
}

// An item's (c n_om + m index, q).  Full launches: items are (c, m, q), q
// fastest.  Symmetry-reduced launches (qlist set): items are (c, m index >= im0,
// k < n_q), k fastest, with q = qlist[k] - one q per point-group orbit and the
// bosonic frequencies Omega >= 0; the others follow by symmetry (k_sym_expand).
// The coordinates are uniform over the work-group: readfirstlane puts them
// (and every address built from them) in scalar registers.  Integer division
// is expanded with vector instructions, and without it the quotients stayed in
// vector registers for the whole item.
__device__ __forceinline__ void item_coords(const LadderArgs &a, int item, int *cm, int *q) {
    if (!a.qlist) {
        *q = __builtin_amdgcn_readfirstlane(item % a.N);
        *cm = __builtin_amdgcn_readfirstlane(item / a.N);
        return;
    }
    const int k = item % a.n_q, r = item / a.n_q;
    const int nm = a.n_om - a.im0;
    *q = __builtin_amdgcn_readfirstlane(a.qlist[k]);
    *cm = __builtin_amdgcn_readfirstlane((r / nm) * a.n_om + a.im0 + r % nm);
}

// Representative of q's orbit under the point group of the hypercubic lattice
// (axis permutations and k_a -> -k_a): per axis the smaller of c_a and nk - c_a,
// sorted ascending from axis 0.  Host and device use this same function.
__host__ __device__ inline int canonical_q(int q, int D, int lognk) {
    const int nk = 1 << lognk;
    int r[4] = {0, 0, 0, 0};
    for (int a = 0; a < D; ++a) {
        const int c = (q >> (a * lognk)) & (nk - 1);
        const int m = (nk - c) & (nk - 1);
        r[a] = c < m ? c : m;
    }
    for (int i = 1; i < D; ++i)          // insertion sort of at most four values
        for (int j = i; j > 0 && r[j - 1] > r[j]; --j) {
            const int t = r[j];
            r[j] = r[j - 1];
            r[j - 1] = t;
        }
    int out = 0;
    for (int a = 0; a < D; ++a) out |= r[a] << (a * lognk);
    return out;
}

struct SymTableArgs {
    int D, lognk, N;
    int *qrep;                       // [N]: representative of each q
    int *qlist;                      // [n_irr]: the representatives, ascending
};

struct SymExpandArgs {
    int n_nu, n_om, N, im0;
    const int *qrep;
    double *w;                       // [2][n_om][n_nu][N]
    double *logdet;                  // [2][n_om][N] or null
    int8_t *status;                  // [2][n_om][N] or null
};

// Work-group b of a launch runs on XCD b % 8 (the dispatcher deals work-groups
// round-robin over the eight XCDs, each with its own L2).  Give every XCD one
// contiguous range of the n items instead, so that the neighbouring q of one
// (channel, Om) - which share the cache lines of chi and W - meet in one L2.
constexpr int kXcd = 8;
__device__ __forceinline__ int xcd_item(int b, int n) {
    const int per = n / kXcd, rem = n % kXcd;
    const int x = b % kXcd, i = b / kXcd;
    return x * per + (x < rem ? x : rem) + i;
}

// Items of a certified ladder launch, handed to body(global item) one at a
// time; uniform over the work-group, which may run several items in turn
// (LDS is reused: a barrier separates them).  The body appears once, so the
// compiler inlines it once.
//   in_queue set: the device-side queue of another kernel, grid-stride.
//   claim null:   XCD x's contiguous range (as xcd_item) split over the
//                 work-groups on that XCD; with one work-group per item this
//                 is exactly the mapping of xcd_item.
//   claim set:    persistent work-groups take the next item of their XCD's
//                 range from its counter, then help the other XCDs' ranges.
// k counts the items this work-group has run; tries (thread 0 only) the XCD
// ranges it found empty.  Contains barriers when claim is set.
__device__ __forceinline__ int next_item(const LadderArgs &a, int k, int *tries, int *s_item) {
    if (a.in_queue) {
        const int u = (int)blockIdx.x + k * (int)gridDim.x;
        return u < *a.in_count ? a.in_queue[u] : -1;
    }
    const int n = a.n_items, per = n / kXcd, rem = n % kXcd;
    const int x = blockIdx.x % kXcd;
    if (!a.claim) {
        const int len = per + (x < rem ? 1 : 0), start = x * per + (x < rem ? x : rem);
        const int wgs = ((int)gridDim.x - x + kXcd - 1) / kXcd;   // work-groups on XCD x
        const int i = (int)blockIdx.x / kXcd + k * wgs;
        return i < len ? a.item0 + start + i : -1;
    }
    if (threadIdx.x == 0) {
        int item = -1;
        while (*tries < kXcd) {
            const int xx = (x + *tries) % kXcd;
            const int len = per + (xx < rem ? 1 : 0);
            const int c = atomicAdd(a.claim + xx, 1);
            if (c < len) {
                item = a.item0 + xx * per + (xx < rem ? xx : rem) + c;
                break;
            }
            ++*tries;
        }
        *s_item = item;
    }
    __syncthreads();
    const int item = *s_item;
    __syncthreads();
    return item;
}

template <typename F>
__device__ __forceinline__ void for_each_item(const LadderArgs &a, F &&body) {
    __shared__ int s_item;
    int tries = 0;
    for (int k = 0;; ++k) {
        const int item = __builtin_amdgcn_readfirstlane(next_item(a, k, &tries, &s_item));
        if (item < 0) break;
        body(item);
        __syncthreads();
    }
}

// Lattice observables (df_lattice.hip)
struct LatticeFieldArgs {
    int n_nu, N;
    double beta, mu;
    const double *g, *delta, *eps, *sigma;   // sigma may be null (Sigma~ = 0)
    double *sigma_lat, *g_lat;               // outputs, may be null
    double *gl, *gd, *fg;                    // [n_nu][N] G_lat, G~, frak G
};

struct LatticeChiArgs {
    int n_nu, N, i0;                         // i0: index of Omega = 0 in the vertex arrays
    int item0;                               // first item (c * N + q) of this launch
    const double *guu, *gud;                 // [n_om][n_nu][n_nu]
    const double *L, *chi0;                  // [n_nu][N]
    double *work;                            // [items][n_nu][n_nu + 1] complex
    double *lad;                             // [2][N]
};

struct LatticeSumArgs {
    int n_nu, N;
    const double *bub, *lad;                 // [n_nu][N], [2][N]
    double *chi_ch, *chi_sp;                 // [N], may be null
};

hipError_t launch_dual_gf(const DualGfArgs &a, hipStream_t s);
hipError_t launch_bubble(const BubbleArgs &a, hipStream_t s);
hipError_t launch_sigma_part(const SigmaArgs &a, hipStream_t s);
hipError_t launch_reduce_mix(const ReduceMixArgs &a, int blocks, hipStream_t s);
hipError_t launch_norm_final(const double *part, int n_part, double *out, hipStream_t s);
hipError_t launch_acc_record(const AccRecordArgs &a, int blocks, hipStream_t s);
hipError_t launch_acc_combine(const AccCombineArgs &a, int blocks, hipStream_t s);
hipError_t launch_gamma_prep(const GammaPrepArgs &a, hipStream_t s);
hipError_t set_fft_lds_limits();

// padded ladder size for n_nu, 0 if unsupported
int ladder_padded_size(int n_nu);
hipError_t launch_ladder_fp64(const LadderArgs &a, hipStream_t s);
// MFMA blocked Gauss-Jordan variant (n_nu <= 64)
int ladder_mfma_padded_size(int n_nu);
hipError_t launch_ladder_mfma_f64(const LadderArgs &a, hipStream_t s);
// certified pivot-free blocked Gauss-Jordan (n_nu <= 128); occ = 3 / 4 select
// the builds capped at three / four waves per SIMD (n_nu <= 64), 0 the
// compiler's budget; grid: work-groups of the launch (n_items for one per
// item; fewer with a.claim set for persistent work-groups, or a queue launch)
int ladder_gjb_padded_size(int n_nu);
bool ladder_gjb_has_occ3(int n_nu);
hipError_t launch_ladder_gjb_f64(const LadderArgs &a, int occ, int grid, hipStream_t s);
int ladder_gjb_occupancy(int n_nu, int occ);   // resident work-groups per CU
// mixed precision: FP32 certified sweep + one FP64 residual correction, and
// the FP32 sweep alone (n_nu <= 128); occ as above (refined: 0, 3 up to 96,
// 4 up to 64; FP32: 0, and 4, 5 up to 64)
int ladder_mixed_padded_size(int n_nu);
int ladder_fp32_padded_size(int n_nu);
bool ladder_mixed_has_occ(int n_nu, int occ);
bool ladder_fp32_has_occ(int n_nu, int occ);
hipError_t launch_ladder_mixed(const LadderArgs &a, int occ, int grid, hipStream_t s);
hipError_t launch_ladder_fp32(const LadderArgs &a, int occ, int grid, hipStream_t s);
int ladder_mixed_occupancy(int n_nu, int occ);
int ladder_fp32_occupancy(int n_nu, int occ);
// pivoting kernel over a device-side queue of items (grid-stride, fixed grid)
hipError_t launch_ladder_fp64_queue(const LadderArgs &a, int blocks, hipStream_t s);
hipError_t launch_zero_ints(int *p, int n, hipStream_t s);
hipError_t launch_sym_tables(const SymTableArgs &a, hipStream_t s);
hipError_t launch_sym_expand(const SymExpandArgs &a, hipStream_t s);
hipError_t launch_lattice_fields(const LatticeFieldArgs &a, hipStream_t s);
hipError_t launch_lattice_chi_ladder(const LatticeChiArgs &a, int items, hipStream_t s);
hipError_t launch_lattice_chi_sum(const LatticeSumArgs &a, hipStream_t s);

}  // namespace df
