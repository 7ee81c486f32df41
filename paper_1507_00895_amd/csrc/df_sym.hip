// Symmetry reduction of the ladder step (eqs. dual_ladder, lin_alg_inv).
//
// With point-group symmetric G~ (and so chi~(Rq) = chi~(q) for every R of the
// hypercubic point group) the ladder of q equals that of its orbit's
// representative; with the conjugation symmetries g(-nu) = g(nu)*,
// Delta(-nu) = Delta(nu)*, gamma_{-Om}(-nu, -nu') = gamma_Om(nu, nu')* and
// Sigma~(-nu) = Sigma~(nu)*, the ladder of -Om is the conjugate of that of Om
// with nu -> -nu.  A reduced launch solves one q per orbit and Om >= 0 only;
//   k_sym_tables   representative of every q, and the list of representatives
//   k_sym_expand   fills every other (c, Om, nu, q) of W, log det and status
#include "df_internal.hpp"

namespace df {

// One block of 1024 threads: each thread takes a contiguous run of q, the
// block scans the runs' representative counts, the list comes out ascending.
__global__ __launch_bounds__(1024) void k_sym_tables(SymTableArgs a) {
    __shared__ int cnt[1024];
    const int t = threadIdx.x;
    const int per = (a.N + 1023) / 1024;
    const int q0 = t * per, q1 = min(a.N, q0 + per);
    int c = 0;
    for (int q = q0; q < q1; ++q) {
        const int r = canonical_q(q, a.D, a.lognk);
        a.qrep[q] = r;
        c += (r == q);
    }
    cnt[t] = c;
    __syncthreads();
    if (t == 0) {   // exclusive scan of 1024 counts (once per plan)
        int s = 0;
        for (int i = 0; i < 1024; ++i) {
            const int v = cnt[i];
            cnt[i] = s;
            s += v;
        }
    }
    __syncthreads();
    int o = cnt[t];
    for (int q = q0; q < q1; ++q)
        if (canonical_q(q, a.D, a.lognk) == q) a.qlist[o++] = q;
}

// One thread per (c, m index, n, q), q fastest.  Sources are always solved
// entries (m index >= im0, q a representative), which this kernel never writes.
__global__ __launch_bounds__(256) void k_sym_expand(SymExpandArgs a) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = 2 * (size_t)a.n_om * a.n_nu * a.N;
    if (e >= total) return;
    const int q = (int)(e % a.N);
    size_t r = e / a.N;
    const int n = (int)(r % a.n_nu);
    r /= a.n_nu;
    const int im = (int)(r % a.n_om);
    const int c = (int)(r / a.n_om);
    const int qs = a.qrep[q];
    if (im >= a.im0 && qs == q) return;
    const bool flip = im < a.im0;                    // Om < 0: conjugate of -Om, nu -> -nu
    const int ims = flip ? a.n_om - 1 - im : im;
    const int ns = flip ? a.n_nu - 1 - n : n;
    cd v = ld(a.w, (((size_t)c * a.n_om + ims) * a.n_nu + ns) * a.N + qs);
    if (flip) v.im = -v.im;
    st(a.w, e, v);
    if (n != 0) return;
    const size_t d = ((size_t)c * a.n_om + im) * a.N + q;
    const size_t ds = ((size_t)c * a.n_om + ims) * a.N + qs;
    if (a.logdet) {
        cd l = ld(a.logdet, ds);
        if (flip) {
            l.im = -l.im;
            if (l.im <= -M_PI) l.im += 2.0 * M_PI;      // phase kept in (-pi, pi]
        }
        st(a.logdet, d, l);
    }
    if (a.status) a.status[d] = a.status[ds];
}

hipError_t launch_sym_tables(const SymTableArgs &a, hipStream_t s) {
    if (a.N < 1 || a.N > 4096) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sym_tables, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sym_expand(const SymExpandArgs &a, hipStream_t s) {
    const size_t total = 2 * (size_t)a.n_om * a.n_nu * a.N;
    hipLaunchKernelGGL(k_sym_expand, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace df
