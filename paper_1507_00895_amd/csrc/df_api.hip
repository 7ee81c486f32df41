// C ABI of libdf: argument validation, workspace layout, launch sequencing,
// the self-consistency loop and its optional hipGraph capture.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../include/df.h"
#include "df_internal.hpp"

using namespace df;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMixBlocks = 512;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

int ilog2_exact(int x) {
    if (x <= 0 || (x & (x - 1))) return -1;
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

struct Shape {
    int D, nk, lognk, N, n_nu, n_om, NP;
    int chunk_len, n_chunks;
};

int check_inst(const df_inst_t &p, Shape *s) {
    if (p.D < 1 || p.D > 3) return DF_E_UNSUPPORTED;
    const int l = ilog2_exact(p.nk);
    if (l < 2 || l > 6) return DF_E_UNSUPPORTED;
    long N = 1;
    for (int a = 0; a < p.D; ++a) N *= p.nk;
    if (N > 4096) return DF_E_UNSUPPORTED;
    if (p.n_nu < 2 || (p.n_nu & 1)) return DF_E_INVAL;
    if (p.n_nu > 128) return DF_E_UNSUPPORTED;
    if (p.n_om < 1 || !(p.n_om & 1) || p.n_om > p.n_nu - 1) return DF_E_INVAL;
    if (!(p.beta > 0.0) || !isfinite(p.beta)) return DF_E_INVAL;
    s->D = p.D;
    s->nk = p.nk;
    s->lognk = l;
    s->N = (int)N;
    s->n_nu = p.n_nu;
    s->n_om = p.n_om;
    s->NP = ladder_padded_size(p.n_nu);
    int nch = (512 + p.n_nu - 1) / p.n_nu;
    if (nch > p.n_om) nch = p.n_om;
    if (nch < 1) nch = 1;
    s->chunk_len = (p.n_om + nch - 1) / nch;
    s->n_chunks = (p.n_om + s->chunk_len - 1) / s->chunk_len;
    return DF_OK;
}

// Per-instance workspace regions (byte offsets from the instance base).
struct Layout {
    size_t gr, gdm, pdm, gtr, queue, part, norm, diff, count, gd, chi, w, sc, total;
};

Layout layout_of(const Shape &s) {
    Layout L;
    const size_t cdb = 16;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const size_t fld = (size_t)s.n_nu * s.N * cdb;
    L.gr = take(fld);
    L.gdm = take(2 * (size_t)s.n_om * s.n_nu * s.n_nu * cdb);
    L.pdm = take(2 * (size_t)s.n_om * s.n_nu * s.n_nu * cdb);
    L.gtr = take(2 * (size_t)s.n_om * s.n_nu * s.n_nu * cdb);
    L.queue = take(2 * (size_t)s.n_om * s.N * sizeof(int));
    L.part = take((size_t)s.n_chunks * fld);
    L.norm = take((size_t)kMixBlocks * 2 * sizeof(double));
    L.diff = take(2 * sizeof(double));
    L.count = take(2 * sizeof(int));   // [0] ladders outside the radius, [1] queue length
    L.gd = take(fld);
    L.chi = take((size_t)s.n_om * fld);
    L.w = take(2 * (size_t)s.n_om * fld);
    L.sc = take(fld);
    L.total = o;
    return L;
}

struct Plan {
    std::vector<Shape> shape;
    std::vector<Layout> lay;
    std::vector<size_t> base;
    size_t total = 0;
};

int make_plan(const df_inst_t *inst, int32_t n_inst, Plan *P) {
    if (!inst || n_inst < 1) return DF_E_INVAL;
    P->shape.resize(n_inst);
    P->lay.resize(n_inst);
    P->base.resize(n_inst);
    size_t off = 0;
    for (int i = 0; i < n_inst; ++i) {
        const int rc = check_inst(inst[i], &P->shape[i]);
        if (rc != DF_OK) return rc;
        P->lay[i] = layout_of(P->shape[i]);
        P->base[i] = off;
        off = align_up(off + P->lay[i].total);
    }
    P->total = off;
    return DF_OK;
}

int check_ws(const Plan &P, void *ws, size_t ws_bytes) {
    if (!ws) return DF_E_WORKSPACE;
    if (((uintptr_t)ws) & (kAlign - 1)) return DF_E_WORKSPACE;
    if (ws_bytes < P.total) return DF_E_WORKSPACE;
    return DF_OK;
}

template <typename T> T *at(void *ws, size_t base, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + base + off);
}

Grid grid_of(const Shape &s) {
    Grid g;
    g.D = s.D;
    g.lognk = s.lognk;
    g.nk = s.nk;
    g.N = s.N;
    return g;
}

#define HIPCHK(x)                                  \
    do {                                           \
        hipError_t e_ = (x);                       \
        if (e_ != hipSuccess) return DF_E_HIP;     \
    } while (0)

// Once per process: raise the dynamic LDS limit of the FFT kernels.  Runs
// before any stream work is queued, never inside a graph capture.  If the
// device refuses, only launches that need more than 64 KiB of LDS fail.
int ensure_attrs() {
    static int done = 0;
    if (!done) {
        (void)set_fft_lds_limits();
        (void)hipGetLastError();
        done = 1;
    }
    return DF_OK;
}

// Ladder kernel choice.  Default: the certified pivot-free blocked kernel on
// the matrix cores, whose uncertified items go to the partial-pivoting kernel.
// DF_LADDER_KERNEL=vector|mfma|gjb overrides the choice (for measurements):
// vector = partial pivoting with vector FMAs for every item, mfma = partial
// pivoting with MFMA trailing updates (n_nu <= 64).
enum LadderKind { LK_GJB = 0, LK_VECTOR = 1, LK_MFMA = 2 };
LadderKind ladder_kind(int n_nu) {
    static int mode = -1;
    if (mode < 0) {
        const char *e = getenv("DF_LADDER_KERNEL");
        mode = LK_GJB;
        if (e && strcmp(e, "vector") == 0) mode = LK_VECTOR;
        if (e && strcmp(e, "mfma") == 0) mode = LK_MFMA;
    }
    if (mode == LK_MFMA && ladder_mfma_padded_size(n_nu) == 0) return LK_VECTOR;
    if (mode == LK_GJB && ladder_gjb_padded_size(n_nu) == 0) return LK_VECTOR;
    return (LadderKind)mode;
}

constexpr int kQueueBlocks = 2048;

// ---- individual stages for one instance ----------------------------------
int stage_dual_gf(const df_inst_t &p, const Shape &s, const double *sigma, double *gd,
                  double *gr, hipStream_t st) {
    DualGfArgs a{};
    a.grid = grid_of(s);
    a.n_nu = s.n_nu;
    a.g = p.g;
    a.delta = p.delta;
    a.eps = p.eps;
    a.sigma = sigma;
    a.gd_in = nullptr;
    a.gd_out = gd;
    a.gr_out = gr;
    a.from_gd = 0;
    HIPCHK(launch_dual_gf(a, st));
    return DF_OK;
}

int stage_transform_gd(const Shape &s, const double *gd, double *gr, hipStream_t st) {
    DualGfArgs a{};
    a.grid = grid_of(s);
    a.n_nu = s.n_nu;
    a.gd_in = gd;
    a.gr_out = gr;
    a.from_gd = 1;
    HIPCHK(launch_dual_gf(a, st));
    return DF_OK;
}

int stage_bubble(const df_inst_t &p, const Shape &s, const double *gr, double *chi,
                 hipStream_t st) {
    BubbleArgs a{};
    a.grid = grid_of(s);
    a.n_nu = s.n_nu;
    a.n_om = s.n_om;
    a.beta = p.beta;
    a.gr = gr;
    a.chi = chi;
    HIPCHK(launch_bubble(a, st));
    return DF_OK;
}

int stage_gamma_prep(const df_inst_t &p, const Shape &s, double *gdm, double *pdm, double *gtr,
                     hipStream_t st) {
    GammaPrepArgs a{};
    a.gtr = gtr;
    a.n_nu = s.n_nu;
    a.n_om = s.n_om;
    a.guu = p.gamma_uu;
    a.gud = p.gamma_ud;
    a.gdm = gdm;
    a.pdm = pdm;
    HIPCHK(launch_gamma_prep(a, st));
    return DF_OK;
}

int stage_ladder(const Shape &s, int prec, const double *gdm, const double *pdm,
                 const double *gtr, const double *chi, double *w, double *logdet, int8_t *status,
                 int *counts, int *queue, hipStream_t st) {
    LadderArgs a{};
    a.gdm = gdm;
    a.pdm = pdm;
    a.gtr = gtr;
    a.chi = chi;
    a.w = w;
    a.logdet = logdet;
    a.status = status;
    a.n_nu = s.n_nu;
    a.n_om = s.n_om;
    a.N = s.N;
    a.item0 = 0;
    a.n_items = 2 * s.n_om * s.N;
    a.fallback_count = counts;
    HIPCHK(launch_zero_ints(counts, 2, st));
    if (prec == DF_FP32_REFINE && ladder_mixed_padded_size(s.n_nu) != 0) {
        a.queue = queue;
        a.queue_count = counts + 1;
        HIPCHK(launch_ladder_mixed(a, st));
        LadderArgs b = a;
        b.queue = nullptr;
        b.queue_count = nullptr;
        b.in_queue = queue;
        b.in_count = counts + 1;
        const int blocks = a.n_items < kQueueBlocks ? a.n_items : kQueueBlocks;
        HIPCHK(launch_ladder_fp64_queue(b, blocks, st));
        return DF_OK;
    }
    switch (ladder_kind(s.n_nu)) {
        case LK_VECTOR: HIPCHK(launch_ladder_fp64(a, st)); break;
        case LK_MFMA: HIPCHK(launch_ladder_mfma_f64(a, st)); break;
        default: {
            a.queue = queue;
            a.queue_count = counts + 1;
            HIPCHK(launch_ladder_gjb_f64(a, st));
            LadderArgs b = a;
            b.queue = nullptr;
            b.queue_count = nullptr;
            b.in_queue = queue;
            b.in_count = counts + 1;
            const int blocks = a.n_items < kQueueBlocks ? a.n_items : kQueueBlocks;
            HIPCHK(launch_ladder_fp64_queue(b, blocks, st));
        }
    }
    return DF_OK;
}

int stage_sigma(const df_inst_t &p, const Shape &s, const double *w, const double *gr,
                double *part, hipStream_t st) {
    SigmaArgs a{};
    a.grid = grid_of(s);
    a.n_nu = s.n_nu;
    a.n_om = s.n_om;
    a.chunk_len = s.chunk_len;
    a.n_chunks = s.n_chunks;
    a.beta = p.beta;
    a.w = w;
    a.gr = gr;
    a.part = part;
    HIPCHK(launch_sigma_part(a, st));
    return DF_OK;
}

int stage_reduce_mix(const Shape &s, const double *part, double *sigma_calc, double *sigma,
                     double alpha, double *norm, double *diff, hipStream_t st) {
    ReduceMixArgs a{};
    a.count = (size_t)s.n_nu * s.N;
    a.n_chunks = s.n_chunks;
    a.alpha = alpha;
    a.part = part;
    a.sigma_calc = sigma_calc;
    a.sigma = sigma;
    a.norm_part = norm;
    int blocks = (int)((a.count + 255) / 256);
    if (blocks > kMixBlocks) blocks = kMixBlocks;
    HIPCHK(launch_reduce_mix(a, blocks, st));
    if (sigma) HIPCHK(launch_norm_final(norm, blocks, diff, st));
    return DF_OK;
}

int check_opts(const df_opts_t *o, bool need_loop) {
    if (!o) return need_loop ? DF_E_INVAL : DF_OK;
    if (o->prec != DF_FP64 && o->prec != DF_FP32_REFINE) return DF_E_INVAL;
    if (o->prec == DF_FP32_REFINE && (o->max_refine < 1 || o->max_refine > 4)) return DF_E_INVAL;
    if (need_loop) {
        if (!(o->mix > 0.0 && o->mix <= 1.0)) return DF_E_INVAL;
        if (o->max_iter < 1) return DF_E_INVAL;
        if (!isfinite(o->tol)) return DF_E_INVAL;
    }
    return DF_OK;
}

}  // namespace

extern "C" {

int df_version(void) { return 100; }

const char *df_strerror(int code) {
    switch (code) {
        case DF_OK: return "success";
        case DF_E_INVAL: return "invalid argument";
        case DF_E_UNSUPPORTED: return "unsupported shape (D in 1..3, nk power of two in [4,64], nk^D <= 4096, n_nu <= 128)";
        case DF_E_WORKSPACE: return "workspace missing, misaligned (256 B) or too small";
        case DF_E_HIP: return "HIP runtime error";
        case DF_E_NONFINITE: return "dual self-energy became non-finite";
        case DF_E_NOT_CONVERGED: return "iteration limit reached before the tolerance";
        case DF_W_FALLBACK: return "success; some ladders were outside the convergence radius";
        default: return "unknown status code";
    }
}

int df_workspace_size(const df_inst_t *inst, int32_t n_inst, const df_opts_t *opts, size_t *bytes) {
    if (!bytes) return DF_E_INVAL;
    int rc = check_opts(opts, false);
    if (rc != DF_OK) return rc;
    Plan P;
    rc = make_plan(inst, n_inst, &P);
    if (rc != DF_OK) return rc;
    *bytes = P.total;
    return DF_OK;
}

int df_dual_gf(const df_inst_t *inst, int32_t n_inst, void *ws, size_t ws_bytes, df_stream_t stream) {
    Plan P;
    int rc = make_plan(inst, n_inst, &P);
    if (rc != DF_OK) return rc;
    rc = check_ws(P, ws, ws_bytes);
    if (rc != DF_OK) return rc;
    rc = ensure_attrs();
    if (rc != DF_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < n_inst; ++i) {
        const df_inst_t &p = inst[i];
        if (!p.g || !p.delta || !p.eps || !p.gd) return DF_E_INVAL;
    }
    for (int i = 0; i < n_inst; ++i) {
        rc = stage_dual_gf(inst[i], P.shape[i], inst[i].sigma, inst[i].gd, nullptr, st);
        if (rc != DF_OK) return rc;
    }
    return DF_OK;
}

int df_bubble(const df_inst_t *inst, int32_t n_inst, void *ws, size_t ws_bytes, df_stream_t stream) {
    Plan P;
    int rc = make_plan(inst, n_inst, &P);
    if (rc != DF_OK) return rc;
    rc = check_ws(P, ws, ws_bytes);
    if (rc != DF_OK) return rc;
    rc = ensure_attrs();
    if (rc != DF_OK) return rc;
    for (int i = 0; i < n_inst; ++i)
        if (!inst[i].gd || !inst[i].chi) return DF_E_INVAL;
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < n_inst; ++i) {
        const Shape &s = P.shape[i];
        double *gr = at<double>(ws, P.base[i], P.lay[i].gr);
        rc = stage_transform_gd(s, inst[i].gd, gr, st);
        if (rc != DF_OK) return rc;
        rc = stage_bubble(inst[i], s, gr, inst[i].chi, st);
        if (rc != DF_OK) return rc;
    }
    return DF_OK;
}

int df_ladder_solve(const df_inst_t *inst, int32_t n_inst, const df_opts_t *opts, void *ws,
                    size_t ws_bytes, df_stream_t stream) {
    int rc = check_opts(opts, false);
    if (rc != DF_OK) return rc;
    Plan P;
    rc = make_plan(inst, n_inst, &P);
    if (rc != DF_OK) return rc;
    rc = check_ws(P, ws, ws_bytes);
    if (rc != DF_OK) return rc;
    rc = ensure_attrs();
    if (rc != DF_OK) return rc;
    for (int i = 0; i < n_inst; ++i)
        if (!inst[i].gamma_uu || !inst[i].gamma_ud || !inst[i].chi || !inst[i].w) return DF_E_INVAL;
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < n_inst; ++i) {
        const Shape &s = P.shape[i];
        const Layout &L = P.lay[i];
        double *gdm = at<double>(ws, P.base[i], L.gdm);
        double *pdm = at<double>(ws, P.base[i], L.pdm);
        double *gtr = at<double>(ws, P.base[i], L.gtr);
        rc = stage_gamma_prep(inst[i], s, gdm, pdm, gtr, st);
        if (rc != DF_OK) return rc;
        rc = stage_ladder(s, opts ? opts->prec : DF_FP64, gdm, pdm, gtr, inst[i].chi,
                          inst[i].w, inst[i].logdet,
                          inst[i].status, at<int>(ws, P.base[i], L.count),
                          at<int>(ws, P.base[i], L.queue), st);
        if (rc != DF_OK) return rc;
    }
    return DF_OK;
}

int df_sigma(const df_inst_t *inst, int32_t n_inst, void *ws, size_t ws_bytes, df_stream_t stream) {
    Plan P;
    int rc = make_plan(inst, n_inst, &P);
    if (rc != DF_OK) return rc;
    rc = check_ws(P, ws, ws_bytes);
    if (rc != DF_OK) return rc;
    rc = ensure_attrs();
    if (rc != DF_OK) return rc;
    for (int i = 0; i < n_inst; ++i)
        if (!inst[i].w || !inst[i].gd || !inst[i].sigma_calc) return DF_E_INVAL;
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < n_inst; ++i) {
        const Shape &s = P.shape[i];
        const Layout &L = P.lay[i];
        double *gr = at<double>(ws, P.base[i], L.gr);
        double *part = at<double>(ws, P.base[i], L.part);
        rc = stage_transform_gd(s, inst[i].gd, gr, st);
        if (rc != DF_OK) return rc;
        rc = stage_sigma(inst[i], s, inst[i].w, gr, part, st);
        if (rc != DF_OK) return rc;
        rc = stage_reduce_mix(s, part, inst[i].sigma_calc, nullptr, 0.0, nullptr, nullptr, st);
        if (rc != DF_OK) return rc;
    }
    return DF_OK;
}

namespace {

// Queue one full iteration of instance i on stream st.
int queue_iteration(const df_inst_t &p, const Shape &s, const Layout &L, void *ws, size_t base,
                    const df_opts_t &o, hipStream_t st) {
    double *gr = at<double>(ws, base, L.gr);
    double *gdm = at<double>(ws, base, L.gdm);
    double *pdm = at<double>(ws, base, L.pdm);
    double *gtr = at<double>(ws, base, L.gtr);
    int *queue = at<int>(ws, base, L.queue);
    double *part = at<double>(ws, base, L.part);
    double *norm = at<double>(ws, base, L.norm);
    double *diff = at<double>(ws, base, L.diff);
    int *count = at<int>(ws, base, L.count);
    double *gd = p.gd ? p.gd : at<double>(ws, base, L.gd);
    double *chi = p.chi ? p.chi : at<double>(ws, base, L.chi);
    double *w = p.w ? p.w : at<double>(ws, base, L.w);
    int rc = stage_dual_gf(p, s, p.sigma, gd, gr, st);
    if (rc != DF_OK) return rc;
    rc = stage_bubble(p, s, gr, chi, st);
    if (rc != DF_OK) return rc;
    rc = stage_ladder(s, o.prec, gdm, pdm, gtr, chi, w, p.logdet, p.status, count, queue, st);
    if (rc != DF_OK) return rc;
    rc = stage_sigma(p, s, w, gr, part, st);
    if (rc != DF_OK) return rc;
    return stage_reduce_mix(s, part, p.sigma_calc, p.sigma, o.mix, norm, diff, st);
}

}  // namespace

int df_iterate(const df_inst_t *inst, int32_t n_inst, const df_opts_t *opts, int32_t *iters_out,
               double *diff_out, void *ws, size_t ws_bytes, df_stream_t stream) {
    int rc = check_opts(opts, true);
    if (rc != DF_OK) return rc;
    Plan P;
    rc = make_plan(inst, n_inst, &P);
    if (rc != DF_OK) return rc;
    rc = check_ws(P, ws, ws_bytes);
    if (rc != DF_OK) return rc;
    rc = ensure_attrs();
    if (rc != DF_OK) return rc;
    for (int i = 0; i < n_inst; ++i) {
        const df_inst_t &p = inst[i];
        if (!p.g || !p.delta || !p.eps || !p.gamma_uu || !p.gamma_ud || !p.sigma) return DF_E_INVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    const bool graph = opts->use_graph != 0 && st != nullptr;

    for (int i = 0; i < n_inst; ++i) {
        const Layout &L = P.lay[i];
        rc = stage_gamma_prep(inst[i], P.shape[i], at<double>(ws, P.base[i], L.gdm),
                              at<double>(ws, P.base[i], L.pdm), at<double>(ws, P.base[i], L.gtr),
                              st);
        if (rc != DF_OK) return rc;
    }

    std::vector<hipGraphExec_t> exec(n_inst, nullptr);
    auto cleanup = [&]() {
        for (auto &e : exec)
            if (e) (void)hipGraphExecDestroy(e);
    };
    if (graph) {
        for (int i = 0; i < n_inst; ++i) {
            hipGraph_t g = nullptr;
            if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                cleanup();
                return DF_E_HIP;
            }
            rc = queue_iteration(inst[i], P.shape[i], P.lay[i], ws, P.base[i], *opts, st);
            hipError_t e = hipStreamEndCapture(st, &g);
            if (rc != DF_OK || e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                cleanup();
                return rc != DF_OK ? rc : DF_E_HIP;
            }
            e = hipGraphInstantiate(&exec[i], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                cleanup();
                return DF_E_HIP;
            }
        }
    }

    std::vector<char> done(n_inst, 0);
    std::vector<double> last(n_inst, INFINITY);
    std::vector<double> host(2);
    int it = 0;
    int result = DF_OK;
    bool any_fallback = false;
    while (it < opts->max_iter) {
        for (int i = 0; i < n_inst; ++i) {
            if (done[i]) continue;
            if (graph) {
                if (hipGraphLaunch(exec[i], st) != hipSuccess) {
                    cleanup();
                    return DF_E_HIP;
                }
            } else {
                rc = queue_iteration(inst[i], P.shape[i], P.lay[i], ws, P.base[i], *opts, st);
                if (rc != DF_OK) {
                    cleanup();
                    return rc;
                }
            }
        }
        ++it;
        bool all_done = true;
        any_fallback = false;
        for (int i = 0; i < n_inst; ++i) {
            if (done[i]) continue;
            double h[2];
            int cnt = 0;
            if (hipMemcpyAsync(h, at<double>(ws, P.base[i], P.lay[i].diff), 2 * sizeof(double),
                               hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipMemcpyAsync(&cnt, at<int>(ws, P.base[i], P.lay[i].count), sizeof(int),
                               hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                cleanup();
                return DF_E_HIP;
            }
            last[i] = h[0];
            if (cnt) any_fallback = true;
            if (h[1] != 0.0 || !isfinite(h[0])) {
                result = DF_E_NONFINITE;
                done[i] = 1;
                continue;
            }
            if (opts->tol > 0.0 && h[0] < opts->tol) done[i] = 1;
            else all_done = false;
        }
        if (result == DF_E_NONFINITE || all_done) break;
    }
    cleanup();
    if (iters_out) *iters_out = it;
    if (diff_out)
        for (int i = 0; i < n_inst; ++i) diff_out[i] = last[i];
    if (result != DF_OK) return result;
    if (opts->tol > 0.0) {
        for (int i = 0; i < n_inst; ++i)
            if (!(last[i] < opts->tol)) return DF_E_NOT_CONVERGED;
    }
    return any_fallback ? DF_W_FALLBACK : DF_OK;
}

}  // extern "C"
