/*
 * df.h - C ABI of the ladder dual-fermion hot path on one MI355X (gfx950).
 *
 * One outer iteration of the ladder dual-fermion method (paper Sec. 2.2):
 *
 *   df_dual_gf       dual Green's function G~ from the DMFT inputs g, Delta,
 *                    the dispersion eps_k (eq. gd0) and the current dual
 *                    self-energy (eq. dyson): G~ = G~0 / (1 - G~0 Sigma~)
 *   df_bubble        dual bubble chi_{Om,nu}(q) = -(T/N) sum_k G~_{nu,k} G~_{nu+Om,k+q}
 *                    (eq. dual_bubble) as FFT convolutions over the k-grid
 *   df_ladder_solve  for every (channel, Om, q): Gamma = [1 - gamma chi]^-1 gamma
 *                    (eqs. dual_ladder, lin_alg_inv), convergence-radius test and
 *                    one-step fallback, and W = diag(Gamma) - diag(gamma chi gamma)/2
 *   df_sigma         dual self-energy of eq. (sd) contracted through a second
 *                    FFT convolution
 *   df_iterate       the whole loop with linear mixing until Sigma~ converges
 *
 * Conventions
 *   - Every array pointer in df_inst_t is a DEVICE pointer on the current HIP
 *     device.  Complex numbers are interleaved (re, im) doubles.
 *   - Fermionic window n in [-n_nu/2, n_nu/2), nu_n = (2n+1) pi / beta.
 *     Bosonic window m in [-(n_om-1)/2, (n_om-1)/2], Om_m = 2 m pi / beta.
 *     Arrays index the windows from 0 (index = n + n_nu/2, m + (n_om-1)/2).
 *   - k-grid: k_j = 2 pi j / nk on each of the D axes; flat index in C order
 *     of the D-dimensional array of shape (nk,)*D; N = nk^D.
 *   - A propagator G~_{nu+Om} whose frequency leaves the window is zero.
 *   - Channel 0 is the density channel gamma^d = gamma^uu + gamma^ud, channel 1
 *     the magnetic channel gamma^m = gamma^uu - gamma^ud (eq. spin_symm).
 *   - Inside the convergence radius <=> Re det(1 - gamma chi) > 0; outside (or
 *     a singular matrix) the ladder takes one step, Gamma = gamma + gamma chi gamma,
 *     and is re-tested on the next iteration.
 *
 * Ownership: the caller allocates every buffer, the workspace included (size
 * it with df_workspace_size; it must be 256-byte aligned).  The library never
 * allocates or frees caller memory; it keeps no state between calls apart
 * from compiled kernels and the autotuner's table of ladder kernel choices
 * (df_autotune).  Calls are asynchronous on the given stream, except
 * df_iterate which synchronises that stream to read back the convergence
 * measure once per iteration, and df_autotune.  Calls on distinct workspaces may run
 * concurrently; two calls sharing a workspace must be ordered by the caller.
 *
 * Errors: argument errors are detected on the host and returned before any
 * work is queued.  No exception crosses the ABI.
 */
#ifndef DF_H
#define DF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define DF_OK                0
#define DF_E_INVAL          -1   /* null pointer, bad size, bad option          */
#define DF_E_UNSUPPORTED    -2   /* shape outside what the kernels handle       */
#define DF_E_WORKSPACE      -3   /* workspace missing, too small or misaligned  */
#define DF_E_HIP            -4   /* a HIP runtime call failed                   */
#define DF_E_NONFINITE      -5   /* Sigma~ became non-finite during df_iterate  */
#define DF_E_NOT_CONVERGED  -6   /* max_iter reached; outputs hold the last iterate */
#define DF_W_FALLBACK        1   /* success, but some ladders were outside the radius */

/* per-(channel, Om, q) ladder status */
#define DF_LADDER_OK         0
#define DF_LADDER_FALLBACK   1
#define DF_LADDER_SINGULAR   2

/* ladder precision */
#define DF_FP64              0   /* plain FP64 inversion                          */
#define DF_FP32_REFINE       1   /* FP32 inversion + FP64 residual refinement     */
#define DF_FP32              2   /* FP32 inversion alone (relative error ~1e-6)   */
#define DF_ADAPTIVE          3   /* df_iterate only: DF_FP32 ladders while an
                                    instance's last diff >= switch_tol, then DF_FP64 */

typedef void *df_stream_t;      /* hipStream_t; NULL is the null stream */

/*
 * One problem instance.
 *   D      lattice dimension, 1..4 (the hypercubic lattices of the paper)
 *   nk     k-points per axis, a power of two in [4, 64]; N = nk^D <= 4096
 *   n_nu   fermionic frequencies, even, 2..128
 *   n_om   bosonic frequencies, odd, 1 <= n_om <= n_nu - 1
 *   beta   inverse temperature, > 0
 * Inputs (read only):
 *   g, delta           [n_nu]              impurity g(nu) and hybridisation Delta(nu)
 *   eps                [N]   (real)        dispersion eps_k
 *   gamma_uu, gamma_ud [n_om][n_nu][n_nu]  impurity vertex gamma^{uu}, gamma^{ud}
 *                                          indexed [m][n][n']
 * State and outputs:
 *   sigma        [n_nu][N]            dual self-energy Sigma~ (df_dual_gf input, NULL = 0;
 *                                     df_iterate in/out)
 *   gd           [n_nu][N]            dual Green's function G~
 *   chi          [n_om][n_nu][N]      dual bubble chi[m][n][q]
 *   w            [2][n_om][n_nu][N]   W^c_{m,n}(q) = Gamma_nn - (gamma chi gamma)_nn / 2
 *   logdet       [2][n_om][N]         complex log det(1 - gamma chi), Im in (-pi, pi]
 *   status       [2][n_om][N] (int8)  DF_LADDER_*
 *   sigma_calc   [n_nu][N]            Sigma~ of eq. (sd) before mixing
 * Which fields a call reads or writes is stated at each entry point.
 */
typedef struct {
    int32_t D, nk, n_nu, n_om;
    double beta;
    const double *g, *delta, *eps, *gamma_uu, *gamma_ud;
    double *sigma, *gd, *chi, *w, *logdet, *sigma_calc;
    int8_t *status;
} df_inst_t;

/*
 * Options.
 *   prec        DF_FP64, DF_FP32_REFINE, DF_FP32, or (df_iterate) DF_ADAPTIVE
 *   max_iter    iteration limit of df_iterate, >= 1
 *   mix         weight alpha of the new Sigma~ in the linear mixing, (0, 1]
 *   tol         df_iterate stops once ||Sigma_new - Sigma_old||_F / ||Sigma_new||_F < tol
 *               (every instance); tol <= 0 runs exactly max_iter iterations
 *   switch_tol  DF_ADAPTIVE: diff below which an instance's ladders switch from
 *               FP32 to FP64 (<= 0: 1e-4).  The FP32 ladders' error (~1e-6
 *               relative) then lies below the iterate's own distance to the
 *               fixed point, and the FP64 iterations that follow contract it
 *               away with the rest, so the converged Sigma~ is that of DF_FP64.
 *   use_graph   nonzero: df_iterate captures one iteration in a hipGraph and replays it
 *   accel       0: linear mixing, Sigma <- (1 - mix) Sigma + mix Sigma_calc.
 *               1..8: Anderson acceleration over the last accel + 1 iterates:
 *               Sigma <- sum_j c_j (Sigma_j + mix (Sigma_calc_j - Sigma_j)), with
 *               real weights c_j (summing to one) from the least-squares fit of
 *               the newest residual by differences of recorded residuals.  Real
 *               weights keep Sigma~(-nu) = Sigma~(nu)* and the lattice
 *               symmetries.  Same fixed point, fewer iterations.  The workspace
 *               grows by (2 accel + 3) n_nu N complex per instance: size it with
 *               the same options.
 *   symmetry    0: every (c, Omega, q) ladder is solved.  1 (df_ladder_solve,
 *               df_iterate): one q per orbit of the lattice point group (axis
 *               permutations and reflections k_a -> -k_a) and Omega >= 0 only are
 *               solved; the others are copied from them, conjugated with
 *               nu -> -nu for Omega < 0 (2D 32x32: 153 of 1024 q, 16 of 31 Omega).
 *               Valid when the inputs carry those symmetries - eps_k invariant
 *               under the group, g(-nu) = g(nu)*, Delta(-nu) = Delta(nu)*,
 *               gamma_{-Om}(-nu, -nu') = gamma_Om(nu, nu')* and a sigma (start value)
 *               that is point-group invariant with Sigma~(-nu) = Sigma~(nu)* - as
 *               those of the hypercubic Hubbard model are; the iteration keeps
 *               them.  Results then equal those of symmetry 0 to rounding.
 *   graph_unroll  df_iterate with use_graph, accel 0 and prec DF_FP64,
 *               DF_FP32_REFINE or DF_FP32: iterations per captured graph, 0..64
 *               (0 and 1: one).  The convergence measure and the fallback
 *               counts are then read once per graph launch, after its last
 *               iteration: an instance may run up to graph_unroll - 1
 *               iterations past the one whose diff fell below tol (iters_out
 *               counts the iterations run), and the host waits once per
 *               graph_unroll iterations instead of once per iteration.  With
 *               tol <= 0 the results are those of graph_unroll 0.  DF_ADAPTIVE
 *               and accel > 0 take a host step every iteration and ignore it.
 */
typedef struct {
    int32_t prec;
    int32_t max_iter;
    double mix;
    double tol;
    double switch_tol;
    int32_t use_graph;
    int32_t accel;
    int32_t symmetry;
    int32_t graph_unroll;
} df_opts_t;

/* Workspace bytes needed by any entry point for these instances and options. */
int df_workspace_size(const df_inst_t *inst, int32_t n_inst, const df_opts_t *opts,
                      size_t *bytes);

/* eq. (gd0), eq. (dyson).  Reads g, delta, eps, sigma (NULL = zero).  Writes gd. */
int df_dual_gf(const df_inst_t *inst, int32_t n_inst, void *ws, size_t ws_bytes,
               df_stream_t stream);

/* eq. (dual_bubble).  Reads gd.  Writes chi. */
int df_bubble(const df_inst_t *inst, int32_t n_inst, void *ws, size_t ws_bytes,
              df_stream_t stream);

/* df_bubble for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): no
 * workspace argument and no allocation.  Its scratch, G~(r) of one instance,
 * is a library-owned device array of 8 MiB per device (n_nu N <= 128 * 4096
 * complex, which every supported shape meets; DF_E_WORKSPACE otherwise).
 * Reads gd, writes chi, as df_bubble.  Every call on a device shares that
 * device's array: calls that overlap in time on one device (two streams, two
 * threads) race and must be ordered by the caller. */
int df_bubble_noalloc(const df_inst_t *inst, int32_t n_inst, df_stream_t stream);

/* eqs. (spin_symm), (dual_ladder), (lin_alg_inv) and the radius test; Gamma^(2) of
 * eq. (sd).  Reads gamma_uu, gamma_ud, chi.  Writes w and, when non-NULL, logdet
 * and status.  opts may be NULL (DF_FP64); DF_ADAPTIVE is rejected here
 * (DF_E_INVAL).  Returns DF_OK; the per-ladder outcome is in status.  Several
 * instances on a stream that is not being captured run as df_iterate runs them,
 * one fused launch per kernel class over a device table of the instances (the
 * table upload synchronises the stream once); under capture, one launch per
 * instance. */
int df_ladder_solve(const df_inst_t *inst, int32_t n_inst, const df_opts_t *opts,
                    void *ws, size_t ws_bytes, df_stream_t stream);

/* eq. (sd).  Reads w, gd.  Writes sigma_calc. */
int df_sigma(const df_inst_t *inst, int32_t n_inst, void *ws, size_t ws_bytes,
             df_stream_t stream);

/* The self-consistency loop.  Reads the inputs and sigma (the start value, e.g.
 * zero or a warm start); writes the final sigma and gd, and the last iteration's
 * chi, w, logdet, status, sigma_calc wherever those pointers are non-NULL.
 * iters_out (host, may be NULL) receives the iterations done; diff_out (host,
 * may be NULL) receives n_inst final diffs.  Returns DF_OK, DF_W_FALLBACK (some
 * ladder of the last iteration fell back), DF_E_NOT_CONVERGED or DF_E_NONFINITE. */
int df_iterate(const df_inst_t *inst, int32_t n_inst, const df_opts_t *opts,
               int32_t *iters_out, double *diff_out, void *ws, size_t ws_bytes,
               df_stream_t stream);

/* Autotuner for the batched ladder (the hot step of every iteration).  For each
 * distinct n_nu among the instances (with opts->prec; opts may be NULL =
 * DF_FP64; DF_ADAPTIVE tunes both of its precisions) it builds the ladder
 * inputs of all instances with that n_nu in the workspace (G~ from sigma,
 * NULL = zero, and chi), times every ladder kernel variant able to run them on
 * one fused launch over those instances - the launch df_iterate makes - (three
 * launches after an untimed one, HIP events on the stream, two passes over the
 * candidates, each variant keeping its faster pass), and keeps the fastest
 * for later calls of this process.  When the environment
 * variable DF_TUNE_CACHE names a file, choices are read from it on first use
 * and the whole table is written back here.  Every variant gives results of
 * the same precision class (bit patterns may differ between variants).
 * Synchronous; instance outputs are not touched.  Must not be called while
 * the stream is being captured (DF_E_INVAL).  The environment variable
 * DF_LADDER_KERNEL, a variant name, overrides both tuned and default choices. */
int df_autotune(const df_inst_t *inst, int32_t n_inst, const df_opts_t *opts, void *ws,
                size_t ws_bytes, df_stream_t stream);

/* Name of the ladder kernel choice that calls for this n_nu and precision use
 * now, for prec DF_FP64, DF_FP32_REFINE or DF_FP32, written to the host buffer
 * name (NUL-terminated, name_len bytes at most).  A choice is a kernel build
 * ("gjb", "gjb_o3", "gjb_o4", "vector", "mfma" for FP64; "mixed", "mixed_o3",
 * "mixed_o4" for the refined class; "fp32", "fp32_o4", "fp32_o5" for FP32
 * alone), optionally with a launch shape: "@p1" / "@p2" = a persistent grid of
 * 1x / 2x the resident work-groups taking items from per-XCD counters (for
 * "gjb" and "gjb_o3"); without it, one work-group per item.  Sizes: every
 * class serves n_nu <= 128; the builds capped at three waves per SIMD ("_o3")
 * exist up to n_nu 64 (refined: 96), those at four or five ("_o4", "_o5") up
 * to 64.  A choice always belongs to the requested precision class; the
 * refined kernels hand their near-instability items to the FP64 kernel, and
 * every certified kernel its uncertified items to "vector", within the call. */
int df_ladder_variant(int32_t n_nu, int32_t prec, char *name, size_t name_len);

/* Record a choice by hand, as df_autotune would: later calls for this n_nu and
 * precision use the named variant.  DF_E_UNSUPPORTED if it cannot serve them. */
int df_ladder_set_variant(int32_t n_nu, int32_t prec, const char *name);

/* Forget the tuned choices of this process (the cache file is left as is). */
int df_autotune_reset(void);

/* Static description of a status code. */
const char *df_strerror(int code);

/* ABI version (major * 100 + minor). */
int df_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DF_H */
