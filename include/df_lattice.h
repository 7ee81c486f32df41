/*
 * df_lattice.h - C ABI of the lattice observables of a dual-fermion solution
 * (Sec. 2.3 of the paper, "Resulting observables"), in libdf.so.
 *
 * From one instance's inputs (g, delta, eps, gamma_uu, gamma_ud, beta; the
 * layouts of df.h) and its dual self-energy sigma (normally the converged
 * Sigma~ of df_iterate; NULL = zero), with nu_n = (2n + 1 - n_nu) pi / beta:
 *
 *   sigma_lat [n_nu][N] complex
 *       Sigma~ / (1 + g Sigma~) + Sigma^DMFT,  Sigma^DMFT = i nu + mu - Delta - 1/g
 *       (eq. sigma_lat; the paper prints Sigma in the denominator with the sign
 *       1 - g Sigma; 1 + g Sigma~ is the form for which eqs. (sigma_lat) and
 *       (glat) obey the lattice Dyson equation G^-1 = i nu + mu - eps - Sigma,
 *       as the paper states they do)
 *   g_lat [n_nu][N] complex
 *       [Delta - eps]^-1 + [Delta - eps]^-1 g^-1 G~ g^-1 [Delta - eps]^-1   (eq. glat)
 *   chi_ch, chi_sp [N] complex: the charge and spin susceptibilities at Omega = 0
 *       -(T/N) sum_{nu,k} G_{nu,k} G_{nu,k+q} + sum_{nu,nu'} L_nu(q) Gamma^{d/m}_{nu nu'}(q) L_nu'(q),
 *       L_nu(q) = -(T/N) sum_k frakG_{nu,k} frakG_{nu,k+q},  frakG = G~ (G~0 + g) / G~0,
 *       Gamma = [1 - gamma chi~]^-1 gamma at Omega = 0 (index (n_om - 1) / 2 of the
 *       vertex arrays), chi~ the dual bubble of G~ (eq. dual_bubble)
 *       (momentum sums per site as in eq. dual_bubble; fermionic sums over the
 *       same n_nu window as the iteration; ch takes the density channel, sp the
 *       magnetic one; Gamma by Gaussian elimination with partial pivoting, FP64)
 *
 * Every output may be NULL (not computed).  All pointers are device pointers;
 * the caller owns every buffer and the workspace (device memory, 256-byte
 * aligned, at least df_lattice_workspace_size bytes).  The call is
 * asynchronous on stream and returns the status codes of df.h: DF_E_INVAL or
 * DF_E_UNSUPPORTED for an instance df_workspace_size would reject (or mu not
 * finite), DF_E_WORKSPACE for a missing, misaligned or short workspace,
 * DF_E_HIP for a failed launch.  Results are deterministic run to run.
 */
#ifndef DF_LATTICE_H
#define DF_LATTICE_H

#include <stddef.h>
#include <stdint.h>

#include "df.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Workspace bytes df_lattice needs for this instance. */
int df_lattice_workspace_size(const df_inst_t *inst, size_t *bytes);

/* The lattice observables above, for one instance with chemical potential mu. */
int df_lattice(const df_inst_t *inst, double mu, double *sigma_lat, double *g_lat,
               double *chi_ch, double *chi_sp, void *ws, size_t ws_bytes, df_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* DF_LATTICE_H */
