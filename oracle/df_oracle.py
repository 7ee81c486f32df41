"""Plain FP64 CPU oracle of the ladder dual-fermion iteration.

TEST INFRASTRUCTURE ONLY.  This module is the independent reference that the
GPU path is checked against.  Only the tests, the smoke check of the entry
module and the CPU-baseline leg of the benchmark may import it; the product
path never does.

Everything is NumPy complex128.  Each function follows one passage of the
paper (Sec. 2.2, "Ladder dual fermion self-consistency loop"):

  dual_gf0        eq. (gd0)            bare dual propagator
  dual_gf         eq. (dyson)          dual Dyson equation
  bubble_direct   eq. (dual_bubble)    plain k-sum (the definition)
  bubble_fft      eq. (dual_bubble)    same sum via the convolution theorem
  spin_channels   eq. (spin_symm)      density / magnetic vertices
  ladder          eqs. (dual_ladder), (lin_alg_inv) and the convergence-radius
                  rule that follows them; Gamma^(2) of eq. (sd)
  sigma_direct    eq. (sd)             plain (Omega, q) sum (the definition)
  sigma_fft       eq. (sd)             same sum via the convolution theorem
  iterate         the self-consistency loop closing Sec. 2.2

Readings of the paper (where it is garbled, silent or ambiguous):
  R1  eq. (dual_ladder) prints Gamma_{Omega'',omega'}; read Gamma_{Omega,omega'',omega'}(q).
      The omega'' sum carries no T: chi already holds it (eq. dual_bubble).
  R2  eq. (sd) closes the diagram with G_{omega+Omega, k+q}, not G_{omega, k+q}:
      the diagonal vertex Gamma_{Omega,omega,omega} has legs omega, omega+Omega,
      omega+Omega, omega, so frequency is conserved only with omega+Omega.
      Gamma^(2) = gamma chi gamma uses the current iteration's chi.
  R3  Outside the fermionic window a propagator G_{nu+Omega} is taken as zero
      (the window is symmetric, so the conjugation symmetry is kept).
  R4  Convergence radius: inside <=> Re det(1 - gamma chi) > 0.  At Omega = 0 the
      determinant is real, so this is exactly the sign test of the paper; a
      singular or non-finite determinant is treated as outside.  Outside, the
      "low-order iterative evaluation" is one ladder step,
      Gamma = gamma + gamma chi gamma, re-tested on the next iteration.
  R5  eq. (dyson) prints G^{(0}; read the bare dual propagator G~^{(0)}.
  R6  Convergence (not specified by the paper): linear mixing of Sigma~ with
      weight alpha, diff = ||Sigma_new - Sigma_old||_F / ||Sigma_new||_F.

Array layouts (shared with the GPU path's ABI, index conventions only):
  g, delta           [n_nu]                 complex
  eps                [N]                    real, flat C order of (nk,)*D
  gamma_uu, gamma_ud [n_om][n_nu][n_nu]     complex
  G, Sigma           [n_nu][N]              complex
  chi                [n_om][n_nu][N]        complex (chi[m][n][q])
  W                  [2][n_om][n_nu][N]     complex, channel 0 = d, 1 = m
  logdet             [2][n_om][N]           complex log det(1 - gamma chi)
  status             [2][n_om][N]           int8: 0 inside, 1 fallback, 2 singular
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

STATUS_OK = 0
STATUS_FALLBACK = 1
STATUS_SINGULAR = 2


# --------------------------------------------------------------------------
# k-grid index arithmetic
# --------------------------------------------------------------------------
def _coords(D: int, nk: int) -> np.ndarray:
    """Integer coordinates of every flat k index, shape [N, D] (C order)."""
    grids = np.meshgrid(*([np.arange(nk)] * D), indexing="ij")
    return np.stack([g.reshape(-1) for g in grids], axis=1)


def _flat(c: np.ndarray, nk: int) -> np.ndarray:
    D = c.shape[-1]
    idx = np.zeros(c.shape[:-1], dtype=np.int64)
    for a in range(D):
        idx = idx * nk + (c[..., a] % nk)
    return idx


def shift_table(D: int, nk: int) -> np.ndarray:
    """kq[k, q] = flat index of (k + q) mod 2 pi, shape [N, N]."""
    c = _coords(D, nk)
    return _flat(c[:, None, :] + c[None, :, :], nk)


def reflect_index(D: int, nk: int) -> np.ndarray:
    """ref[r] = flat index of -r mod nk on every axis."""
    return _flat(-_coords(D, nk), nk)


def _shifted_window(X: np.ndarray, m: int) -> np.ndarray:
    """Y[n] = X[n + m] along axis 0, zero where n + m leaves the window (R3)."""
    n_nu = X.shape[0]
    Y = np.zeros_like(X)
    if m >= 0:
        Y[: n_nu - m] = X[m:]
    else:
        Y[-m:] = X[: n_nu + m]
    return Y


def bosonic_offsets(n_om: int) -> np.ndarray:
    h = (n_om - 1) // 2
    return np.arange(-h, h + 1)


# --------------------------------------------------------------------------
# eq. (gd0) and eq. (dyson)
# --------------------------------------------------------------------------
def dual_gf0(g: np.ndarray, delta: np.ndarray, eps: np.ndarray) -> np.ndarray:
    """G~0_{nu,k} = [g^-1 + Delta - eps_k]^-1 - g   (eq. gd0)."""
    g = np.asarray(g, dtype=np.complex128)[:, None]
    delta = np.asarray(delta, dtype=np.complex128)[:, None]
    eps = np.asarray(eps, dtype=np.float64)[None, :]
    return 1.0 / (1.0 / g + delta - eps) - g


def dual_gf(G0: np.ndarray, sigma: Optional[np.ndarray]) -> np.ndarray:
    """G~ = [G~0^-1 - Sigma~]^-1   (eq. dyson, reading R5)."""
    if sigma is None:
        return G0.copy()
    return 1.0 / (1.0 / G0 - sigma)


# --------------------------------------------------------------------------
# eq. (dual_bubble)
# --------------------------------------------------------------------------
def bubble_direct(G: np.ndarray, D: int, nk: int, n_om: int, beta: float) -> np.ndarray:
    """chi_{Om,nu}(q) = -(T/N) sum_k G_{nu,k} G_{nu+Om,k+q}, the plain k-sum."""
    N = nk ** D
    T = 1.0 / beta
    kq = shift_table(D, nk)
    chi = np.zeros((n_om, G.shape[0], N), dtype=np.complex128)
    for im, m in enumerate(bosonic_offsets(n_om)):
        Gs = _shifted_window(G, m)                 # Gs[n, k] = G_{n+m, k}
        for q in range(N):
            chi[im, :, q] = -(T / N) * np.sum(G * Gs[:, kq[:, q]], axis=1)
    return chi


def bubble_fft(G: np.ndarray, D: int, nk: int, n_om: int, beta: float) -> np.ndarray:
    """Same sum as bubble_direct through the convolution theorem.

    With a = IFFT_k G_nu and b = IFFT_k G_{nu+Om} (numpy conventions),
    sum_k A(k) B(k+q) = N FFT_r[a(-r) b(r)](q), so chi = -T FFT_r[a(-r) b(r)].
    """
    n_nu, N = G.shape
    shape = (n_nu,) + (nk,) * D
    axes = tuple(range(1, D + 1))
    T = 1.0 / beta
    Gr = np.fft.ifftn(G.reshape(shape), axes=axes).reshape(n_nu, N)
    ref = reflect_index(D, nk)
    a = Gr[:, ref]                                  # a_n(-r)
    chi = np.zeros((n_om, n_nu, N), dtype=np.complex128)
    for im, m in enumerate(bosonic_offsets(n_om)):
        b = _shifted_window(Gr, m)                  # b_n(r) = G_{n+m}(r)
        p = (a * b).reshape(shape)
        chi[im] = -T * np.fft.fftn(p, axes=axes).reshape(n_nu, N)
    return chi


# --------------------------------------------------------------------------
# eq. (spin_symm), eqs. (dual_ladder)/(lin_alg_inv), Gamma^(2) of eq. (sd)
# --------------------------------------------------------------------------
def spin_channels(gamma_uu: np.ndarray, gamma_ud: np.ndarray) -> np.ndarray:
    """gamma^{d/m} = gamma^{uu} +- gamma^{ud}; channel 0 = d, 1 = m."""
    return np.stack([gamma_uu + gamma_ud, gamma_uu - gamma_ud])


@dataclasses.dataclass
class LadderResult:
    W: np.ndarray          # [2][n_om][n_nu][N]
    logdet: np.ndarray     # [2][n_om][N] complex
    status: np.ndarray     # [2][n_om][N] int8
    lam: Optional[np.ndarray] = None   # [2][n_om][N] max Re eig(gamma chi), or max |eig| (diagnostic)


def ladder(gamma_dm: np.ndarray, chi: np.ndarray, with_eigs: bool = False,
           mode: str = "auto", abs_eigs: bool = False) -> LadderResult:
    """Ladder for every (channel, Omega, q).

    mode "auto" applies the convergence-radius rule (R4); mode "fallback"
    takes the one-step ladder everywhere (second-order truncation).

    For each (c, m, q):  M = gamma^c_m diag(chi_m(q)),  D = 1 - M,
      inside (Re det D > 0, reading R4):  Gamma = solve(D, gamma)   (eq. lin_alg_inv)
      outside:                            Gamma = gamma + M gamma  (one ladder step)
      Gamma2 = M gamma                    (second-order term of eq. sd)
      W = diag(Gamma) - Gamma2_diag / 2
    """
    n_ch, n_om, n_nu, _ = gamma_dm.shape
    N = chi.shape[2]
    W = np.zeros((n_ch, n_om, n_nu, N), dtype=np.complex128)
    logdet = np.zeros((n_ch, n_om, N), dtype=np.complex128)
    status = np.zeros((n_ch, n_om, N), dtype=np.int8)
    lam = np.zeros((n_ch, n_om, N)) if with_eigs else None
    eye = np.eye(n_nu, dtype=np.complex128)
    for c in range(n_ch):
        for im in range(n_om):
            gam = gamma_dm[c, im]
            X = chi[im].T                                    # [N][n_nu]
            M = gam[None, :, :] * X[:, None, :]              # M[q] = gamma diag(chi_q)
            Dm = eye[None] - M
            sign, logabs = np.linalg.slogdet(Dm)
            ld = logabs + 1j * np.angle(sign)
            Gam2 = M @ gam[None]                             # gamma chi gamma
            g2d = np.diagonal(Gam2, axis1=1, axis2=2)        # [N][n_nu]
            ok = np.isfinite(logabs) & (np.real(sign) > 0)
            if mode == "fallback":
                ok = np.zeros_like(ok)
            singular = ~np.isfinite(logabs)
            Wq = np.empty((N, n_nu), dtype=np.complex128)
            if np.any(ok):
                Gam = np.linalg.solve(Dm[ok], np.broadcast_to(gam, (int(ok.sum()), n_nu, n_nu)))
                Wq[ok] = np.diagonal(Gam, axis1=1, axis2=2) - 0.5 * g2d[ok]
            bad = ~ok
            if np.any(bad):
                Wq[bad] = np.diagonal(gam)[None, :] + 0.5 * g2d[bad]
            W[c, im] = Wq.T
            logdet[c, im] = ld
            st = np.where(ok, STATUS_OK, STATUS_FALLBACK).astype(np.int8)
            st[singular] = STATUS_SINGULAR
            status[c, im] = st
            if with_eigs:
                ev = np.linalg.eigvals(M)
                lam[c, im] = np.max(np.abs(ev) if abs_eigs else np.real(ev), axis=1)
    return LadderResult(W=W, logdet=logdet, status=status, lam=lam)


# --------------------------------------------------------------------------
# eq. (sd)
# --------------------------------------------------------------------------
def sigma_vertex(W: np.ndarray) -> np.ndarray:
    """V = 3 W^m + W^d  (the channel weights of eq. sd)."""
    return 3.0 * W[1] + W[0]


def sigma_direct(W: np.ndarray, G: np.ndarray, D: int, nk: int, beta: float) -> np.ndarray:
    """Sigma~_{nu,k} = T/(2N) sum_{Om,q} V_{Om,nu}(q) G_{nu+Om,k+q}  (eq. sd, R2, R3)."""
    n_om = W.shape[1]
    N = nk ** D
    T = 1.0 / beta
    V = sigma_vertex(W)
    kq = shift_table(D, nk)
    S = np.zeros_like(G)
    for im, m in enumerate(bosonic_offsets(n_om)):
        Gs = _shifted_window(G, m)
        for k in range(N):
            S[:, k] += np.sum(V[im] * Gs[:, kq[k, :]], axis=1)
    return (T / (2.0 * N)) * S


def sigma_fft(W: np.ndarray, G: np.ndarray, D: int, nk: int, beta: float) -> np.ndarray:
    """Same sum as sigma_direct through the convolution theorem.

    With v = IFFT_q V and g = IFFT_k G, sum_q V(q) G(k+q) = N FFT_r[v(-r) g(r)](k).
    """
    n_om = W.shape[1]
    n_nu, N = G.shape
    shape = (n_nu,) + (nk,) * D
    axes = tuple(range(1, D + 1))
    T = 1.0 / beta
    V = sigma_vertex(W)
    Gr = np.fft.ifftn(G.reshape(shape), axes=axes).reshape(n_nu, N)
    ref = reflect_index(D, nk)
    acc = np.zeros((n_nu, N), dtype=np.complex128)
    for im, m in enumerate(bosonic_offsets(n_om)):
        v = np.fft.ifftn(V[im].reshape(shape), axes=axes).reshape(n_nu, N)
        acc += v[:, ref] * _shifted_window(Gr, m)
    return 0.5 * T * np.fft.fftn(acc.reshape(shape), axes=axes).reshape(n_nu, N)


# --------------------------------------------------------------------------
# self-consistency loop
# --------------------------------------------------------------------------
def rel_diff(new: np.ndarray, old: np.ndarray) -> float:
    """||new - old||_F / ||new||_F (reading R6); 0 when both vanish."""
    num = float(np.linalg.norm((new - old).ravel()))
    den = float(np.linalg.norm(new.ravel()))
    if den == 0.0:
        return 0.0 if num == 0.0 else math.inf
    return num / den


@dataclasses.dataclass
class IterResult:
    sigma: np.ndarray
    G: np.ndarray
    chi: np.ndarray
    ladder: LadderResult
    sigma_calc: np.ndarray
    iters: int
    diff: float
    history: list


def iterate(g, delta, eps, gamma_uu, gamma_ud, D: int, nk: int, beta: float,
            n_om: int, alpha: float = 0.5, tol: float = 0.0, max_iter: int = 10,
            sigma0: Optional[np.ndarray] = None, direct: bool = False) -> IterResult:
    """Repeat G~ -> chi -> Gamma -> Sigma~ -> mix until diff < tol or max_iter."""
    G0 = dual_gf0(g, delta, eps)
    gam = spin_channels(gamma_uu, gamma_ud)
    sigma = np.zeros_like(G0) if sigma0 is None else np.array(sigma0, dtype=np.complex128)
    bub = bubble_direct if direct else bubble_fft
    sig = sigma_direct if direct else sigma_fft
    history = []
    it = 0
    diff = math.inf
    G = chi = lr = scalc = None
    while it < max_iter:
        G = dual_gf(G0, sigma)
        chi = bub(G, D, nk, n_om, beta)
        lr = ladder(gam, chi)
        scalc = sig(lr.W, G, D, nk, beta)
        new = (1.0 - alpha) * sigma + alpha * scalc
        diff = rel_diff(new, sigma)
        sigma = new
        it += 1
        history.append(diff)
        if diff < tol:
            break
    return IterResult(sigma=sigma, G=G, chi=chi, ladder=lr, sigma_calc=scalc,
                      iters=it, diff=diff, history=history)


def leading_eigenvalue(gamma_dm: np.ndarray, chi: np.ndarray, im: int, c: int) -> np.ndarray:
    """max Re eig(gamma^c_m diag(chi_m(q))) for every q (diagnostic)."""
    gam = gamma_dm[c, im]
    X = chi[im].T
    M = gam[None, :, :] * X[:, None, :]
    return np.max(np.real(np.linalg.eigvals(M)), axis=1)
