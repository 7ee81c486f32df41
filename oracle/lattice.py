"""Plain FP64 CPU oracle of the lattice observables of the converged dual solution.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check of the entry
module and the CPU-baseline leg of the benchmark may import it; the product
path never does.

NumPy complex128 throughout.  The functions follow Sec. 2.3 of the paper
("Resulting observables"):

  matsubara_nu   the fermionic window nu_n = (2n + 1) pi / beta, n = -n_nu/2 .. n_nu/2 - 1
  sigma_dmft     Sigma^DMFT = i nu + mu - Delta - 1/g           (after eq. sigma_lat)
  sigma_lat      eq. (sigma_lat), reading L1
  g_lat          eq. (glat)
  frak_g         the dressed propagator of the susceptibility formula
  chi_lattice    chi^{ch/sp}(Omega = 0, q): lattice bubble plus the ladder
                 term sum_{nu nu'} L_nu Gamma_{nu nu'} L_nu' (readings L2, L3)

Readings of the paper (where it is garbled, silent or ambiguous):
  L1  eq. (sigma_lat) prints Sigma (not Sigma~) in the denominator and the sign
      1 - g Sigma.  The paper states that eqs. (sigma_lat) and (glat) are
      related by the lattice Dyson equation G^-1 = i nu + mu - eps - Sigma;
      with eqs. (gd0) and (dyson) that holds exactly for
      Sigma = Sigma~ / (1 + g Sigma~) + Sigma^DMFT, which is used here (the
      Dyson relation is a test of this module).
  L2  The momentum sums of the susceptibility formula (the lattice bubble and
      L) carry the 1/N_k^D of eq. (dual_bubble): susceptibilities per site.
  L3  The fermionic sums run over the same window as the rest of the
      iteration (no tail correction), and Gamma^{d/m} at Omega = 0 is the full
      matrix [1 - gamma chi~]^-1 gamma of eq. (lin_alg_inv) with the converged
      chi~; chi^ch takes the density channel, chi^sp the magnetic one.

Array layouts follow df_oracle: g, delta [n_nu]; eps [N]; Sigma~, G~, G [n_nu][N];
gamma_uu, gamma_ud [n_om][n_nu][n_nu]; chi~ [n_om][n_nu][N].
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import df_oracle as O


def matsubara_nu(n_nu: int, beta: float) -> np.ndarray:
    """nu_n = (2n + 1) pi / beta for n = -n_nu/2 .. n_nu/2 - 1."""
    n = np.arange(n_nu) - n_nu // 2
    return (2 * n + 1) * np.pi / beta


def sigma_dmft(g: np.ndarray, delta: np.ndarray, mu: float, beta: float) -> np.ndarray:
    """Sigma^DMFT_nu = i nu + mu - Delta_nu - 1/g_nu  [n_nu]."""
    nu = matsubara_nu(len(g), beta)
    return 1j * nu + mu - np.asarray(delta) - 1.0 / np.asarray(g)


def sigma_lat(sigma: np.ndarray, g: np.ndarray, delta: np.ndarray, mu: float,
              beta: float) -> np.ndarray:
    """Sigma_{nu,k} = Sigma~ / (1 + g Sigma~) + Sigma^DMFT_nu  (eq. sigma_lat, L1)."""
    gg = np.asarray(g)[:, None]
    return sigma / (1.0 + gg * sigma) + sigma_dmft(g, delta, mu, beta)[:, None]


class _Q:
    """Complex number with exact rational parts (fractions.Fraction)."""
    __slots__ = ("re", "im")

    def __init__(self, re, im=0):
        self.re, self.im = Fraction(re), Fraction(im)

    def __add__(self, o):
        return _Q(self.re + o.re, self.im + o.im)

    def __sub__(self, o):
        return _Q(self.re - o.re, self.im - o.im)

    def __mul__(self, o):
        return _Q(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    def inv(self):
        d = self.re * self.re + self.im * self.im
        return _Q(self.re / d, -self.im / d)

    def to_complex(self) -> complex:
        return complex(float(self.re), float(self.im))


def g_lat(sigma, g: np.ndarray, delta: np.ndarray, eps: np.ndarray) -> np.ndarray:
    """G_{nu,k} = a + a g^-1 G~ g^-1 a with a = [Delta_nu - eps_k]^-1  (eq. glat), G~ from
    eqs. (gd0) and (dyson) with self-energy sigma (None = zero).

    Evaluated exactly, in rational arithmetic on the FP64 inputs, and rounded once:
    where Delta - eps is small the two terms of eq. (glat) are large and cancel
    (to a part in 1e4-1e6 on the workloads of the tests), and G~0 is itself a
    small difference of O(g) terms there, so that FP64 (and even long double)
    arithmetic loses up to 1e-10 of the result.
    """
    n_nu, N = len(g), len(eps)
    out = np.empty((n_nu, N), dtype=np.complex128)
    for n in range(n_nu):
        gq = _Q(float(np.real(g[n])), float(np.imag(g[n])))
        ginv = gq.inv()
        for k in range(N):
            dme = _Q(float(np.real(delta[n])) - Fraction(float(eps[k])), float(np.imag(delta[n])))
            G = (ginv + dme).inv() - gq                                   # eq. (gd0)
            if sigma is not None:
                S = _Q(float(np.real(sigma[n, k])), float(np.imag(sigma[n, k])))
                G = (G.inv() - S).inv()                                   # eq. (dyson)
            a = dme.inv()
            out[n, k] = (a + a * ginv * G * ginv * a).to_complex()
    return out


def frak_g(G: np.ndarray, G0: np.ndarray, g: np.ndarray) -> np.ndarray:
    """frak G_{nu,k} = G~ (G~0 + g) / G~0."""
    return G * (G0 + np.asarray(g)[:, None]) / G0


def lattice_bubble0(X: np.ndarray, D: int, nk: int, beta: float) -> np.ndarray:
    """-(T/N) sum_k X_{nu,k} X_{nu,k+q} at Omega = 0, per nu: [n_nu][N]  (L2)."""
    return O.bubble_fft(X, D, nk, 1, beta)[0]


def chi_lattice(sigma: np.ndarray, g: np.ndarray, delta: np.ndarray, eps: np.ndarray,
                gamma_uu: np.ndarray, gamma_ud: np.ndarray, D: int, nk: int,
                beta: float, Gl: np.ndarray = None):
    """chi^{ch/sp}(Omega = 0, q) of the dual solution with self-energy sigma.

    chi = -(T/N) sum_{nu,k} G_{nu,k} G_{nu,k+q} + sum_{nu,nu'} L_nu Gamma_{nu nu'} L_nu'
    with L_nu(q) = -(T/N) sum_k frakG_{nu,k} frakG_{nu,k+q} and Gamma = solve(1 - gamma chi~, gamma)
    at Omega = 0 (index (n_om - 1) / 2 of the vertex arrays).  Gl: g_lat(sigma, ...) if the
    caller has it.  Returns (chi_ch, chi_sp), [N] each.
    """
    n_om = gamma_uu.shape[0]
    i0 = (n_om - 1) // 2
    G0 = O.dual_gf0(g, delta, eps)
    G = O.dual_gf(G0, sigma)
    if Gl is None:
        Gl = g_lat(sigma, g, delta, eps)
    bub = lattice_bubble0(Gl, D, nk, beta).sum(axis=0)           # [N]
    L = lattice_bubble0(frak_g(G, G0, g), D, nk, beta)           # [n_nu][N]
    chi0 = O.bubble_fft(G, D, nk, 1, beta)[0]                    # chi~ at Omega = 0
    gam = O.spin_channels(gamma_uu[i0][None], gamma_ud[i0][None])[:, 0]   # [2][n_nu][n_nu]
    n_nu = len(g)
    eye = np.eye(n_nu, dtype=np.complex128)
    out = []
    for c in range(2):
        lad = np.empty(L.shape[1], dtype=np.complex128)
        for q in range(L.shape[1]):
            Dm = eye - gam[c] * chi0[None, :, q]                 # 1 - gamma diag(chi~)
            Gam = np.linalg.solve(Dm, gam[c])                    # eq. (lin_alg_inv)
            lad[q] = L[:, q] @ Gam @ L[:, q]
        out.append(bub + lad)
    return out[0], out[1]
