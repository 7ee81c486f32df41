"""Exact diagonalisation of the Hubbard atom: g and the two-particle vertex.

TEST INFRASTRUCTURE ONLY.  This module is a pin for the closed-form
atomic-limit inputs (paper Sec. 4, eqs. atomic_limit1-4) and for the vertex
definition of eq. (vertex).  It is imported by the tests, never by the
product path.

Method (brute force on the 4-state Fock space, no closed forms used):
  H = U n_up n_dn - mu (n_up + n_dn), c_up / c_dn as 4x4 Jordan-Wigner
  matrices.  The imaginary-time ordered correlator
      <T c_1(t1) c+_2(t2) c_3(t3) c+_4(0)>
  is integrated over the three times for every one of the 3! time orderings.
  On each ordering the Lehmann sum turns the integrand into a product of
  exponentials over the four time intervals, and the integral over the
  simplex of interval lengths is a divided difference of exp(-beta z)
  (Hermite-Genocchi); the divided difference is evaluated exactly (also at
  coinciding points, which produce the beta-proportional terms) as the
  corner element of the matrix exponential of a bidiagonal matrix (Opitz).
  Fourier convention: c(tau) picks +i w tau, c+(tau) picks -i w tau; with
  w1 = nu, w2 = nu + Om, w3 = nu' + Om, w4 = nu' frequency is conserved.
  The connected part subtracts the two Wick pairings, and the vertex is the
  connected part divided by the four legs g1 g2 g3 g4.

Reading of eq. (vertex) fixed by this pin: the printed formula has a garbled
spin delta and omits the division by the legs; the closed forms of Sec. 4
are the amputated connected part.  The closed-form "gamma^{ud}" equals the
amputated connected part of the spin arrangement (up, up, dn, dn) in this
operator order, i.e. both c / c+ pairs of the particle-hole channel carry one
spin each; the tests establish which arrangement and which overall sign
reproduce the closed form.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy.linalg import expm


def fock_operators():
    """Annihilators c_up, c_dn on |n_up n_dn>: basis |00>,|10>,|01>,|11>."""
    c_up = np.zeros((4, 4))
    c_dn = np.zeros((4, 4))
    c_up[0, 1] = 1.0          # c_up |10> = |00>
    c_up[2, 3] = 1.0          # c_up |11> = c_up c+_up c+_dn |0> = |01>
    c_dn[0, 2] = 1.0          # c_dn |01> = |00>
    c_dn[1, 3] = -1.0         # c_dn c+_up c+_dn |0> = -c+_up |0>
    return c_up, c_dn


def energies(U: float, mu: float) -> np.ndarray:
    return np.array([0.0, -mu, -mu, U - 2.0 * mu])


def lehmann_g(nu: np.ndarray, beta: float, U: float, mu: float) -> np.ndarray:
    """g(i nu) = -<T c c+>(i nu) by the Lehmann sum (spin up)."""
    c_up, _ = fock_operators()
    E = energies(U, mu)
    E = E - E.min()
    w = np.exp(-beta * E)
    Z = w.sum()
    out = np.zeros(np.shape(nu), dtype=np.complex128)
    for i in range(4):
        for j in range(4):
            a = c_up[i, j]
            if a == 0.0:
                continue
            out += a * a * (w[i] + w[j]) / (Z * (1j * np.asarray(nu) - (E[j] - E[i])))
    return out


def divided_difference_exp(beta: float, z) -> complex:
    """f[z0..zn] for f(z) = exp(-beta z), exact at coinciding points."""
    n = len(z)
    J = np.diag(np.asarray(z, dtype=np.complex128)) + np.diag(np.ones(n - 1), 1)
    return expm(-beta * J)[0, n - 1]


def g2_ordered(ops, freqs, beta: float, U: float, mu: float) -> complex:
    """int_0^beta dt1 dt2 dt3 e^{i sum_a s_a w_a t_a} <T O1(t1) O2(t2) O3(t3) O4(0)>.

    ops  : four 4x4 matrices O1..O4 (O4 sits at tau = 0)
    freqs: three signed frequencies x_a (O_a(t_a) carries e^{i x_a t_a})
    """
    E = energies(U, mu)
    E = E - E.min()
    Z = np.exp(-beta * E).sum()
    total = 0.0 + 0.0j
    for perm in itertools.permutations(range(3)):
        # perm lists operator indices from the latest time to the earliest
        # time (tau_a > tau_b > tau_c > 0); fermionic sign of the reordering
        inv = sum(1 for x in range(3) for y in range(x + 1, 3) if perm[x] > perm[y])
        sign = -1.0 if inv % 2 else 1.0
        A, B, C = (ops[p] for p in perm)
        xa, xb, xc = (freqs[p] for p in perm)
        D = ops[3]
        for i in range(4):
            for j in range(4):
                if A[i, j] == 0.0:
                    continue
                for k in range(4):
                    if B[j, k] == 0.0:
                        continue
                    for l in range(4):
                        if C[k, l] == 0.0 or D[l, i] == 0.0:
                            continue
                        amp = A[i, j] * B[j, k] * C[k, l] * D[l, i]
                        pts = [E[i], E[j] - 1j * xa, E[k] - 1j * (xa + xb),
                               E[l] - 1j * (xa + xb + xc)]
                        total += sign * amp * (-1.0) ** 3 * divided_difference_exp(beta, pts)
    return total / Z


def vertex_ed(spins, nu, nup, Om, beta: float, U: float, mu: float) -> complex:
    """Amputated connected two-particle function for spins (s1, s2, s3, s4).

    Operator string c_{s1}(w1) c+_{s2}(w2) c_{s3}(w3) c+_{s4}(w4) with
    w1 = nu, w2 = nu + Om, w3 = nu' + Om, w4 = nu'.  Returns
    [G2 - disconnected] / (g1 g2 g3 g4); spins are 0 (up) or 1 (dn).
    """
    c = fock_operators()
    s1, s2, s3, s4 = spins
    ops = [c[s1], c[s2].T, c[s3], c[s4].T]
    w1, w2, w3, w4 = nu, nu + Om, nup + Om, nup
    G2 = g2_ordered(ops, [w1, -w2, w3], beta, U, mu)
    g = lambda w: complex(lehmann_g(np.array([w]), beta, U, mu)[0])
    disc = 0.0 + 0.0j
    tol = 1e-12 * max(1.0, abs(nu) + abs(nup) + abs(Om))
    # <T c1 c+2><T c3 c+4>: both pairs diagonal in spin, needs w1 == w2
    if s1 == s2 and s3 == s4 and abs(Om) < tol:
        disc += beta * g(w1) * g(w3)
    # -<T c1 c+4><T c3 c+2>: needs w2 == w3, i.e. nu == nu'
    if s1 == s4 and s2 == s3 and abs(nu - nup) < tol:
        disc -= beta * g(w1) * g(w3)
    return (G2 - disc) / (g(w1) * g(w2) * g(w3) * g(w4))
