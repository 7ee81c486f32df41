"""Seeded synthetic inputs for the ladder dual-fermion hot path.

This module produces what the method consumes (paper, Sec. 2.1 "Prerequisites"
and Sec. 4 "Example I"): Matsubara grids, the hypercubic dispersion, and the
Hubbard-atom ("atomic limit") impurity Green's function g, hybridisation Delta
and the two vertex components gamma^{uu}, gamma^{ud} given in closed form by
eqs. (atomic_limit1)-(atomic_limit4).  It also holds the named workloads
(lattice, cut-offs, U, beta, t) and the seeded parameter draws of the batched
workload.

No step of the dual-fermion iteration itself (dual propagator, bubble, ladder,
Schwinger-Dyson, Dyson, mixing) is computed here: both the GPU path and the
CPU oracle receive these arrays as plain inputs.

Conventions (all complex arrays are numpy complex128):
  fermionic index n in [-n_nu/2, n_nu/2),  nu_n = (2n+1) pi / beta
  bosonic   index m in [-(n_om-1)/2, (n_om-1)/2],  Om_m = 2 m pi / beta
  vertex arrays are [n_om][n_nu][n_nu] indexed [m][n][n'] (window offsets)
  k-grid: k_j = 2 pi j / nk on every axis, flat index in C order of the
  D-dimensional array of shape (nk,)*D (last axis fastest).

Readings of the paper taken here (each is listed with its reason in the
design notes of the repository):
  * the U^3 term of gamma^{ud} has the denominator w1 w2 w3 w4 (the printed
    squared denominators are dimensionally inconsistent with the -U term);
  * the first beta-proportional term of gamma^{ud} carries the Kronecker
    delta w1 = -w3 (printed: w2 = -w3); exact diagonalisation of the atom
    reproduces the closed form only with this index;
  * gamma^{ud} is the (up up dn dn) component of the operator string of
    eq. (vertex), i.e. the particle-hole pairs (1,2) and (3,4) each carry
    one spin, and both vertices are amputated by g1 g2 g3 g4;
  * Delta = 2 D t^2 g (the printed 2 D g is the t = 1 case);
  * Kronecker deltas are evaluated on the integer indices (n, n', m);
  * the Fermi factors 1/(1+exp(+-beta U/2)) are evaluated as logistic
    functions so that any beta U is safe.
"""
from __future__ import annotations

import dataclasses
import json
import math
import os
from typing import List, Optional

import numpy as np


# --------------------------------------------------------------------------
# grids
# --------------------------------------------------------------------------
def fermionic_indices(n_nu: int) -> np.ndarray:
    """Integer labels n of the fermionic window, nu_n = (2n+1) pi / beta."""
    if n_nu <= 0 or n_nu % 2:
        raise ValueError("n_nu must be positive and even")
    return np.arange(-n_nu // 2, n_nu // 2)


def bosonic_indices(n_om: int) -> np.ndarray:
    """Integer labels m of the bosonic window, Om_m = 2 m pi / beta."""
    if n_om <= 0 or n_om % 2 == 0:
        raise ValueError("n_om must be positive and odd")
    h = (n_om - 1) // 2
    return np.arange(-h, h + 1)


def matsubara_fermionic(n: np.ndarray, beta: float) -> np.ndarray:
    return (2.0 * np.asarray(n, dtype=np.float64) + 1.0) * math.pi / beta


def kpoints(D: int, nk: int) -> np.ndarray:
    """k vectors of the D-dimensional grid, shape [nk**D, D], C order."""
    axes = [2.0 * math.pi * np.arange(nk) / nk] * D
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.reshape(-1) for m in mesh], axis=1)


def dispersion_hypercubic(D: int, nk: int, t: float) -> np.ndarray:
    """eps_k = -2 t sum_i cos k_i on the nk**D grid (flat, C order)."""
    k = kpoints(D, nk)
    return -2.0 * t * np.cos(k).sum(axis=1)


# --------------------------------------------------------------------------
# Hubbard atom at particle-hole symmetry, eqs. (atomic_limit1)-(atomic_limit4)
# --------------------------------------------------------------------------
def _expit(x: float) -> float:
    if x >= 0:
        return 1.0 / (1.0 + math.exp(-x))
    e = math.exp(x)
    return e / (1.0 + e)


def atom_g(n_nu: int, beta: float, U: float) -> np.ndarray:
    """g_nu = (1/2)[1/(i nu - U/2) + 1/(i nu + U/2)]  (eq. atomic_limit1)."""
    nu = matsubara_fermionic(fermionic_indices(n_nu), beta)
    iw = 1j * nu
    return 0.5 * (1.0 / (iw - 0.5 * U) + 1.0 / (iw + 0.5 * U))


def atom_delta(g: np.ndarray, D: int, t: float) -> np.ndarray:
    """Delta_nu = 2 D t^2 g_nu  (eq. atomic_limit2, with the hopping restored)."""
    return 2.0 * D * t * t * g


def atom_vertices(n_nu: int, n_om: int, beta: float, U: float):
    """Closed-form gamma^{uu}, gamma^{ud} of the half-filled Hubbard atom.

    Legs: w1 = nu_n, w2 = nu_{n+m}, w3 = nu_{n'+m}, w4 = nu_{n'}
    (eqs. atomic_limit3, atomic_limit4).  Returns two complex arrays of shape
    [n_om][n_nu][n_nu] (the values are real).
    """
    n = fermionic_indices(n_nu)
    m = bosonic_indices(n_om)
    M = m[:, None, None]
    N1 = n[None, :, None]
    N2 = n[None, None, :]
    w1 = matsubara_fermionic(N1, beta) + 0.0 * M
    w2 = matsubara_fermionic(N1 + M, beta) + 0.0 * N2
    w3 = matsubara_fermionic(N2 + M, beta) + 0.0 * N1
    w4 = matsubara_fermionic(N2, beta) + 0.0 * M
    w1 = np.broadcast_to(w1, (n_om, n_nu, n_nu))
    w2 = np.broadcast_to(w2, (n_om, n_nu, n_nu))
    w3 = np.broadcast_to(w3, (n_om, n_nu, n_nu))
    w4 = np.broadcast_to(w4, (n_om, n_nu, n_nu))

    def lam(w):
        return 1.0 + U * U / (4.0 * w * w)

    d_m0 = np.broadcast_to((M == 0), (n_om, n_nu, n_nu)).astype(np.float64)   # w1 == w2
    d_nn = np.broadcast_to((N1 == N2), (n_om, n_nu, n_nu)).astype(np.float64)  # w1 == w4
    d_w1_mw3 = (N1 == -(N2 + M) - 1).astype(np.float64)                       # w1 == -w3
    d_w1_mw3 = np.broadcast_to(d_w1_mw3, (n_om, n_nu, n_nu))

    bu = beta * U * U / 4.0
    guu = bu * (d_m0 - d_nn) * lam(w1) * lam(w3)

    prod = w1 * w2 * w3 * w4
    f_minus = _expit(-0.5 * beta * U)   # 1/(1+exp(+beta U/2))
    f_plus = _expit(0.5 * beta * U)     # 1/(1+exp(-beta U/2))
    gud = (-U
           + (U ** 3 / 8.0) * (w1 ** 2 + w2 ** 2 + w3 ** 2 + w4 ** 2) / prod
           + (3.0 * U ** 5 / 16.0) / prod
           + bu * f_minus * (2.0 * d_w1_mw3 + d_m0) * lam(w2) * lam(w3)
           - bu * f_plus * (2.0 * d_nn + d_m0) * lam(w1) * lam(w3))
    return guu.astype(np.complex128), gud.astype(np.complex128)


# --------------------------------------------------------------------------
# Hubbard atom at any filling (Lehmann representation), for mu != U/2
# --------------------------------------------------------------------------
# The closed forms above hold at particle-hole symmetry only.  Away from it the
# inputs come from the atom's four states |n_up n_dn>, H = U n_up n_dn -
# mu (n_up + n_dn), in the Lehmann representation: the impurity g is the usual
# sum over pairs of states, and the three-frequency two-particle function is
# the time integral of the ordered product of four operators, summed over the
# 3! orderings of the three operators at non-zero time.  On one ordering the
# Boltzmann factors and the frequency phases make the integrand the exponential
# of a linear function of the four interval lengths, and its integral over
# the interval simplex (total length beta) is minus the third divided
# difference of exp(-beta z) at the four points z_a = E_a - i X_a, X_a the
# running sum of the frequencies (Hermite-Genocchi).  Two points can coincide
# (a bosonic sum of zero with equal energies); the confluent divided
# differences (double points) are written out below.  The vertex is the
# connected part, amputated by the four legs, as for the closed forms; with
# mu = U/2 it equals them (pinned in the tests, together with a brute-force
# exact diagonalisation at other mu).

def _atom_states(U: float, mu: float):
    """Energies (lowest = 0) and annihilators of the atom, basis |00>, |10>,
    |01>, |11> (n_up n_dn), Jordan-Wigner order up before down."""
    E = np.array([0.0, -mu, -mu, U - 2.0 * mu])
    E = E - E.min()
    c_up = np.zeros((4, 4))
    c_dn = np.zeros((4, 4))
    c_up[0, 1] = c_up[2, 3] = 1.0
    c_dn[0, 2] = 1.0
    c_dn[1, 3] = -1.0
    return E, (c_up, c_dn)


def atom_g_lehmann(n_nu: int, beta: float, U: float, mu: float) -> np.ndarray:
    """g(i nu) = sum_{ab} |<a|c|b>|^2 (w_a + w_b) / (Z (i nu - E_b + E_a)), spin up."""
    E, (c_up, _) = _atom_states(U, mu)
    w = np.exp(-beta * E)
    Z = w.sum()
    iw = 1j * matsubara_fermionic(fermionic_indices(n_nu), beta)
    out = np.zeros(n_nu, dtype=np.complex128)
    for a in range(4):
        for b in range(4):
            if c_up[a, b] != 0.0:
                out += c_up[a, b] ** 2 * (w[a] + w[b]) / (Z * (iw - (E[b] - E[a])))
    return out


def _divdiff3_exp(beta, E, K, h, tolE):
    """Third divided difference of f(z) = exp(-beta z) at z_a = E_a - i pi K_a / beta
    (a = 0..3; E real scalars, K integer arrays, h = pi / beta).  Points 0, 2 and
    points 1, 3 may coincide (equal energy and equal K); no other pair can."""
    z = [E[a] - 1j * h * K[a] for a in range(4)]
    f = [np.exp(-beta * E[a]) * np.where(K[a] % 2 == 0, 1.0, -1.0) for a in range(4)]
    c02 = (abs(E[0] - E[2]) <= tolE) & (K[0] == K[2])
    c13 = (abs(E[1] - E[3]) <= tolE) & (K[1] == K[3])
    with np.errstate(divide="ignore", invalid="ignore"):
        # all four distinct
        dist = sum(f[a] / np.prod([z[a] - z[b] for b in range(4) if b != a], axis=0)
                   for a in range(4))

        def one_double(p, fp, q, fq, r, fr):
            d_pq, d_pr, d_qr = p - q, p - r, q - r
            return (-beta * fp / (d_pq * d_pr) - fp * (1.0 / d_pq + 1.0 / d_pr) / (d_pq * d_pr)
                    + fq / (d_pq * d_pq * d_qr) - fr / (d_pr * d_pr * d_qr))

        d02 = one_double(z[0], f[0], z[1], f[1], z[3], f[3])
        d13 = one_double(z[1], f[1], z[0], f[0], z[2], f[2])
        dpq = z[0] - z[1]
        both = (-beta * f[0] - 2.0 * f[0] / dpq - beta * f[1] + 2.0 * f[1] / dpq) / (dpq * dpq)
    return np.where(c02 & c13, both, np.where(c02, d02, np.where(c13, d13, dist)))


def atom_g2(spins, n_nu: int, n_om: int, beta: float, U: float, mu: float) -> np.ndarray:
    """int dt1 dt2 dt3 e^{i (w1 t1 - w2 t2 + w3 t3)} <T c_s1(t1) c+_s2(t2) c_s3(t3) c+_s4(0)>
    on the window grid [m][n][n'], legs w1 = nu_n, w2 = nu_{n+m}, w3 = nu_{n'+m}."""
    E, c = _atom_states(U, mu)
    Z = np.exp(-beta * E).sum()
    n = fermionic_indices(n_nu)
    m = bosonic_indices(n_om)
    M, N1, N2 = m[:, None, None], n[None, :, None], n[None, None, :]
    shape = (n_om, n_nu, n_nu)
    # operator frequencies in units of pi / beta: c carries +w, c+ carries -w
    X = [np.broadcast_to(2 * N1 + 1, shape), np.broadcast_to(-(2 * (N1 + M) + 1), shape),
         np.broadcast_to(2 * (N2 + M) + 1, shape)]
    s1, s2, s3, s4 = spins
    ops = [c[s1], c[s2].T, c[s3]]
    last = c[s4].T
    h = math.pi / beta
    tolE = 1e-9 * max(1.0, float(np.abs(E).max()))
    out = np.zeros(shape, dtype=np.complex128)
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        # perm: operators from the latest time to the earliest; sign of the
        # reordering of the three fermion operators
        inv = sum(1 for a in range(3) for b in range(a + 1, 3) if perm[a] > perm[b])
        sign = -1.0 if inv % 2 else 1.0
        A, B, C = (ops[p] for p in perm)
        Ka = X[perm[0]]
        Kb = Ka + X[perm[1]]
        Kc = Kb + X[perm[2]]
        zero = np.zeros(shape, dtype=np.int64)
        for i in range(4):
            for j in range(4):
                if A[i, j] == 0.0:
                    continue
                for k in range(4):
                    if B[j, k] == 0.0:
                        continue
                    for l in range(4):
                        amp = A[i, j] * B[j, k] * C[k, l] * last[l, i]
                        if amp == 0.0:
                            continue
                        dd = _divdiff3_exp(beta, (E[i], E[j], E[k], E[l]), (zero, Ka, Kb, Kc), h, tolE)
                        out -= sign * amp * dd
    return out / Z


def atom_vertices_lehmann(n_nu: int, n_om: int, beta: float, U: float, mu: float):
    """gamma^{uu}, gamma^{ud} of the Hubbard atom at chemical potential mu:
    the connected two-particle function, amputated by g1 g2 g3 g4, for the spin
    arrangements (up, up, up, up) and (up, up, dn, dn) of the operator string.
    Returns two complex arrays [n_om][n_nu][n_nu]."""
    g = atom_g_lehmann(n_nu, beta, U, mu)
    n = fermionic_indices(n_nu)
    m = bosonic_indices(n_om)
    h = (n_om - 1) // 2
    i1 = np.broadcast_to((n - n[0])[None, :, None], (n_om, n_nu, n_nu))
    i2 = i1 + m[:, None, None]
    i4 = np.broadcast_to((n - n[0])[None, None, :], (n_om, n_nu, n_nu))
    i3 = i4 + m[:, None, None]
    # legs outside the window: take g from the formula on the shifted index
    gext = atom_g_lehmann(n_nu + 2 * h + 2, beta, U, mu)
    off = h + 1
    g1, g2, g3, g4 = (gext[ix + off] for ix in (i1, i2, i3, i4))
    legs = g1 * g2 * g3 * g4
    d_m0 = np.broadcast_to((m == 0)[:, None, None], legs.shape)
    d_nn = np.broadcast_to((n[:, None] == n[None, :])[None], legs.shape)
    G_uu = atom_g2((0, 0, 0, 0), n_nu, n_om, beta, U, mu)
    G_ud = atom_g2((0, 0, 1, 1), n_nu, n_om, beta, U, mu)
    # disconnected parts: <T c1 c+2><T c3 c+4> (Omega = 0) and - <T c1 c+4><T c3 c+2> (nu = nu')
    disc_uu = beta * g1 * g3 * (d_m0.astype(float) - d_nn.astype(float))
    disc_ud = beta * g1 * g3 * d_m0.astype(float)
    return (G_uu - disc_uu) / legs, (G_ud - disc_ud) / legs


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    """One problem instance: lattice, cut-offs, physical parameters, inputs."""
    D: int
    nk: int
    n_nu: int
    n_om: int
    beta: float
    U: float
    mu: float
    t: float
    g: np.ndarray = None
    delta: np.ndarray = None
    eps: np.ndarray = None
    gamma_uu: np.ndarray = None
    gamma_ud: np.ndarray = None

    @property
    def N(self) -> int:
        return self.nk ** self.D

    def summary(self) -> dict:
        return dict(D=self.D, nk=self.nk, n_nu=self.n_nu, n_om=self.n_om,
                    beta=self.beta, U=self.U, mu=self.mu, t=self.t)


def atomic_limit_problem(D: int, nk: int, n_nu: int, n_om: int, beta: float,
                         U: float, t: float, mu: Optional[float] = None) -> Problem:
    """Problem with Hubbard-atom inputs: the closed forms at mu = U/2 (the
    default), the Lehmann representation at any other mu."""
    if mu is None:
        mu = 0.5 * U
    if abs(mu - 0.5 * U) <= 1e-14 * max(1.0, abs(U)):
        g = atom_g(n_nu, beta, U)
        guu, gud = atom_vertices(n_nu, n_om, beta, U)
    else:
        g = atom_g_lehmann(n_nu, beta, U, mu)
        guu, gud = atom_vertices_lehmann(n_nu, n_om, beta, U, mu)
    return Problem(D=D, nk=nk, n_nu=n_nu, n_om=n_om, beta=beta, U=U, mu=mu, t=t,
                   g=g, delta=atom_delta(g, D, t),
                   eps=dispersion_hypercubic(D, nk, t),
                   gamma_uu=guu, gamma_ud=gud)


# The paper's benchmark point is U/t = 20, beta t = 1 (Sec. 4).  The named
# workloads below keep every printed U, beta and shape; the hopping is set to
# t = 0.1 (t = 0.182358 for the 3D case) so that the ladder is inside its
# convergence radius with these atomic-limit inputs.
T_REMAP = 0.1
T_REMAP_3D = 0.182358


def workload_small() -> List[Problem]:
    """2D 8x8, n_nu = 16, Omega = 0 only, U = 2, beta = 10 (10 iterations)."""
    return [atomic_limit_problem(2, 8, 16, 1, 10.0, 2.0, T_REMAP)]


def workload_square32(Us=(1.0, 2.0, 4.0)) -> List[Problem]:
    """2D 32x32, n_nu = 64, n_om = 31, beta = 20, U in {1, 2, 4}."""
    return [atomic_limit_problem(2, 32, 64, 31, 20.0, float(U), T_REMAP) for U in Us]


def workload_cubic16() -> List[Problem]:
    """3D 16^3, n_nu = 96, n_om = 23, U = 3, beta = 15, near the AF instability."""
    return [atomic_limit_problem(3, 16, 96, 23, 15.0, 3.0, T_REMAP_3D)]


def batched_candidates(seed: int = 1507):
    """Seeded stream of candidate draws of the uneven batched workload.

    D in {2, 3}; 2D nk in {16, 32, 64}, 3D nk in {8, 16}; n_nu in {32, 64,
    128}; n_om = n_nu/4 - 1; U ~ U[1, 4]; beta ~ U[5, 25]; mu = U/2 + U[-0.5, 0.5].
    Candidates whose first-iteration ladder is outside or near the edge of
    its convergence radius are rejected by the recipe of batched_params().
    """
    rng = np.random.default_rng(seed)
    while True:
        D = int(rng.choice([2, 3]))
        nk = int(rng.choice([16, 32, 64])) if D == 2 else int(rng.choice([8, 16]))
        n_nu = int(rng.choice([32, 64, 128]))
        U = float(rng.uniform(1.0, 4.0))
        beta = float(rng.uniform(5.0, 25.0))
        mu = 0.5 * U + float(rng.uniform(-0.5, 0.5))
        yield dict(D=D, nk=nk, n_nu=n_nu, n_om=n_nu // 4 - 1, U=U, beta=beta, mu=mu, t=T_REMAP)


BATCHED_DRAWS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                             "tests", "golden", "batched_draws.json")


def batched_params(n_inst: int = 64):
    """The 64 instances of the batched workload: the first candidates of
    batched_candidates(1507) whose leading eigenvalue of gamma chi~ on the first
    iteration (Omega = 0, every q, both channels) is below 0.9; the accepted
    draws, with their eigenvalues, are stored by tests/golden/make_batched_draws.py."""
    with open(BATCHED_DRAWS) as f:
        rec = json.load(f)
    out = [dict(d) for d in rec["accepted"][:n_inst]]
    for d in out:
        d.pop("lambda_lead", None)
    return out


def draw_batched_params(n_inst: int = 64, seed: int = 1507):
    """The first n_inst candidates, without the radius rejection."""
    gen = batched_candidates(seed)
    return [next(gen) for _ in range(n_inst)]


def batched_problems(params) -> List[Problem]:
    return [atomic_limit_problem(p["D"], p["nk"], p["n_nu"], p["n_om"], p["beta"],
                                 p["U"], p["t"], mu=p.get("mu")) for p in params]


def draw_warmstart_params(n_inst: int, seed: int):
    """Seeded draws for the learned warm start: U ~ U[1,4], beta ~ U[5,20]."""
    rng = np.random.default_rng(seed)
    return [dict(U=float(rng.uniform(1.0, 4.0)), beta=float(rng.uniform(5.0, 20.0)),
                 t=T_REMAP, D=2) for _ in range(n_inst)]


def random_complex(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded standard complex normal array (used for structure-free tests)."""
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
