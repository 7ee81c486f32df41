"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks one oracle function against something other than itself:
exact diagonalisation, algebraic identities, brute force, library special
cases, closed-form sum rules and symmetries.  None of these needs a GPU.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import atom_ed
from oracle import df_oracle as O
from paper_1507_00895_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def nu_of(n, beta):
    return (2 * n + 1) * math.pi / beta


def small_problem(D=2, nk=4, n_nu=6, n_om=3, beta=2.0, U=4.0, t=0.2):
    return I.atomic_limit_problem(D, nk, n_nu, n_om, beta, U, t)


# ---------------------------------------------------------------- P1, P2: inputs
@pytest.mark.parametrize("beta,U", [(2.0, 1.5), (1.0, 2.0), (5.0, 3.0)])
def test_p1_closed_form_vertex_matches_exact_diagonalisation(beta, U):
    """eqs. atomic_limit3/4 (with the readings of the inputs module) == ED of the atom."""
    n_nu, n_om = 6, 5
    guu, gud = I.atom_vertices(n_nu, n_om, beta, U)
    ns, ms = I.fermionic_indices(n_nu), I.bosonic_indices(n_om)
    scale = max(np.abs(guu).max(), np.abs(gud).max())
    for im, m in enumerate(ms):
        for i, n in enumerate(ns):
            for j, npr in enumerate(ns):
                args = (nu_of(n, beta), nu_of(npr, beta), 2 * m * math.pi / beta, beta, U, U / 2)
                a = atom_ed.vertex_ed((0, 0, 0, 0), *args)
                b = atom_ed.vertex_ed((0, 0, 1, 1), *args)
                assert abs(a - guu[im, i, j]) <= 1e-12 * scale
                assert abs(b - gud[im, i, j]) <= 1e-12 * scale


def test_p1_printed_delta_would_fail():
    """The printed delta(w2, -w3) of the first beta-term disagrees with ED."""
    beta, U = 2.0, 1.5
    # entry where w2 = -w3 but w1 != -w3: m = -2, n = 1, n' = 2
    n, npr, m = 1, 2, -2
    assert (n + m) == -(npr + m) - 1 and n != -(npr + m) - 1
    ed = atom_ed.vertex_ed((0, 0, 1, 1), nu_of(n, beta), nu_of(npr, beta), 2 * m * math.pi / beta,
                           beta, U, U / 2)
    _, gud = I.atom_vertices(6, 5, beta, U)
    assert abs(ed - gud[0, n + 3, npr + 3]) < 1e-12
    lam = lambda w: 1 + U * U / (4 * w * w)
    printed_extra = (beta * U * U / 4) / (1 + math.exp(beta * U / 2)) * 2 * \
        lam(nu_of(n + m, beta)) * lam(nu_of(npr + m, beta))
    assert abs(printed_extra) > 0.1


def test_p2_g_matches_lehmann_and_identity():
    beta, U = 3.0, 2.5
    g = I.atom_g(16, beta, U)
    nu = I.matsubara_fermionic(I.fermionic_indices(16), beta)
    assert np.allclose(g, atom_ed.lehmann_g(nu, beta, U, U / 2), rtol=1e-14, atol=0)
    lam = 1 + U * U / (4 * nu * nu)
    assert np.allclose(1.0 / g, 1j * nu * lam, rtol=1e-14, atol=0)


def test_high_frequency_limit_of_vertex():
    """gamma^{ud} -> -U and gamma^{uu} -> 0 far from the low frequencies."""
    beta, U = 10.0, 1.0
    guu, gud = I.atom_vertices(400, 3, beta, U)
    # m = -1, n = -200, n' = -197: no Kronecker delta is active
    assert abs(gud[0, 0, 3] + U) < 1e-3
    assert abs(guu[0, 0, 3]) == 0.0


# ---------------------------------------------------------------- P3: dual propagator
def test_p3_gd0_identity_and_symmetries():
    p = I.atomic_limit_problem(2, 8, 16, 1, 10.0, 2.0, 0.1)
    G0 = O.dual_gf0(p.g, p.delta, p.eps)
    x = (p.delta[:, None] - p.eps[None, :])
    alt = -p.g[:, None] ** 2 * x / (1 + p.g[:, None] * x)
    assert np.allclose(G0, alt, rtol=1e-13, atol=0)
    # conjugation: G(-nu) = G(nu)*  (nu_{-n-1} = -nu_n)
    assert np.allclose(G0[::-1], np.conj(G0), rtol=1e-14, atol=0)
    # particle-hole at mu = U/2: G0(k+Q) = -G0(k)*
    c = O._coords(2, 8)
    kQ = O._flat(c + 4, 8)
    assert np.allclose(G0[:, kQ], -np.conj(G0), rtol=1e-13, atol=1e-30)
    # point group: swap the two axes and reflect one
    G2 = G0.reshape(16, 8, 8)
    assert np.allclose(G2, G2.transpose(0, 2, 1), rtol=1e-14)
    assert np.allclose(G2, G2[:, (-np.arange(8)) % 8, :], rtol=1e-14)


def test_dual_dyson_through_the_lattice_dyson_equation():
    """eq. (dyson) checked through physics, not by restating it: the G~ of
    O.dual_gf, put into the lattice Green's function of eq. (glat), must obey
    the lattice Dyson equation G^-1 = i nu + mu - eps - Sigma that the paper
    states between eqs. (sigma_lat) and (glat), with Sigma from eq. (sigma_lat)
    (denominator 1 + g Sigma~, the reading that makes the stated relation hold
    for the G~ of eqs. gd0 and dyson) and Sigma^DMFT = i nu + mu - Delta - 1/g.
    Both are written out here.  Generic complex g, Delta, Sigma~ and real eps; a
    wrong sign of Sigma~ or an inverted G~0 in the dual Dyson equation fails."""
    rng = np.random.default_rng(31)
    n_nu, N, mu, beta = 6, 10, 0.4, 2.5
    c = lambda *sh: rng.standard_normal(sh) + 1j * rng.standard_normal(sh)
    g, delta, eps, S = c(n_nu), c(n_nu), rng.standard_normal(N), 0.3 * c(n_nu, N)
    G = O.dual_gf(O.dual_gf0(g, delta, eps), S)
    nu = ((2 * I.fermionic_indices(n_nu) + 1) * math.pi / beta)[:, None]
    gg, dd, ee = g[:, None], delta[:, None], eps[None, :]
    a = 1.0 / (dd - ee)
    G_lat = a + a * (1.0 / gg) * G * (1.0 / gg) * a                       # eq. (glat)
    sigma_dmft = 1j * nu + mu - dd - 1.0 / gg
    sigma_lat = S / (1.0 + gg * S) + sigma_dmft                           # eq. (sigma_lat)
    lhs = G_lat * (1j * nu + mu - ee - sigma_lat)
    assert np.abs(lhs - 1.0).max() <= 1e-11
    # the opposite sign of Sigma~ in the dual Dyson equation breaks the relation
    Gw = O.dual_gf(O.dual_gf0(g, delta, eps), -S)
    lhs_w = (a + a * (1.0 / gg) * Gw * (1.0 / gg) * a) * (1j * nu + mu - ee - sigma_lat)
    assert np.abs(lhs_w - 1.0).max() > 1e-2


def test_leading_eigenvalue_of_a_rank_one_vertex():
    """For gamma = u v^T the matrix gamma diag(chi) has the single nonzero
    eigenvalue sum_j v_j chi_j u_j (closed form); the diagnostic returns its
    real part when it is positive, else zero."""
    rng = np.random.default_rng(41)
    n_nu, N, n_om = 5, 7, 3
    u = rng.standard_normal(n_nu) + 1j * rng.standard_normal(n_nu)
    v = rng.standard_normal(n_nu) + 1j * rng.standard_normal(n_nu)
    gam = np.zeros((2, n_om, n_nu, n_nu), dtype=complex)
    gam[1, 1] = np.outer(u, v)
    chi = rng.standard_normal((n_om, n_nu, N)) + 1j * rng.standard_normal((n_om, n_nu, N))
    lam = O.leading_eigenvalue(gam, chi, 1, 1)
    want = np.maximum(np.real(np.einsum("j,jq,j->q", v, chi[1], u)), 0.0)
    assert np.allclose(lam, want, rtol=1e-10, atol=1e-12)


def test_dyson_definition():
    rng = np.random.default_rng(3)
    G0 = rng.standard_normal((4, 9)) + 1j * rng.standard_normal((4, 9))
    S = 0.1 * (rng.standard_normal((4, 9)) + 1j * rng.standard_normal((4, 9)))
    G = O.dual_gf(G0, S)
    assert np.allclose(1.0 / G, 1.0 / G0 - S, rtol=1e-13)
    assert np.allclose(G, G0 / (1 - G0 * S), rtol=1e-13)


# ---------------------------------------------------------------- P4: bubble
def _brute_bubble(G, D, nk, n_om, beta):
    """Explicit nested loops over (m, n, q, k) with per-axis index arithmetic."""
    n_nu, N = G.shape
    T = 1.0 / beta
    coords = list(np.ndindex(*((nk,) * D)))
    index = {c: i for i, c in enumerate(coords)}
    out = np.zeros((n_om, n_nu, N), dtype=complex)
    h = (n_om - 1) // 2
    for im in range(n_om):
        m = im - h
        for n in range(n_nu):
            if not (0 <= n + m < n_nu):
                continue
            for q, qc in enumerate(coords):
                s = 0j
                for k, kc in enumerate(coords):
                    kq = index[tuple((a + b) % nk for a, b in zip(kc, qc))]
                    s += G[n, k] * G[n + m, kq]
                out[im, n, q] = -T / N * s
    return out


@pytest.mark.parametrize("D,nk", [(2, 4), (2, 6), (3, 4), (1, 8), (4, 4)])
def test_p4_bubble_fft_and_direct_match_brute_force(D, nk):
    N = nk ** D
    G = I.random_complex((4, N), seed=10 + D * nk)
    ref = _brute_bubble(G, D, nk, 3, 2.5)
    for f in (O.bubble_direct, O.bubble_fft):
        chi = f(G, D, nk, 3, 2.5)
        assert np.abs(chi - ref).max() <= 1e-14 * np.abs(ref).max()


def test_p4_bubble_sum_rule_and_conjugation():
    p = I.atomic_limit_problem(2, 8, 16, 5, 10.0, 2.0, 0.1)
    G = O.dual_gf0(p.g, p.delta, p.eps)
    chi = O.bubble_fft(G, 2, 8, 5, p.beta)
    T = 1 / p.beta
    Gloc = G.mean(axis=1)
    for im, m in enumerate(O.bosonic_offsets(5)):
        for n in range(16):
            expect = -T * Gloc[n] * Gloc[n + m] if 0 <= n + m < 16 else 0
            assert abs(chi[im, n].mean() - expect) <= 1e-14 * np.abs(chi).max()
    # chi_{-m,-n-1}(q) = chi_{m,n}(q)*
    for im in range(5):
        for n in range(16):
            assert np.allclose(chi[4 - im, 15 - n], np.conj(chi[im, n]), rtol=1e-12, atol=1e-20)


# ---------------------------------------------------------------- P5: ladder
def test_p5_ladder_matches_neumann_series_and_eigenvalues():
    p = I.workload_small()[0]
    G = O.dual_gf0(p.g, p.delta, p.eps)
    chi = O.bubble_fft(G, p.D, p.nk, p.n_om, p.beta)
    gam = O.spin_channels(p.gamma_uu, p.gamma_ud)
    lr = O.ladder(gam, chi, with_eigs=True)
    assert np.all(lr.status == 0)
    for c in range(2):
        for q in (0, 9, 36):
            g_ = gam[c, 0]
            M = g_ * chi[0, :, q][None, :]
            # Neumann series sum_j M^j gamma (spectral radius 0.185 here)
            term = g_.copy()
            acc = g_.copy()
            for _ in range(60):
                term = M @ term
                acc = acc + term
            W = np.diag(acc) - 0.5 * np.diag(M @ g_)
            assert np.abs(W - lr.W[c, 0, :, q]).max() <= 1e-12 * np.abs(W).max()
            ev = np.linalg.eigvals(M)
            det = np.prod(1 - ev)
            assert abs(np.exp(lr.logdet[c, 0, q]) - det) <= 1e-12 * abs(det)
            # det is real at Omega = 0
            assert abs(det.imag) <= 1e-12 * abs(det)
            assert abs(lr.logdet[c, 0, q].imag) < 1e-12
    # the magnetic ladder is most unstable at Q = (pi, pi)
    Q = 4 * 8 + 4
    assert np.argmax(lr.lam[1, 0]) == Q


def test_p5_fallback_outside_radius():
    """Outside the radius: one ladder step, flagged, and det has Re <= 0."""
    p = I.atomic_limit_problem(2, 8, 16, 1, 10.0, 2.0, 0.3)
    G = O.dual_gf0(p.g, p.delta, p.eps)
    chi = O.bubble_fft(G, p.D, p.nk, p.n_om, p.beta)
    gam = O.spin_channels(p.gamma_uu, p.gamma_ud)
    lr = O.ladder(gam, chi, with_eigs=True)
    out = lr.status == 1
    assert out.any() and (~out).any()
    assert np.all(lr.lam[out] > 1.0)
    assert np.all(np.cos(lr.logdet[out].imag) <= 0)
    c, im, q = [a[0] for a in np.nonzero(out)]
    g_ = gam[c, im]
    M = g_ * chi[im, :, q][None, :]
    W = np.diag(g_) + 0.5 * np.diag(M @ g_)
    assert np.allclose(lr.W[c, im, :, q], W, rtol=1e-13)


# ---------------------------------------------------------------- P6: Schwinger-Dyson
def _brute_sigma_second_order(G, gam, D, nk, n_om, beta):
    """Second-order dual self-energy by explicit nested sums over (m, q, n'', k').

    Sigma_{n,k} = T/(2N) sum_{m,q} [3 (g^m_nn + 1/2 sum_n'' g^m_{n n''} chi_{m n''}(q) g^m_{n'' n})
                                   +   (g^d_nn + 1/2 sum_n'' g^d_{n n''} chi_{m n''}(q) g^d_{n'' n})]
                 * G_{n+m, k+q},
    chi_{m n''}(q) = -T/N sum_k' G_{n'',k'} G_{n''+m, k'+q}.
    """
    n_nu, N = G.shape
    T = 1.0 / beta
    coords = list(np.ndindex(*((nk,) * D)))
    index = {c: i for i, c in enumerate(coords)}
    add = lambda a, b: index[tuple((x + y) % nk for x, y in zip(coords[a], coords[b]))]
    h = (n_om - 1) // 2
    Gw = lambda n, k: G[n, k] if 0 <= n < n_nu else 0.0
    S = np.zeros((n_nu, N), dtype=complex)
    for n in range(n_nu):
        for k in range(N):
            s = 0j
            for im in range(n_om):
                m = im - h
                for q in range(N):
                    chi = [-T / N * sum(Gw(n2, kp) * Gw(n2 + m, add(kp, q)) for kp in range(N))
                           for n2 in range(n_nu)]
                    V = 0j
                    for c, w in ((1, 3.0), (0, 1.0)):
                        g_ = gam[c, im]
                        V += w * (g_[n, n] + 0.5 * sum(g_[n, n2] * chi[n2] * g_[n2, n]
                                                       for n2 in range(n_nu)))
                    s += V * Gw(n + m, add(k, q))
            S[n, k] = T / (2 * N) * s
    return S


def test_p6_second_order_sigma_matches_direct_diagrams():
    p = small_problem(D=2, nk=4, n_nu=4, n_om=3, beta=2.0, U=3.0, t=0.3)
    G = O.dual_gf0(p.g, p.delta, p.eps)
    gam = O.spin_channels(p.gamma_uu, p.gamma_ud)
    chi = O.bubble_fft(G, 2, 4, 3, p.beta)
    lr = O.ladder(gam, chi, mode="fallback")
    ref = _brute_sigma_second_order(G, gam, 2, 4, 3, p.beta)
    for f in (O.sigma_fft, O.sigma_direct):
        S = f(lr.W, G, 2, 4, p.beta)
        assert np.abs(S - ref).max() <= 1e-13 * np.abs(ref).max()


def test_p6_zero_vertex_gives_zero_sigma():
    p = I.workload_small()[0]
    z = np.zeros_like(p.gamma_uu)
    r = O.iterate(p.g, p.delta, p.eps, z, z, p.D, p.nk, p.beta, p.n_om, max_iter=3)
    assert np.all(r.sigma == 0)
    assert np.allclose(r.G, O.dual_gf0(p.g, p.delta, p.eps), rtol=1e-15, atol=0)


def test_p6_sigma_k_sum_rule_and_point_group():
    p = I.atomic_limit_problem(2, 8, 16, 5, 10.0, 2.0, 0.1)
    G = O.dual_gf0(p.g, p.delta, p.eps)
    gam = O.spin_channels(p.gamma_uu, p.gamma_ud)
    chi = O.bubble_fft(G, 2, 8, 5, p.beta)
    lr = O.ladder(gam, chi)
    S = O.sigma_fft(lr.W, G, 2, 8, p.beta)
    V = O.sigma_vertex(lr.W)
    T = 1 / p.beta
    Gloc = G.mean(axis=1)
    for n in range(16):
        expect = 0j
        for im, m in enumerate(O.bosonic_offsets(5)):
            if 0 <= n + m < 16:
                expect += 0.5 * T * V[im, n].mean() * Gloc[n + m]
        assert abs(S[n].mean() - expect) <= 1e-13 * np.abs(S).max()
    S2 = S.reshape(16, 8, 8)
    assert np.allclose(S2, S2.transpose(0, 2, 1), rtol=1e-11, atol=1e-15 * np.abs(S).max())
    assert np.allclose(S2, S2[:, (-np.arange(8)) % 8, :], rtol=1e-11, atol=1e-15 * np.abs(S).max())
    # conjugation symmetry of the dual self-energy
    assert np.allclose(S[::-1], np.conj(S), rtol=1e-11, atol=1e-15 * np.abs(S).max())


# ---------------------------------------------------------------- P7: loop
def test_p7_fixed_point_independent_of_mixing_and_start():
    p = I.workload_small()[0]
    args = (p.g, p.delta, p.eps, p.gamma_uu, p.gamma_ud, p.D, p.nk, p.beta, p.n_om)
    a = O.iterate(*args, alpha=0.5, tol=1e-12, max_iter=300)
    b = O.iterate(*args, alpha=0.3, tol=1e-12, max_iter=300)
    assert a.diff < 1e-12 and b.diff < 1e-12
    assert O.rel_diff(a.sigma, b.sigma) < 1e-10
    # residual of the fixed point map
    G = O.dual_gf(O.dual_gf0(p.g, p.delta, p.eps), a.sigma)
    gam = O.spin_channels(p.gamma_uu, p.gamma_ud)
    chi = O.bubble_fft(G, p.D, p.nk, p.n_om, p.beta)
    F = O.sigma_fft(O.ladder(gam, chi).W, G, p.D, p.nk, p.beta)
    assert O.rel_diff(F, a.sigma) < 1e-11
    # warm start from a perturbed solution reaches the same point
    c = O.iterate(*args, alpha=0.5, tol=1e-12, max_iter=300, sigma0=1.3 * a.sigma)
    assert O.rel_diff(c.sigma, a.sigma) < 1e-10


def test_iteration_direct_equals_fft_path():
    p = small_problem(D=2, nk=4, n_nu=6, n_om=3, beta=2.0, U=4.0, t=0.2)
    args = (p.g, p.delta, p.eps, p.gamma_uu, p.gamma_ud, p.D, p.nk, p.beta, p.n_om)
    a = O.iterate(*args, max_iter=4, direct=True)
    b = O.iterate(*args, max_iter=4, direct=False)
    assert O.rel_diff(a.sigma, b.sigma) < 1e-13


# ---------------------------------------------------------------- regression markers
def test_regression_markers_from_golden():
    """First-iteration leading eigenvalues and determinants (regression only)."""
    with open(os.path.join(GOLDEN, "regression_markers.json")) as f:
        gold = json.load(f)
    p = I.workload_small()[0]
    G = O.dual_gf0(p.g, p.delta, p.eps)
    chi = O.bubble_fft(G, p.D, p.nk, p.n_om, p.beta)
    gam = O.spin_channels(p.gamma_uu, p.gamma_ud)
    lr = O.ladder(gam, chi, with_eigs=True)
    Q = 4 * 8 + 4
    s = gold["small"]
    assert abs(lr.lam[1, 0, Q] - s["lam_m_Q"]) < 1e-12
    assert abs(np.exp(lr.logdet[1, 0, Q]).real - s["det_m_Q"]) < 1e-12
    assert abs(lr.lam[0, 0, 0] - s["lam_d_0"]) < 1e-12
    assert abs(np.exp(lr.logdet[0, 0, 0]).real - s["det_d_0"]) < 1e-12
    r = O.iterate(p.g, p.delta, p.eps, p.gamma_uu, p.gamma_ud, p.D, p.nk, p.beta, p.n_om,
                  alpha=0.5, max_iter=10)
    assert np.allclose(r.history, s["diff_history_10"], rtol=1e-10)


# ---------------------------------------------------------------- warm-start network reference
def test_mlp_reference_gradient_matches_finite_differences():
    from oracle import mlp_ref as R
    rng = np.random.default_rng(11)
    dims = [5, 7, 6, 3]
    n_par = sum(dims[l + 1] * dims[l] + dims[l + 1] for l in range(3))
    p = 0.4 * rng.standard_normal(n_par)
    X = rng.standard_normal((9, 5))
    T = rng.standard_normal((9, 3))
    loss, g = R.loss_grad(p, dims, X, T)
    h = 1e-6
    for i in rng.choice(n_par, 25, replace=False):
        e = np.zeros(n_par)
        e[i] = h
        fd = (R.loss_grad(p + e, dims, X, T)[0] - R.loss_grad(p - e, dims, X, T)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd))
    # a single linear layer reduces to least squares: gradient closed form
    W = rng.standard_normal((2, 4))
    b = rng.standard_normal(2)
    X1 = rng.standard_normal((6, 4))
    T1 = rng.standard_normal((6, 2))
    _, g1 = R.loss_grad(np.concatenate([W.ravel(), b]), [4, 2], X1, T1)
    r = X1 @ W.T + b - T1
    assert np.allclose(g1[:8].reshape(2, 4), 2 * r.T @ X1 / r.size)
    assert np.allclose(g1[8:], 2 * r.sum(0) / r.size)


# ---------------------------------------------------------------- warm-start host logic
def test_warmstart_features_are_point_group_invariant():
    from paper_1507_00895_amd import warmstart as W
    nk = 16
    f = W.k_features(nk).reshape(nk, nk, -1)
    i = np.arange(nk)
    assert np.allclose(f, f.transpose(1, 0, 2))                    # k_x <-> k_y
    assert np.allclose(f, f[(-i) % nk])                            # k_x -> -k_x
    assert np.allclose(f, f[:, (-i) % nk])                         # k_y -> -k_y
    # the 15 wedge points of the 8x8 grid cover every C4v orbit once
    orbits = set()
    for x in range(8):
        for y in range(8):
            a, b = min(x, 8 - x), min(y, 8 - y)
            orbits.add((max(a, b), min(a, b)))
    assert sorted(orbits) == sorted(W.WEDGE)


def test_warmstart_target_layout_round_trip():
    from paper_1507_00895_amd import warmstart as W
    cfg = W.WarmStartConfig(nk=4, n_nu=8, n_om=3)
    rng = np.random.default_rng(2)
    pos = rng.standard_normal((4, 16)) + 1j * rng.standard_normal((4, 16))
    sig = np.concatenate([np.conj(pos[::-1]), pos], axis=0)          # Sigma(-nu) = Sigma(nu)*
    rows = W.targets_from_sigma([sig], cfg)
    assert rows.shape == (16, 12)
    assert np.allclose(W.sigma_from_rows(rows, cfg), sig, rtol=1e-14, atol=0)
    assert np.allclose(rows[:, 8:], np.log(np.sqrt(np.mean(np.abs(sig) ** 2))))
