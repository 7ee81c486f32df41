"""Pins of the Hubbard-atom inputs away from half filling (the Lehmann
generator of the inputs module): against brute-force exact diagonalisation of
the atom (oracle/atom_ed.py) at mu != U/2, against the closed forms of Sec. 4
at mu = U/2, and the conjugation symmetry that the symmetry-reduced ladder
relies on."""
import math

import numpy as np
import pytest

from oracle import atom_ed
from paper_1507_00895_amd import inputs as I


@pytest.mark.parametrize("beta,U,mu", [(2.0, 1.5, 0.3), (2.0, 1.5, 1.4), (10.0, 3.0, 1.0),
                                       (5.0, 2.0, 2.6)])
def test_lehmann_vertex_matches_exact_diagonalisation(beta, U, mu):
    n_nu, n_om = 6, 5
    g = I.atom_g_lehmann(n_nu, beta, U, mu)
    nu = I.matsubara_fermionic(I.fermionic_indices(n_nu), beta)
    assert np.abs(g - atom_ed.lehmann_g(nu, beta, U, mu)).max() <= 1e-14 * np.abs(g).max()
    guu, gud = I.atom_vertices_lehmann(n_nu, n_om, beta, U, mu)
    scale = max(np.abs(guu).max(), np.abs(gud).max())
    for im, m in enumerate(I.bosonic_indices(n_om)):
        for i, n in enumerate(I.fermionic_indices(n_nu)):
            for j, npr in enumerate(I.fermionic_indices(n_nu)):
                args = ((2 * n + 1) * math.pi / beta, (2 * npr + 1) * math.pi / beta,
                        2 * m * math.pi / beta, beta, U, mu)
                assert abs(atom_ed.vertex_ed((0, 0, 0, 0), *args) - guu[im, i, j]) <= 1e-12 * scale
                assert abs(atom_ed.vertex_ed((0, 0, 1, 1), *args) - gud[im, i, j]) <= 1e-12 * scale


@pytest.mark.parametrize("beta,U", [(10.0, 2.0), (20.0, 4.0), (5.0, 1.0)])
def test_lehmann_vertex_equals_closed_form_at_half_filling(beta, U):
    cu, cd = I.atom_vertices(16, 7, beta, U)
    lu, ld = I.atom_vertices_lehmann(16, 7, beta, U, U / 2)
    assert np.abs(lu - cu).max() <= 1e-12 * np.abs(cu).max()
    assert np.abs(ld - cd).max() <= 1e-12 * np.abs(cd).max()
    assert np.abs(I.atom_g_lehmann(16, beta, U, U / 2) - I.atom_g(16, beta, U)).max() <= 1e-15


def test_off_half_filling_breaks_particle_hole_but_keeps_conjugation():
    """mu != U/2: g is no longer purely imaginary, the vertex no longer real;
    g(-nu) = g(nu)* and gamma_{-Om}(-nu, -nu') = gamma_Om(nu, nu')* still hold."""
    beta, U, mu = 8.0, 2.5, 1.6
    g = I.atom_g_lehmann(12, beta, U, mu)
    assert np.abs(g.real).max() > 1e-3
    assert np.abs(g[::-1] - g.conj()).max() <= 1e-15
    for gam in I.atom_vertices_lehmann(12, 5, beta, U, mu):
        assert np.abs(gam.imag).max() > 1e-6 * np.abs(gam).max()
        flipped = gam[::-1, ::-1, ::-1]
        assert np.abs(flipped - gam.conj()).max() <= 1e-12 * np.abs(gam).max()


def test_atomic_limit_problem_off_half_filling():
    p = I.atomic_limit_problem(2, 4, 8, 3, 10.0, 2.0, 0.1, mu=1.3)
    assert p.mu == 1.3
    assert np.allclose(p.g, I.atom_g_lehmann(8, 10.0, 2.0, 1.3), rtol=0, atol=0)
    assert np.allclose(p.delta, 2 * 2 * 0.01 * p.g, rtol=1e-15)
