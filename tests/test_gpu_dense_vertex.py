"""The ladder on a dense complex vertex, the general input of Sec. 2.1 (a
vertex measured by an impurity solver has no atomic-limit structure).

gamma^uu and gamma^ud are seeded dense complex matrices, scaled so that the
largest eigenvalue modulus of gamma^c diag(chi~) over all (c, Omega, q) is 0.8:
every item is inside the convergence radius, but rho(|M|) exceeds max |lambda|
(median about 0.46, up to 1.4), so the H-matrix certificate of the pivot-free
kernels fails on part of the items (about 13 %), which then go through the
partial-pivoting queue in the same call.  Parity with the
oracle at each precision's bar, status bit-exact; the fraction of items with
rho(|M|) < 0.999 (an upper bound on the certificate's pass rate, whose bound is
never below rho(|M|)) and the ladder time are printed."""
import time

import numpy as np
import pytest

from oracle import df_oracle as O
from paper_1507_00895_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-9, 2: 2e-5}


def rel(x, ref):
    return float(np.abs(np.asarray(x) - ref).max() / np.abs(ref).max())


def dense_problem(D, nk, n_nu, n_om, target=0.8, seed=77):
    p = I.atomic_limit_problem(D, nk, n_nu, n_om, 10.0, 2.0, 0.1)
    rng = np.random.default_rng(seed)
    shape = (n_om, n_nu, n_nu)
    guu = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    gud = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    G0 = O.dual_gf0(p.g, p.delta, p.eps)
    chi = O.bubble_fft(G0, p.D, p.nk, p.n_om, p.beta)
    gam = O.spin_channels(guu, gud)
    lam = 0.0
    rho_abs = []
    for c in range(2):
        for m in range(n_om):
            M = gam[c, m][None, :, :] * chi[m].T[:, None, :]
            lam = max(lam, float(np.abs(np.linalg.eigvals(M)).max()))
            rho_abs.append(np.abs(np.linalg.eigvals(np.abs(M))).max(axis=1))
    s = target / lam
    p.gamma_uu, p.gamma_ud = s * guu, s * gud
    return p, s * np.concatenate(rho_abs)


@pytest.mark.parametrize("shape", [(2, 8, 32, 3), (2, 8, 64, 3)], ids=lambda s: "nu{}".format(s[2]))
def test_dense_complex_vertex_parity(shape):
    import torch
    from paper_1507_00895_amd import binding as B
    B.load()
    p, rho_abs = dense_problem(*shape)
    print(f"dense vertex {shape}: rho(|M|) median {np.median(rho_abs):.2f}, max {rho_abs.max():.2f}; "
          f"items with rho(|M|) < 0.999: {np.mean(rho_abs < 0.999):.3f}", flush=True)
    inst = B.make_instance(p)
    ws = B.workspace([inst])
    B.df_dual_gf([inst], ws)
    B.df_bubble([inst], ws)
    torch.cuda.synchronize()
    lr = O.ladder(O.spin_channels(p.gamma_uu, p.gamma_ud), inst.chi.cpu().numpy())
    assert (lr.status == 0).all()            # inside the radius everywhere
    for prec in (B.DF_FP64, B.DF_FP32_REFINE, B.DF_FP32):
        inst.w.zero_()
        B.df_ladder_solve([inst], ws, B.make_opts(prec=prec))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.df_ladder_solve([inst], ws, B.make_opts(prec=prec))
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        print(f"  prec {prec}: {2 * p.n_om * p.N} ladders in {ms:.2f} ms", flush=True)
        assert np.array_equal(inst.status.cpu().numpy(), lr.status)
        # FP32 alone is not refined; for the others the bar of the precision class
        assert rel(inst.w.cpu().numpy(), lr.W) <= TOL[prec], prec
