"""Parity of the mixed-precision ladder (FP32 matrix cores + one FP64 residual
correction) with the FP64 CPU oracle: 1e-9 relative per result array.

log det of a certified item comes from its FP32 pivots accumulated in FP64,
so its accuracy is that of an FP32 factorisation, about kappa * n * eps32
(kappa <= 200 after diagonal scaling for certified items): the stated
tolerance is 1e-4 absolute on log|det| and on the phase.  Items near the
instability fail the certificate and get the FP64 determinant.
"""
import numpy as np
import pytest

from oracle import df_oracle as O
from paper_1507_00895_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-9
TOL_LOGDET32 = 1e-4


def rel(x, ref):
    den = np.abs(ref).max()
    return float(np.abs(np.asarray(x) - ref).max() / den) if den > 0 else float(np.abs(x).max())


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_1507_00895_amd import binding
    binding.load()
    return binding


SHAPES = [
    (2, 8, 16, 5, 10.0, 2.0, 0.1),
    (2, 4, 14, 3, 5.0, 2.0, 0.2),
    (1, 64, 20, 7, 10.0, 2.0, 0.1),
    (2, 16, 48, 9, 10.0, 2.0, 0.1),
    (2, 32, 64, 7, 20.0, 1.0, 0.1),       # the hardest 32x32 instance (lambda 0.75)
    (3, 8, 64, 7, 15.0, 3.0, I.T_REMAP_3D),
    (2, 8, 16, 1, 10.0, 2.0, 0.3),         # outside the radius: uncertified, FP64 path
    (2, 16, 96, 3, 10.0, 2.0, 0.1),        # n_nu > 64: FP64 path
]


@pytest.mark.parametrize("shape", SHAPES, ids=["D{}nk{}nu{}om{}".format(*s[:4]) for s in SHAPES])
def test_mixed_ladder_parity(B, shape):
    import torch
    p = I.atomic_limit_problem(*shape)
    inst = B.make_instance(p)
    ws = B.workspace([inst])
    B.df_dual_gf([inst], ws)
    B.df_bubble([inst], ws)
    B.df_ladder_solve([inst], ws, B.make_opts(prec=B.DF_FP32_REFINE))
    torch.cuda.synchronize()
    chi = host(inst.chi)
    gam = O.spin_channels(p.gamma_uu, p.gamma_ud)
    N = p.N
    qs = np.arange(N) if N * p.n_nu ** 3 * p.n_om <= 3e8 else \
        np.unique(np.concatenate([[0, N - 1], np.random.default_rng(1).choice(N, 30, replace=False)]))
    lr = O.ladder(gam, chi[:, :, qs])
    assert np.array_equal(host(inst.status)[:, :, qs], lr.status)
    assert rel(host(inst.w)[..., qs], lr.W) <= TOL_MIXED
    ld = host(inst.logdet)[:, :, qs]
    assert np.abs(ld.real - lr.logdet.real).max() <= TOL_LOGDET32
    assert np.abs(np.exp(1j * ld.imag) - np.exp(1j * lr.logdet.imag)).max() <= TOL_LOGDET32


def test_mixed_iterate_small_ten_iterations(B):
    p = I.workload_small()[0]
    inst = B.make_instance(p)
    ws = B.workspace([inst])
    B.df_iterate([inst], ws, B.make_opts(prec=B.DF_FP32_REFINE, mix=0.5, max_iter=10))
    r = O.iterate(p.g, p.delta, p.eps, p.gamma_uu, p.gamma_ud, p.D, p.nk, p.beta, p.n_om,
                  alpha=0.5, max_iter=10)
    assert rel(host(inst.sigma), r.sigma) <= TOL_MIXED


def test_mixed_full_square32_one_iteration_sampled(B):
    """2D 32x32, n_nu 64, n_om 31, U in {1, 2, 4}: the benchmark workload."""
    import torch
    probs = I.workload_square32()
    insts = [B.make_instance(p) for p in probs]
    ws = B.workspace(insts)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    B.df_iterate(insts, ws, B.make_opts(prec=B.DF_FP32_REFINE, mix=0.5, max_iter=1, use_graph=1),
                 stream=s.cuda_stream)
    s.synchronize()
    for p, x in zip(probs, insts):
        chi = host(x.chi)
        gam = O.spin_channels(p.gamma_uu, p.gamma_ud)
        qs = np.unique(np.concatenate([[0, 528, p.N - 1],
                                       np.random.default_rng(2).choice(p.N, 13, replace=False)]))
        lr = O.ladder(gam, chi[:, :, qs])
        W = host(x.w)
        assert rel(W[..., qs], lr.W) <= TOL_MIXED
        sc = host(x.sigma_calc)
        # Sigma~ from the mixed W, checked against the FP64 sums of that W
        assert rel(sc, O.sigma_fft(W, host(x.gd), p.D, p.nk, p.beta)) <= 1e-12


def test_mixed_converges_to_fp64_fixed_point(B):
    """Cold start to tol 1e-11 on both paths: the fixed points agree to 1e-9."""
    import torch
    p = I.atomic_limit_problem(2, 16, 32, 7, 20.0, 1.0, 0.1)
    out = {}
    for prec in (B.DF_FP64, B.DF_FP32_REFINE):
        inst = B.make_instance(p)
        ws = B.workspace([inst])
        code, iters, d = B.df_iterate([inst], ws, B.make_opts(prec=prec, mix=0.5, tol=1e-11,
                                                              max_iter=300))
        torch.cuda.synchronize()
        out[prec] = host(inst.sigma)
    assert rel(out[B.DF_FP32_REFINE], out[B.DF_FP64]) <= TOL_MIXED


# ---------------------------------------------------------------- FP32 ladders and the adaptive loop
# A certified FP32 ladder (rho(|M|) < 0.99, so kappa <= 100 after diagonal
# scaling) carries a relative error of about kappa * n * eps32 in the worst
# case; 2e-5 is the bound stated for W.
TOL_FP32 = 2e-5


@pytest.mark.parametrize("shape", SHAPES[:6], ids=["D{}nk{}nu{}om{}".format(*s[:4]) for s in SHAPES[:6]])
def test_fp32_ladder_parity(B, shape):
    import torch
    p = I.atomic_limit_problem(*shape)
    inst = B.make_instance(p)
    ws = B.workspace([inst])
    B.df_dual_gf([inst], ws)
    B.df_bubble([inst], ws)
    B.df_ladder_solve([inst], ws, B.make_opts(prec=B.DF_FP32))
    torch.cuda.synchronize()
    chi = host(inst.chi)
    N = p.N
    qs = np.arange(N) if N * p.n_nu ** 3 * p.n_om <= 3e8 else \
        np.unique(np.concatenate([[0, N - 1], np.random.default_rng(1).choice(N, 30, replace=False)]))
    lr = O.ladder(O.spin_channels(p.gamma_uu, p.gamma_ud), chi[:, :, qs])
    assert np.array_equal(host(inst.status)[:, :, qs], lr.status)
    assert rel(host(inst.w)[..., qs], lr.W) <= TOL_FP32


@pytest.mark.parametrize("use_graph", [0, 1])
def test_adaptive_converges_to_fp64_fixed_point(B, use_graph):
    """FP32 ladders until the diff drops below switch_tol, FP64 after: the
    converged Sigma~ is the FP64 path's (both to tol 1e-11)."""
    import torch
    probs = [I.atomic_limit_problem(2, 16, 32, 7, 20.0, 1.0, 0.1),
             I.atomic_limit_problem(2, 8, 64, 5, 10.0, 3.0, 0.1)]
    out = {}
    for prec in (B.DF_FP64, B.DF_ADAPTIVE):
        insts = [B.make_instance(p) for p in probs]
        ws = B.workspace(insts)
        s = torch.cuda.Stream()
        torch.cuda.synchronize()
        code, iters, d = B.df_iterate(insts, ws, B.make_opts(prec=prec, mix=0.5, tol=1e-11,
                                                             max_iter=300, use_graph=use_graph,
                                                             switch_tol=1e-5),
                                      stream=s.cuda_stream)
        s.synchronize()
        assert max(d) < 1e-11
        out[prec] = [host(x.sigma) for x in insts]
    for a, b in zip(out[B.DF_ADAPTIVE], out[B.DF_FP64]):
        assert rel(a, b) <= TOL_MIXED


def test_adaptive_at_large_n_nu(B):
    """n_nu = 96 and 128: the FP32 phase runs the FP32 ladder of those sizes
    (six and eight waves), the FP64 phase the certified FP64 kernels; the
    converged Sigma~ is the FP64 path's."""
    import torch
    probs = [I.atomic_limit_problem(3, 4, 96, 3, 10.0, 2.0, I.T_REMAP_3D),
             I.atomic_limit_problem(2, 4, 128, 3, 10.0, 2.0, 0.1)]
    assert B.df_ladder_variant(96, B.DF_FP32) == "fp32"
    assert B.df_ladder_variant(128, B.DF_FP32) == "fp32"
    out = {}
    for prec in (B.DF_FP64, B.DF_ADAPTIVE):
        insts = [B.make_instance(p) for p in probs]
        ws = B.workspace(insts)
        print(f"adaptive large n_nu, prec {prec}", flush=True)
        code, iters, d = B.df_iterate(insts, ws, B.make_opts(prec=prec, mix=0.5, tol=1e-11,
                                                             max_iter=300, use_graph=1,
                                                             switch_tol=1e-5))
        torch.cuda.synchronize()
        assert max(d) < 1e-11
        out[prec] = [host(x.sigma) for x in insts]
    for a, b in zip(out[B.DF_ADAPTIVE], out[B.DF_FP64]):
        assert rel(a, b) <= TOL_MIXED


def test_adaptive_never_converges_in_fp32(B):
    """A switch threshold below tol must not let an instance stop on FP32 ladders."""
    import torch
    p = I.workload_small()[0]
    res = {}
    for prec, sw in ((B.DF_FP64, 0.0), (B.DF_ADAPTIVE, 1e-12)):
        inst = B.make_instance(p)
        ws = B.workspace([inst])
        B.df_iterate([inst], ws, B.make_opts(prec=prec, mix=0.5, tol=1e-9, max_iter=300,
                                             switch_tol=sw))
        torch.cuda.synchronize()
        res[prec] = host(inst.sigma)
    assert rel(res[B.DF_ADAPTIVE], res[B.DF_FP64]) <= 1e-8
