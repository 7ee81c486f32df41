"""Anderson-accelerated self-consistency (df_opts_t.accel): the fixed point of
the plain loop, reached in fewer iterations."""
import numpy as np
import pytest

from oracle import df_oracle as O
from paper_1507_00895_amd import inputs as I

pytestmark = pytest.mark.gpu


def rel(x, ref):
    return float(np.abs(np.asarray(x) - ref).max() / np.abs(ref).max())


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1507_00895_amd import binding
    binding.load()
    return binding


def _run(B, probs, graph=1, **kw):
    import torch
    insts = [B.make_instance(p) for p in probs]
    opts = B.make_opts(**kw, use_graph=graph)
    ws = B.workspace(insts, opts)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    code, iters, d = B.df_iterate(insts, ws, opts, stream=s.cuda_stream,
                                  allow=(B.DF_OK, B.DF_W_FALLBACK))
    s.synchronize()
    return insts, iters, d


def test_accelerated_fixed_point_matches_oracle(B):
    """Small 2D workload: the oracle's plain loop and the accelerated GPU loop,
    both to a diff below 1e-12, agree to 1e-10."""
    p = I.workload_small()[0]
    r = O.iterate(p.g, p.delta, p.eps, p.gamma_uu, p.gamma_ud, p.D, p.nk, p.beta, p.n_om,
                  alpha=0.5, tol=1e-12, max_iter=400)
    insts, iters, d = _run(B, [p], mix=0.5, tol=1e-12, max_iter=400, accel=5)
    assert d[0] < 1e-12
    assert iters < r.iters
    assert rel(insts[0].sigma.cpu().numpy(), r.sigma) <= 1e-10


@pytest.mark.parametrize("accel", [1, 3, 5, 8])
def test_accelerated_loop_fewer_iterations_same_fixed_point(B, accel):
    p = I.atomic_limit_problem(2, 16, 32, 7, 20.0, 1.0, 0.1)
    lin, it_lin, _ = _run(B, [p], mix=0.5, tol=1e-11, max_iter=400)
    acc, it_acc, d = _run(B, [p], mix=0.5, tol=1e-11, max_iter=400, accel=accel)
    assert d[0] < 1e-11
    assert it_acc < it_lin
    a, l = acc[0].sigma.cpu().numpy(), lin[0].sigma.cpu().numpy()
    assert rel(a, l) <= 1e-9
    # real weights keep the conjugation symmetry Sigma(-nu) = Sigma(nu)*
    assert rel(np.conj(a[::-1]), a) <= 1e-13
    # sigma_calc is F of the last iterate: at the fixed point it equals sigma
    assert rel(acc[0].sigma_calc.cpu().numpy(), a) <= 1e-9


def test_accelerated_fused_instances_deterministic(B):
    """Uneven instances in fused launches: graph and eager runs, and each
    instance run alone, give identical bits."""
    shapes = [(2, 16, 32, 7, 12.0, 1.5, 0.1), (3, 4, 64, 7, 20.0, 2.5, 0.1),
              (2, 8, 16, 3, 6.0, 3.5, 0.1), (2, 8, 48, 11, 24.0, 3.0, 0.1)]
    probs = [I.atomic_limit_problem(*s) for s in shapes]
    kw = dict(mix=0.5, tol=1e-10, max_iter=200, accel=5)
    g1, it1, d1 = _run(B, probs, graph=1, **kw)
    g0, it0, d0 = _run(B, probs, graph=0, **kw)
    assert it1 == it0 and max(d1) < 1e-10
    for a, b in zip(g1, g0):
        assert np.array_equal(a.sigma.cpu().numpy(), b.sigma.cpu().numpy())
    for p, a in zip(probs, g1):
        one, _, _ = _run(B, [p], graph=1, **kw)
        assert np.array_equal(one[0].sigma.cpu().numpy(), a.sigma.cpu().numpy())


def test_accelerated_adaptive_reaches_fp64_fixed_point(B):
    probs = [I.atomic_limit_problem(2, 16, 32, 7, 20.0, 1.0, 0.1),
             I.atomic_limit_problem(2, 8, 64, 5, 10.0, 3.0, 0.1)]
    f64, _, _ = _run(B, probs, prec=B.DF_FP64, mix=0.5, tol=1e-11, max_iter=400, accel=5)
    ad, _, d = _run(B, probs, prec=B.DF_ADAPTIVE, mix=0.5, tol=1e-11, max_iter=400, accel=5,
                    switch_tol=1e-5)
    assert max(d) < 1e-11
    for a, b in zip(ad, f64):
        assert rel(a.sigma.cpu().numpy(), b.sigma.cpu().numpy()) <= 1e-9


@pytest.mark.parametrize("accel", [0, 5], ids=["linear", "anderson"])
def test_adaptive_fixed_point_matches_oracle(B, accel):
    """The adaptive loop (FP32 ladders until the diff falls below switch_tol,
    FP64 ladders from then on), with linear mixing or Anderson acceleration,
    against the oracle's plain FP64 loop (eq. dyson and the ladder of Sec. 2.2
    iterated to a diff below 1e-12) on the small 2D workload: the same fixed
    point to 1e-10."""
    p = I.workload_small()[0]
    r = O.iterate(p.g, p.delta, p.eps, p.gamma_uu, p.gamma_ud, p.D, p.nk, p.beta, p.n_om,
                  alpha=0.5, tol=1e-12, max_iter=400)
    insts, iters, d = _run(B, [p], prec=B.DF_ADAPTIVE, mix=0.5, tol=1e-12, max_iter=400,
                           accel=accel, switch_tol=1e-5)
    assert d[0] < 1e-12
    assert rel(insts[0].sigma.cpu().numpy(), r.sigma) <= 1e-10
