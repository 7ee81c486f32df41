"""df_iterate's outcomes other than plain convergence, and one point of the
paper's own sweeps (Sec. 4) converged on both sides.

The error paths are host-side outcomes of the loop: every kernel runs and
exits normally, the host reads the convergence measures and decides."""
import numpy as np
import pytest

from oracle import df_oracle as O
from paper_1507_00895_amd import inputs as I

pytestmark = pytest.mark.gpu


def rel(x, ref):
    return float(np.abs(np.asarray(x) - ref).max() / np.abs(ref).max())


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1507_00895_amd import binding
    binding.load()
    return binding


def test_nonfinite_start_value_is_reported(B):
    """A NaN in the start value of Sigma~ makes the first diff non-finite:
    DF_E_NONFINITE after one iteration."""
    import torch
    p = I.workload_small()[0]
    inst = B.make_instance(p)
    ws = B.workspace([inst])
    inst.sigma[3, 5] = complex(float("nan"), 0.0)
    code, iters, d = B.df_iterate([inst], ws, B.make_opts(mix=0.5, tol=1e-8, max_iter=20),
                                  allow=(B.DF_E_NONFINITE,))
    torch.cuda.synchronize()
    assert code == B.DF_E_NONFINITE
    assert iters == 1


@pytest.mark.parametrize("use_graph", [0, 1])
def test_iteration_limit_is_reported_with_the_last_iterate(B, use_graph):
    """max_iter = 2 with a tolerance the loop cannot reach: DF_E_NOT_CONVERGED,
    and Sigma~ holds the second iterate (the oracle's, to 1e-12)."""
    import torch
    p = I.workload_small()[0]
    inst = B.make_instance(p)
    ws = B.workspace([inst])
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    code, iters, d = B.df_iterate([inst], ws, B.make_opts(mix=0.5, tol=1e-14, max_iter=2,
                                                          use_graph=use_graph),
                                  stream=s.cuda_stream, allow=(B.DF_E_NOT_CONVERGED,))
    s.synchronize()
    assert code == B.DF_E_NOT_CONVERGED and iters == 2 and d[0] > 1e-14
    r = O.iterate(p.g, p.delta, p.eps, p.gamma_uu, p.gamma_ud, p.D, p.nk, p.beta, p.n_om,
                  alpha=0.5, max_iter=2)
    assert rel(host(inst.sigma), r.sigma) <= 1e-12
    assert abs(d[0] - r.diff) <= 1e-12 * r.diff


def test_fallback_flag_of_an_instance_that_converged_first(B):
    """Two instances converge at different iterations; only the first has a
    ladder outside the radius on its last iteration (oracle: 57 iterations
    with one fallback ladder against 64 without).  The fallback warning must
    survive the first instance leaving the active set."""
    import torch
    pa = I.atomic_limit_problem(2, 4, 8, 1, 10.0, 2.0, 0.27)
    pb = I.atomic_limit_problem(2, 8, 16, 3, 10.0, 2.0, 0.26)
    ra = O.iterate(pa.g, pa.delta, pa.eps, pa.gamma_uu, pa.gamma_ud, pa.D, pa.nk, pa.beta,
                   pa.n_om, alpha=0.5, tol=1e-8, max_iter=300)
    rb = O.iterate(pb.g, pb.delta, pb.eps, pb.gamma_uu, pb.gamma_ud, pb.D, pb.nk, pb.beta,
                   pb.n_om, alpha=0.5, tol=1e-8, max_iter=300)
    assert ra.iters < rb.iters
    assert (ra.ladder.status != 0).any() and not (rb.ladder.status != 0).any()
    for use_graph in (0, 1):
        insts = [B.make_instance(pa), B.make_instance(pb)]
        ws = B.workspace(insts)
        s = torch.cuda.Stream()
        torch.cuda.synchronize()
        code, iters, d = B.df_iterate(insts, ws, B.make_opts(mix=0.5, tol=1e-8, max_iter=300,
                                                             use_graph=use_graph),
                                      stream=s.cuda_stream)
        s.synchronize()
        assert code == B.DF_W_FALLBACK, use_graph
        assert iters == rb.iters
        assert rel(host(insts[0].sigma), ra.sigma) <= 1e-9
        assert rel(host(insts[1].sigma), rb.sigma) <= 1e-9
    # alone, the second instance ends without a warning
    one = B.make_instance(pb)
    code, _, _ = B.df_iterate([one], B.workspace([one]), B.make_opts(mix=0.5, tol=1e-8,
                                                                     max_iter=300))
    assert code == B.DF_OK


def test_paper_sweep_point_converged_against_oracle(B):
    """One point of the paper's sweeps (Sec. 4, Figs. 1-3): the 2D atomic limit
    at U = 20, beta = 1, t = 1 with N_Omega = 3, N_omega = 48, N_k = 8,
    converged to tol 1e-10 on the GPU and by the oracle.  Sigma~ agrees to 1e-9
    and so does g = G~(i pi / beta, k = 0), the quantity whose convergence in
    the cut-offs eq. (deltag) measures."""
    import torch
    p = I.atomic_limit_problem(2, 8, 48, 3, 1.0, 20.0, 1.0)
    inst = B.make_instance(p)
    ws = B.workspace([inst])
    code, iters, d = B.df_iterate([inst], ws, B.make_opts(mix=0.5, tol=1e-10, max_iter=500))
    torch.cuda.synchronize()
    r = O.iterate(p.g, p.delta, p.eps, p.gamma_uu, p.gamma_ud, p.D, p.nk, p.beta, p.n_om,
                  alpha=0.5, tol=1e-10, max_iter=500)
    assert d[0] < 1e-10 and r.diff < 1e-10
    assert abs(iters - r.iters) <= 1
    assert rel(host(inst.sigma), r.sigma) <= 1e-9
    n0 = p.n_nu // 2                     # nu_{n0} = pi / beta
    G = O.dual_gf(O.dual_gf0(p.g, p.delta, p.eps), r.sigma)
    g_gpu = host(inst.gd)[n0, 0]
    assert abs(g_gpu - G[n0, 0]) <= 1e-9 * abs(G[n0, 0])


@pytest.mark.parametrize("unroll", [3, 4])
def test_graph_unroll_runs_the_same_iterations(B, unroll):
    """graph_unroll captures several iterations per graph and reads the
    convergence measure once per launch.  With tol = 0 the iterations are
    those of one iteration per graph (10 = 3 + 3 + 3 + 1 or 4 + 4 + 2, the
    remainder queued one by one): Sigma~ bit-identical.  With tol > 0 the
    loop stops at the end of a graph launch whose last diff is below tol, at
    most unroll - 1 iterations after the plain loop would, and stays within
    the plain loop's tolerance of the oracle's fixed point."""
    import torch
    p = I.atomic_limit_problem(2, 8, 16, 3, 10.0, 2.0, 0.1)
    s = torch.cuda.Stream()

    def run(**kw):
        inst = B.make_instance(p)
        ws = B.workspace([inst])
        torch.cuda.synchronize()
        code, iters, d = B.df_iterate([inst], ws, B.make_opts(mix=0.5, use_graph=1, **kw),
                                      stream=s.cuda_stream,
                                      allow=(B.DF_OK, B.DF_W_FALLBACK, B.DF_E_NOT_CONVERGED))
        s.synchronize()
        return code, iters, d, host(inst.sigma)

    _, it0, _, s0 = run(tol=0.0, max_iter=10)
    _, it1, _, s1 = run(tol=0.0, max_iter=10, graph_unroll=unroll)
    assert it0 == it1 == 10
    assert np.array_equal(s0, s1)

    c0, n0, d0, t0 = run(tol=1e-11, max_iter=200)
    c1, n1, d1, t1 = run(tol=1e-11, max_iter=200, graph_unroll=unroll)
    assert c0 == c1 == B.DF_OK and d0[0] < 1e-11 and d1[0] < 1e-11
    assert n0 <= n1 <= n0 + unroll - 1 and n1 % unroll == 0
    assert rel(t1, t0) <= 1e-10
