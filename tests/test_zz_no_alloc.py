"""df_bubble_noalloc (the workspace-free entry point) against df_bubble,
through the C ABI: two calls in a row, the second on a smaller input, both
bit-identical to df_bubble's chi (same kernels, same arithmetic); also a
two-instance call, whose instances take turns on the one scratch array."""
import numpy as np
import pytest

from paper_1507_00895_amd import inputs as I

pytestmark = pytest.mark.gpu


def _reference_chi(B, p, sigma_seed):
    import torch
    inst = B.make_instance(p)
    inst.sigma.copy_(torch.as_tensor(1e-3 * I.random_complex((p.n_nu, p.N), seed=sigma_seed)))
    ws = B.workspace([inst])
    B.df_dual_gf([inst], ws)
    B.df_bubble([inst], ws)
    torch.cuda.synchronize()
    return inst


def test_bubble_noalloc_matches_bubble():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1507_00895_amd import binding as B
    B.load()
    big = I.atomic_limit_problem(3, 16, 96, 7, 15.0, 3.0, I.T_REMAP_3D)     # 6.3 MB of G~(r)
    small = I.atomic_limit_problem(2, 8, 16, 3, 10.0, 2.0, 0.1)
    for p, seed in ((big, 1), (small, 2)):
        ref = _reference_chi(B, p, seed)
        print(f"noalloc bubble D{p.D} nk{p.nk} n_nu{p.n_nu} n_om{p.n_om}", flush=True)
        want = ref.chi.clone()
        ref.chi.fill_(float("nan"))
        B.df_bubble_noalloc([ref])
        torch.cuda.synchronize()
        assert torch.equal(ref.chi, want)
    # two instances in one call
    a, b = _reference_chi(B, small, 3), _reference_chi(B, big, 4)
    wa, wb = a.chi.clone(), b.chi.clone()
    a.chi.zero_()
    b.chi.zero_()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    B.df_bubble_noalloc([a, b], stream=s.cuda_stream)
    s.synchronize()
    assert torch.equal(a.chi, wa) and torch.equal(b.chi, wb)
