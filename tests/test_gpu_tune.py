"""Every ladder kernel variant the autotuner can pick matches the oracle, and
the autotuner records a choice that the following calls use."""
import os

import numpy as np
import pytest

from oracle import df_oracle as O
from paper_1507_00895_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-9, 2: 2e-5}


def rel(x, ref):
    return float(np.abs(np.asarray(x) - ref).max() / np.abs(ref).max())


@pytest.fixture()
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1507_00895_amd import binding
    binding.load()
    binding.df_autotune_reset()
    yield binding
    binding.df_autotune_reset()


# (D, nk, n_nu, n_om): every padded size of the certified kernels and a ragged one
SHAPES = [(2, 8, 16, 5), (2, 8, 30, 3), (2, 16, 48, 5), (2, 8, 64, 5), (3, 4, 96, 3),
          (2, 4, 128, 3), (2, 4, 112, 3)]


def _ladder_case(B, shape, prec):
    import torch
    D, nk, n_nu, n_om = shape
    p = I.atomic_limit_problem(D, nk, n_nu, n_om, 10.0, 2.0, 0.1 if D == 2 else I.T_REMAP_3D)
    inst = B.make_instance(p)
    ws = B.workspace([inst])
    inst.sigma.copy_(torch.as_tensor(1e-3 * I.random_complex((n_nu, p.N), seed=5)))
    B.df_dual_gf([inst], ws)
    B.df_bubble([inst], ws)
    torch.cuda.synchronize()
    return p, inst, ws


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "D{}nk{}nu{}om{}".format(*s))
def test_every_variant_matches_oracle(B, shape):
    import torch
    n_nu = shape[2]
    for prec in (B.DF_FP64, B.DF_FP32_REFINE, B.DF_FP32):
        p, inst, ws = _ladder_case(B, shape, prec)
        chi = inst.chi.cpu().numpy()
        lr = O.ladder(O.spin_channels(p.gamma_uu, p.gamma_ud), chi)
        ran = []
        for name in B.LADDER_VARIANTS:
            try:
                B.df_ladder_set_variant(n_nu, prec, name)
            except B.DfError as e:
                assert e.code == B.DF_E_UNSUPPORTED
                continue
            assert B.df_ladder_variant(n_nu, prec) == name
            inst.w.zero_()
            inst.status.fill_(-1)
            B.df_ladder_solve([inst], ws, B.make_opts(prec=prec))
            torch.cuda.synchronize()
            assert np.array_equal(inst.status.cpu().numpy(), lr.status), name
            assert rel(inst.w.cpu().numpy(), lr.W) <= TOL[prec], name
            ran.append(name)
        assert ran, (shape, prec)
        B.df_autotune_reset()


def test_autotune_records_choice_and_cache(B, tmp_path):
    import torch
    cache = tmp_path / "tune.txt"
    os.environ["DF_TUNE_CACHE"] = str(cache)
    try:
        p, inst, ws = _ladder_case(B, (2, 16, 48, 5), B.DF_FP64)
        B.df_autotune([inst], ws, B.make_opts(prec=B.DF_FP64))
        choice = B.df_ladder_variant(48, B.DF_FP64)
        assert choice in B.LADDER_VARIANTS
        lines = cache.read_text().split()
        assert lines == ["0", "48", choice]
        # the tuned choice still gives oracle results
        lr = O.ladder(O.spin_channels(p.gamma_uu, p.gamma_ud), inst.chi.cpu().numpy())
        B.df_ladder_solve([inst], ws, B.make_opts(prec=B.DF_FP64))
        torch.cuda.synchronize()
        assert rel(inst.w.cpu().numpy(), lr.W) <= TOL[0]
    finally:
        del os.environ["DF_TUNE_CACHE"]
    B.df_autotune_reset()
    assert B.df_ladder_variant(48, B.DF_FP64) == "gjb_o3"   # the untuned default
