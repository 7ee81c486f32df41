"""Learned warm start: trained on the method's own converged Sigma~, it must
reach the same fixed point as a cold start in fewer iterations."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_warm_start_gain_same_fixed_point():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1507_00895_amd import warmstart as W
    cfg = W.WarmStartConfig(nk=8, n_nu=16, n_om=5)
    r = W.train_and_evaluate(n_train=64, n_test=4, steps=800, cfg=cfg)
    print(r)
    first, last = r["train_loss_first_last"]
    assert last < 0.05 * first
    assert r["prediction_rel_error_mean"] < 0.2
    assert all(w <= c for w, c in zip(r["iterations_warm"], r["iterations_cold"]))
    assert r["mean_iterations_warm"] < r["mean_iterations_cold"]
    # both runs stop at diff < 1e-8; their fixed points agree well within that
    # bound divided by the contraction gap
    assert r["fixed_point_rel_diff_max"] <= 1e-6
