"""Pins of the warm-start network's Adam reference (oracle/mlp_ref.py).

Adam (Kingma and Ba, 2015, Algorithm 1) has closed forms that do not restate
its recurrence: under a gradient held constant from m = v = 0, the
bias-corrected moments are exactly g and g^2 on every step, so every step moves
each parameter by lr g / (|g| + eps).  A missing bias correction (first step
lr (1 - b1) g / (sqrt(1 - b2) |g|), about 3.2 lr), a wrong sign or a swapped
pair of decay rates fails these.
"""
import numpy as np

from oracle import mlp_ref as R


def test_adam_constant_gradient_steps_are_lr_sign():
    g = np.array([0.5, -2.0, 1e-3, 7.0])
    lr, eps = 0.01, 1e-8
    p = np.zeros_like(g)
    m = np.zeros_like(g)
    v = np.zeros_like(g)
    for step in range(1, 26):
        p, m, v = R.adam(p, g, m, v, step, lr, eps=eps)
        want = -step * lr * g / (np.abs(g) + eps)
        assert np.allclose(p, want, rtol=1e-12, atol=0), step


def test_adam_first_step_and_a_sign_change():
    """Step 1 from zero moments moves by lr sign(g) whatever |g| is; a gradient
    that flips sign on step 2 leaves the bias-corrected first moment at
    (b1 (1 - b1) g1 + (1 - b1) g2) / (1 - b1^2), a weighted mean evaluated here
    in closed form for g1 = 1, g2 = -1: (0.09 - 0.1) / 0.19."""
    lr, b1, b2 = 0.1, 0.9, 0.999
    p, m, v = R.adam(np.array([1.0]), np.array([1.0]), np.zeros(1), np.zeros(1), 1, lr)
    assert abs(p[0] - (1.0 - lr / (1.0 + 1e-8))) < 1e-14
    p, m, v = R.adam(p, np.array([-1.0]), m, v, 2, lr)
    mhat = (b1 * (1 - b1) * 1.0 + (1 - b1) * -1.0) / (1 - b1 ** 2)
    vhat = (b2 * (1 - b2) + (1 - b2)) / (1 - b2 ** 2)   # = 1: both squares are 1
    assert abs(mhat - (-0.01 / 0.19)) < 1e-15 and abs(vhat - 1.0) < 1e-12
    assert abs(p[0] - (1.0 - lr / (1.0 + 1e-8) - lr * mhat / (np.sqrt(vhat) + 1e-8))) < 1e-14
