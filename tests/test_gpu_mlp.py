"""Warm-start network kernels (df_mlp_*) against the FP64 NumPy reference.

The kernels compute in FP32 on the matrix cores; the reference runs in FP64
on the same FP32 parameters and inputs.  Tolerance: every output and every
gradient block within 2e-5 of its largest magnitude (FP32 accumulation over
at most a few hundred terms of mixed sign: about sqrt(K) * 6e-8 relative,
with headroom).
"""
import numpy as np
import pytest

from oracle import mlp_ref as R

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 2e-5


@pytest.fixture(scope="module")
def B():
    from paper_1507_00895_amd import binding
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()
    return binding


def _net(dims, batch, seed):
    rng = np.random.default_rng(seed)
    flat = []
    for l in range(len(dims) - 1):
        flat.append(rng.standard_normal(dims[l + 1] * dims[l]) / np.sqrt(dims[l]))
        flat.append(0.1 * rng.standard_normal(dims[l + 1]))
    p = np.concatenate(flat).astype(np.float32)
    X = rng.standard_normal((batch, dims[0])).astype(np.float32)
    T = rng.standard_normal((batch, dims[-1])).astype(np.float32)
    return p, X, T


def _dev(a):
    return torch.as_tensor(a, device="cuda").contiguous()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


def _blocks(flat, dims):
    out, o = [], 0
    for l in range(len(dims) - 1):
        for n in (dims[l + 1] * dims[l], dims[l + 1]):
            out.append(flat[o:o + n])
            o += n
    return out


# (dims, batch): ragged tiles in every GEMM dimension, split-K over the batch
# (batch 300 -> 2 splits with a ragged last chunk, 1000 -> 4), a single row,
# one layer, and the warm-start shape.
CASES = [
    ([7, 70, 130, 5], 300),
    ([7, 70, 130, 5], 1),
    ([33, 65, 17], 1000),
    ([12, 9], 77),
    ([129, 256, 256, 256, 32], 512),
]


@pytest.mark.parametrize("dims,batch", CASES)
def test_forward_matches_reference(B, dims, batch):
    p, X, _ = _net(dims, batch, 3)
    assert B.df_mlp_param_count(dims) == p.size
    Y = torch.empty((batch, dims[-1]), dtype=torch.float32, device="cuda")
    ws = B.mlp_workspace(dims, batch)
    B.df_mlp_forward(dims, _dev(p), _dev(X), Y, ws)
    ref, _ = R.forward(p.astype(np.float64), dims, X.astype(np.float64))
    assert _rel(Y.cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("dims,batch", CASES)
def test_loss_grad_matches_reference(B, dims, batch):
    p, X, T = _net(dims, batch, 5)
    grads = torch.full((p.size,), np.nan, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = B.mlp_workspace(dims, batch)
    B.df_mlp_loss_grad(dims, _dev(p), _dev(X), _dev(T), grads, loss, ws)
    ref_loss, ref_g = R.loss_grad(p.astype(np.float64), dims, X.astype(np.float64),
                                  T.astype(np.float64))
    assert abs(float(loss.item()) - ref_loss) <= TOL * ref_loss
    g = grads.cpu().numpy()
    assert np.all(np.isfinite(g))
    for got, ref in zip(_blocks(g, dims), _blocks(ref_g, dims)):
        assert _rel(got, ref) <= TOL


def test_loss_grad_reproducible_and_null_loss(B):
    dims, batch = [20, 64, 64, 8], 700
    p, X, T = _net(dims, batch, 9)
    ws = B.mlp_workspace(dims, batch)
    g1 = torch.zeros(p.size, dtype=torch.float32, device="cuda")
    g2 = torch.zeros_like(g1)
    B.df_mlp_loss_grad(dims, _dev(p), _dev(X), _dev(T), g1, None, ws)
    B.df_mlp_loss_grad(dims, _dev(p), _dev(X), _dev(T), g2, None, ws)
    assert torch.equal(g1, g2)


def test_adam_matches_reference(B):
    rng = np.random.default_rng(4)
    n = 5000
    p = rng.standard_normal(n).astype(np.float32)
    pd, m, v = _dev(p), torch.zeros(n, dtype=torch.float32, device="cuda"), \
        torch.zeros(n, dtype=torch.float32, device="cuda")
    rp, rm, rv = p.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in range(1, 4):
        g = rng.standard_normal(n).astype(np.float32)
        B.df_mlp_adam(pd, _dev(g), m, v, step, 1e-2)
        rp, rm, rv = R.adam(rp, g.astype(np.float64), rm, rv, step, 1e-2)
    assert np.max(np.abs(pd.cpu().numpy() - rp)) <= 1e-6
    assert _rel(m.cpu().numpy(), rm) <= 1e-6
    assert _rel(v.cpu().numpy(), rv) <= 1e-5


def test_argument_errors(B):
    dims = [4, 8, 2]
    ws = B.mlp_workspace(dims, 4)
    X = torch.zeros((4, 4), dtype=torch.float32, device="cuda")
    Y = torch.zeros((4, 2), dtype=torch.float32, device="cuda")
    p = torch.zeros(B.df_mlp_param_count(dims), dtype=torch.float32, device="cuda")
    with pytest.raises(B.DfError):
        B.df_mlp_param_count([4] + [2000] + [2])
    with pytest.raises(B.DfError):
        B.df_mlp_forward(dims, p, X, Y, ws[:16])
    with pytest.raises(TypeError):
        B.df_mlp_forward(dims, p.double(), X, Y, ws)


def test_training_reduces_loss(B):
    """Adam on a smooth regression target: the kernels' gradients descend."""
    rng = np.random.default_rng(8)
    X = rng.uniform(-1, 1, (2048, 3)).astype(np.float32)
    T = np.stack([np.sin(2 * X[:, 0]) * X[:, 1], np.cos(X[:, 2] + X[:, 0])], 1).astype(np.float32)
    dims = [3, 64, 64, 2]
    p, _, _ = _net(dims, 1, 2)
    pd = _dev(p)
    g = torch.zeros_like(pd)
    m, v = torch.zeros_like(pd), torch.zeros_like(pd)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = B.mlp_workspace(dims, 2048)
    Xd, Td = _dev(X), _dev(T)
    first = None
    for step in range(1, 401):
        B.df_mlp_loss_grad(dims, pd, Xd, Td, g, loss, ws)
        if step == 1:
            first = float(loss.item())
        B.df_mlp_adam(pd, g, m, v, step, 3e-3)
    B.df_mlp_loss_grad(dims, pd, Xd, Td, g, loss, ws)
    assert float(loss.item()) < 0.05 * first
