"""NumPy reference of the warm-start network: forward, backward, Adam.

TEST INFRASTRUCTURE ONLY (gradient checks of the GPU kernels).  FP64.

Network: affine layers dims[0] -> ... -> dims[L], SiLU after every layer but
the last; loss = mean over all outputs of (Y - T)^2.  Parameters are one flat
vector, layer by layer: W_l (dims[l+1] x dims[l], row-major) then b_l.
"""
import numpy as np


def unpack(params, dims):
    out, o = [], 0
    for l in range(len(dims) - 1):
        n_w = dims[l + 1] * dims[l]
        W = params[o:o + n_w].reshape(dims[l + 1], dims[l])
        o += n_w
        b = params[o:o + dims[l + 1]]
        o += dims[l + 1]
        out.append((W, b))
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, dims, X):
    layers = unpack(np.asarray(params, dtype=np.float64), dims)
    a = np.asarray(X, dtype=np.float64)
    cache = [(None, a)]
    for l, (W, b) in enumerate(layers):
        z = a @ W.T + b
        a = z if l == len(layers) - 1 else silu(z)
        cache.append((z, a))
    return a, cache


def loss_grad(params, dims, X, T):
    """(loss, flat gradient) of the mean squared error."""
    params = np.asarray(params, dtype=np.float64)
    layers = unpack(params, dims)
    Y, cache = forward(params, dims, X)
    T = np.asarray(T, dtype=np.float64)
    n = Y.size
    loss = float(np.sum((Y - T) ** 2) / n)
    dz = 2.0 * (Y - T) / n
    grads = []
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        a_prev = cache[l][1]
        grads.append((dz.T @ a_prev, dz.sum(axis=0)))
        if l > 0:
            dz = (dz @ W) * dsilu(cache[l][0])
    flat = []
    for dW, db in reversed(grads):
        flat.append(dW.ravel())
        flat.append(db)
    return loss, np.concatenate(flat)


def adam(params, grads, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grads
    v = b2 * v + (1 - b2) * grads * grads
    p = params - lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
    return p, m, v
