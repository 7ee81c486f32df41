"""Learned warm start of the dual self-energy.

A small MLP maps per-(instance, k) features to Sigma~(k, nu) at the positive
fermionic frequencies; Sigma~ at negative frequencies follows by conjugation
(Sigma~(-nu) = Sigma~(nu)*).  The prediction only replaces the zero start of
df_iterate, which still runs to the same tolerance: results stay those of the
method, only the iteration count changes.

Every numeric step runs in libdf's HIP kernels: the training data come from
df_iterate, the coarse dual-propagator features from df_dual_gf, training and
inference from df_mlp_loss_grad / df_mlp_adam / df_mlp_forward.  torch holds
device buffers and does index bookkeeping (minibatch gathers, reshapes).

Features (one row per k point of an instance; 2D square lattices):
  * instance: U, beta, log U, log beta, 1/beta, t, D (standardised over the
    training set);
  * k: five point-group-invariant combinations of cos k_i and cos 2k_i;
  * coarse dual propagator: G~0 of the instance on an 8 x 8 grid at the four
    lowest positive Matsubara frequencies, at the 15 points of the irreducible
    wedge 0 <= k_y <= k_x <= pi (real and imaginary parts: 120 numbers).
Targets: Re and Im of the converged Sigma~(k, nu_n), n = 0 .. n_nu/2 - 1,
divided by the instance's rms |Sigma~|, plus the log of that scale;
standardised per output.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import List, Optional

import numpy as np

from . import binding as B
from . import inputs as I

HIDDEN = (256, 256, 256)


@dataclasses.dataclass
class WarmStartConfig:
    nk: int = 16
    n_nu: int = 32
    n_om: int = 7
    t: float = 0.1
    U_range: tuple = (1.0, 4.0)
    beta_range: tuple = (5.0, 20.0)
    tol: float = 1e-8
    mix: float = 0.5

    def problem(self, U: float, beta: float):
        return I.atomic_limit_problem(2, self.nk, self.n_nu, self.n_om, beta, U, self.t)


def draw(n: int, seed: int, cfg: WarmStartConfig, corners: bool = False):
    """n (U, beta) pairs, Latin-hypercube stratified over the two ranges; with
    corners, the four corners of the (U, beta) box replace four of them (a
    network interpolates poorly towards corners it has not seen)."""
    rng = np.random.default_rng(seed)
    out = []
    cols = []
    for lo, hi in (cfg.U_range, cfg.beta_range):
        u = (rng.permutation(n) + rng.uniform(size=n)) / n
        cols.append(lo + (hi - lo) * u)
    for U, beta in zip(*cols):
        out.append((float(U), float(beta)))
    if corners and n >= 8:
        (u0, u1), (b0, b1) = cfg.U_range, cfg.beta_range
        out[:4] = [(u0, b0), (u0, b1), (u1, b0), (u1, b1)]
    return out


# ---------------------------------------------------------------- features
WEDGE = [(x, y) for x in range(5) for y in range(x + 1)]          # 15 points of the 8x8 wedge


def wedge_rows(nk: int) -> np.ndarray:
    """Flat indices of the irreducible wedge 0 <= k_y <= k_x <= pi of the nk x nk
    grid: one k per point-group orbit.  The features are invariant under the
    group, so rows on the wedge train the network for the whole grid."""
    h = nk // 2
    return np.array([x * nk + y for x in range(h + 1) for y in range(x + 1)])


def k_features(nk: int) -> np.ndarray:
    """Point-group-invariant functions of k on the nk x nk grid, [N, 5]."""
    k = I.kpoints(2, nk)
    c1, c2 = np.cos(k[:, 0]), np.cos(k[:, 1])
    d1, d2 = np.cos(2 * k[:, 0]), np.cos(2 * k[:, 1])
    return np.stack([(c1 + c2) / 2, c1 * c2, (d1 + d2) / 2, d1 * d2, (c1 * d2 + d1 * c2) / 2], axis=1)


def coarse_gd0(params: List[tuple], cfg: WarmStartConfig, device="cuda") -> np.ndarray:
    """G~0 on the 8x8 grid at the 4 lowest positive nu, wedge points: [n, 120] (df_dual_gf)."""
    import torch
    insts = []
    for U, beta in params:
        g = I.atom_g(8, beta, U)
        c = dict(dtype=torch.complex128, device=device)
        insts.append(B.Instance(
            D=2, nk=8, n_nu=8, n_om=1, beta=beta,
            g=torch.as_tensor(g, **c), delta=torch.as_tensor(I.atom_delta(g, 2, cfg.t), **c),
            eps=torch.as_tensor(I.dispersion_hypercubic(2, 8, cfg.t), dtype=torch.float64, device=device),
            gamma_uu=None, gamma_ud=None, gd=torch.zeros((8, 64), **c)))
    ws = B.workspace(insts, device=device)
    B.df_dual_gf(insts, ws)
    torch.cuda.synchronize()
    idx = [x * 8 + y for x, y in WEDGE]
    out = []
    for x in insts:
        gd = x.gd[4:8][:, idx].cpu().numpy()                        # nu_0 .. nu_3
        out.append(np.concatenate([gd.real.ravel(), gd.imag.ravel()]))
    return np.array(out)


def build_features(params: List[tuple], cfg: WarmStartConfig, device="cuda",
                   rows: Optional[np.ndarray] = None) -> np.ndarray:
    """[n * len(rows), 132] feature rows (FP32), instance-major; rows: the k
    indices to include (default: all N)."""
    kf = k_features(cfg.nk)
    if rows is not None:
        kf = kf[rows]
    nr = kf.shape[0]
    g0 = coarse_gd0(params, cfg, device)
    out = np.empty((len(params) * nr, 7 + kf.shape[1] + g0.shape[1]), dtype=np.float32)
    for i, ((U, beta), gsum) in enumerate(zip(params, g0)):
        inst = np.array([U, beta, math.log(U), math.log(beta), 1.0 / beta, cfg.t, 2.0])
        out[i * nr:(i + 1) * nr] = np.concatenate([np.tile(inst, (nr, 1)), kf, np.tile(gsum, (nr, 1))],
                                                  axis=1)
    return out


# ---------------------------------------------------------------- data from the method
def converge(params: List[tuple], cfg: WarmStartConfig, sigma0: Optional[list] = None,
             batch: int = 64, device="cuda", accel: int = 0, prec: int = B.DF_FP64,
             symmetry: int = 0, keep=None, log=None):
    """Run df_iterate to cfg.tol for every instance (fused batches; accel > 0:
    Anderson-accelerated, prec DF_ADAPTIVE: FP32 ladders far from the fixed
    point, symmetry 1: one ladder per point-group orbit - each the same fixed
    point).

    Returns (per instance keep(sigma) - by default the converged Sigma~ as a
    numpy [n_nu x N] array -, iteration counts, seconds per batch).
    """
    import torch
    keep = keep or (lambda s: s)
    sig, its, secs = [], [], []
    stream = torch.cuda.Stream(device=device)
    for s in range(0, len(params), batch):
        chunk = params[s:s + batch]
        insts = [B.make_instance(cfg.problem(U, beta), device=device, outputs=False)
                 for U, beta in chunk]
        if sigma0 is not None:
            for x, s0 in zip(insts, sigma0[s:s + batch]):
                x.sigma.copy_(torch.as_tensor(s0))
        ws = B.workspace(insts, B.make_opts(accel=accel), device=device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        code, it, diffs = B.df_iterate(insts, ws, B.make_opts(prec=prec, mix=cfg.mix, tol=cfg.tol,
                                                              max_iter=500, use_graph=1, accel=accel,
                                                              symmetry=symmetry),
                                       stream=stream.cuda_stream,
                                       allow=(B.DF_OK, B.DF_W_FALLBACK, B.DF_E_NOT_CONVERGED))
        stream.synchronize()
        secs.append(time.perf_counter() - t0)
        its.append(it)
        sig.extend(keep(x.sigma.cpu().numpy()) for x in insts)
        del insts, ws
        if log and len(params) > batch:
            log(f"converged {min(s + batch, len(params))} of {len(params)} ({secs[-1]:.2f} s, "
                f"{it} iterations)")
    return sig, its, secs


def targets_from_sigma(sigmas, cfg: WarmStartConfig, rows: Optional[np.ndarray] = None) -> np.ndarray:
    """[n * N, 3 n_nu / 2] rows: Re and Im of Sigma~ / S at the positive
    frequencies, then n_nu / 2 copies of log S, with S the instance's
    root-mean-square |Sigma~|.

    Sigma~ spans orders of magnitude over the (U, beta) range; splitting off
    the instance scale makes the regression error relative.  The copies give
    the scale the same weight in the mean squared error as the shape.
    """
    h = cfg.n_nu // 2
    out = []
    for s in sigmas:
        S = max(float(np.sqrt(np.mean(np.abs(s) ** 2))), 1e-300)
        pos = s[h:].T / S                                          # [N, h], nu_0 .. nu_{h-1}
        if rows is not None:
            pos = pos[rows]
        out.append(np.concatenate([pos.real, pos.imag, np.full((pos.shape[0], h), math.log(S))],
                                  axis=1))
    return np.concatenate(out, axis=0)


def sigma_from_rows(rows: np.ndarray, cfg: WarmStartConfig) -> np.ndarray:
    """Inverse of targets_from_sigma for one instance, with Sigma~(-nu) = Sigma~(nu)*."""
    h = cfg.n_nu // 2
    S = math.exp(float(np.mean(rows[:, 2 * h:])))
    pos = S * (rows[:, :h] + 1j * rows[:, h:2 * h]).T               # [h, N]
    return np.concatenate([np.conj(pos[::-1]), pos], axis=0)


# ---------------------------------------------------------------- the network on the GPU
def _scale(std: np.ndarray) -> np.ndarray:
    return np.where(std > 1e-12 * max(float(np.max(std)), 1e-300), std, 1.0)


class WarmStartNet:
    def __init__(self, n_in: int, n_out: int, seed: int = 0, device="cuda"):
        import torch
        self.dims = [n_in, *HIDDEN, n_out]
        self.device = device
        rng = np.random.default_rng(seed)
        flat = []
        for l in range(len(self.dims) - 1):
            fan_in = self.dims[l]
            flat.append(rng.standard_normal(self.dims[l + 1] * fan_in) * math.sqrt(2.0 / fan_in))
            flat.append(np.zeros(self.dims[l + 1]))
        p = np.concatenate(flat).astype(np.float32)
        assert p.size == B.df_mlp_param_count(self.dims)
        self.params = torch.as_tensor(p, device=device)
        self.x_mean = self.x_std = self.y_mean = self.y_std = None

    def fit(self, X: np.ndarray, Y: np.ndarray, steps: int = 2000, batch: int = 4096,
            lr: float = 2e-3, seed: int = 1, log_every: int = 0):
        import torch
        dev = self.device
        # constant columns (t and D of a one-lattice training set) stay unscaled
        self.x_mean, self.x_std = X.mean(0), _scale(X.std(0))
        self.y_mean, self.y_std = Y.mean(0), _scale(Y.std(0))
        Xs = torch.as_tensor(((X - self.x_mean) / self.x_std).astype(np.float32), device=dev)
        Ys = torch.as_tensor(((Y - self.y_mean) / self.y_std).astype(np.float32), device=dev)
        n = Xs.shape[0]
        batch = min(batch, n)
        grads = torch.zeros_like(self.params)
        m = torch.zeros_like(self.params)
        v = torch.zeros_like(self.params)
        loss = torch.zeros(1, dtype=torch.float32, device=dev)
        ws = B.mlp_workspace(self.dims, batch, device=dev)
        gen = torch.Generator(device=dev)
        gen.manual_seed(seed)
        history = []
        for step in range(1, steps + 1):
            idx = torch.randint(0, n, (batch,), device=dev, generator=gen)
            xb = Xs.index_select(0, idx).contiguous()
            yb = Ys.index_select(0, idx).contiguous()
            B.df_mlp_loss_grad(self.dims, self.params, xb, yb, grads, loss, ws)
            cur_lr = lr * 0.5 * (1.0 + math.cos(math.pi * step / steps)) + 1e-5
            B.df_mlp_adam(self.params, grads, m, v, step, cur_lr)
            if step == 1 or step == steps or (log_every and step % log_every == 0):
                history.append((step, float(loss.item())))
        return history

    def predict(self, X: np.ndarray) -> np.ndarray:
        import torch
        Xs = torch.as_tensor(((X - self.x_mean) / self.x_std).astype(np.float32), device=self.device)
        Y = torch.empty((Xs.shape[0], self.dims[-1]), dtype=torch.float32, device=self.device)
        ws = B.mlp_workspace(self.dims, Xs.shape[0], device=self.device)
        B.df_mlp_forward(self.dims, self.params, Xs, Y, ws)
        return Y.cpu().numpy().astype(np.float64) * self.y_std + self.y_mean


def train_and_evaluate(n_train: int = 256, n_test: int = 16, steps: int = 2000,
                       cfg: Optional[WarmStartConfig] = None, seed_train: int = 895,
                       seed_test: int = 896, test_params: Optional[List[tuple]] = None,
                       device="cuda", log=None, loop: Optional[dict] = None,
                       data_loop: Optional[dict] = None, batch: int = 64,
                       more_loops: Optional[dict] = None):
    """Generate converged Sigma~ with the method, train, compare cold and warm starts.

    The training set is a Latin-hypercube draw over the (U, beta) box with its
    corners (seed_train); the test points are n_test fresh draws (seed_test)
    or test_params, and none of them may be a training point (held out).
    Training rows are the k of the irreducible wedge of each instance.
    loop: df_iterate options of the cold / warm comparison (default: FP64,
    linear mixing); data_loop: those of the data generation (default: FP64,
    Anderson m = 5); more_loops: {name: (options, number of test points)},
    further cold / warm comparisons on the first test points.  Every loop runs to cfg.tol, so both starts end at the
    same fixed point.  log: optional callable receiving progress strings.
    """
    log = log or (lambda msg: None)
    cfg = cfg or WarmStartConfig()
    loop = dict(loop or {})
    data_loop = dict(data_loop or {"accel": 5})
    N = cfg.nk ** 2
    rows = wedge_rows(cfg.nk)
    t0 = time.perf_counter()
    ptrain = draw(n_train, seed_train, cfg, corners=True)
    ptest = list(test_params) if test_params is not None else draw(n_test, seed_test, cfg)
    train_set = set(ptrain)
    if any(q in train_set for q in ptest):
        raise ValueError("a test point is a training point")
    n_test = len(ptest)
    # training data: the method's own fixed points, kept as wedge rows of targets
    Y, its_train, _ = converge(ptrain, cfg, device=device, batch=batch,
                               keep=lambda s: targets_from_sigma([s], cfg, rows), log=log,
                               **data_loop)
    Y = np.concatenate(Y, axis=0)
    t_data = time.perf_counter() - t0
    log(f"warm start: {n_train} converged training instances in {t_data:.1f} s")
    X = build_features(ptrain, cfg, device, rows=rows)
    net = WarmStartNet(X.shape[1], Y.shape[1], device=device)
    t1 = time.perf_counter()
    hist = net.fit(X, Y, steps=steps)
    t_train = time.perf_counter() - t1
    log(f"warm start: {steps} training steps in {t_train:.1f} s, loss {hist[0][1]:.3g} -> {hist[-1][1]:.3g}")
    del X, Y

    ta = time.perf_counter()
    pred = net.predict(build_features(ptest, cfg, device))
    t_inf = time.perf_counter() - ta
    warm0 = [sigma_from_rows(pred[i * N:(i + 1) * N], cfg) for i in range(n_test)]
    sig_cold, it_cold, sec_cold = converge(ptest, cfg, batch=1, device=device, **loop)
    sig_warm, it_warm, sec_warm = converge(ptest, cfg, sigma0=warm0, batch=1, device=device, **loop)
    rel_pred = [float(np.linalg.norm(w - c) / np.linalg.norm(c)) for w, c in zip(warm0, sig_cold)]
    rel_fixed = [float(np.linalg.norm(w - c) / np.linalg.norm(c)) for w, c in zip(sig_warm, sig_cold)]
    more = {}
    for name, (opts, n_sub) in (more_loops or {}).items():
        sub = ptest[:n_sub]
        _, ic, sc = converge(sub, cfg, batch=1, device=device, keep=lambda s: None, **opts)
        _, iw, sw = converge(sub, cfg, sigma0=warm0[:n_sub], batch=1, device=device,
                             keep=lambda s: None, **opts)
        more[name] = {"loop": {k: int(v) for k, v in opts.items()}, "n_test": len(sub),
                      "mean_iterations_cold": float(np.mean(ic)),
                      "mean_iterations_warm": float(np.mean(iw)),
                      "mean_seconds_cold": float(np.mean(sc)),
                      "mean_seconds_warm": float(np.mean(sw)) + t_inf / n_test}
        log(f"warm start, {name}: iterations {more[name]['mean_iterations_cold']:.1f} -> "
            f"{more[name]['mean_iterations_warm']:.1f}")
    return {
        "more_loops": more,
        "workload": f"2D {cfg.nk}x{cfg.nk}, n_nu {cfg.n_nu}, n_om {cfg.n_om}, t {cfg.t}, "
                    f"U in {cfg.U_range}, beta in {cfg.beta_range}, tol {cfg.tol}",
        "n_train": n_train, "n_test": n_test, "train_steps": steps,
        "test_held_out": True, "train_rows_per_instance": int(len(rows)),
        "loop": {k: int(v) for k, v in loop.items()},
        "data_loop": {k: int(v) for k, v in data_loop.items()},
        "train_loss_first_last": [hist[0][1], hist[-1][1]],
        "seconds_data": t_data, "seconds_train": t_train, "seconds_inference": t_inf,
        "iterations_cold": it_cold, "iterations_warm": it_warm,
        "mean_iterations_cold": float(np.mean(it_cold)), "mean_iterations_warm": float(np.mean(it_warm)),
        "mean_seconds_cold": float(np.mean(sec_cold)),
        "mean_seconds_warm": float(np.mean(sec_warm)) + t_inf / n_test,
        "prediction_rel_error_mean": float(np.mean(rel_pred)),
        "fixed_point_rel_diff_max": float(np.max(rel_fixed)),
        "train_iterations_mean": float(np.mean(its_train)),
    }


if __name__ == "__main__":
    import json
    import sys
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 256
    print(json.dumps(train_and_evaluate(n_train=n)))
