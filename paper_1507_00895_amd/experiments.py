"""The paper's convergence and cost sweeps (Sec. 4, "Example I and performance
analysis") on the GPU path.

The 2D Hubbard model with the closed-form atomic-limit inputs at U = 20,
mu = U/2, beta = 1 (t = 1) is converged with df_iterate for a range of one
control parameter x while the others stay at the paper's values:

  om   N_Omega (bosonic frequencies)  at N_omega = 48, N_k = 16
  nu   N_omega (fermionic window)     at N_Omega = 3,  N_k = 8
  k    N_k (k-points per axis)        at N_Omega = 3,  N_omega = 48

For each point it records the wall time to convergence (tol 1e-10) and
g = G~(i pi / beta, k = 0), and reports delta_g = |g_x - g_inf| / |g_inf|, with
g_inf from a fit g_x = g_inf + a x^-p over the five largest points of the
sweep (the paper extrapolates N_x -> infinity, eq. deltag, without saying
how; a power law is what its Figs. 1 and 2 show).

    python -m paper_1507_00895_amd.experiments --sweep om|nu|k|all [--repeat R] [--graph-unroll U]

prints one JSON object per sweep.  Every step runs in libdf's kernels.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

U, BETA, T_HOP = 20.0, 1.0, 1.0

SWEEPS = {
    "om": dict(param="n_om", values=[1, 3, 5, 7, 9, 13, 17, 23, 31, 39, 47], n_nu=48, nk=16, n_om=None),
    "nu": dict(param="n_nu", values=[8, 12, 16, 24, 32, 48, 64, 96, 128], n_nu=None, nk=8, n_om=3),
    "k": dict(param="nk", values=[4, 8, 16, 32, 64], n_nu=48, nk=None, n_om=3),
}


def converge_point(B, inputs, D, nk, n_nu, n_om, repeat=3, tol=1e-10, unroll=4):
    """Converge one point; returns (best wall seconds, g = G~(i pi/beta, k=0), iterations,
    whether tol was reached).  unroll: iterations per captured graph (the
    convergence measure is read once per graph launch, so up to unroll - 1
    iterations run past convergence; the per-iteration host wait goes)."""
    import torch
    p = inputs.atomic_limit_problem(D, nk, n_nu, n_om, BETA, U, T_HOP)
    x = B.make_instance(p)
    opts = B.make_opts(mix=0.5, tol=tol, max_iter=500, use_graph=1, graph_unroll=unroll)
    ws = B.workspace([x], opts)
    stream = torch.cuda.Stream()
    best, it, code = None, 0, 0
    for _ in range(repeat):
        x.sigma.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        code, it, d = B.df_iterate([x], ws, opts, stream=stream.cuda_stream,
                                   allow=(B.DF_OK, B.DF_W_FALLBACK, B.DF_E_NOT_CONVERGED))
        stream.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    n0 = n_nu // 2                                   # nu_n0 = pi / beta
    g = complex(x.gd[n0, 0].item())
    return best, g, it, code != B.DF_E_NOT_CONVERGED


def extrapolate(xs, gs, tail=5):
    """g_inf of the fit g = g_inf + a x^-p on the last `tail` points.  For a fixed p
    the model is linear in (g_inf, a): those come from least squares, and p from
    the smallest residual over a grid refined twice (variable projection).
    Returns (g_inf, p); (last g, None) when the last two points already agree
    to rounding (exponential convergence, as in N_k) or there are too few."""
    xs = np.asarray(xs[-tail:], float)
    gs = np.asarray(gs[-tail:], complex)
    if len(xs) < 3 or abs(gs[-1] - gs[-2]) <= 1e-13 * abs(gs[-1]):
        return complex(gs[-1]), None   # converged to rounding: nothing to extrapolate

    def fit(p):
        A = np.stack([np.ones_like(xs), xs ** (-p)], axis=1).astype(complex)
        c, *_ = np.linalg.lstsq(A, gs, rcond=None)
        return c, float(np.linalg.norm(A @ c - gs))

    lo, hi = 0.05, 8.0
    best = None
    for _ in range(3):
        grid = np.linspace(lo, hi, 401)
        res = [fit(p)[1] for p in grid]
        i = int(np.argmin(res))
        best = grid[i]
        step = grid[1] - grid[0]
        lo, hi = max(0.05, best - 2 * step), min(8.0, best + 2 * step)
    c, _ = fit(best)
    return complex(c[0]), float(best)


def run_sweep(name, repeat=3, unroll=4):
    from paper_1507_00895_amd import binding as B
    from paper_1507_00895_amd import inputs
    cfg = SWEEPS[name]
    rows = []
    for v in cfg["values"]:
        kw = dict(nk=cfg["nk"], n_nu=cfg["n_nu"], n_om=cfg["n_om"])
        kw[cfg["param"]] = v
        sec, g, it, ok = converge_point(B, inputs, 2, kw["nk"], kw["n_nu"], kw["n_om"], repeat,
                                        unroll=unroll)
        rows.append({cfg["param"]: v, "seconds": sec, "iterations": it, "converged": ok,
                     "g": [g.real, g.imag]})
        print(f"[experiments] {name} {cfg['param']}={v}: {sec * 1e3:.2f} ms, {it} iterations",
              file=sys.stderr, flush=True)
    xs = [r[cfg["param"]] for r in rows]
    gs = [complex(*r["g"]) for r in rows]
    ginf, power = extrapolate(xs, gs)
    for r, g in zip(rows, gs):
        r["delta_g"] = abs(g - ginf) / abs(ginf)
    return {"sweep": name, "fixed": {k: cfg[k] for k in ("n_nu", "nk", "n_om") if cfg[k] is not None},
            "U": U, "beta": BETA, "t": T_HOP, "tol": 1e-10, "graph_unroll": unroll,
            "g_inf": [ginf.real, ginf.imag],
            "fit_power": power, "points": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sweep", choices=["om", "nu", "k", "all"], default="all")
    ap.add_argument("--repeat", type=int, default=3)
    ap.add_argument("--graph-unroll", type=int, default=4,
                    help="iterations per captured graph (df_opts_t.graph_unroll)")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the sweeps run on the GPU path"
    names = ["om", "nu", "k"] if args.sweep == "all" else [args.sweep]
    for n in names:
        print(json.dumps(run_sweep(n, args.repeat, args.graph_unroll)), flush=True)


if __name__ == "__main__":
    main()
