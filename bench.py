"""Benchmark of the ladder dual-fermion hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec fp64|mixed|fp32]
                    [--no-cpu-baseline] [--no-converge] [--no-warm] [--batched-only]

Workload: 2D square lattice 32x32, n_nu = 64, n_om = 31, beta = 20,
U in {1, 2, 4} (three instances, t = 0.1), Hubbard-atom inputs.  A step is
one full outer iteration (dual propagator, bubble, both ladder channels for
every (Om, q), Schwinger-Dyson, mixing and the convergence measure) of all
three instances.  Inputs are resident in HBM before the timed region.

Prints one JSON line.  value = (q, Om, channel) ladder solves per second of
whole iterations of the --prec path; beside it: the ladder kernel's own rate
and roofline, and under "paths" the ladder rate and seconds per converged
Sigma~ (tol 1e-8) of the plain FP64 path, the per-ladder mixed-precision
path (FP32 + FP64 residual correction), the adaptive path (FP32 ladders while
the diff exceeds 1e-4, FP64 after), the FP64 and adaptive paths with Anderson
acceleration of the mixing, and paths warm-started by the learned network
(trained inside the run on converged Sigma~ of the same shape; its cost is
reported separately), and the CPU oracle rate.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 matrix (= FP64 vector) peak
FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 matrix peak
ACCEL = 5                    # Anderson history depth of the accelerated paths
HBM_PEAK_GBS = 8000.0


def measured_traffic(kernel: str, workgroups: int, per: int = 1):
    """HBM bytes per instance from the committed PMC summary, if it still matches.

    profiles/ladder_traffic.json records calibrated FETCH_SIZE + WRITE_SIZE of
    the ladder kernels per dispatch of `workgroups` work-groups, together with
    a hash of their sources; the figure is divided by the `per` instances such
    a dispatch covers.  When the sources have changed since, the figures no
    longer apply and None is returned.
    """
    import hashlib
    path = os.path.join(ROOT, "profiles", "ladder_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        entry = rec["kernels"].get(f"{kernel}@{workgroups}")
        if entry is None:
            return None
        h = hashlib.sha256()
        for name in rec["source_files"]:
            with open(os.path.join(ROOT, "paper_1507_00895_amd", "csrc", name), "rb") as f:
                h.update(f.read())
        if h.hexdigest()[:16] != rec["source_sha256_16"]:
            return None
        return float(entry["traffic_bytes"]) / per
    except (OSError, KeyError, ValueError):
        return None


def ladder_flops(n_nu: int) -> float:
    """Algorithmic real flops of one complex n_nu x n_nu inversion: 8 n^3."""
    return 8.0 * n_nu ** 3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", choices=["fp64", "mixed", "fp32"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-converge", action="store_true",
                    help="skip the seconds-per-converged-Sigma~ legs of all paths")
    ap.add_argument("--no-warm", action="store_true", help="skip the warm-started path")
    ap.add_argument("--no-tune", action="store_true", help="keep the default ladder kernels")
    ap.add_argument("--c5-train", type=int, default=2000,
                    help="training instances of the full-scale warm start (64x64, n_nu 128)")
    ap.add_argument("--c5-test", type=int, default=50, help="its held-out evaluation draws")
    ap.add_argument("--no-c5", action="store_true", help="skip the full-scale warm start")
    ap.add_argument("--no-cubic16", action="store_true", help="skip the 3D 16^3 leg")
    ap.add_argument("--warm-train", type=int, default=128,
                    help="converged instances the warm-start network is trained on")
    ap.add_argument("--warm-steps", type=int, default=6000)
    ap.add_argument("--graph", type=int, default=1)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--traffic-table", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/ladder_traffic.json from the counter_collection.csv "
                         "files of two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of "
                         "--profile-ladders --copy-calibration, then exit (no GPU needed)")
    ap.add_argument("--profile-ladders", action="store_true",
                    help="only the ladder launches of the main kernel builds (square 32x32 and "
                         "cubic 16^3 workloads), for rocprofv3 runs")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched uneven workload leg and print its JSON object")
    return ap.parse_args()


def cpu_baseline(problems, budget_s: float = 8.0):
    """Time the CPU oracle on one outer iteration of the first instance, on the
    host's cores: 1 process, and P processes (P = the cores this process may
    run on) with the ladder split over the bosonic slices; BLAS threads = 1 in
    every process.

    The dual propagator, bubble and Schwinger-Dyson steps run once in this
    process (FFTs, single-threaded).  The 1-process ladder runs on as many
    slices as fit in about budget_s and is scaled to all n_om; the P-process
    ladder runs every slice.  Returns solves/s of whole iterations (P
    processes as the value, the 1-process figure beside it).
    """
    import multiprocessing as mp
    import numpy as np
    from oracle import df_oracle as O
    from oracle.timing import ladder_seconds
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"     # inherited by the worker processes started below
    p = problems[0]
    t0 = time.perf_counter()
    G0 = O.dual_gf0(p.g, p.delta, p.eps)
    G = O.dual_gf(G0, np.zeros_like(G0))
    chi = O.bubble_fft(G, p.D, p.nk, p.n_om, p.beta)
    gam = O.spin_channels(p.gamma_uu, p.gamma_ud)
    t_pre = time.perf_counter() - t0
    W = np.zeros((2, p.n_om, p.n_nu, p.N), dtype=np.complex128)
    t2 = time.perf_counter()
    O.sigma_fft(W, G, p.D, p.nk, p.beta)
    t_sig = time.perf_counter() - t2
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    P = max(1, min(cores, 16, p.n_om))
    ctx = mp.get_context("spawn")          # no fork of a process that holds the GPU
    tasks = [(gam[:, m:m + 1], chi[m:m + 1]) for m in range(p.n_om)]
    with ctx.Pool(1) as pool:
        n_sl, t1 = 0, 0.0
        pool.apply(ladder_seconds, (tasks[0],))           # imports, first touch
        while n_sl < p.n_om and t1 < budget_s:
            t1 += pool.apply(ladder_seconds, (tasks[n_sl],))
            n_sl += 1
    t_lad1 = t1 * p.n_om / n_sl
    with ctx.Pool(P) as pool:
        pool.map(ladder_seconds, tasks[:P], chunksize=1)  # imports, first touch
        ta = time.perf_counter()
        pool.map(ladder_seconds, tasks, chunksize=1)
        t_ladP = time.perf_counter() - ta
    solves = 2 * p.n_om * p.N
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    one = solves / (t_pre + t_lad1 + t_sig)
    return {"value": solves / (t_pre + t_ladP + t_sig), "unit": "solves/s", "cores": P,
            "kind": "oracle", "processes": P, "blas_threads_per_process": 1,
            "single_process": {"value": one, "cores": 1,
                               "sample": f"ladder on {n_sl} of {p.n_om} bosonic slices, scaled"},
            "cpu_model": model, "cpu_count": os.cpu_count(), "affinity_cores": cores,
            "seconds_per_iteration": {"1_process": t_pre + t_lad1 + t_sig,
                                      f"{P}_processes": t_pre + t_ladP + t_sig},
            "sample": (f"one outer iteration of the U={p.U} instance of the 2D 32x32 workload: "
                       f"dual GF, bubble and Schwinger-Dyson in one process; the ladder "
                       f"({solves} solves) over all {p.n_om} bosonic slices on {P} processes "
                       f"({t_ladP:.1f} s); 1 process: {n_sl} slices timed and scaled")}


def orbit_count(D, nk):
    """Orbits of the hypercubic point group (axis permutations, k_a -> -k_a) on the q-grid."""
    import itertools
    return len({tuple(sorted(min(c, (nk - c) % nk) for c in q))
                for q in itertools.product(range(nk), repeat=D)})


def ladder_launch_ms(B, insts, ws, prec, stream, reps, symmetry=0):
    """Ladder time per instance: df_ladder_solve over all instances (one fused launch
    per kernel class, as in the loop), HIP events on the launch stream, divided by
    the instance count."""
    import numpy as np
    import torch
    ms = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        B.df_ladder_solve(insts, ws, B.make_opts(prec=prec, symmetry=symmetry),
                          stream=stream.cuda_stream)
        e1.record(stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    return float(np.mean(ms)) / len(insts)


def converge_each(B, problems, insts, ws, prec, stream, graph, sigma0=None, accel=0, symmetry=0):
    """Cold (or given) start to tol 1e-8, one instance at a time (DF_ADAPTIVE:
    FP32 ladders down to a diff of 1e-4, FP64 after; accel > 0: Anderson
    acceleration over accel + 1 iterates)."""
    import torch
    out = []
    for i, (p, x) in enumerate(zip(problems, insts)):
        if sigma0 is None:
            x.sigma.zero_()
        else:
            x.sigma.copy_(torch.as_tensor(sigma0[i]))
        torch.cuda.synchronize()
        ta = time.perf_counter()
        code, it, d = B.df_iterate([x], ws, B.make_opts(prec=prec, mix=0.5, tol=1e-8, max_iter=500,
                                                        use_graph=graph, switch_tol=1e-4,
                                                        accel=accel, symmetry=symmetry),
                                   stream=stream.cuda_stream,
                                   allow=(B.DF_OK, B.DF_W_FALLBACK, B.DF_E_NOT_CONVERGED))
        stream.synchronize()
        out.append({"U": p.U, "iterations": it, "seconds": time.perf_counter() - ta,
                    "final_diff": d[0], "code": code})
    return out


def kernel_symbol(variant: str, np_: int, full: bool = True) -> str:
    """Kernel of a variant name at padded size np_; full: the launch's instances
    all have n_nu = np_ (the mask-free builds).  Persistent grids ("@p1", "@p2")
    run the item-loop build of the same kernel; at np_ = 96 the one-item-per-slot
    launches of gjb and fp32 hold two items per work-group."""
    base, _, persist = variant.partition("@")
    f = "true" if full else "false"
    loop = "true" if persist else "false"
    if base == "gjb" and np_ == 96 and full and not persist:
        return "k_ladder_gjb_f64_xk<96, true, 2>"
    if base == "fp32" and np_ == 96 and full:
        return "k_ladder_fp32_x2<96, true>"
    table = {"gjb": f"k_ladder_gjb_f64<{np_}, {loop}, {f}>",
             "gjb_o3": f"k_ladder_gjb_f64_o3<{np_}, {loop}, {f}>",
             "gjb_o4": f"k_ladder_gjb_f64_o4<{np_}, {f}>",
             "vector": f"k_ladder_fp64<{np_},...>", "mfma": f"k_ladder_mfma_f64<{np_}>"}
    for k in ("mixed", "mixed_o3", "mixed_o4", "fp32", "fp32_o4", "fp32_o5"):
        table[k] = f"k_ladder_{k}<{np_}, {f}>"
    return table[base]


def roofline_of(prec, B, n_om, N, n_nu, lad_ms, n_inst=1):
    """Roofline of the ladder kernel per instance; lad_ms is the time per instance
    (launches fused over n_inst instances, as the loop runs them)."""
    flops_launch = 2 * n_om * N * ladder_flops(n_nu)
    variant = B.df_ladder_variant(n_nu, prec)
    kernel_name = kernel_symbol(variant, n_nu)
    base = variant.partition("@")[0]
    if base in ("fp32", "fp32_o4", "fp32_o5"):
        peak = FP32_PEAK_TFLOPS
    elif base not in ("mixed", "mixed_o3", "mixed_o4"):
        peak = FP64_PEAK_TFLOPS
    else:
        # The refined solve's own work per solve: the inverse and Z0 = X gamma in
        # FP32 (2 x 8 n^3 flops) and the residual in FP64 (8 n^3).  Each part is
        # priced at its own peak; the blended peak is that work over its time.
        flops_launch *= 3
        t_unit = 2.0 / FP32_PEAK_TFLOPS + 1.0 / FP64_PEAK_TFLOPS
        peak = 3.0 / t_unit
    achieved = flops_launch / (lad_ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": measured_traffic(kernel_name, 2 * n_om * N * n_inst, n_inst),
            "traffic_source": "profiles/ladder_traffic.json: rocprofv3 FETCH_SIZE + WRITE_SIZE of "
                              "this build and launch shape, scaled by a 256 MiB copy; null once "
                              "the ladder sources differ from the profiled ones",
            "kernel": kernel_name, "variant": variant, "launch_ms": lad_ms,
            "algorithmic_flops_per_launch": flops_launch}


def lattice_leg(B, problems, insts, stream, log):
    """df_lattice (Sigma_lat, G_lat, chi^{ch/sp} at Omega = 0) on each instance's last
    converged Sigma~: time per instance (HIP events) and where chi^sp peaks."""
    import numpy as np
    import torch
    out = []
    for p, x in zip(problems, insts):
        c = dict(dtype=torch.complex128, device=x.g.device)
        sl, gl = torch.empty((p.n_nu, p.N), **c), torch.empty((p.n_nu, p.N), **c)
        ch, sp = torch.empty(p.N, **c), torch.empty(p.N, **c)
        ws = B.lattice_workspace(x, device=x.g.device)
        B.df_lattice(x, p.mu, sl, gl, ch, sp, ws=ws, stream=stream.cuda_stream)   # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        B.df_lattice(x, p.mu, sl, gl, ch, sp, ws=ws, stream=stream.cuda_stream)
        e1.record(stream)
        e1.synchronize()
        s = sp.cpu().numpy().real
        q = int(np.argmax(s))
        Q = sum((p.nk // 2) * p.nk ** a for a in range(p.D))
        out.append({"U": p.U, "ms": e0.elapsed_time(e1), "chi_sp_max": float(s[q]),
                    "chi_sp_peak_at_Q": q == Q, "chi_ch_at_Q": float(ch.cpu().numpy().real[Q])})
    log(f"lattice observables: {[round(o['ms'], 2) for o in out]} ms per instance")
    return out


def batched_leg(B, log):
    """The uneven batched workload (64 seeded instances, D in {2, 3}, 2D 16^2..64^2,
    3D 8^3..16^3, n_nu in {32, 64, 128}) in fused, graph-captured iterations:
    time per outer iteration of all 64 and the ladder solves per second, FP64,
    after autotuning each n_nu class on its fused launch."""
    import numpy as np
    import torch
    from paper_1507_00895_amd import inputs as I
    probs = I.batched_problems(I.batched_params())
    insts = [B.make_instance(p) for p in probs]
    ws = B.workspace(insts)
    s = torch.cuda.Stream()
    B.df_autotune(insts, ws, B.make_opts(prec=B.DF_FP64), stream=s.cuda_stream)
    opts = B.make_opts(mix=0.5, tol=0.0, max_iter=1, use_graph=1)
    B.df_iterate(insts, ws, opts, stream=s.cuda_stream, allow=(B.DF_OK, B.DF_W_FALLBACK))
    s.synchronize()
    steps = 3
    opts = B.make_opts(mix=0.5, tol=0.0, max_iter=steps, use_graph=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.df_iterate(insts, ws, opts, stream=s.cuda_stream, allow=(B.DF_OK, B.DF_W_FALLBACK))
    s.synchronize()
    dt = (time.perf_counter() - t0) / steps
    solves = sum(2 * p.n_om * p.N for p in probs)
    out = {"instances": len(probs), "ms_per_iteration": dt * 1e3,
           "ladder_solves_per_iteration": solves, "solves_per_s": solves / dt,
           "ladder_classes": sorted({p.n_nu for p in probs}),
           "variants": {n: B.df_ladder_variant(n, B.DF_FP64) for n in sorted({p.n_nu for p in probs})}}
    log(f"batched uneven workload: {out['ms_per_iteration']:.1f} ms per iteration of "
        f"{len(probs)} instances, {out['solves_per_s'] / 1e6:.1f} M solves/s")
    del insts, ws
    torch.cuda.empty_cache()
    return out


def warm_start_leg(args, log):
    """The learned warm start at the bench shape (2D 32x32, n_nu 64, n_om 31):
    trained on args.warm_train converged Sigma~ (Latin-hypercube draws over
    U in [1, 4], beta in [5, 20] with the box corners, seed 895), evaluated on
    8 held-out draws (seed 896; none is a training point): iterations and
    seconds to tol 1e-8, warm against cold, for the plain FP64 loop, the
    adaptive loop and the adaptive Anderson-accelerated loop."""
    from paper_1507_00895_amd import binding as B
    from paper_1507_00895_amd import warmstart as W
    cfg = W.WarmStartConfig(nk=32, n_nu=64, n_om=31, t=0.1)
    r = W.train_and_evaluate(n_train=args.warm_train, n_test=8, steps=args.warm_steps, cfg=cfg,
                             log=log, loop=dict(prec=B.DF_FP64),
                             data_loop=dict(prec=B.DF_ADAPTIVE, accel=ACCEL),
                             more_loops={"adaptive": (dict(prec=B.DF_ADAPTIVE), 8),
                                         "adaptive_anderson": (dict(prec=B.DF_ADAPTIVE, accel=ACCEL), 8),
                                         "adaptive_anderson_sym": (dict(prec=B.DF_ADAPTIVE, accel=ACCEL,
                                                                        symmetry=1), 8)})
    log(f"warm start (32x32, held out): FP64 loop {r['mean_iterations_cold']:.1f} -> "
        f"{r['mean_iterations_warm']:.1f} iterations")
    return r


def warm_config5_leg(args, log):
    """The learned warm start at its stated scale: 2D 64x64, n_nu 128, n_om 15,
    U in [1, 4], beta in [5, 20], mu = U/2, t = 0.1; trained on args.c5_train
    converged Sigma~ (seed 895, box corners included) generated by the
    adaptive, Anderson-accelerated, symmetry-reduced loop, and evaluated on
    args.c5_test held-out draws (seed 896): iterations and seconds to tol 1e-8,
    warm against cold, with that loop and with the FP64 linear-mixing loop
    (symmetry-reduced ladders) on the first 10 test points."""
    from paper_1507_00895_amd import binding as B
    from paper_1507_00895_amd import warmstart as W
    cfg = W.WarmStartConfig(nk=64, n_nu=128, n_om=15, t=0.1)
    fast = dict(prec=B.DF_ADAPTIVE, accel=ACCEL, symmetry=1)
    r = W.train_and_evaluate(n_train=args.c5_train, n_test=args.c5_test, steps=args.warm_steps,
                             cfg=cfg, log=log, loop=fast, data_loop=fast, batch=32,
                             more_loops={"fp64_linear_mixing_sym": (dict(prec=B.DF_FP64, symmetry=1),
                                                                    10)})
    log(f"warm start (config 5, {args.c5_train} training, {args.c5_test} held out): "
        f"{r['mean_iterations_cold']:.1f} -> {r['mean_iterations_warm']:.1f} iterations, "
        f"{r['mean_seconds_cold']:.3f} -> {r['mean_seconds_warm']:.3f} s")
    return r


def cubic16_leg(B, args, log):
    """3D 16^3, n_nu 96, n_om 23, U 3, beta 15, t 0.182358 (leading ladder
    eigenvalue 0.97 at Q on the first iteration): after autotuning, the ladder
    rate and roofline fraction of the FP64, refined (FP32 + FP64 residual,
    FP64 determinants near the instability) and FP32 kernels, and seconds per
    converged Sigma~ (tol 1e-8) of the FP64, refined and adaptive loops with
    Anderson acceleration, plus the plain FP64 loop with symmetry-reduced
    ladders."""
    import numpy as np
    import torch
    from paper_1507_00895_amd import inputs as I
    probs = I.workload_cubic16()
    p = probs[0]
    insts = [B.make_instance(q) for q in probs]
    ws = B.workspace(insts, B.make_opts(accel=ACCEL))
    stream = torch.cuda.Stream()
    out = {"workload": "3D 16^3, n_nu 96, n_om 23, U 3, beta 15, t 0.182358, Hubbard-atom inputs"}
    for name, pr in (("fp64", B.DF_FP64), ("mixed", B.DF_FP32_REFINE), ("fp32", B.DF_FP32)):
        if not args.no_tune:
            B.df_autotune(insts, ws, B.make_opts(prec=pr), stream=stream.cuda_stream)
        ms = ladder_launch_ms(B, insts, ws, pr, stream, 3)
        roof = roofline_of(pr, B, p.n_om, p.N, p.n_nu, ms)
        out[name] = {"ladder_variant": B.df_ladder_variant(p.n_nu, pr), "ladder_launch_ms": ms,
                     "ladder_solves_per_s": 2 * p.n_om * p.N / (ms * 1e-3),
                     "roofline_frac": roof["frac"], "roofline_achieved": roof["achieved"],
                     "roofline_peak": roof["peak"]}
        log(f"cubic16 {name}: ladder {ms:.2f} ms ({out[name]['ladder_variant']}), "
            f"{roof['frac']:.3f} of its roofline")
    for name, pr, ac, sy in (("fp64", B.DF_FP64, ACCEL, 0), ("mixed", B.DF_FP32_REFINE, ACCEL, 0),
                             ("adaptive", B.DF_ADAPTIVE, ACCEL, 0), ("fp64_sym_linear", B.DF_FP64, 0, 1)):
        conv = converge_each(B, probs, insts, ws, pr, stream, 1, accel=ac, symmetry=sy)
        out.setdefault(name, {}).update({"s_per_converged_sigma": conv[0]["seconds"],
                                         "iterations": conv[0]["iterations"],
                                         "final_diff": conv[0]["final_diff"], "code": conv[0]["code"],
                                         "accel": ac, "symmetry": sy})
        log(f"cubic16 {name}: {conv[0]['seconds']:.3f} s per converged Sigma~ "
            f"({conv[0]['iterations']} iterations)")
    # determinant of the magnetic ladder at Q, Omega = 0, first iteration and converged
    i0 = (p.n_om - 1) // 2
    Q = (p.nk // 2) * (p.nk * p.nk + p.nk + 1)
    ld = insts[0].logdet[1, i0, Q].item()
    out["det_magnetic_Q_converged"] = float(np.exp(ld.real) * np.cos(ld.imag))
    del insts, ws
    torch.cuda.empty_cache()
    return out


TRAFFIC_SOURCES = ["df_ladder_gjb.hpp", "df_ladder_mixed.hpp", "df_gj_core.hpp", "df_device.hpp",
                   "df_internal.hpp"]


def write_traffic_table(fetch_csv: str, write_csv: str) -> dict:
    """profiles/ladder_traffic.json from two rocprofv3 counter_collection.csv
    files: per ladder kernel and work-group count, FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch, averaged), each scaled by the factor that maps the same
    counter on the plain 256 MiB device copy (the 256-work-group
    __amd_rocclr_copyBuffer dispatch of --copy-calibration) to its 256 MiB;
    with the hash of the kernel sources, so that the figures are used only
    while those sources are unchanged."""
    import csv
    import hashlib
    from collections import defaultdict

    def per_kernel(path):
        acc = defaultdict(list)
        for r in csv.DictReader(open(path)):
            name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("df::", "")
            wgs = int(r["Grid_Size"]) // int(r["Workgroup_Size"])
            acc[(name, wgs)].append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in acc.items()}

    fetch, write = per_kernel(fetch_csv), per_kernel(write_csv)
    copy_mib = 256.0
    f_copy = fetch[("__amd_rocclr_copyBuffer", 256)]
    w_copy = write[("__amd_rocclr_copyBuffer", 256)]
    ff, wf = copy_mib * 1024 / f_copy, copy_mib * 1024 / w_copy
    kernels = {}
    for (name, wgs), fk in fetch.items():
        if "k_ladder" not in name or wgs < 1000 or (name, wgs) not in write:
            continue
        wk = write[(name, wgs)]
        kernels[f"{name}@{wgs}"] = {"fetch_kib_raw": fk, "write_kib_raw": wk,
                                    "fetch_bytes": fk * 1024 * ff, "write_bytes": wk * 1024 * wf,
                                    "traffic_bytes": (fk * ff + wk * wf) * 1024}
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1507_00895_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    rec = {"workload": "bench.py --profile-ladders: 2D 32x32, n_nu 64, n_om 31 (three fused instances, "
                       "190464 work-groups) and 3D 16^3, n_nu 96, n_om 23 (188416 work-groups)",
           "source_files": TRAFFIC_SOURCES, "source_sha256_16": h.hexdigest()[:16],
           "calibration": {"copy_bytes": int(copy_mib * 2 ** 20), "fetch_kib_raw": f_copy,
                           "write_kib_raw": w_copy, "fetch_factor": ff, "write_factor": wf},
           "kernels": kernels}
    with open(os.path.join(ROOT, "profiles", "ladder_traffic.json"), "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def profile_ladders(B, args, log):
    """One untimed and three timed df_ladder_solve calls per kernel build, on
    the 2D 32x32 workload (three fused instances: gjb_o4, gjb_o3, fp32_o4,
    mixed_o3, gjb_o3@p1) and the 3D 16^3 one (gjb, fp32, mixed); with
    --copy-calibration also one plain 256 MiB device copy.  For rocprofv3
    (kernel times, counters); prints the HIP-event time per call."""
    import torch
    from paper_1507_00895_amd import inputs as I
    stream = torch.cuda.Stream()
    for wl, probs, cases in (("square32", I.workload_square32(),
                              [(B.DF_FP64, "gjb_o4"), (B.DF_FP64, "gjb_o3"), (B.DF_FP32, "fp32_o4"),
                               (B.DF_FP32_REFINE, "mixed_o3"), (B.DF_FP64, "gjb_o3@p1")]),
                             ("cubic16", I.workload_cubic16(),
                              [(B.DF_FP64, "gjb"), (B.DF_FP32, "fp32"), (B.DF_FP32_REFINE, "mixed")])):
        insts = [B.make_instance(p) for p in probs]
        ws = B.workspace(insts)
        B.df_dual_gf(insts, ws)
        B.df_bubble(insts, ws)
        torch.cuda.synchronize()
        for prec, name in cases:
            B.df_ladder_set_variant(probs[0].n_nu, prec, name)
            ms = ladder_launch_ms(B, insts, ws, prec, stream, 4)
            log(f"{wl} {name}: {ms:.3f} ms per instance")
        # one outer iteration (graph off): every kernel of the path in the trace
        B.df_autotune_reset()
        B.df_iterate(insts, ws, B.make_opts(mix=0.5, max_iter=1), stream=stream.cuda_stream)
        stream.synchronize()
        del insts, ws
        torch.cuda.empty_cache()
    if args.copy_calibration:
        src = torch.ones(32 * 2 ** 20, dtype=torch.float64)
        src = src.cuda()
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()


def main():
    args = parse()
    if args.traffic_table:
        rec = write_traffic_table(*args.traffic_table)
        print(json.dumps({k: v["traffic_bytes"] for k, v in rec["kernels"].items()}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1507_00895_amd import binding as B
    from paper_1507_00895_amd import inputs as I

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.profile_ladders:
        profile_ladders(B, args, log)
        return
    if args.batched_only:
        print(json.dumps({"batched_uneven": batched_leg(B, log)}), flush=True)
        return
    problems = I.workload_square32()
    insts = [B.make_instance(p, device=dev) for p in problems]
    prec = {"fp64": B.DF_FP64, "mixed": B.DF_FP32_REFINE, "fp32": B.DF_FP32}[args.prec]
    opts = B.make_opts(prec=prec, mix=0.5, tol=0.0, max_iter=1, use_graph=args.graph,
                       accel=ACCEL)
    ws = B.workspace(insts, opts, device=dev)
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    sh = stream.cuda_stream

    # autotune the ladder kernel for both precisions on this workload's data
    tuned = {}
    if not args.no_tune:
        for name, pr in (("fp64", B.DF_FP64), ("mixed", B.DF_FP32_REFINE), ("fp32", B.DF_FP32)):
            t_a = time.perf_counter()
            B.df_autotune(insts, ws, B.make_opts(prec=pr), stream=sh)
            tuned[name] = {"variant": B.df_ladder_variant(problems[0].n_nu, pr),
                           "seconds": time.perf_counter() - t_a}
        log(f"autotuned: {tuned}")

    # warmup
    if args.warmup > 0:
        B.df_iterate(insts, ws, B.make_opts(prec=prec, mix=0.5, tol=0.0, max_iter=args.warmup,
                                            use_graph=args.graph), stream=sh)
    stream.synchronize()
    # timed: K outer iterations of the three instances
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    code, iters, diffs = B.df_iterate(insts, ws, B.make_opts(prec=prec, mix=0.5, tol=0.0,
                                                             max_iter=args.steps,
                                                             use_graph=args.graph), stream=sh)
    stream.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert iters == args.steps
    solves_per_step = sum(2 * p.n_om * p.N for p in problems)
    ms_per_step = 1e3 * dt / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step")

    p0 = problems[0]
    reps = max(3, args.steps)
    lad_ms = ladder_launch_ms(B, insts, ws, prec, stream, reps)
    roof = roofline_of(prec, B, p0.n_om, p0.N, p0.n_nu, lad_ms, len(insts))

    if args.copy_calibration:
        # a plain copy kernel of known size: 256 MiB read + 256 MiB written
        src = torch.ones(32 * 2 ** 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # the three paths on the same GPU: ladder rate and seconds per converged
    # Sigma~ (tol 1e-8), per instance
    paths = {}
    if not args.no_converge:
        for name, pr in (("fp64", B.DF_FP64), ("mixed", B.DF_FP32_REFINE), ("fp32", B.DF_FP32),
                         ("adaptive", B.DF_ADAPTIVE)):
            entry = {}
            if pr != B.DF_ADAPTIVE:
                ms = lad_ms if pr == prec else ladder_launch_ms(B, insts, ws, pr, stream, reps)
                entry = {"ladder_variant": B.df_ladder_variant(p0.n_nu, pr), "ladder_launch_ms": ms,
                         "ladder_solves_per_s": 2 * p0.n_om * p0.N / (ms * 1e-3),
                         "roofline_frac": roofline_of(pr, B, p0.n_om, p0.N, p0.n_nu, ms,
                                                     len(insts))["frac"]}
            if pr != B.DF_FP32:       # FP32 alone does not reach the FP64 fixed point
                conv = converge_each(B, problems, insts, ws, pr, stream, args.graph)
                entry.update({"s_per_converged_sigma": float(np.mean([c["seconds"] for c in conv])),
                              "mean_iterations": float(np.mean([c["iterations"] for c in conv])),
                              "converged": conv})
                log(f"{name}: {entry['s_per_converged_sigma']:.3f} s per converged Sigma~")
            paths[name] = entry
        # the same loops with Anderson acceleration of the mixing
        for name, pr in (("fp64_anderson", B.DF_FP64), ("adaptive_anderson", B.DF_ADAPTIVE)):
            conv = converge_each(B, problems, insts, ws, pr, stream, args.graph, accel=ACCEL)
            paths[name] = {"s_per_converged_sigma": float(np.mean([c["seconds"] for c in conv])),
                           "mean_iterations": float(np.mean([c["iterations"] for c in conv])),
                           "accel": ACCEL, "converged": conv}
            log(f"{name}: {paths[name]['s_per_converged_sigma']:.3f} s per converged Sigma~")
        # symmetry-reduced ladders (one q per point-group orbit, Omega >= 0): a different
        # unit of work, so reported apart; "effective" rates count the full 2 n_om N ladders
        ms = ladder_launch_ms(B, insts, ws, B.DF_FP64, stream, reps, symmetry=1)
        paths["fp64_sym"] = {"ladder_launch_ms": ms,
                             "ladders_solved_per_launch":
                                 2 * (p0.n_om - (p0.n_om - 1) // 2) * orbit_count(p0.D, p0.nk),
                             "effective_solves_per_s": 2 * p0.n_om * p0.N / (ms * 1e-3)}
        for name, pr, ac in (("fp64_sym", B.DF_FP64, 0), ("adaptive_anderson_sym", B.DF_ADAPTIVE, ACCEL)):
            conv = converge_each(B, problems, insts, ws, pr, stream, args.graph, accel=ac, symmetry=1)
            paths.setdefault(name, {}).update(
                {"s_per_converged_sigma": float(np.mean([c["seconds"] for c in conv])),
                 "mean_iterations": float(np.mean([c["iterations"] for c in conv])),
                 "converged": conv})
            log(f"{name}: {paths[name]['s_per_converged_sigma']:.3f} s per converged Sigma~")
        if not args.no_warm:
            paths["warm_square32"] = warm_start_leg(args, log)
        paths["lattice_observables"] = lattice_leg(B, problems, insts, stream, log)
        paths["batched_uneven"] = batched_leg(B, log)
        if not args.no_cubic16:
            paths["cubic16"] = cubic16_leg(B, args, log)
        if not args.no_warm and not args.no_c5:
            paths["warm_config5"] = warm_config5_leg(args, log)

    out = {
        "metric": "ladder (q,omega) solves/s + s per converged Sigma~: FP64 vs FP32-MFMA+refine at 1e-9 rel",
        "value": solves_per_step / (ms_per_step * 1e-3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed": "f32+f64", "fp32": "f32"}[args.prec],
        "data": "synthetic",
        "config": {"workload": "2D square 32x32, n_nu 64, n_om 31, beta 20, U in {1,2,4}, t 0.1, "
                               "Hubbard-atom inputs; one step = one outer iteration of all 3",
                   "path": args.prec, "hip_graph": bool(args.graph), "autotuned": tuned,
                   "solves_per_step": solves_per_step},
        "roofline": roof,
        "ladder_solves_per_s": 2 * p0.n_om * p0.N / (lad_ms * 1e-3),
        "paths": paths,
    }
    if args.prec in paths:
        out["s_per_converged_sigma"] = paths[args.prec]["s_per_converged_sigma"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(problems)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
