"""Benchmark: assemble + solve + evaluate of the multilevel 2D Poisson least-squares system.

Workload (default): -Lap u = f on [0,1]^2, u = sum_{k in 1,4,16} sin(k pi x) sin(k pi y)/k,
three levels of 1x1, 4x4 and 16x16 subdomains (width ratio 2.9), 96 tanh random features per
subdomain, 400 x 400 collocation grid: 160,000 rows, 26,208 columns, 2.42e8 stored entries.

One step = the whole hot path on one synthetic input already resident in HBM: assemble the
block-sparse matrix (FP64, plus an FP32 copy) and right-hand side, build the block-Jacobi
preconditioner from the FP64 diagonal Gram blocks, run the solver until the solution on a
128 x 128 check grid is within rel-L2 1e-6 of the exact solution (or the iteration budget of
15,000 iterations is spent), evaluate the solution on the 480 x 480 test grid.

Default solver: FP64 iterative refinement (residual with the FP64 matrix) around block-Jacobi
preconditioned LSQR on the FP32 copy.  For comparison the same step is also timed once with
block-Jacobi LSQR in FP64 and with plain FP64 LSQR (the method's own solver and budget).

Prints one JSON line.  value = collocation rows per second of time-to-solution.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("time-to-solution at rel-L2 1e-6 (s) and collocation rows/s; "
          "mixed/batched vs plain FP64")
HBM_PEAK_GBS = 8000.0
# dense matrix-core peaks of MI355X (TFLOP/s), per input type
MFMA_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="poisson3l")
    p.add_argument("--method", default="mixed_ir",
                   choices=["lsqr", "cgls", "mixed_ir", "normal_cg", "mixed_ir_cg"])
    p.add_argument("--gram-prec", default=None, choices=["fp64", "fp32"],
                   help="Gram blocks for normal_cg / mixed_ir_cg (default fp64 / fp32)")
    p.add_argument("--no-precond", action="store_true", help="no block-Jacobi preconditioning")
    p.add_argument("--shift", type=float, default=1e-12)
    p.add_argument("--store", default=None, choices=["fp64", "fp32", "bf16", "fp16"],
                   help="low-precision stored copy for the inner solves of mixed_ir (default: "
                        "fp16 for single problems, fp32 for the batched workloads)")
    p.add_argument("--inner", type=int, default=None,
                   help="inner LSQR steps per refinement step (default: 500 on a 16-bit copy, "
                        "2500 on fp32)")
    p.add_argument("--no-gram", action="store_true", help="skip the Gram-phase MFMA timing")
    p.add_argument("--no-compare", action="store_true",
                   help="skip the FP64 comparison solves")
    p.add_argument("--iters", type=int, default=15000)
    p.add_argument("--target", type=float, default=1e-6)
    p.add_argument("--check-every", type=int, default=100)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--kernel-reps", type=int, default=20)
    p.add_argument("--compare-iters", type=int, default=15000,
                   help="iteration budget of the FP64 comparison solves")
    p.add_argument("--batch-n", type=int, default=512)
    p.add_argument("--batch-btol", type=float, default=1e-6)
    p.add_argument("--epochs", type=int, default=100, help="warm workload: MLP training epochs")
    p.add_argument("--copy-bytes", type=int, default=0,
                   help="only run device copies of this many bytes (traffic-counter reference)")
    args = p.parse_args()
    gram_method = args.method in ("normal_cg", "mixed_ir_cg")
    if args.gram_prec is None:
        args.gram_prec = "fp32" if args.method == "mixed_ir_cg" else "fp64"
    if args.store is None:
        if gram_method:
            args.store = "fp32" if args.gram_prec == "fp32" else "fp64"
        else:
            args.store = "fp16" if args.workload in ("poisson3l", "poisson5l") else "fp32"
    if args.inner is None:
        args.inner = 500 if args.store in ("fp16", "bf16") else 2500
    return args


def _threads():
    """Threads the oracle's BLAS actually runs with (threadpoolctl's view of the loaded BLAS)."""
    from threadpoolctl import threadpool_info
    n = [int(i["num_threads"]) for i in threadpool_info() if i.get("user_api") == "blas"]
    return max(n) if n else 1


def cpu_baseline(spec, W, b, f, n_iters_solve, budget_s=20.0):
    """The oracle (numpy/scipy float64, untuned) on the host: a bounded sample of the same
    workload, scaled to the full step.  Sample: assembly of a subset of subdomain blocks on every
    level (per-entry cost), and LSQR iterations on those blocks (per-entry matvec cost)."""
    import numpy as np
    from oracle import assemble as asm
    from oracle import geometry as geo
    from oracle import linalg
    from oracle import basis

    x = geo.points(spec)
    subs = geo.subdomains(spec)
    N = x.shape[0]
    L = len(spec.levels)
    rng = np.random.default_rng(0)
    # pick up to 6 subdomains per level
    picked = []
    for l in range(L):
        lev = [sd for sd in subs if sd.level == l]
        idx = rng.choice(len(lev), size=min(6, len(lev)), replace=False)
        picked += [(l, lev[i]) for i in sorted(idx)]
    t0 = time.perf_counter()
    ans = basis.ansatz(x, spec)
    sums = {}
    blocks = []
    ent = 0
    scale = 1.0 / (np.sqrt(float(N)) * L)
    for l, sd in picked:
        if l not in sums:
            sums[l] = basis.level_sum(x, [s for s in subs if s.level == l])
        rows = np.nonzero(geo.in_support(x, sd))[0]
        q = slice(sd.q0, sd.q0 + spec.K)
        val, grad, lap = basis.localized_function(x[rows], spec, sd, W[q], b[q],
                                                  tuple(s[rows] for s in sums[l]),
                                                  tuple(a[rows] for a in ans))
        blocks.append(asm.Block(sd, rows, basis.apply_operator(spec, val, grad, lap) * scale))
        ent += rows.size * spec.K
        if time.perf_counter() - t0 > budget_s / 2:
            break
    t_asm = time.perf_counter() - t0
    # LSQR iterations restricted to the sampled blocks
    n = len(subs) * spec.K
    h = asm.rhs(spec, f)
    t1 = time.perf_counter()
    its = 0
    while True:
        its += 5
        linalg.lsqr(lambda v: asm.matvec(blocks, v, N), lambda u: asm.rmatvec(blocks, u, n), h, n,
                    atol=0, btol=0, iter_lim=5)
        if time.perf_counter() - t1 > budget_s / 2 or its >= 200:
            break
    t_it = (time.perf_counter() - t1) / its
    total_nnz = sum(int(np.sum(geo.in_support(x, sd))) for sd in subs) * spec.K
    t_full = t_asm * total_nnz / ent + t_it * total_nnz / ent * n_iters_solve
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": N / t_full,
        "unit": "rows/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{len(blocks)} of {len(subs)} subdomain blocks ({ent} entries of "
                   f"{total_nnz}) assembled in {t_asm:.2f} s and {its} LSQR iterations on them "
                   f"({t_it * 1e3:.1f} ms each), scaled by entry count to the full assembly and "
                   f"{n_iters_solve} iterations: {t_full:.0f} s per step"),
    }


def run_batch(args):
    """The ragged batch: 512 independent 2D Poisson instances (J~U{4..24}^2, K~U{64..128},
    20..60 points per subdomain cell), 8 right-hand sides each, every kernel one launch over the
    batch.  A step is assembly, block-Jacobi factors and the solve of every (instance, rhs) pair
    until ||h - M c|| <= btol ||h|| (istop 1), least-squares optimality ||M^T r|| <= btol ||M|| ||r||
    (istop 2; pairs whose features cannot represent the solution) or the iteration budget."""
    import numpy as np
    import torch

    from inputs import configs, feature_params
    from paper_2409_01949_amd import Batch

    specs, _ = configs.batch_instances(n=args.batch_n, seed=3, n_rhs=8)
    feats = [feature_params(s) for s in specs]
    mixed = args.method == "mixed_ir"
    store = args.store if mixed else "fp64"
    t0 = time.perf_counter()
    B = Batch(specs, [w for w, _ in feats], [b for _, b in feats], 8, store_prec=store)
    t_define = time.perf_counter() - t0
    print(f"# batch defined in {t_define:.1f} s: {B.sizes}", file=sys.stderr, flush=True)
    f = np.concatenate([configs.batch_forcing(s).ravel() for s in specs])
    fd = torch.as_tensor(f).cuda()
    coef = torch.empty(8 * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
    btol = args.batch_btol
    precond = not args.no_precond
    B.assemble(fd)
    tune = {p: B.autotune(p, reps=3) for p in sorted({"fp64", store})}
    print(f"# autotuned A^T U tiles: {tune}", file=sys.stderr, flush=True)

    def step():
        ta = time.perf_counter()
        B.assemble(fd)
        if precond:
            B.precondition(args.shift)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        if mixed:
            inf = B.solve(coef, method="mixed_ir", inner_iters=args.inner,
                          outer_lim=max(1, args.iters // args.inner), atol=btol, btol=btol,
                          check_every=args.check_every, precond=precond)
        else:
            inf = B.solve(coef, iter_lim=args.iters, atol=btol, btol=btol,
                          check_every=args.check_every, precond=precond)
        torch.cuda.synchronize()
        return inf, tb - ta, time.perf_counter() - tb

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(args.steps):
        infos, t_setup, t_solve = step()
        print(f"# step {k}: assemble+factors {t_setup * 1e3:.1f} ms, solve {t_solve:.2f} s",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t1) / args.steps
    its = np.array([i["iters"] for i in infos])
    stops = np.array([i["istop"] for i in infos])
    # ||h|| per pair from the forcing (h = f / sqrt(N_i)); relative residuals of the solve
    hn = np.concatenate([np.linalg.norm(configs.batch_forcing(s), axis=1) / np.sqrt(s.n_rows)
                         for s in specs])
    rel = np.array([i["rnorm"] for i in infos]) / hn
    rows_rhs = B.sizes["n_rows"] * 8
    nnz = B.sizes["nnz"]
    method = (f"batched {'bj-' if precond else ''}"
              + (f"mixed-ir ({store} inner)" if mixed else "lsqr-fp64"))
    out = {
        "metric": METRIC, "value": rows_rhs / dt, "unit": "rows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": f"f64+{store}" if mixed else "f64", "data": "synthetic",
        "config": {"workload": f"batch{args.batch_n}x8", "instances": args.batch_n, "n_rhs": 8,
                   "rows": B.sizes["n_rows"], "cols": B.sizes["n_phi"], "nnz": nnz,
                   "method": method, "btol": btol, "iter_budget": args.iters,
                   "inner": args.inner if mixed else None, "shift": args.shift if precond else None},
        "define_s": t_define, "setup_ms": t_setup * 1e3, "solve_s": t_solve,
        "autotune_ms": {p: v[0] for p, v in tune.items()},
        "tiles": {p: v[1] for p, v in tune.items()},
        "pairs_converged": int(np.sum(stops == 1)), "pairs": int(len(stops)),
        "pairs_ls_optimal": int(np.sum(stops == 2)), "pairs_budget": int(np.sum(stops == 7)),
        "iters_max": int(its.max()), "iters_median": float(np.median(its)),
        "rel_residual_quantiles": {q: float(np.quantile(rel, float(q)))
                                   for q in ("0.5", "0.9", "0.99", "1.0")},
        "ms_per_iteration": t_solve * 1e3 / max(1, int(its.max())),
    }
    B.destroy()
    print(json.dumps(out), flush=True)


def run_warm(args):
    """Learned warm start on the 1D parameterised family (omega ~ U[5,50], c ~ N(0,1)^3, J=64,
    K=32, 6000 points): 4,096 training solves (512 omega x 8 c) by the batched solver, the MLP
    (3 x 512 tanh, BF16 products) trained on them, then the 1,024 held-out pairs (128 x 8) solved
    to ||h - M c|| <= btol ||h|| from its prediction.  A step is prediction + warm solve; the cold
    solve of the same batch is reported beside it."""
    import numpy as np
    import torch

    from inputs import configs
    from paper_2409_01949_amd import warmstart as ws

    def log(m):
        print("# " + m, file=sys.stderr, flush=True)

    om, C = configs.warm_groups(512, 5)
    B, specs, _ = ws.family_batch(om, C)
    coef, infos, t_data = ws.solve_batch(B, btol=args.batch_btol * 0.1, inner=2000, outer=6)
    X, F = ws.family_inputs(specs, om, C)
    Y = ws.coef_blocks(coef, specs, C.shape[1])
    B.destroy()
    log(f"training data: {len(X)} samples from {len(infos)} solves in {t_data:.1f} s")
    W = ws.WarmStart(n_in=X.shape[1], K=Y.shape[1], max_batch=4096, seed=0)
    t0 = time.perf_counter()
    hist = W.fit(X, F, Y, epochs=args.epochs, lr=1e-3, seed=0, log=log)
    t_train = time.perf_counter() - t0
    om2, C2 = configs.warm_groups(128, 6)
    B2, specs2, hn2 = ws.family_batch(om2, C2)
    X2, F2 = ws.family_inputs(specs2, om2, C2)
    btol = args.batch_btol
    # a pair is solved at ||r|| <= btol ||h|| or, for the pairs whose optimal residual lies above
    # that, at least-squares optimality with atol = btol
    _, cold, t_cold = ws.solve_batch(B2, btol=btol, inner=2000, outer=10, atol=btol)

    def step():
        torch.cuda.synchronize()
        ta = time.perf_counter()
        x0 = torch.as_tensor(np.ascontiguousarray(W.predict(X2, F2)).reshape(-1)).cuda()
        _, warm, _ = ws.solve_batch(B2, x0=x0, btol=btol, inner=2000, outer=10,
                                    precondition=False, atol=btol)
        torch.cuda.synchronize()
        return warm, time.perf_counter() - ta

    for _ in range(args.warmup):
        step()
    ts = []
    for _ in range(args.steps):
        warm, dt = step()
        ts.append(dt)
    dt = float(np.mean(ts))
    itc = np.array([i["iters"] for i in cold])
    itw = np.array([i["iters"] for i in warm])
    rows_rhs = B2.sizes["n_rows"] * C2.shape[1]
    out = {
        "metric": METRIC, "value": rows_rhs / dt, "unit": "rows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+fp32",
        "data": "synthetic",
        "config": {"workload": "warm1d_128x8", "instances": 128, "n_rhs": 8,
                   "train_solves": len(infos), "rows": B2.sizes["n_rows"],
                   "cols": B2.sizes["n_phi"], "method": "bj-mixed-ir (fp32 inner), MLP x0",
                   "btol": btol, "epochs": args.epochs,
                   "mlp": "65-512-512-512-192 tanh, bf16, output modulated by 6 weights"},
        "warm_s": dt, "cold_s": t_cold, "speedup_vs_cold": t_cold / dt,
        "iters_mean": {"cold": float(itc.mean()), "warm": float(itw.mean())},
        "iters_max": {"cold": int(itc.max()), "warm": int(itw.max())},
        "converged": {"cold": int(sum(i["istop"] == 1 for i in cold)),
                      "warm": int(sum(i["istop"] == 1 for i in warm)), "pairs": len(cold)},
        "ls_optimal": {"cold": int(sum(i["istop"] == 2 for i in cold)),
                       "warm": int(sum(i["istop"] == 2 for i in warm))},
        "training": {"data_s": t_data, "train_s": t_train, "loss_first": hist[0],
                     "loss_last": hist[-1]},
    }
    B2.destroy()
    W.destroy()
    print(json.dumps(out), flush=True)


def krylov_sigma(P):
    """Extreme singular values of the bidiagonal the last solve's LSQR built (a lower bound on
    the condition number of the operator it ran on), or None."""
    try:
        smax, smin, k = P.condition_estimate()
    except Exception:
        return None
    return {"sigma_max": smax, "sigma_min": smin, "kappa_lower_bound": smax / smin, "steps": k}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter summary
    (profiles/<kernel>_<workload>_traffic.json: FETCH_SIZE + WRITE_SIZE per dispatch, scaled by
    the same counters on a plain copy of known size), or None when there is none or the kernel's
    sources changed since the counters were taken (the SHA-256 of the listed source files, read
    in order and concatenated, is recorded there)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
        h = hashlib.sha256()
        for src in d.get("sources", [d.get("source")]):
            with open(os.path.join(ROOT, src), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != d["source_sha256"]:
            return None
        return float(d["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def run_copy(args):
    """Plain device-to-device copies of a known size (the reference for scaling the HBM traffic
    counters of the other kernels): prints bytes read and written per copy."""
    import torch

    n = args.copy_bytes // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8,
                      "copies": args.steps}), flush=True)


def _one_wg_us_per_step(P, coef, n_it, reps):
    """Microseconds per LSQR step of the one-workgroup solve on P: n_it steps in one launch, less
    a solve of no steps (the set-up kernels), HIP events on the stream the solve runs on."""
    import torch
    stream = torch.cuda.current_stream()

    def timed(k):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        P.solve(coef, method="lsqr", iter_lim=k, atol=0.0, btol=0.0, check_every=max(k, 1))
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1)

    timed(n_it)
    ms = min(timed(n_it) for _ in range(reps)) - min(timed(0) for _ in range(reps))
    return ms, ms * 1e3 / max(n_it, 1)


def run_oscillator(args):
    """The damped oscillator of Sec. 4.2 (eq. harm_oscillator) at the paper's baseline
    (omega0 = 80, one level of 20 subdomains, K = 12, delta = 2.9, 260 collocation points, soft
    initial conditions with lambda_u0 = omega0^4 and lambda_v0 = omega0^2), solved as the paper
    does (Sec. 4.1): FP64 LSQR for its whole budget of 15,000 iterations (atol = btol = 0, no
    early stop).  A step is assembly (operator rows and the two constraint rows) and that solve;
    the error is e_L1 against the exact solution on 1,000 test points."""
    import numpy as np
    import torch

    from inputs import configs, feature_params
    from paper_2409_01949_amd import Problem

    budget = 15000
    spec = configs.oscillator()
    W, b = feature_params(spec)
    f = configs.forcing(spec)
    P = Problem.from_spec(spec, W, b, "fp64")
    fd = torch.as_tensor(f).cuda()
    n = P.sizes["n_phi"]
    rows = P.sizes["n_rows"] + P.sizes["n_bc"]
    coef = torch.empty(n, dtype=torch.float64, device="cuda")
    xt = np.linspace(0.0, 1.0, 1000)[:, None]
    ue = configs.exact(spec, xt)
    xt_d = torch.as_tensor(xt).cuda()
    u_d = torch.empty(1000, dtype=torch.float64, device="cuda")

    def step():
        P.assemble(fd)
        return P.solve(coef, method="lsqr", iter_lim=budget, atol=0.0, btol=0.0,
                       check_every=budget)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    info = infos[-1]
    P.evaluate(coef, xt_d, u_d)
    u = u_d.cpu().numpy()
    rel = float(np.linalg.norm(u - ue) / np.linalg.norm(ue))
    e_l1 = float(np.mean(np.abs(u - ue)) / np.std(ue))
    sigma = krylov_sigma(P)
    # The dominant kernel is the one-workgroup LSQR: the system (8,880 entries) sits in one CU's
    # LDS, so a step is bound by its barriers, reductions and dependent LDS reads, not by HBM.
    # Its yardstick is the fixed cost of a step: the same kernel on the smallest system (the
    # 3-subdomain 1D problem, 200 block points) measured alongside.
    k = info["iters"]
    reps = max(2, args.kernel_reps // 10)
    ms_launch, us_step = _one_wg_us_per_step(P, coef, k, reps)
    tiny = configs.tiny1d()
    Wt, bt = feature_params(tiny)
    Pt = Problem.from_spec(tiny, Wt, bt, "fp64")
    Pt.assemble(torch.as_tensor(configs.forcing(tiny)).cuda())
    ct = torch.empty(Pt.sizes["n_phi"], dtype=torch.float64, device="cuda")
    _, us_floor = _one_wg_us_per_step(Pt, ct, 2000, reps)
    Pt.destroy()
    out = {
        "metric": METRIC,
        "value": rows / dt, "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "oscillator80", "omega0": 80.0, "J": 20, "K": spec.K,
                   "delta": spec.delta, "collocation_points": spec.n_rows,
                   "constraint_rows": P.sizes["n_bc"], "method": "lsqr fp64",
                   "atol": 0.0, "btol": 0.0, "iter_budget": budget},
        "time_to_solution_s": dt, "iters": info["iters"], "istop": info["istop"],
        "rel_l2_test_vs_exact": rel, "e_l1_test": e_l1, "krylov_sigma": sigma,
        "roofline": {"bound": "latency", "achieved": us_step, "peak": us_floor,
                     "unit": "us/step", "frac": us_floor / us_step, "traffic": None,
                     "kernel": f"k_lsqr_persistent ({k} LSQR steps in one workgroup, the "
                               f"system's {P.sizes['nnz']} entries in LDS)",
                     "peak_meaning": "fixed cost of one step: the same kernel on the 200-point "
                                     "3-subdomain 1D system",
                     "ms_per_launch": ms_launch},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = oscillator_cpu_baseline(spec, W, b, f, xt, ue, budget, rows)
    P.destroy()
    print(json.dumps(out), flush=True)


def oscillator_cpu_baseline(spec, W, b, f, xt, ue, budget, rows):
    """The oracle's whole step (assembly of [N; B] and LSQR for the same budget) timed on the
    host, 1 warm-up and 3 repeats; the e_L1 of its solution and of the dense QR solution of the
    same system (what the features can reach) are reported beside it, untimed."""
    import numpy as np
    from oracle import assemble as asm
    from oracle import evaluate as ev_o
    from oracle import linalg

    n = len(W)

    def oracle_step():
        blocks = asm.assemble_blocks(spec, W, b)
        M = np.vstack([asm.dense_from_blocks(blocks, spec.n_rows, n), asm.bc_rows(spec, W, b)])
        h = asm.rhs(spec, f)
        return M, h, linalg.lsqr(lambda v: M @ v, lambda r: M.T @ r, h, n, atol=0.0, btol=0.0,
                                 iter_lim=budget)

    oracle_step()
    ts = []
    for _ in range(3):
        t1 = time.perf_counter()
        M, h, ref = oracle_step()
        ts.append(time.perf_counter() - t1)
    e_l1 = lambda c: float(np.mean(np.abs(ev_o.evaluate(spec, W, b, c, xt) - ue)) / np.std(ue))
    xq = linalg.householder_lstsq(M, h)
    t_med = float(np.median(ts))
    return {"value": rows / t_med, "unit": "rows/s", "cores": _threads(), "kind": "oracle",
            "sample": (f"the whole step: assembly and {ref.itn} LSQR iterations (istop "
                       f"{ref.istop}), median of 3 repeats after 1 warm-up "
                       f"{t_med:.2f} s (min {min(ts):.2f}, max {max(ts):.2f})"),
            "oracle_e_l1_test": e_l1(ref.x), "dense_qr_e_l1_test": e_l1(xq)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU build: run with --gpus 1 (the multi-GPU "
                                   "sharding is a design only)"}))
        sys.exit(2)
    if args.copy_bytes:
        run_copy(args)
        return
    if args.workload.startswith("batch"):
        run_batch(args)
        return
    if args.workload == "warm":
        run_warm(args)
        return
    if args.workload == "oscillator":
        run_oscillator(args)
        return
    import numpy as np
    import torch

    from inputs import configs, feature_params
    from inputs.problems import grid_points
    from paper_2409_01949_amd import Problem

    spec = getattr(configs, args.workload)()
    W, b = feature_params(spec)
    f = configs.forcing(spec)
    precond = not args.no_precond
    P = Problem.from_spec(spec, W, b, args.store)
    fd = torch.as_tensor(f).cuda()
    xc = torch.as_tensor(grid_points(spec, spec.meta["n_check"])).cuda()
    uc_np = configs.exact(spec, grid_points(spec, spec.meta["n_check"]))
    uc = torch.as_tensor(uc_np).cuda()
    xt_np = grid_points(spec, spec.meta["n_test"])
    xt = torch.as_tensor(xt_np).cuda()
    ut_np = configs.exact(spec, xt_np)
    n = P.sizes["n_phi"]
    coef = torch.empty(n, dtype=torch.float64, device="cuda")
    u_test = torch.empty(xt.shape[0], dtype=torch.float64, device="cuda")

    gram_method = args.method in ("normal_cg", "mixed_ir_cg")

    def step(method=args.method, pre=precond, iters=args.iters):
        P.assemble(fd)
        if pre:
            P.precondition(args.shift)
        if method in ("normal_cg", "mixed_ir_cg"):
            P.gram(args.gram_prec, "all")
        if method in ("mixed_ir", "mixed_ir_cg"):
            info = P.solve(coef, method=method, inner_iters=args.inner,
                           outer_lim=max(1, iters // args.inner), atol=0.0, btol=0.0,
                           check_every=min(args.check_every, args.inner), check_pts=xc,
                           check_ref=uc, target_rel_l2=args.target, precond=pre)
        else:
            info = P.solve(coef, method=method, iter_lim=iters, atol=0.0, btol=0.0,
                           check_every=args.check_every, check_pts=xc, check_ref=uc,
                           target_rel_l2=args.target, precond=pre)
        P.evaluate(coef, xt, u_test)
        return info

    def note(msg):
        print("# " + msg, file=sys.stderr, flush=True)

    for w in range(args.warmup):
        wi = step()
        note(f"warmup step {w}: {wi['iters']} iterations")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(args.steps):
        infos.append(step())
        note(f"step {k}: {infos[-1]['iters']} iterations, rel-L2 {infos[-1]['rel_l2']:.3e}")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    info = infos[-1]
    # the operator of the timed solve's last LSQR run (for the refinement: its last inner solve)
    main_sigma = krylov_sigma(P)
    u = u_test.cpu().numpy()
    e_l1 = float(np.mean(np.abs(u - ut_np)) / np.std(ut_np))
    rel_test = float(np.linalg.norm(u - ut_np) / np.linalg.norm(ut_np))

    # roofline of the dominant kernel: the per-chunk pass of x = M^T u over the matrix copy the
    # inner iterations stream (the low-precision copy for the mixed path)
    kprec = args.store if args.method == "mixed_ir" else "fp64"
    es = {"fp64": 8, "fp32": 4, "bf16": 2, "fp16": 2}[kprec]
    ms_mv, ms_rmv = P.time_kernels(args.kernel_reps, prec=kprec)
    ms_mv64, ms_rmv64 = P.time_kernels(args.kernel_reps, prec="fp64")
    nnz, nbp = P.sizes["nnz"], P.sizes["n_block_points"]
    n_chunks = sum(-(-int(v) // 2048) for v in [r[4] * r[6] for r in P.copy_blocks()])
    rmv_bytes = lambda e: nnz * e + nbp * 8 + n_chunks * spec.K * 8
    mv_bytes = lambda e: nnz * e + nbp * 8
    achieved = rmv_bytes(es) / (ms_rmv * 1e-3) / 1e9
    kname = {"fp64": "FP64", "fp32": "FP32", "bf16": "BF16", "fp16": "FP16"}[kprec]
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic(f"k_rmv_chunks_{kprec}", spec.name),
                "kernel": f"k_rmv_chunks<{kname}> (x = M^T u, per-chunk pass)",
                "ms_per_launch": ms_rmv, "algorithmic_bytes_per_launch": rmv_bytes(es),
                "also": [
                    {"kernel": f"k_mv_blocks<{kname}> (y = M v, per-block-point pass)",
                     "ms_per_launch": ms_mv,
                     "achieved_GBs": mv_bytes(es) / (ms_mv * 1e-3) / 1e9},
                    {"kernel": "k_rmv_chunks<FP64>", "ms_per_launch": ms_rmv64,
                     "achieved_GBs": rmv_bytes(8) / (ms_rmv64 * 1e-3) / 1e9},
                    {"kernel": "k_mv_blocks<FP64>", "ms_per_launch": ms_mv64,
                     "achieved_GBs": mv_bytes(8) / (ms_mv64 * 1e-3) / 1e9}]}
    if gram_method:
        # CG on the Gram blocks: the per-block pass of y = G p reads every stored block once
        # and writes two K-vectors of partials per block
        ms_pairs, ms_gmv = P.time_gram_mv(args.kernel_reps)
        n_pairs = P.sizes["n_pairs"]
        esg = 8 if args.gram_prec == "fp64" else 4
        g_bytes = n_pairs * spec.K * spec.K * esg + 2 * n_pairs * spec.K * 8
        gname = "FP64" if esg == 8 else "FP32"
        lsqr_roof = roofline
        roofline = {"bound": "hbm", "achieved": g_bytes / (ms_pairs * 1e-3) / 1e9,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": g_bytes / (ms_pairs * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                    "kernel": f"k_gmv_pairs<{gname}> (y = G p, per stored Gram block)",
                    "ms_per_launch": ms_pairs, "algorithmic_bytes_per_launch": g_bytes,
                    "also": [{"kernel": "G p, both passes", "ms_per_launch": ms_gmv}] +
                            [{"kernel": lsqr_roof["kernel"], "ms_per_launch": ms_rmv,
                              "achieved_GBs": achieved}] + lsqr_roof["also"]}

    # the Gram phase on the matrix cores: all overlapping pairs, FP64 and the stored copy's type
    gram_mfma = []
    if not args.no_gram:
        for gp in ["fp64"] + ([args.store] if args.store in ("fp32", "bf16", "fp16") else []):
            ms_g, fl = P.time_gram(gp, "all", reps=3)
            tf = fl / (ms_g * 1e-3) / 1e12
            # a pair's 2 K^2 S flops read both blocks' S shared rows (2 K S entries): K / es flop
            # per input byte, so the pass is bound by the matrix cores (FP64) or by reading its
            # inputs (16-bit entries) when no row is shared between pairs in cache
            es = {"fp64": 8, "fp32": 4, "bf16": 2, "fp16": 2}[gp]
            in_bytes = fl * es / spec.K
            bw_tf = fl / (in_bytes / (HBM_PEAK_GBS * 1e9)) / 1e12
            ceiling = min(MFMA_PEAK_TFLOPS[gp], bw_tf)
            gram_mfma.append({"kernel": f"k_gram<{gp.upper()}> (+ chunk reduction), "
                                        f"{P.sizes['n_pairs']} pairs", "ms": ms_g, "flops": fl,
                              "achieved_tflops": tf, "peak_tflops": MFMA_PEAK_TFLOPS[gp],
                              "frac": tf / MFMA_PEAK_TFLOPS[gp], "input_bytes": in_bytes,
                              "bound": "mfma" if MFMA_PEAK_TFLOPS[gp] <= bw_tf else "hbm",
                              "ceiling_tflops": ceiling, "frac_of_ceiling": tf / ceiling})
            note(f"gram {gp}: {ms_g:.2f} ms, {tf:.1f} TFLOP/s")

    compare = {}
    if not args.no_compare:
        for label, meth, pre in (("fp64_block_jacobi_lsqr", "lsqr", True),
                                 ("fp64_plain_lsqr", "lsqr", False)):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ci = step(meth, pre, args.compare_iters)
            torch.cuda.synchronize()
            compare[label] = {"time_to_solution_s": time.perf_counter() - t1,
                              "reached_target": bool(ci["istop"] == 8), "iters": ci["iters"],
                              "iter_budget": args.compare_iters,
                              "rel_l2_check_at_stop": ci["rel_l2"],
                              "krylov_sigma": krylov_sigma(P)}
            note(f"{label}: {compare[label]['time_to_solution_s']:.2f} s, {ci['iters']} iterations")
        compare["speedup_vs_fp64_block_jacobi"] = \
            compare["fp64_block_jacobi_lsqr"]["time_to_solution_s"] / dt
        compare["speedup_vs_fp64_plain_lsqr"] = compare["fp64_plain_lsqr"]["time_to_solution_s"] / dt

    out = {
        "metric": METRIC,
        "value": spec.n_rows / dt,
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": (f"f64+{args.store}" if args.method == "mixed_ir" else
                  f"f64+{args.gram_prec}" if gram_method else "f64"),
        "data": "synthetic",
        "config": {"workload": spec.name, "rows": spec.n_rows, "cols": n, "nnz": nnz,
                   "levels": [list(J) for J in spec.levels], "K": spec.K,
                   "grid": list(spec.n_points),
                   "method": (f"{args.method}" + ("+block-jacobi" if precond else "") +
                              (f" (inner {args.store} x{args.inner})" if args.method == "mixed_ir"
                               else f" (gram {args.gram_prec}" +
                               (f", inner x{args.inner})" if args.method == "mixed_ir_cg" else ")")
                               if gram_method else "-fp64")),
                   "iter_budget": args.iters, "target_rel_l2": args.target,
                   "reference": "exact solution on the 128x128 check grid"},
        "time_to_solution_s": dt,
        "reached_target": bool(info["istop"] == 8),
        "iters": info["iters"],
        "outer_iters": info["outer_iters"],
        "rel_l2_check_at_stop": info["rel_l2"],
        "rel_l2_test_vs_exact": rel_test,
        "e_l1_test": e_l1,
        "roofline": roofline,
        "gram_mfma": gram_mfma,
        "krylov_sigma": main_sigma,
        "compare": compare,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, W, b, f, info["iters"])
    P.destroy()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
