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
    p.add_argument("--ref-iters", type=int, default=15000,
                   help="iteration budget of the FP64 reference solution (atol = btol = 1e-10)")
    p.add_argument("--secondary", default="ode1d,helmholtz,batch,poisson5l",
                   help="workloads measured after the headline in the default run, each with a "
                        "fixed budget (empty: none)")
    p.add_argument("--secondary-deadline", type=float, default=300.0,
                   help="seconds after which the remaining secondary workloads are skipped")
    p.add_argument("--secondary-ref-iters", type=int, default=1000,
                   help="iteration budget of the FP64 reference solution of a secondary "
                        "multilevel workload")
    p.add_argument("--secondary-iters", type=int, default=3000,
                   help="inner-iteration budget of the secondary multilevel and batched steps")
    p.add_argument("--batch-n", type=int, default=512)
    p.add_argument("--batch-patch", type=int, default=2,
                   help="batched workload: block-Jacobi over patches of P x P neighbouring "
                        "subdomains (1: per subdomain)")
    p.add_argument("--batch-btol", type=float, default=None,
                   help="batched workloads: residual tolerance (default 1e-6 for batch, 1e-4 "
                        "for warm, 1e-3 for warm2d)")
    p.add_argument("--epochs", type=int, default=None,
                   help="warm workloads: MLP training epochs (default 100 for warm, 300 for warm2d)")
    p.add_argument("--warm-inner", type=int, default=None,
                   help="warm workloads: inner LSQR steps per refinement step")
    p.add_argument("--warm-outer", type=int, default=None,
                   help="warm workloads: refinement steps")
    p.add_argument("--warm-train-groups", type=int, default=512,
                   help="warm workloads: training omegas (8 coefficient vectors each)")
    p.add_argument("--warm-test-groups", type=int, default=128,
                   help="warm workloads: held-out omegas (8 coefficient vectors each)")
    p.add_argument("--copy-bytes", type=int, default=0,
                   help="only run device copies of this many bytes (traffic-counter reference)")
    p.add_argument("--write-traffic", default=None, metavar="NAME",
                   help="host only: write profiles/traffic_NAME.json from rocprofv3 counter runs "
                        "(--pmc-fetch/--pmc-write of the workload, --copy-fetch/--copy-write of "
                        "`--copy-bytes 1073741824` copies) for --traffic-kernels, hashing "
                        "--traffic-sources")
    p.add_argument("--pmc-fetch", default=None)
    p.add_argument("--pmc-write", default=None)
    p.add_argument("--copy-fetch", default=None)
    p.add_argument("--copy-write", default=None)
    p.add_argument("--copy-ref-bytes", type=int, default=1 << 30)
    p.add_argument("--traffic-kernels", default="",
                   help="';'-separated kernel names as bench.py reports them, e.g. k_bt_mvb<FP32,16>")
    p.add_argument("--traffic-sources", default="",
                   help="','-separated source files (from the repository root) of those kernels")
    p.add_argument("--traffic-out", default=None,
                   help="where --write-traffic writes (default profiles/traffic_NAME.json)")
    args = p.parse_args()
    args.store_given, args.inner_given = args.store, args.inner
    args.batch_btol_given = args.batch_btol
    if args.batch_btol is None:
        args.batch_btol = 1e-6
    return _defaults(args)


def _defaults(args):
    """Per-workload defaults of the stored copy and the inner step count."""
    gram_method = args.method in ("normal_cg", "mixed_ir_cg")
    if args.gram_prec is None:
        args.gram_prec = "fp32" if args.method == "mixed_ir_cg" else "fp64"
    args.store, args.inner = args.store_given, args.inner_given
    if args.store is None:
        if gram_method:
            args.store = "fp32" if args.gram_prec == "fp32" else "fp64"
        else:
            args.store = "fp16" if args.workload in ("poisson3l", "poisson5l") else "fp32"
    if args.inner is None:
        args.inner = 500 if args.store in ("fp16", "bf16") else 2500
    return args


def _args_for(args, workload):
    import copy
    a = copy.copy(args)
    a.workload = workload
    return _defaults(a)


def _threads():
    """Threads the oracle's BLAS actually runs with (threadpoolctl's view of the loaded BLAS)."""
    from threadpoolctl import threadpool_info
    n = [int(i["num_threads"]) for i in threadpool_info() if i.get("user_api") == "blas"]
    return max(n) if n else 1


def _oracle_sample(spec, W, b, max_per_level=4, seed=0):
    """A fixed sample of subdomain blocks for timing the oracle: up to `max_per_level` blocks of
    every level, chosen by a seeded draw (so every level's block sizes are represented)."""
    import numpy as np
    from oracle import geometry as geo

    subs = geo.subdomains(spec)
    rng = np.random.default_rng(seed)
    picked = []
    for l in range(len(spec.levels)):
        lev = [sd for sd in subs if sd.level == l]
        idx = rng.choice(len(lev), size=min(max_per_level, len(lev)), replace=False)
        picked += [lev[i] for i in sorted(idx)]
    return subs, picked


def _oracle_fixed(spec, subs, picked, max_rows):
    """The oracle's per-level work that does not grow with the stored entries: the ansatz factor
    and the window sums of every level (each subdomain's window at each grid point), evaluated at
    the rows the sampled blocks use and scaled by point count to the whole grid (the work is the
    same per point).  Returns (seconds for the whole grid, points, ansatz, sums) with the
    ansatz and sums filled in at the sampled rows."""
    import numpy as np
    from oracle import basis
    from oracle import geometry as geo

    x = geo.points(spec)
    rows = np.unique(np.concatenate([np.nonzero(geo.in_support(x, sd))[0][:max_rows]
                                     for sd in picked]))
    xs = x[rows]
    t0 = time.perf_counter()
    ans_s = basis.ansatz(xs, spec)
    sums_s = {l: basis.level_sum(xs, [s for s in subs if s.level == l])
              for l in range(len(spec.levels))}
    t = (time.perf_counter() - t0) * x.shape[0] / rows.size

    def full(parts):
        out = []
        for a in parts:
            z = np.zeros((x.shape[0],) + a.shape[1:])
            z[rows] = a
            out.append(z)
        return tuple(out)

    return t, x, full(ans_s), {l: full(v) for l, v in sums_s.items()}


def _oracle_sample_step(spec, W, b, f, subs, picked, n_lsqr, max_rows, x, ans, sums):
    """The oracle on the sampled blocks, each cut to its first max_rows rows: their entries
    (features, windows from the level sums, operator rows), then n_lsqr LSQR iterations with the
    oracle's block products restricted to them, and the same products timed alone.  Returns
    (seconds of entries, seconds per LSQR iteration, seconds per product pair, entries)."""
    import numpy as np
    from oracle import assemble as asm
    from oracle import basis
    from oracle import geometry as geo
    from oracle import linalg

    N = x.shape[0]
    L = len(spec.levels)
    scale = 1.0 / (np.sqrt(float(N)) * L)
    t0 = time.perf_counter()
    blocks = []
    ent = 0
    for sd in picked:
        l = sd.level
        rows = np.nonzero(geo.in_support(x, sd))[0][:max_rows]
        q = slice(sd.q0, sd.q0 + spec.K)
        val, grad, lap = basis.localized_function(x[rows], spec, sd, W[q], b[q],
                                                  tuple(s[rows] for s in sums[l]),
                                                  tuple(a[rows] for a in ans))
        blocks.append(asm.Block(sd, rows, basis.apply_operator(spec, val, grad, lap) * scale))
        ent += rows.size * spec.K
    t_ent = time.perf_counter() - t0
    n = len(subs) * spec.K
    h = asm.rhs(spec, f)
    mv = lambda v: asm.matvec(blocks, v, N)
    rmv = lambda u: asm.rmatvec(blocks, u, n)
    t1 = time.perf_counter()
    linalg.lsqr(mv, rmv, h, n, atol=0, btol=0, iter_lim=n_lsqr)
    t_it = (time.perf_counter() - t1) / n_lsqr
    v, u = np.ones(n), np.ones(N)
    t2 = time.perf_counter()
    for _ in range(n_lsqr):
        mv(v)
        rmv(u)
    t_prod = (time.perf_counter() - t2) / n_lsqr
    return t_ent, t_it, t_prod, ent


def cpu_baseline(spec, W, b, f, n_iters_solve, total_nnz, rows_per_step=None, max_per_level=2,
                 n_lsqr=20, repeats=3, repeats_1t=2, max_rows=8192):
    """The oracle (NumPy/SciPy FP64, untuned) on the host, on a bounded sample of the same
    workload, scaled to the full step:
      * the per-level work that does not grow with the entries (ansatz, the window sums of every
        level at every point) is timed once in full;
      * the entries of a fixed sample of subdomain blocks of every level (each cut to its first
        max_rows rows) and the oracle's block products on them are scaled by entry count;
      * an LSQR iteration costs its vector work (timed on the full-length vectors: the LSQR
        iteration on the sample less its products) plus the scaled products.
    Protocol: 1 warm-up, then `repeats` timed repeats of the sampled part with the BLAS on all
    the threads it uses, and 1 warm-up + `repeats_1t` repeats at 1 thread; value = collocation
    rows per second of the scaled step (median of the repeats at all threads)."""
    import numpy as np
    from oracle import geometry as geo
    from threadpoolctl import threadpool_limits

    subs, picked = _oracle_sample(spec, W, b, max_per_level)
    t_fixed, x, ans, sums = _oracle_fixed(spec, subs, picked, max_rows)
    rows = rows_per_step or spec.n_rows

    def series(k):
        out = []
        for i in range(k + 1):
            t_ent, t_it, t_prod, ent = _oracle_sample_step(spec, W, b, f, subs, picked, n_lsqr,
                                                           max_rows, x, ans, sums)
            sc = total_nnz / ent
            if i > 0:
                out.append(t_fixed + t_ent * sc +
                           n_iters_solve * (max(t_it - t_prod, 0.0) + t_prod * sc))
        return out, ent

    full, ent = series(repeats)
    threads = _threads()
    with threadpool_limits(limits=1, user_api="blas"):
        one, _ = series(repeats_1t)
    stat = lambda v: {"median_s": float(np.median(v)), "min_s": float(min(v)),
                      "max_s": float(max(v)), "repeats": len(v)}
    t_full = float(np.median(full))
    return {
        "value": rows / t_full,
        "unit": "rows/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"the oracle's per-level window sums and ansatz at the sampled rows, timed "
                   f"once and scaled by point count to the grid ({t_fixed:.1f} s); the entries of {len(picked)} of {len(subs)} subdomain blocks "
                   f"(up to {max_per_level} per level, each cut to its first {max_rows} rows: "
                   f"{ent} of {total_nnz} entries) and {n_lsqr} LSQR iterations with the "
                   f"oracle's block products on them, scaled by entry count (products) to the "
                   f"full assembly plus the step's {n_iters_solve} iterations. 1 warm-up + "
                   f"{repeats} repeats with BLAS on {threads} threads (element-wise NumPy work "
                   f"runs on one), 1 warm-up + {repeats_1t} at 1 thread; value from the median "
                   f"at {threads} threads: {t_full:.1f} s per step"),
        "runs": {f"{threads}_threads": stat(full), "1_thread": stat(one)},
        "value_1_thread": rows / float(np.median(one)),
    }


def run_batch(args, steps=None, warmup=None, iters=None):
    """The ragged batch: 512 independent 2D Poisson instances (J~U{4..24}^2, K~U{64..128},
    20..60 points per subdomain cell), 8 right-hand sides each, every kernel one launch over the
    batch.  A step is assembly, block-Jacobi factors (per subdomain, or over patches of
    --batch-patch^2 neighbouring subdomains) and the solve of every (instance, rhs) pair until
    ||h - M c|| <= btol ||h|| (istop 1), for the refinement also least-squares optimality
    ||M^T r|| <= btol ||M|| ||r|| (istop 2; pairs whose features cannot represent the solution),
    or the iteration budget."""
    import numpy as np
    import torch

    from inputs import configs, feature_params
    from paper_2409_01949_amd import Batch

    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    iters = args.iters if iters is None else iters
    specs, _ = configs.batch_instances(n=args.batch_n, seed=3, n_rhs=8)
    feats = [feature_params(s) for s in specs]
    mixed = args.method == "mixed_ir"
    store = args.store if mixed else "fp64"
    # one inner solve over the whole budget unless --inner is given: every refinement step
    # restarts LSQR, and fewer restarts reach the target on more pairs (6,000 iterations:
    # 1,820 pairs with 4 x 1,500, 1,925 with 2 x 3,000, 1,957 with 1 x 6,000)
    inner = min(args.inner, iters) if args.inner_given else iters
    t0 = time.perf_counter()
    B = Batch(specs, [w for w, _ in feats], [b for _, b in feats], 8, store_prec=store)
    t_define = time.perf_counter() - t0
    print(f"# batch defined in {t_define:.1f} s: {B.sizes}", file=sys.stderr, flush=True)
    f = np.concatenate([configs.batch_forcing(s).ravel() for s in specs])
    fd = torch.as_tensor(f).cuda()
    coef = torch.empty(8 * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
    btol = args.batch_btol
    precond = not args.no_precond
    patch = args.batch_patch if precond else 1
    B.assemble(fd)
    if precond:
        # the passes run on the folded matrix (in the patch layout for patches): tune on it
        B.precondition(args.shift, patch=patch)
    # launch shapes of the three matrix passes, timed per precision (or from the process's cache)
    tune = {p: B.tune(p, reps=3) for p in sorted({"fp64", store})}
    print(f"# tuned shapes: {tune}", file=sys.stderr, flush=True)

    def step(budget):
        ta = time.perf_counter()
        B.assemble(fd)
        if precond:
            B.precondition(args.shift, patch=patch)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        if mixed:
            inf = B.solve(coef, method="mixed_ir", inner_iters=min(inner, budget),
                          outer_lim=max(1, budget // inner), atol=btol, btol=btol,
                          check_every=args.check_every, precond=precond)
        else:
            # the refinement's residual test ||r|| <= btol ||h|| (atol = 0: Paige and Saunders'
            # first test without its atol ||A|| ||x|| term, the second test off)
            inf = B.solve(coef, iter_lim=budget, atol=0.0, btol=btol,
                          check_every=args.check_every, precond=precond)
        torch.cuda.synchronize()
        return inf, tb - ta, time.perf_counter() - tb

    for _ in range(warmup):
        # the warm-up runs the step with a short budget: every kernel, graph and table is
        # exercised once before the timed steps
        step(min(iters, 2 * args.check_every))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(steps):
        infos, t_setup, t_solve = step(iters)
        print(f"# step {k}: assemble+factors {t_setup * 1e3:.1f} ms, solve {t_solve:.2f} s",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t1) / steps
    its = np.array([i["iters"] for i in infos])
    stops = np.array([i["istop"] for i in infos])
    # ||h|| per pair from the forcing (h = f / sqrt(N_i)); relative residuals of the solve
    hn = np.concatenate([np.linalg.norm(configs.batch_forcing(s), axis=1) / np.sqrt(s.n_rows)
                         for s in specs])
    rel = np.array([i["rnorm"] for i in infos]) / hn
    rows_rhs = B.sizes["n_rows"] * 8
    nnz, nbp = B.sizes["nnz"], B.sizes["n_block_points"]
    N, n_phi = B.sizes["n_rows"], B.sizes["n_phi"]
    bj_name = f"bj{patch}x{patch}-" if patch > 1 else "bj-"
    method = (f"batched {bj_name if precond else ''}"
              + (f"mixed-ir ({store} inner)" if mixed else "lsqr-fp64"))
    # rooflines of the three matrix passes of a step, on the matrix the inner steps stream
    kp = store if mixed else "fp64"
    label = f"batch{args.batch_n}x8" + (f"_p{patch}" if patch > 1 else "")
    roof = _batch_pass_roofline(B, kp, tune[kp], label,
                                "the longest matrix pass of a batched Krylov step, 8 rhs",
                                folded=precond)
    n_ok = int(np.sum((stops == 1) | (stops == 2)))
    out = {
        "metric": METRIC, "value": rows_rhs / dt, "unit": "rows/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": f"f64+{store}" if mixed else "f64", "data": "synthetic",
        "config": {"workload": f"batch{args.batch_n}x8", "instances": args.batch_n, "n_rhs": 8,
                   "rows": N, "cols": n_phi, "nnz": nnz,
                   "method": method, "btol": btol, "iter_budget": iters,
                   "inner": inner if mixed else None, "shift": args.shift if precond else None,
                   "patch": patch if precond else None},
        "define_s": t_define, "setup_ms": t_setup * 1e3, "solve_s": t_solve,
        "tuned_shapes": tune,
        "pairs_meeting_stop_test": n_ok, "pairs": int(len(stops)),
        "fraction_meeting_stop_test": n_ok / len(stops),
        "pairs_converged": int(np.sum(stops == 1)),
        "pairs_ls_optimal": int(np.sum(stops == 2)), "pairs_budget": int(np.sum(stops == 7)),
        "iters_max": int(its.max()), "iters_median": float(np.median(its)),
        "rel_residual_quantiles": {q: float(np.quantile(rel, float(q)))
                                   for q in ("0.5", "0.9", "0.99", "1.0")},
        "ms_per_iteration": t_solve * 1e3 / max(1, int(its.max())),
        "roofline": roof,
    }
    B.destroy()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = batch_cpu_baseline(specs, feats, int(its.max()), nnz, rows_rhs,
                                                 patch=patch if precond else None,
                                                 shift=args.shift)
    return out


def batch_cpu_baseline(specs, feats, n_iters, nnz_total, rows_rhs, n_sample=4, n_lsqr=20,
                       forcing=None, patch=None, shift=1e-12):
    """The oracle on a sample of the batch: the smallest, the largest and two seeded instances,
    each assembled (FP64 blocks) and n_lsqr LSQR iterations run for each of its 8 right-hand
    sides (with patch: on the oracle's block-Jacobi fold over patches of patch^2 subdomains,
    factors and fold included in the assembly time); scaled by entry count to the whole batch
    and the step's iterations.  1 warm-up + 2 repeats at the BLAS's threads, 1 warm-up + 1
    repeat at 1 thread."""
    import numpy as np
    from inputs import configs
    from oracle import assemble as asm
    from oracle import linalg
    from threadpoolctl import threadpool_limits

    sizes = [s.n_rows * s.K for s in specs]
    rng = np.random.default_rng(1)
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)),
                   *[int(i) for i in rng.choice(len(specs), size=n_sample - 2, replace=False)]})

    def once():
        t_asm = t_it = 0.0
        ent = 0
        for i in pick:
            spec, (W, b) = specs[i], feats[i]
            t0 = time.perf_counter()
            blocks = asm.assemble_blocks(spec, W, b)
            n = len(blocks) * spec.K
            if patch is not None:
                pb = linalg.patch_blocks(blocks, patch)
                fold = linalg.fold_blocks(pb, linalg.block_jacobi_factors(pb, shift))
                mv = lambda v: linalg.patch_matvec(fold, v, spec.n_rows)
                rmv = lambda u: linalg.patch_rmatvec(fold, u)
            else:
                mv = lambda v: asm.matvec(blocks, v, spec.n_rows)
                rmv = lambda u: asm.rmatvec(blocks, u, n)
            t_asm += time.perf_counter() - t0
            ent += sum(blk.M.size for blk in blocks)
            F = configs.batch_forcing(spec) if forcing is None else forcing(i)
            t1 = time.perf_counter()
            for r in range(F.shape[0]):
                h = asm.rhs(spec, F[r])
                linalg.lsqr(mv, rmv, h, n, atol=0, btol=0, iter_lim=n_lsqr)
            t_it += (time.perf_counter() - t1) / n_lsqr
        return (t_asm + t_it * n_iters) * nnz_total / ent, ent

    def series(k):
        ts = []
        for j in range(k + 1):
            t, ent = once()
            if j > 0:
                ts.append(t)
        return ts, ent

    ts, ent = series(2)
    threads = _threads()
    with threadpool_limits(limits=1, user_api="blas"):
        t1s, _ = series(1)
    t_med = float(np.median(ts))
    return {"value": rows_rhs / t_med, "unit": "rows/s", "cores": threads, "kind": "oracle",
            "sample": (f"instances {pick} ({ent} of {nnz_total} entries): oracle assembly"
                       + (f", block-Jacobi factors and fold over {patch} x {patch} patches"
                          if patch is not None else "") + " and "
                       f"{n_lsqr} LSQR iterations per right-hand side (8 each), scaled by entry "
                       f"count to the batch and the step's {n_iters} iterations; 1 warm-up + 2 "
                       f"repeats at {threads} BLAS threads, median {t_med:.0f} s per step (min "
                       f"{min(ts):.0f}, max {max(ts):.0f}); 1 thread: {t1s[0]:.0f} s"),
            "value_1_thread": rows_rhs / t1s[0]}


def _batch_pass_roofline(B, kp, shape, workload, label, folded=False):
    """HBM roofline of the longest of the three matrix passes of a batched Krylov step (8 right-
    hand sides) on the stored copy of precision kp, with the other two under "also".  With
    folded, the entries and block points are those of the folded matrix the solves stream (the
    patch blocks when the factors are of patches)."""
    es = {"fp64": 8, "fp32": 4, "bf16": 2, "fp16": 2}[kp]
    nnz, nbp = B.sizes["nnz"], B.sizes["n_block_points"]
    if folded:
        tab = B.copy_blocks(folded=True)
        nnz = int((tab[:, 3] * tab[:, 5] * tab[:, 6]).sum())
        nbp = int((tab[:, 3] * tab[:, 5]).sum())
    N, n_phi = B.sizes["n_rows"], B.sizes["n_phi"]
    ms_mv, ms_g, ms_rmv = B.time_kernels(kp, reps=5)
    R = 8
    prods = {f"k_bt_mvb<{_kname(kp)},{shape['mvb_ahead']}>": (ms_mv, nnz * es + 8 * R * (n_phi + nbp)),
             f"k_bt_gather<{shape['gather_rows']}>": (ms_g, 8 * R * (nbp + N)),
             f"k_bt_rmvb<{_kname(kp)},{shape['rmvb_tile']}>": (ms_rmv,
                                                            nnz * es + 8 * R * (nbp + n_phi))}
    dom = max(prods, key=lambda k: prods[k][0])
    roof = {"bound": "hbm", "achieved": prods[dom][1] / (prods[dom][0] * 1e-3) / 1e9,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": measured_traffic(dom, workload),
            "kernel": f"{dom} ({label})", "ms_per_launch": prods[dom][0],
            "algorithmic_bytes_per_launch": prods[dom][1],
            "also": [{"kernel": k, "ms_per_launch": t, "algorithmic_bytes_per_launch": a,
                      "achieved_GBs": a / (t * 1e-3) / 1e9,
                      "frac": a / (t * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "traffic": measured_traffic(k, workload)}
                     for k, (t, a) in prods.items() if k != dom]}
    roof["frac"] = roof["achieved"] / HBM_PEAK_GBS
    return roof


def _warm_errors(specs, om, C, coef_y, B, groups):
    """rel-L2 of u against the exact solution on each sampled group's test grid, for every
    right-hand side, from batch coefficients in block-Jacobi coordinates (mapped back by the
    batch, evaluated by a single-problem handle of the instance)."""
    import numpy as np
    import torch

    from inputs import configs, feature_params
    from inputs.problems import grid_points
    from paper_2409_01949_amd import Problem

    x = torch.empty(B.n_rhs * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
    B.from_coords(torch.as_tensor(coef_y).cuda(), x)
    xh = x.cpu().numpy()
    R = C.shape[1]
    out = []
    o = 0
    offs = []
    for s in specs:
        offs.append(o)
        o += R * int(np.prod(s.levels[0])) * s.K
    for g in groups:
        s = specs[g]
        n = int(np.prod(s.levels[0])) * s.K
        W, b = feature_params(s)
        P = Problem.from_spec(s, W, b)
        tp = grid_points(s, s.meta["n_test"])
        u = torch.empty(R * tp.shape[0], dtype=torch.float64, device="cuda")
        P.evaluate(torch.as_tensor(xh[offs[g]:offs[g] + R * n]).cuda(),
                   torch.as_tensor(tp).cuda(), u, n_rhs=R)
        uh = u.cpu().numpy().reshape(R, -1)
        for r in range(R):
            ue = configs.warm_exact(s, C[g, r], tp)
            out.append(float(np.linalg.norm(uh[r] - ue) / np.linalg.norm(ue)))
        P.destroy()
    return np.array(out)


def run_warm(args):
    """Learned warm start on a parameterised family (omega ~ U[5,50], c ~ N(0,1)^3): 1D
    (`warm`, J=64, K=32, 6000 points) or 2D (`warm2d`, -Lap u = f on [0,1]^2, 16 x 16
    subdomains, K=48, 200^2 points).  4,096 training solves (512 omega x 8 c) by the batched
    solver, the MLP (3 x 512 tanh, BF16 products) trained on them, then the 1,024 held-out pairs
    (128 x 8) solved to ||h - M c|| <= btol ||h|| (or least-squares optimality at atol = btol)
    from its prediction.  A step is prediction + warm solve; the cold solve of the same batch is
    reported beside it, with both solutions' rel-L2 against the exact solution on sampled
    groups."""
    import numpy as np
    import torch

    from inputs import configs, feature_params
    from paper_2409_01949_amd import warmstart as ws

    def log(m):
        print("# " + m, file=sys.stderr, flush=True)

    dim = 2 if args.workload == "warm2d" else 1
    inner = args.warm_inner or (2000 if dim == 1 else 4000)
    outer = args.warm_outer or (10 if dim == 1 else 4)
    btol = args.batch_btol_given if args.batch_btol_given else (1e-4 if dim == 1 else 1e-3)
    epochs = args.epochs or (100 if dim == 1 else 300)
    chunk = 512 if dim == 1 else 64
    store = "fp32"
    om, C = configs.warm_groups(args.warm_train_groups, 5)
    parts, infos, t_data = [], [], 0.0
    for c0 in range(0, len(om), chunk):
        B, specs, _ = ws.family_batch(om[c0:c0 + chunk], C[c0:c0 + chunk], dim=dim)
        B.tune(store, reps=3)
        log(f"training omegas {c0}..{c0 + len(specs) - 1}: batch assembled")
        coef, inf, t = ws.solve_batch(B, btol=btol * 0.1, atol=btol * 0.1, inner=inner,
                                      outer=outer)
        log(f"training omegas {c0}..{c0 + len(specs) - 1}: solved in {t:.1f} s")
        X, F, T = ws.training_set(specs, om[c0:c0 + chunk], C[c0:c0 + chunk],
                                  ws.coef_blocks(coef, specs, C.shape[1]))
        parts.append((X.astype(np.float32), None if F is None else F.astype(np.float32), T))
        infos += inf
        t_data += t
        B.destroy()
        torch.cuda.empty_cache()
    X = np.concatenate([p[0] for p in parts])
    F = None if parts[0][1] is None else np.concatenate([p[1] for p in parts])
    Y = np.concatenate([p[2] for p in parts])
    parts = None
    log(f"training data: {len(X)} samples from {len(infos)} solves in {t_data:.1f} s")
    Wn = ws.WarmStart(n_in=X.shape[1], K=Y.shape[1], max_batch=4096, seed=0,
                      n_mod=1 if F is None else F.shape[1])
    t0 = time.perf_counter()
    hist = Wn.fit(X, F, Y, epochs=epochs, lr=1e-3, seed=0, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n_steps = epochs * (len(X) // 4096)
    flop_step = sum(6 * 4096 * a * b for a, b in zip(Wn.dims[:-1], Wn.dims[1:]))
    X = F = Y = None
    om2, C2 = configs.warm_groups(args.warm_test_groups, 6)
    B2, specs2, hn2 = ws.family_batch(om2, C2, dim=dim)
    shape = B2.tune(store, reps=3)
    log("held-out batch assembled")
    # a pair is solved at ||r|| <= btol ||h|| or, for the pairs whose optimal residual lies above
    # that, at least-squares optimality with atol = btol
    yc, cold, t_cold = ws.solve_batch(B2, btol=btol, inner=inner, outer=outer, atol=btol)
    log(f"cold solve {t_cold:.2f} s")

    def step():
        torch.cuda.synchronize()
        ta = time.perf_counter()
        x0 = torch.as_tensor(np.ascontiguousarray(ws.predict(Wn, specs2, om2, C2))
                             .reshape(-1)).cuda()
        yw, warm, _ = ws.solve_batch(B2, x0=x0, btol=btol, inner=inner, outer=outer,
                                     precondition=False, atol=btol)
        torch.cuda.synchronize()
        return yw, warm, time.perf_counter() - ta

    for _ in range(args.warmup):
        step()
    ts = []
    for _ in range(args.steps):
        yw, warm, dt = step()
        ts.append(dt)
    dt = float(np.mean(ts))
    itc = np.array([i["iters"] for i in cold])
    itw = np.array([i["iters"] for i in warm])
    groups = sorted({0, len(om2) // 2, len(om2) - 1})
    ec = _warm_errors(specs2, om2, C2, yc, B2, groups)
    ew = _warm_errors(specs2, om2, C2, yw, B2, groups)
    rows_rhs = B2.sizes["n_rows"] * C2.shape[1]
    name = f"warm{dim}d_{len(om2)}x{C2.shape[1]}"
    roof = _batch_pass_roofline(B2, store, shape, name,
                                "the longest matrix pass of the warm-started solve")
    roof["also"].append({"kernel": "k_mlp_gemm (training, whole Adam step)",
                         "ms_per_step": t_train / max(1, n_steps) * 1e3,
                         "achieved_TFLOPs": flop_step * n_steps / t_train / 1e12,
                         "peak_TFLOPs": 2500.0, "bound": "mfma"})
    mlp = "-".join(str(d) for d in Wn.dims) + " tanh, bf16" + (
        f", output modulated by {Wn.net.n_mod}" if Wn.net.n_mod > 1 else
        ", one mode per sample, combined over the distinct modes")
    out = {
        "metric": METRIC, "value": rows_rhs / dt, "unit": "rows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+fp32",
        "data": "synthetic",
        "config": {"workload": name, "instances": len(om2), "n_rhs": C2.shape[1],
                   "train_solves": len(infos), "rows": B2.sizes["n_rows"],
                   "cols": B2.sizes["n_phi"], "method": "bj-mixed-ir (fp32 inner), MLP x0",
                   "btol": btol, "atol": btol, "inner": inner, "outer": outer,
                   "epochs": epochs, "mlp": mlp},
        "warm_s": dt, "cold_s": t_cold, "speedup_vs_cold": t_cold / dt,
        "iters_mean": {"cold": float(itc.mean()), "warm": float(itw.mean())},
        "iters_max": {"cold": int(itc.max()), "warm": int(itw.max())},
        "converged": {"cold": int(sum(i["istop"] == 1 for i in cold)),
                      "warm": int(sum(i["istop"] == 1 for i in warm)), "pairs": len(cold)},
        "ls_optimal": {"cold": int(sum(i["istop"] == 2 for i in cold)),
                       "warm": int(sum(i["istop"] == 2 for i in warm))},
        "rel_l2_vs_exact": {"groups": groups, "cold_median": float(np.median(ec)),
                            "cold_max": float(ec.max()), "warm_median": float(np.median(ew)),
                            "warm_max": float(ew.max())},
        "training": {"data_s": t_data, "train_s": t_train, "adam_steps": n_steps,
                     "loss_first": hist[0], "loss_last": hist[-1]},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        feats2 = [feature_params(s) for s in specs2]
        out["cpu_baseline"] = batch_cpu_baseline(
            specs2, feats2, int(itw.max()), B2.sizes["nnz"], rows_rhs,
            forcing=lambda i: configs.warm_batch_forcing(specs2[i], C2[i]))
    B2.destroy()
    Wn.destroy()
    return out

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
    profiles/traffic_<workload>.json (rocprofv3 FETCH_SIZE and WRITE_SIZE per dispatch, each
    scaled by the same counter on a plain copy of known size), or None when the kernel is not in
    it or the library's kernel sources changed since the counters were taken (the SHA-256 of
    the listed source files, read in order and concatenated, is recorded there)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
        h = hashlib.sha256()
        for src in d["sources"]:
            with open(os.path.join(ROOT, src), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != d["source_sha256"]:
            return None
        return float(d["kernels"][kernel]["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError, TypeError):
        return None


_PREC_NAMES = {"0": "FP64", "1": "FP32", "2": "BF16", "3": "FP16"}


def _kernel_label(name):
    """A rocprofv3 kernel name in the form bench.py reports it: namespace and return type
    dropped, the precision argument of the matrix-pass templates named (k_mv_blocks<FP16,2>)."""
    s = name.strip()
    if s.startswith("void "):
        s = s[5:]
    s = s.replace("elmfb::", "")
    base, _, rest = s.partition("<")
    base = base.split("(")[0]
    if not rest or "(" in base:
        return base
    targs = [t.strip() for t in rest.split(">")[0].split(",")]
    if base in ("k_mv_blocks", "k_bt_mvb", "k_bt_rmvb", "k_rmv_chunks"):
        targs[0] = _PREC_NAMES.get(targs[0], targs[0])
        if base == "k_rmv_chunks":
            targs = targs[:1]
    return f"{base}<{','.join(targs)}>"


def _counter_values(run_dir, counter):
    """Per kernel label, the counter's value (KiB) of every dispatch in a rocprofv3 --pmc run."""
    import csv
    import glob
    out = {}
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {run_dir}")
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    out.setdefault(_kernel_label(r["Kernel_Name"]), []).append(
                        float(r["Counter_Value"]))
    return out


def _copy_scale(run_dir, counter, nbytes):
    """Bytes per counted KiB, from the copy kernel's dispatches of a plain copy of nbytes (the
    runtime's copy kernel; dispatches below a fifth of nbytes, other copies, are left out)."""
    vals = _counter_values(run_dir, counter)
    name, v = max(((n, v) for n, v in vals.items() if "copy" in n.lower()),
                  key=lambda kv: max(kv[1]))
    big = [x for x in v if x * 1024 > 0.2 * nbytes]
    return nbytes / (sum(big) / len(big) * 1024), name


def write_traffic(args):
    """profiles/traffic_<name>.json: HBM bytes per dispatch of the named kernels, FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch, averaged over the run's dispatches) each scaled by what the
    same counter reads for a plain copy of known size, with the SHA-256 of the kernels' source
    files (read in order and concatenated) so that measured_traffic() drops them once a source
    changes."""
    import hashlib
    fs, fname = _copy_scale(args.copy_fetch, "FETCH_SIZE", args.copy_ref_bytes)
    ws, _ = _copy_scale(args.copy_write, "WRITE_SIZE", args.copy_ref_bytes)
    F = _counter_values(args.pmc_fetch, "FETCH_SIZE")
    W = _counter_values(args.pmc_write, "WRITE_SIZE")
    sources = [x for x in args.traffic_sources.split(",") if x]
    h = hashlib.sha256()
    for src in sources:
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    out = {"workload": args.write_traffic, "sources": sources, "source_sha256": h.hexdigest(),
           "scale": {"fetch": fs, "write": ws, "copy_kernel": fname},
           "unit": "bytes per dispatch (FETCH_SIZE x scale.fetch + WRITE_SIZE x scale.write)",
           "kernels": {}}
    for k in [x for x in args.traffic_kernels.split(";") if x]:
        if k not in F or k not in W:
            raise SystemExit(f"{k}: not in both counter runs (kernels seen: {sorted(F)})")
        rd = sum(F[k]) / len(F[k]) * 1024 * fs
        wr = sum(W[k]) / len(W[k]) * 1024 * ws
        out["kernels"][k] = {"hbm_bytes_per_launch": rd + wr, "read_bytes": rd,
                             "write_bytes": wr, "dispatches_fetch": len(F[k]),
                             "dispatches_write": len(W[k])}
    path = args.traffic_out or os.path.join(ROOT, "profiles", f"traffic_{args.write_traffic}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


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
    """Microseconds per LSQR step of the one-workgroup solve on P: up to n_it steps in one launch,
    less a solve of no steps (the set-up kernels), HIP events on the stream the solve runs on,
    divided by the steps the solve actually took (at atol = btol = 0 a small system can still end
    early on LSQR's machine-precision tests)."""
    import torch
    stream = torch.cuda.current_stream()

    def timed(k):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        info = P.solve(coef, method="lsqr", iter_lim=k, atol=0.0, btol=0.0, check_every=max(k, 1))
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1), info["iters"]

    steps = timed(n_it)[1]
    runs = [timed(n_it) for _ in range(reps)]
    assert all(r[1] == steps for r in runs), "the solve's step count changed between repeats"
    ms = min(r[0] for r in runs) - min(timed(0)[0] for _ in range(reps))
    return ms, ms * 1e3 / max(steps, 1), steps


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
    ms_launch, us_step, _ = _one_wg_us_per_step(P, coef, k, reps)
    tiny = configs.tiny1d()
    Wt, bt = feature_params(tiny)
    Pt = Problem.from_spec(tiny, Wt, bt, "fp64")
    Pt.assemble(torch.as_tensor(configs.forcing(tiny)).cuda())
    ct = torch.empty(Pt.sizes["n_phi"], dtype=torch.float64, device="cuda")
    _, us_floor, floor_steps = _one_wg_us_per_step(Pt, ct, 2000, reps)
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
                                     f"3-subdomain 1D system ({floor_steps} steps, where its "
                                     "solve ends)",
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

    from threadpoolctl import threadpool_limits

    def series(k):
        ts = []
        for i in range(k + 1):
            t1 = time.perf_counter()
            res = oracle_step()
            if i > 0:
                ts.append(time.perf_counter() - t1)
        return ts, res

    ts, (M, h, ref) = series(3)
    with threadpool_limits(limits=1, user_api="blas"):
        t1s, _ = series(1)
    e_l1 = lambda c: float(np.mean(np.abs(ev_o.evaluate(spec, W, b, c, xt) - ue)) / np.std(ue))
    xq = linalg.householder_lstsq(M, h)
    t_med = float(np.median(ts))
    return {"value": rows / t_med, "unit": "rows/s", "cores": _threads(), "kind": "oracle",
            "sample": (f"the whole step: assembly and {ref.itn} LSQR iterations (istop "
                       f"{ref.istop}), median of 3 repeats after 1 warm-up at {_threads()} BLAS "
                       f"threads {t_med:.2f} s (min {min(ts):.2f}, max {max(ts):.2f}); 1 warm-up "
                       f"+ 1 repeat at 1 thread {t1s[0]:.2f} s"),
            "value_1_thread": rows / t1s[0],
            "oracle_e_l1_test": e_l1(ref.x), "dense_qr_e_l1_test": e_l1(xq)}


def _multi_wg_us_per_step(P, coef, n_it, reps):
    """Microseconds per LSQR step of the multi-workgroup solve on P (graph replays of n_it
    steps), less a solve of no steps, with HIP events on the stream the solve runs on."""
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


def run_ode1d(args, steps, warmup):
    """The 1D first-order ODE du/dx = cos(15x) on [-2 pi, 2 pi], u(0) = 0 by the ansatz
    tanh(15x) NN: 20 subdomains (width ratio 1.3), K = 64, 2,000 collocation points, FP64,
    plain LSQR to atol = btol = 1e-10 within the 15,000-iteration budget.  A step is assembly
    and that solve; the error is against the exact solution on 1,000 test points.  The system
    (166,400 entries, 1.3 MB) lives in the caches, so a step of the multi-workgroup LSQR is bound
    by its dozen dependent launches, not by HBM: the roofline reports microseconds per step
    against the same graph of kernels on the smallest system."""
    import numpy as np
    import torch

    from inputs import configs, feature_params
    from paper_2409_01949_amd import Problem

    budget = 15000
    spec = configs.ode1d()
    W, b = feature_params(spec)
    f = configs.forcing(spec)
    P = Problem.from_spec(spec, W, b, "fp64")
    fd = torch.as_tensor(f).cuda()
    n = P.sizes["n_phi"]
    coef = torch.empty(n, dtype=torch.float64, device="cuda")
    xt = np.linspace(spec.lo[0], spec.hi[0], 1000)[:, None]
    ue = configs.exact(spec, xt)
    xt_d = torch.as_tensor(xt).cuda()
    u_d = torch.empty(1000, dtype=torch.float64, device="cuda")

    def step(pre=False):
        P.assemble(fd)
        if pre:
            P.precondition(args.shift)
        return P.solve(coef, method="lsqr", iter_lim=budget, atol=1e-10, btol=1e-10,
                       check_every=1000, precond=pre)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    info = infos[-1]
    P.evaluate(coef, xt_d, u_d)
    u = u_d.cpu().numpy()
    rel = float(np.linalg.norm(u - ue) / np.linalg.norm(ue))
    # block-Jacobi LSQR (not the workload's solver) to the same test, for comparison
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bi = step(True)
    torch.cuda.synchronize()
    t_bj = time.perf_counter() - t1
    P.evaluate(coef, xt_d, u_d)
    rel_bj = float(np.linalg.norm(u_d.cpu().numpy() - ue) / np.linalg.norm(ue))
    P.assemble(fd)
    reps = max(2, args.kernel_reps // 10)
    ms_l, us_step = _multi_wg_us_per_step(P, coef, 2000, reps)
    tiny = configs.tiny1d()
    Wt, bt = feature_params(tiny)
    Pt = Problem.from_spec(tiny, Wt, bt, "fp64")
    Pt.assemble(torch.as_tensor(configs.forcing(tiny)).cuda())
    ct = torch.empty(Pt.sizes["n_phi"], dtype=torch.float64, device="cuda")
    old = os.environ.get("ELMFB_PERSISTENT")
    os.environ["ELMFB_PERSISTENT"] = "0"
    try:
        _, us_floor = _multi_wg_us_per_step(Pt, ct, 2000, reps)
    finally:
        if old is None:
            del os.environ["ELMFB_PERSISTENT"]
        else:
            os.environ["ELMFB_PERSISTENT"] = old
    Pt.destroy()
    out = {
        "metric": METRIC, "value": spec.n_rows / dt, "unit": "rows/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "ode1d", "J": 20, "K": spec.K, "delta": spec.delta,
                   "collocation_points": spec.n_rows, "method": "lsqr fp64 (plain)",
                   "atol": 1e-10, "btol": 1e-10, "iter_budget": budget},
        "time_to_solution_s": dt, "iters": info["iters"], "istop": info["istop"],
        "rnorm": info["rnorm"], "arnorm": info["arnorm"],
        "rel_l2_test_vs_exact": rel,
        "note": ("LSQR does not meet atol = btol = 1e-10 within the budget on this system (istop "
                 "7); the CPU oracle's own LSQR runs on row-permuted copies differ in u by ~3e-3 "
                 "there, which bounds what any implementation reproduces"),
        "block_jacobi_lsqr": {"s": t_bj, "iters": bi["iters"], "istop": bi["istop"],
                              "rnorm": bi["rnorm"], "rel_l2_test_vs_exact": rel_bj},
        "roofline": {"bound": "latency", "achieved": us_step, "peak": us_floor,
                     "unit": "us/step", "frac": us_floor / us_step, "traffic": None,
                     "kernel": "multi-workgroup LSQR step (graph of the product passes, the row "
                               "gather, the column pass and the scalar kernels)",
                     "peak_meaning": "the same graph of kernels on the 200-point 3-subdomain 1D "
                                     "system (ELMFB_PERSISTENT=0)",
                     "ms_per_2000_steps": ms_l},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = ode1d_cpu_baseline(spec, W, b, f, info["iters"])
    P.destroy()
    return out


def ode1d_cpu_baseline(spec, W, b, f, n_iters, n_lsqr=1000):
    """The oracle on the 1D ODE: assembly of the dense matrix and n_lsqr dense LSQR iterations,
    scaled to the GPU step's n_iters iterations; 1 warm-up + 3 repeats at the BLAS's threads,
    1 warm-up + 2 repeats at 1 thread."""
    import numpy as np
    from oracle import assemble as asm
    from oracle import linalg
    from threadpoolctl import threadpool_limits

    n = len(W)

    def once():
        t0 = time.perf_counter()
        blocks = asm.assemble_blocks(spec, W, b)
        M = asm.dense_from_blocks(blocks, spec.n_rows, n)
        h = asm.rhs(spec, f)
        t1 = time.perf_counter()
        linalg.lsqr(lambda v: M @ v, lambda r: M.T @ r, h, n, atol=0.0, btol=0.0,
                    iter_lim=n_lsqr)
        t2 = time.perf_counter()
        return (t1 - t0) + (t2 - t1) * n_iters / n_lsqr

    def series(k):
        return [t for i, t in enumerate(once() for _ in range(k + 1)) if i > 0]

    ts = series(3)
    threads = _threads()
    with threadpool_limits(limits=1, user_api="blas"):
        t1s = series(2)
    t_med = float(np.median(ts))
    return {"value": spec.n_rows / t_med, "unit": "rows/s", "cores": threads, "kind": "oracle",
            "sample": (f"assembly and {n_lsqr} dense LSQR iterations, scaled to the step's "
                       f"{n_iters}; 1 warm-up + 3 repeats at {threads} BLAS threads, median "
                       f"{t_med:.2f} s per step (min {min(ts):.2f}, max {max(ts):.2f}); 1 warm-up "
                       f"+ 2 repeats at 1 thread, median {float(np.median(t1s)):.2f} s"),
            "value_1_thread": spec.n_rows / float(np.median(t1s))}


def run_helmholtz(args, steps, warmup, levels=((16, 16),)):
    """The L-shaped Helmholtz problem of Sec. 4.4 at the paper's baseline: omega = 8, k = 1, one
    level of 16 x 16 subdomains less the 8 x 8 outside the L (192), K = 16, width ratio 2.9,
    R = 1, the 80 x 80 grid's 4,800 points inside the L as interior rows, 320 Dirichlet rows at
    the boundary points with lambda_bc = 25 omega^4.  Solved as the paper does (Sec. 4.1): FP64
    LSQR for its whole 15,000-iteration budget (atol = btol = 0).  A step is assembly (interior
    and boundary rows) and that solve; the error is e_L1 against the exact solution on the
    96 x 96 grid's points inside the L (the paper's ELM-FBPINN: 1.3 +- 0.8e-2, context only)."""
    import numpy as np
    import torch

    from inputs import configs, feature_params
    from paper_2409_01949_amd import Problem

    budget = 15000
    spec = configs.helmholtz(levels=levels)
    Wf, bf = feature_params(spec)
    f = configs.forcing(spec)
    xb = configs.boundary_points(spec)
    g = configs.exact(spec, xb)
    wgt = float(np.sqrt(spec.meta["lambda_bc"] / xb.shape[0]))
    P = Problem.from_spec(spec, Wf, bf, "fp64", bc_pts=xb, bc_vals=g, bc_weight=wgt)
    fd = torch.as_tensor(f).cuda()
    n = P.sizes["n_phi"]
    rows = P.sizes["n_interior"] + P.sizes["n_bc"]
    coef = torch.empty(n, dtype=torch.float64, device="cuda")
    from inputs.problems import grid_points
    xt_all = grid_points(spec, spec.meta["n_test"])
    xt = xt_all[configs.in_l_shape(spec, xt_all)]
    ue = configs.exact(spec, xt)
    xt_d = torch.as_tensor(xt).cuda()
    u_d = torch.empty(xt.shape[0], dtype=torch.float64, device="cuda")

    def step():
        P.assemble(fd)
        return P.solve(coef, method="lsqr", iter_lim=budget, atol=0.0, btol=0.0,
                       check_every=1000)

    print(f"# {spec.name}: {P.sizes}", file=sys.stderr, flush=True)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    info = infos[-1]
    print(f"# {spec.name}: {dt:.3f} s per step, {info['iters']} iterations", file=sys.stderr,
          flush=True)
    P.evaluate(coef, xt_d, u_d)
    u = u_d.cpu().numpy()
    e_l1 = float(np.mean(np.abs(u - ue)) / np.std(ue))
    rel = float(np.linalg.norm(u - ue) / np.linalg.norm(ue))
    sigma = krylov_sigma(P)
    reps = max(2, args.kernel_reps // 10)
    ms_l, us_step = _multi_wg_us_per_step(P, coef, 2000, reps)
    tiny = configs.tiny1d()
    Wt, bt = feature_params(tiny)
    Pt = Problem.from_spec(tiny, Wt, bt, "fp64")
    Pt.assemble(torch.as_tensor(configs.forcing(tiny)).cuda())
    ct = torch.empty(Pt.sizes["n_phi"], dtype=torch.float64, device="cuda")
    old = os.environ.get("ELMFB_PERSISTENT")
    os.environ["ELMFB_PERSISTENT"] = "0"
    try:
        _, us_floor = _multi_wg_us_per_step(Pt, ct, 2000, reps)
    finally:
        if old is None:
            del os.environ["ELMFB_PERSISTENT"]
        else:
            os.environ["ELMFB_PERSISTENT"] = old
    Pt.destroy()
    out = {
        "metric": METRIC, "value": rows / dt, "unit": "rows/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": spec.name, "omega": spec.meta["omega"], "k": spec.meta["k"],
                   "levels": [list(J) for J in spec.levels], "K": spec.K,
                   "subdomains": P.sizes["n_blocks"], "interior_rows": P.sizes["n_interior"],
                   "boundary_rows": P.sizes["n_bc"], "lambda_bc": spec.meta["lambda_bc"],
                   "method": "lsqr fp64", "atol": 0.0, "btol": 0.0, "iter_budget": budget},
        "time_to_solution_s": dt, "iters": info["iters"], "istop": info["istop"],
        "rnorm": info["rnorm"], "e_l1_test": e_l1, "rel_l2_test_vs_exact": rel,
        "paper_e_l1_context": "1.3 +- 0.8e-2 (ELM-FBPINN, 37 s on one CPU core)",
        "krylov_sigma": sigma,
        "roofline": {"bound": "latency", "achieved": us_step, "peak": us_floor,
                     "unit": "us/step", "frac": us_floor / us_step, "traffic": None,
                     "kernel": "multi-workgroup LSQR step (the product passes, the row gather, "
                               "the boundary rows, the column pass and the scalar kernels)",
                     "peak_meaning": "the same graph of kernels on the 200-point 3-subdomain 1D "
                                     "system (ELMFB_PERSISTENT=0)",
                     "ms_per_2000_steps": ms_l},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = helmholtz_cpu_baseline(spec, Wf, bf, f, xb, g, info["iters"],
                                                     rows)
    P.destroy()
    return out


def helmholtz_cpu_baseline(spec, Wf, bf, f_grid, xb, g, n_iters, rows, n_lsqr=1000):
    """The oracle on the Helmholtz problem: assembly of the interior blocks and the Dirichlet
    rows, then n_lsqr LSQR iterations on the sparse [N; B], scaled to the GPU step's n_iters;
    1 warm-up + 2 repeats at the BLAS's threads, 1 warm-up + 1 repeat at 1 thread."""
    import numpy as np
    import scipy.sparse as sp
    from inputs import configs
    from oracle import assemble as asm
    from oracle import geometry as geo
    from oracle import linalg
    from threadpoolctl import threadpool_limits

    inside = configs.in_l_shape(spec, geo.grid(spec))

    def once():
        t0 = time.perf_counter()
        W, b = geo.kept_parameters(spec, Wf, bf)
        blocks = asm.assemble_blocks(spec, W, b)
        N, n = int(inside.sum()), len(blocks) * spec.K
        S = sp.csr_matrix(np.vstack([asm.dense_from_blocks(blocks, N, n),
                                     asm.dirichlet_rows(spec, W, b, xb)]))
        h = asm.rhs(spec, f_grid[inside], g)
        t1 = time.perf_counter()
        linalg.lsqr(lambda v: S @ v, lambda u: S.T @ u, h, n, atol=0.0, btol=0.0,
                    iter_lim=n_lsqr)
        return (t1 - t0) + (time.perf_counter() - t1) * n_iters / n_lsqr

    def series(k):
        return [t for i, t in enumerate(once() for _ in range(k + 1)) if i > 0]

    ts = series(2)
    threads = _threads()
    with threadpool_limits(limits=1, user_api="blas"):
        t1s = series(1)
    t_med = float(np.median(ts))
    return {"value": rows / t_med, "unit": "rows/s", "cores": threads, "kind": "oracle",
            "sample": (f"assembly and {n_lsqr} LSQR iterations on the sparse [N; B], scaled to "
                       f"the step's {n_iters}; 1 warm-up + 2 repeats at {threads} BLAS threads, "
                       f"median {t_med:.2f} s per step (min {min(ts):.2f}, max {max(ts):.2f}); "
                       f"1 thread {t1s[0]:.2f} s"),
            "value_1_thread": rows / t1s[0]}


def _kname(prec):
    return {"fp64": "FP64", "fp32": "FP32", "bf16": "BF16", "fp16": "FP16"}[prec]


def product_rooflines(P, spec, prec, reps):
    """HBM rooflines of the two products of one Krylov step on the matrix copy of precision
    `prec`, timed with HIP events on the stream they run on (elmfb_time_kernels).  Algorithmic
    bytes per launch (entries of s bytes):
      k_mv_blocks   (first pass of y = M v): nnz s + 8 N_Phi (v) + 8 block points (partials out)
      k_gather_rows (completes y):           8 block points (partials in) + 8 N (y out)
      y = M v as a whole:                    nnz s + 8 (N + N_Phi)
      k_rmv_chunks  (first pass of M^T u):   nnz s + 8 block points (u gathered) + 8 chunks K
      k_rmv_finish  (completes x):           8 chunks K + 8 N_Phi
      x = M^T u as a whole:                  nnz s + 8 (N + N_Phi)
    Returns {name: (ms, algorithmic bytes)}."""
    es = {"fp64": 8, "fp32": 4, "bf16": 2, "fp16": 2}[prec]
    ms_mv, ms_rmv, ms_g, ms_f = P.time_kernels(reps, prec=prec)
    nnz, nbp = P.sizes["nnz"], P.sizes["n_block_points"]
    N, n_phi = P.sizes["n_rows"], P.sizes["n_phi"]
    n_chunks = sum(-(-int(r[4] * r[6]) // 2048) for r in P.copy_blocks())
    k = _kname(prec)
    pts = 2 if es == 2 else 1
    return {
        f"k_mv_blocks<{k},{pts}>": (ms_mv, nnz * es + 8 * n_phi + 8 * nbp),
        "k_gather_rows": (ms_g, 8 * nbp + 8 * N),
        f"k_rmv_chunks<{k}>": (ms_rmv, nnz * es + 8 * nbp + 8 * n_chunks * spec.K),
        "k_rmv_finish": (ms_f, 8 * n_chunks * spec.K + 8 * n_phi),
        "y = M v": (ms_mv + ms_g, nnz * es + 8 * (N + n_phi)),
        "x = M^T u": (ms_rmv + ms_f, nnz * es + 8 * (N + n_phi)),
    }


def hbm_roofline(prods, workload, label):
    """The roofline object of the dominant kernel (the longer of the two first passes, which
    rocprofv3 ranks first: each runs once per step), with the other kernels and the two products
    as a whole under "also"."""
    first = [k for k in prods if k.startswith("k_mv_blocks") or k.startswith("k_rmv_chunks")]
    dom = max(first, key=lambda k: prods[k][0])
    ms, alg = prods[dom]
    ach = alg / (ms * 1e-3) / 1e9
    traffic = measured_traffic(dom, workload)
    also = []
    for k, (t, a) in prods.items():
        if k == dom:
            continue
        also.append({"kernel": k, "ms_per_launch": t, "algorithmic_bytes_per_launch": a,
                     "achieved_GBs": a / (t * 1e-3) / 1e9,
                     "frac": a / (t * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": measured_traffic(k, workload) if k.startswith("k_") else None})
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "kernel": f"{dom} ({label})",
            "ms_per_launch": ms, "algorithmic_bytes_per_launch": alg, "also": also}


def run_single(args, workload, steps, warmup, secondary=False):
    """One multilevel 2D Poisson problem (poisson3l: the headline; poisson5l: the 5-level one).
    A step: assemble (FP64 + the low-precision copy) and h, block-Jacobi factors and the folded
    M R^-1, the solve until rel-L2 <= target against the exact solution on the check grid (or
    the budget), evaluation on the test grid."""
    import numpy as np
    import torch

    from inputs import configs, feature_params
    from inputs.problems import grid_points
    from paper_2409_01949_amd import Problem

    def note(msg):
        print("# " + msg, file=sys.stderr, flush=True)

    spec = getattr(configs, workload)()
    W, b = feature_params(spec)
    f = configs.forcing(spec)
    precond = not args.no_precond
    iters = args.iters if not secondary else args.secondary_iters
    t_def = time.perf_counter()
    P = Problem.from_spec(spec, W, b, args.store)
    t_def = time.perf_counter() - t_def
    fd = torch.as_tensor(f).cuda()
    xc = torch.as_tensor(grid_points(spec, spec.meta["n_check"])).cuda()
    uc = torch.as_tensor(configs.exact(spec, grid_points(spec, spec.meta["n_check"]))).cuda()
    xt_np = grid_points(spec, spec.meta["n_test"])
    xt = torch.as_tensor(xt_np).cuda()
    ut_np = configs.exact(spec, xt_np)
    n = P.sizes["n_phi"]
    coef = torch.empty(n, dtype=torch.float64, device="cuda")
    u_test = torch.empty(xt.shape[0], dtype=torch.float64, device="cuda")
    gram_method = args.method in ("normal_cg", "mixed_ir_cg")

    def step(method=args.method, pre=precond, iters=iters, target=args.target, tol=0.0):
        P.assemble(fd)
        if pre:
            P.precondition(args.shift)
        if method in ("normal_cg", "mixed_ir_cg"):
            P.gram(args.gram_prec, "all")
        chk = dict(check_pts=xc, check_ref=uc, target_rel_l2=target) if target > 0 else {}
        if method in ("mixed_ir", "mixed_ir_cg"):
            info = P.solve(coef, method=method, inner_iters=args.inner,
                           outer_lim=max(1, iters // args.inner), atol=tol, btol=tol,
                           check_every=min(args.check_every, args.inner), precond=pre, **chk)
        else:
            info = P.solve(coef, method=method, iter_lim=iters, atol=tol, btol=tol,
                           check_every=args.check_every, precond=pre, **chk)
        P.evaluate(coef, xt, u_test)
        return info

    for w in range(warmup):
        # a secondary workload warms up on a short budget: every kernel, graph and table once
        wi = step(iters=min(iters, 2 * args.check_every)) if secondary else step()
        note(f"{workload} warmup step {w}: {wi['iters']} iterations")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(steps):
        infos.append(step())
        note(f"{workload} step {k}: {infos[-1]['iters']} iterations, rel-L2 "
             f"{infos[-1]['rel_l2']:.3e}")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    info = infos[-1]
    main_sigma = krylov_sigma(P)
    u = u_test.cpu().numpy()
    e_l1 = float(np.mean(np.abs(u - ut_np)) / np.std(ut_np))
    rel_test = float(np.linalg.norm(u - ut_np) / np.linalg.norm(ut_np))

    kprec = args.store if args.method == "mixed_ir" else "fp64"
    prods = product_rooflines(P, spec, kprec, args.kernel_reps)
    roofline = hbm_roofline(prods, f"{spec.name}_{kprec}",
                            "the longer matrix-streaming pass of a Krylov step")
    if kprec != "fp64" and not secondary:
        roofline["also"] += [{"kernel": f"{k} [fp64]", "ms_per_launch": t,
                              "achieved_GBs": a / (t * 1e-3) / 1e9}
                             for k, (t, a) in product_rooflines(P, spec, "fp64",
                                                                args.kernel_reps).items()]
    if gram_method:
        # CG on the Gram blocks: the per-block pass of y = G p reads every stored block once
        # and writes two K-vectors of partials per block
        ms_pairs, ms_gmv = P.time_gram_mv(args.kernel_reps)
        n_pairs = P.sizes["n_pairs"]
        esg = 8 if args.gram_prec == "fp64" else 4
        g_bytes = n_pairs * spec.K * spec.K * esg + 2 * n_pairs * spec.K * 8
        lsqr_roof = roofline
        roofline = {"bound": "hbm", "achieved": g_bytes / (ms_pairs * 1e-3) / 1e9,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": g_bytes / (ms_pairs * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                    "kernel": f"k_gmv_pairs<{'FP64' if esg == 8 else 'FP32'}> (y = G p, per "
                              f"stored Gram block)",
                    "ms_per_launch": ms_pairs, "algorithmic_bytes_per_launch": g_bytes,
                    "also": [{"kernel": "G p, both passes", "ms_per_launch": ms_gmv},
                             {k: lsqr_roof[k] for k in ("kernel", "ms_per_launch", "achieved")}]
                            + lsqr_roof["also"]}

    # the Gram phase on the matrix cores: all overlapping pairs, FP64 and the stored copy's type
    gram_mfma = []
    if not args.no_gram and not secondary:
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

    # the FP64 reference solution (the method's accuracy yardstick): FP64 block-Jacobi LSQR on
    # the GPU -- the FP64 path checked against the oracle by the parity tests -- run to
    # atol = btol = 1e-10 within the 15,000-iteration budget, evaluated on the test grid
    fp64_ref = None
    if not args.no_compare:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ri = step("lsqr", True, args.ref_iters, target=0.0, tol=1e-10)
        torch.cuda.synchronize()
        u_ref = u_test.cpu().numpy()
        fp64_ref = {
            "what": ("u_ref = FP64 block-Jacobi LSQR on the GPU (the FP64 path the parity tests "
                     "check against the CPU oracle), atol = btol = 1e-10, "
                     f"{args.ref_iters}-iteration budget, on the {spec.meta['n_test']} test grid"),
            "istop": ri["istop"], "iters": ri["iters"], "s": time.perf_counter() - t1,
            "u_ref_rel_l2_vs_exact": float(np.linalg.norm(u_ref - ut_np) / np.linalg.norm(ut_np)),
            "rel_l2_test_vs_u_ref": float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)),
        }
        note(f"FP64 reference: istop {ri['istop']} after {ri['iters']}, rel-L2 of the step's u "
             f"vs it {fp64_ref['rel_l2_test_vs_u_ref']:.2e}")

    compare = {}
    if not args.no_compare and not secondary:
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

    method_txt = (f"{args.method}" + ("+block-jacobi" if precond else "") +
                  (f" (inner {args.store} x{args.inner})" if args.method == "mixed_ir"
                   else f" (gram {args.gram_prec}" +
                   (f", inner x{args.inner})" if args.method == "mixed_ir_cg" else ")")
                   if gram_method else "-fp64"))
    out = {
        "metric": METRIC, "value": spec.n_rows / dt, "unit": "rows/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": (f"f64+{args.store}" if args.method == "mixed_ir" else
                  f"f64+{args.gram_prec}" if gram_method else "f64"),
        "data": "synthetic",
        "config": {"workload": spec.name, "rows": spec.n_rows, "cols": n, "nnz": P.sizes["nnz"],
                   "levels": [list(J) for J in spec.levels], "K": spec.K,
                   "grid": list(spec.n_points), "method": method_txt, "iter_budget": iters,
                   "target_rel_l2": args.target,
                   "reference": "exact solution on the check grid (stop test); FP64 reference "
                                "solution and exact solution on the test grid (reported)"},
        "define_s": t_def,
        "time_to_solution_s": dt,
        "reached_target": bool(info["istop"] == 8),
        "iters": info["iters"],
        "outer_iters": info["outer_iters"],
        "rel_l2_check_at_stop": info["rel_l2"],
        "rel_l2_test_vs_exact": rel_test,
        "rel_l2_test_vs_fp64_ref": fp64_ref["rel_l2_test_vs_u_ref"] if fp64_ref else None,
        "fp64_reference": fp64_ref,
        "e_l1_test": e_l1,
        "roofline": roofline,
        "gram_mfma": gram_mfma,
        "krylov_sigma": main_sigma,
        "compare": compare,
    }
    if not args.no_cpu_baseline:
        note("cpu_baseline: the oracle on a sample of the workload")
        # the stored-entry count of the plan (equal to the oracle's, by the parity tests) scales
        # the sample; the 5-level grid takes a smaller sample (1 block per level, 2,048 rows)
        big = spec.n_rows > 500_000
        out["cpu_baseline"] = cpu_baseline(spec, W, b, f, info["iters"], P.sizes["nnz"],
                                           max_per_level=1 if big else 2,
                                           max_rows=2048 if big else 8192)
    P.destroy()
    return out


def main():
    args = parse()
    if args.write_traffic:
        write_traffic(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU build: run with --gpus 1 (the multi-GPU "
                                   "sharding is a design only)"}))
        sys.exit(2)
    if args.copy_bytes:
        run_copy(args)
        return
    if args.workload.startswith("batch"):
        print(json.dumps(run_batch(args)), flush=True)
        return
    if args.workload in ("warm", "warm2d"):
        print(json.dumps(run_warm(args)), flush=True)
        return
    if args.workload == "oscillator":
        run_oscillator(args)
        return
    if args.workload == "ode1d":
        print(json.dumps(run_ode1d(args, args.steps, args.warmup)), flush=True)
        return
    if args.workload in ("helmholtz", "helmholtz_ml"):
        lv = ((16, 16),) if args.workload == "helmholtz" else ((1, 1), (8, 8), (16, 16))
        print(json.dumps(run_helmholtz(args, args.steps, args.warmup, lv)), flush=True)
        return
    t_start = time.perf_counter()
    out = run_single(args, args.workload, args.steps, args.warmup)
    # the other workloads, each one step with a fixed budget after a short warm-up, reported
    # beside the headline (skipped, with the reason, once the run has taken too long)
    sec = [w for w in args.secondary.split(",") if w] if args.workload == "poisson3l" else []
    if sec:
        out["secondary"] = []
    for w in sec:
        elapsed = time.perf_counter() - t_start
        if elapsed > args.secondary_deadline:
            out["secondary"].append({"workload": w, "skipped": f"run already took {elapsed:.0f} "
                                     f"s (> {args.secondary_deadline:.0f} s)"})
            continue
        print(f"# secondary workload {w}", file=sys.stderr, flush=True)
        try:
            a = _args_for(args, w)
            if w == "ode1d":
                r = run_ode1d(a, 3, 1)
            elif w == "helmholtz":
                r = run_helmholtz(a, 2, 1)
            elif w == "batch":
                r = run_batch(a, 1, 1, args.secondary_iters)
            else:
                a.no_gram = True
                a.iters = args.secondary_iters
                a.ref_iters = args.secondary_ref_iters
                r = run_single(a, w, 1, 1, secondary=True)
        except Exception as exc:   # a secondary failure must not lose the headline line
            r = {"workload": w, "error": f"{type(exc).__name__}: {exc}"}
        out["secondary"].append(r)
        import torch
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
