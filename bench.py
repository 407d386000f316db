#!/usr/bin/env python
"""Benchmark of the FMM-compressed EFIE matvec (y = A_q x) on one MI355X.

Workload (matvec configuration): six-patch NURBS unit sphere (cube-sphere map),
refinement level 5 (32 x 32 elements per patch), div-conforming splines of degree
p = 2 (N = 13,068 complex unknowns), wavenumber kappa = 8, Chebyshev interpolation
degree q = 8, 5 x 5 Gauss rule for regular near-field element pairs, random
coefficient vector N(0,1) + i N(0,1) with seed 0, FP64 throughout.

A step is one application of the whole compressed operator (P2M, M2M, M2L, L2L,
L2P and the near-field product) to the device-resident vector; the operator is
assembled once before timing.  The JSON line reports DOF/s = N / t_step.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]

--mode serve instead measures the serving loop: a stream of independent scattering
solves (seeded synthetic requests: sphere or torus with jittered control points,
level 3..6, degree 1..2, kappa in [1, 20], one random plane wave each, GMRES to a
relative residual of 1e-6) arriving with exponential inter-arrival times; it
reports completed solves per second and the p50 / p99 latency from arrival to the
solution in host memory.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector
FP64_MFMA_PEAK_TFLOPS = 78.6    # MI355X FP64 dense matrix cores
BF16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix cores


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--eta", type=float, default=1.6)
    ap.add_argument("--leaf-depth", type=int, default=3)
    ap.add_argument("--level", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=64, help="rows of the larger bounded oracle sample")
    ap.add_argument("--no-solve", action="store_true",
                    help="matvec mode: skip the batched-solve leg (level 6, kappa 16, 64 plane waves)")
    ap.add_argument("--nrhs", type=int, default=1, help="right-hand sides per apply (batched kernels when > 1)")
    ap.add_argument("--prec", type=int, default=0, choices=(0, 1, 2, 3, 4),
                    help="coupling precision: 0 FP64, 1 FP32, 2 BF16 matrix cores, 3 split BF16 (3 products), "
                         "4 split BF16 coupling and near field")
    ap.add_argument("--store-coupling", type=int, default=-1, choices=(-1, 0, 1),
                    help="coupling blocks: 1 stored, 0 evaluated per apply, -1 stored if they fit")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--mode", choices=("matvec", "serve", "solve"), default="matvec")
    ap.add_argument("--p", type=int, default=2, help="solve: spline degree")
    ap.add_argument("--kappa", type=float, default=8.0, help="solve: wavenumber")
    ap.add_argument("--q", type=int, default=8, help="solve: interpolation degree")
    ap.add_argument("--tol", type=float, default=1e-6, help="solve: relative residual")
    ap.add_argument("--jitter", type=float, default=0.0,
                    help="solve: standard deviation of the control-point jitter of the cube-sphere (0: none)")
    ap.add_argument("--jitter-seed", type=int, default=7, help="solve: seed of the jitter")
    ap.add_argument("--restart", type=int, default=1500, help="solve: GMRES restart")
    ap.add_argument("--inner-prec", type=int, default=3, choices=(0, 1, 2, 3, 4),
                    help="solve: precision of refined inner solves (as --prec)")
    ap.add_argument("--inner-tol", type=float, default=1e-4, help="solve: relative residual of the inner solves")
    ap.add_argument("--compare-fp64", action="store_true", help="solve: also solve in FP64 and report the difference")
    ap.add_argument("--autotune", action="store_true",
                    help="time the candidate tile shapes of the apply first and keep the fastest (ige_op_autotune)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (calibrates HBM byte counters)")
    ap.add_argument("--kappa-cap", type=float, default=0.0,
                    help="matvec/solve: admissible blocks also need kappa * diam <= this (0: the paper's condition)")
    ap.add_argument("--q-level", type=str, default="",
                    help="matvec: interpolation degree per cluster-tree level, comma separated (0: --q); "
                         "'rule' takes the kappa * diam rule of the binding on the levels with far blocks")
    ap.add_argument("--requests", type=int, default=32, help="serve: number of requests")
    ap.add_argument("--rate", type=float, default=20.0, help="serve: mean arrivals per second")
    ap.add_argument("--workers", type=int, default=4, help="serve: concurrent requests (one stream each)")
    ap.add_argument("--sphere-only", action="store_true", help="serve: every request on the sphere")
    ap.add_argument("--same-object", action="store_true",
                    help="serve: every request on the object, level, degree and kappa of the first one "
                         "(a stream of incident directions on one scatterer)")
    ap.add_argument("--waves", type=int, default=1,
                    help="serve: plane waves per request, solved together (solves/s counts waves)")
    ap.add_argument("--maxit", type=int, default=3000, help="serve: GMRES iteration cap per request")
    ap.add_argument("--srv-restart", type=int, default=300, help="serve: GMRES restart of every request")
    ap.add_argument("--max-merge", type=int, default=64,
                    help="serve: plane waves of waiting requests on one operator solved together (1: no merging)")
    ap.add_argument("--refine", action="store_true",
                    help="serve / solve: FP64 refinement around solves with the --inner-prec coupling")
    return ap.parse_args()


PREC_NAMES = ["f64", "f32 coupling", "bf16 coupling", "split-bf16 coupling", "split-bf16 coupling and near field"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_traffic(r, kernel):
    """HBM bytes per launch of the near-field product from the committed counter
    summary, valid only while the source file of that kernel is the one the counters
    were taken on."""
    import hashlib
    files = {"k_near_cmp": ("k_near_cmp_sphere_l5_p2_traffic.json", "near_once.hip"),
             "k_near_blk": ("k_near_blk_sphere_l5_p2_traffic.json", "kernels.hip")}
    if r != 1 or kernel not in files:
        return None
    path = os.path.join(ROOT, "profiles", files[kernel][0])
    src = os.path.join(ROOT, "paper_1807_03097_amd", "csrc", files[kernel][1])
    if not os.path.exists(path):
        return None
    ref = json.load(open(path))
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    return ref["traffic_bytes"] if ref.get("source_sha256", ref.get("kernels_hip_sha256")) == h else None


def host_cpu():
    """model, physical cores and thread settings of the host (CPU baseline disclosure)"""
    model, phys = None, set()
    try:
        cur = {}
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                if cur:
                    phys.add((cur.get("physical id"), cur.get("core id")))
                cur = {}
                continue
            k, v = [t.strip() for t in line.split(":", 1)]
            cur[k] = v
            if k == "model name" and model is None:
                model = v
        if cur:
            phys.add((cur.get("physical id"), cur.get("core id")))
    except OSError:
        pass
    return {"model": model, "physical_cores": len(phys) or None, "logical_cpus": os.cpu_count(),
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS"), "OMP_PROC_BIND": os.environ.get("OMP_PROC_BIND")}


def cpu_baseline(pats, p, m, kappa, q, eta, d, x, rows):
    """The oracle, as it stands, on a bounded sample of the same operator: complete
    rows of A_q x for two sample sizes, the fixed cost (the whole-mesh moment pass)
    and the cost per row fitted to them, and the full apply extrapolated to N rows."""
    import numpy as np
    from oracle import oracle as O

    o = O.Oracle(pats, p, m, kappa, g=5, gs=5)
    tree = o.block_tree(eta, d)
    times, ys = [], []
    for nr in (max(1, rows // 4), rows):
        sel = np.unique(np.linspace(0, o.N - 1, nr).astype(int))
        t0 = time.perf_counter()
        y = o.fmm_apply(x, q, eta, d, rows=sel, tree=tree)
        times.append((len(sel), time.perf_counter() - t0))
        ys.append((sel, y))
    (n1, t1), (n2, t2) = times
    per_row = max((t2 - t1) / (n2 - n1), 1e-12)
    fixed = max(t1 - n1 * per_row, 0.0)
    t_full = fixed + o.N * per_row
    return {"value": o.N / t_full, "unit": "DOF/s", "cores": int(O.lib().or_num_threads()), "kind": "oracle",
            "sample": f"complete rows of the same A_q x: {n1} rows in {t1:.2f} s and {n2} rows in {t2:.2f} s; "
                      f"fixed cost {fixed:.2f} s + {per_row * 1e3:.1f} ms per row, extrapolated to the "
                      f"{o.N} rows of one apply ({t_full:.0f} s)",
            "extrapolated": True, "host": host_cpu()}, ys[-1][0], ys[-1][1]


def serve_requests(n, seed, waves=1, sphere_only=False):
    """Seeded request parameters: geometry, jitter seed, level, degree, kappa, waves
    (sphere_only: every request on the sphere, the other draws unchanged)."""
    import numpy as np
    from paper_1807_03097_amd import workloads as W
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0, n)
    out = []
    for i in range(n):
        ri = np.random.default_rng(i)
        geo = "sphere" if ri.random() < 0.5 or sphere_only else "torus"
        m = int(ri.integers(3, 7))
        p = int(ri.integers(1, 3))
        kappa = float(ri.uniform(1.0, 20.0))
        d, pol = W.random_plane_waves(waves, 1000 + i)
        if waves == 1:
            d, pol = d[0], pol[0]
        out.append({"geo": geo, "jitter_seed": i, "m": m, "p": p, "kappa": kappa, "dir": d, "pol": pol,
                    "gap": float(gaps[i])})
    return out


def run_solve(args):
    """Solves of plane-wave scattering problems on the cube-sphere (Fibonacci
    directions, theta polarisation), all right-hand sides at once."""
    import numpy as np
    import torch

    from paper_1807_03097_amd import binding as B
    from paper_1807_03097_amd import workloads as W

    torch.cuda.set_device(0)
    ctx = B.Context(0)
    pats = W.cube_sphere()
    if args.jitter > 0:
        pats = W.jitter(pats, args.jitter, args.jitter_seed)
    geom = B.Geometry(ctx, pats)
    q_level = None
    if args.q_level == "rule":
        plan = B.Operator(geom, args.p, args.level, args.kappa, args.q, args.eta, 5, 5, args.leaf_depth,
                          kappa_cap=args.kappa_cap, plan_only=True)
        q_level = B.degree_rule(plan.info, args.kappa, args.q, set(plan.partition()["far"][:, 0].tolist()))
        plan.close()
    elif args.q_level:
        q_level = [int(v) for v in args.q_level.split(",")]
    t0 = time.perf_counter()
    op = B.Operator(geom, args.p, args.level, args.kappa, args.q, args.eta, 5, 5, args.leaf_depth,
                    kappa_cap=args.kappa_cap, q_level=q_level)
    t_asm = time.perf_counter() - t0
    dirs, pols = W.fibonacci_plane_waves(args.nrhs)
    F = op.rhs_plane_wave(dirs, pols)
    log(f"N={op.N} near entries={op.info.near_nnz} far pairs={op.info.far_pairs} assembled in {t_asm:.2f} s")
    tuned = {}
    if args.autotune:
        t2 = time.perf_counter()
        for pr in sorted({0, args.inner_prec if args.refine else 0}):
            tuned[str(pr)] = op.autotune(args.nrhs, pr)
        log(f"autotuned {tuned} in {time.perf_counter() - t2:.2f} s")
    runs = []
    modes = [("refined" if args.refine else "fp64", args.refine)]
    if args.compare_fp64 and args.refine:
        modes.append(("fp64", False))
    sols = {}
    for name, refine in modes:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        X, st, rc = op.solve(F, tol=args.tol, restart=args.restart, maxit=args.maxit, refine=refine,
                             inner_tol=args.inner_tol, inner_prec=args.inner_prec)
        dt = time.perf_counter() - t1
        sols[name] = X
        iters = [s_[0] for s_ in st]
        log(f"{name}: {dt:.2f} s, rc={rc}, iterations {min(iters)}..{max(iters)}, outer {max(s_[1] for s_ in st)}, "
            f"max relres {max(s_[2] for s_ in st):.2e}")
        runs.append({"mode": name, "seconds": dt, "rc": rc, "solves_per_s": args.nrhs / dt,
                     "iters_max": max(iters), "iters_mean": float(np.mean(iters)),
                     "outer_max": max(s_[1] for s_ in st), "relres_max": max(s_[2] for s_ in st)})
    diff = None
    if "refined" in sols and "fp64" in sols:
        diff = max(float(np.linalg.norm(sols["refined"][c] - sols["fp64"][c]) / np.linalg.norm(sols["fp64"][c]))
                   for c in range(args.nrhs))
        log(f"refined vs FP64 solutions: max relative difference {diff:.2e}")
    prec_name = PREC_NAMES[args.inner_prec]
    out = {
        "metric": "EFIE solves/s",
        "value": runs[0]["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f64" if not args.refine else f"f64 refinement around {prec_name}",
        "data": "synthetic",
        "config": {"workload": f"cube-sphere" + (f" jittered N(0,{args.jitter}^2) seed {args.jitter_seed}"
                                                  if args.jitter > 0 else "")
                               + f", level {args.level}, p={args.p}, kappa={args.kappa}, q={args.q}, "
                               f"eta={args.eta}, {args.nrhs} Fibonacci plane waves, GMRES tol {args.tol}, "
                               f"restart {args.restart}", "n_dof": op.N, "kappa_cap": args.kappa_cap,
                   "q_level": op.q_levels(), "far_pairs": int(op.info.far_pairs)},
        "assemble_s": t_asm,
        "runs": runs,
        "refined_vs_fp64_max_rel_diff": diff,
        "autotuned": tuned or None,
    }
    print(json.dumps(out), flush=True)
    op.close()
    geom.close()
    ctx.close()


def solve_leg(level=6, kappa=16.0, nrhs=64, tol=1e-6, restart=300, inner_prec=4, eta=1.6, d=3):
    """The batched-solve configuration: cube-sphere, level 6, p = 2, kappa = 16, q = 8,
    64 Fibonacci plane waves (theta polarisation), GMRES to a relative residual of 1e-6,
    refined (FP64 residuals around split-BF16 inner solves) and plain FP64; solves/s of
    both, the true FP64 residuals, the difference of the two solutions and the residual
    of that difference (at most the sum of the two residuals: the tolerance-aware bound
    on solutions that agree only to about tol * cond(A))."""
    import numpy as np

    from paper_1807_03097_amd import binding as B
    from paper_1807_03097_amd import workloads as W

    ctx = B.Context(0)
    geom = B.Geometry(ctx, W.cube_sphere())
    t0 = time.perf_counter()
    op = B.Operator(geom, 2, level, kappa, 8, eta, 5, 5, d)
    t_asm = time.perf_counter() - t0
    dirs, pols = W.fibonacci_plane_waves(nrhs)
    F = op.rhs_plane_wave(dirs, pols)
    t1 = time.perf_counter()
    tuned = {str(pr): op.autotune(nrhs, pr) for pr in (0, inner_prec)}
    t_tune = time.perf_counter() - t1
    runs, sols = {}, {}
    for name, refine in (("refined", True), ("fp64", False)):
        t2 = time.perf_counter()
        X, st, rc = op.solve(F, tol=tol, restart=restart, maxit=6000, refine=refine, inner_tol=1e-4,
                             inner_prec=inner_prec)
        dt = time.perf_counter() - t2
        sols[name] = X
        runs[name] = {"seconds": dt, "solves_per_s": nrhs / dt, "rc": rc, "iters_max": max(c[0] for c in st),
                      "relres_fp64_max": max(c[2] for c in st)}
        log(f"solve leg {name}: {dt:.2f} s ({nrhs / dt:.2f} solves/s), iterations <= {runs[name]['iters_max']}, "
            f"max FP64 relres {runs[name]['relres_fp64_max']:.2e}")
    Dx = sols["refined"] - sols["fp64"]
    AD = op.apply(np.ascontiguousarray(Dx))
    diff = max(float(np.linalg.norm(Dx[c]) / np.linalg.norm(sols["fp64"][c])) for c in range(nrhs))
    res_diff = max(float(np.linalg.norm(AD[c]) / np.linalg.norm(F[c])) for c in range(nrhs))
    bound = runs["refined"]["relres_fp64_max"] + runs["fp64"]["relres_fp64_max"]
    log(f"solve leg: refined vs FP64 solutions {diff:.2e}; residual of the difference {res_diff:.2e} "
        f"(bound {bound:.2e}); implied cond(A) >= {diff / max(res_diff, 1e-300):.0f}")
    out = {"workload": f"cube-sphere level {level}, p=2, N={op.N}, kappa={kappa}, q=8, eta={eta}, d={d}, "
                       f"{nrhs} Fibonacci plane waves, GMRES tol {tol}, restart {restart}, "
                       f"refined inner precision {PREC_NAMES[inner_prec]}",
           "assemble_s": t_asm, "autotune_s": t_tune, "autotuned": tuned, "refined": runs["refined"],
           "fp64": runs["fp64"], "speedup_refined_over_fp64": runs["fp64"]["seconds"] / runs["refined"]["seconds"],
           "refined_vs_fp64_max_rel_diff": diff, "residual_of_difference_max": res_diff,
           "residual_bound": bound, "difference_within_bound": bool(res_diff <= 1.01 * bound)}
    op.close()
    geom.close()
    ctx.close()
    return out


def run_serving(args):
    import numpy as np
    import torch

    from paper_1807_03097_amd import binding as B
    from paper_1807_03097_amd import workloads as W

    torch.cuda.set_device(0)
    ctx = B.Context(0)
    reqs = serve_requests(args.requests, 4, args.waves, args.sphere_only)
    restart = args.srv_restart
    if args.same_object:
        for rq in reqs[1:]:
            rq.update({k: reqs[0][k] for k in ("geo", "jitter_seed", "m", "p", "kappa")})
    geoms = []
    for k, rq in enumerate(reqs):
        if args.same_object and k > 0:
            geoms.append(geoms[0])
            continue
        base = W.cube_sphere() if rq["geo"] == "sphere" else W.torus()
        geoms.append(B.Geometry(ctx, W.jitter(base, 0.01, rq["jitter_seed"])))
    srv = B.Server(ctx, args.workers, max_merge=args.max_merge)
    t0 = time.perf_counter()
    arrival, tickets = [], []
    t_next = 0.0
    for k, rq in enumerate(reqs):
        t_next += rq["gap"] / args.rate
        dt = t0 + t_next - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        arrival.append(time.perf_counter() - t0)
        tickets.append(srv.submit(geoms[k], rq["p"], rq["m"], rq["kappa"], rq["dir"], rq["pol"], q=8, eta=args.eta,
                                  tol=1e-6, restart=restart, maxit=args.maxit, refine=args.refine,
                                  inner_tol=1e-4, inner_prec=args.inner_prec))
    stats = []
    for k, t in enumerate(tickets):
        stats.append(srv.wait(t))
        log(f"done {k + 1}/{len(tickets)} at {time.perf_counter() - t0:.1f} s")
    srv.close()
    # server clock starts at Server(); t0 was taken right after it
    lat = np.array([st["t_done"] - a for st, a in zip(stats, arrival)])
    done = [st for st in stats if st["rc"] == 0]
    capped = [st for st in stats if st["rc"] == -3]
    span = max(st["t_done"] for st in stats) - min(arrival)
    for k, (rq, st) in enumerate(zip(reqs, stats)):
        log(f"req {k:3d} {rq['geo']:6s} m={rq['m']} p={rq['p']} kappa={rq['kappa']:5.2f} N={st['n_dof']:6d} "
            f"iters={st['iters']:5d} relres={st['relres']:.1e} rc={st['rc']} asm={st['assemble_s']:.3f}s "
            f"solve={st['solve_s']:.3f}s latency={lat[k]:.3f}s merged={st['merged']} reused={st['reused']}")
    out = {
        "metric": "EFIE serving solves/s",
        "value": len(done) * args.waves / span,
        "unit": "solves/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f64" if not args.refine else PREC_NAMES[args.inner_prec] + " + f64 refinement",
        "data": "synthetic",
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "completed": len(done),
        "capped_at_maxit": len(capped),
        "requests": len(stats),
        "span_s": span,
        "config": {"workload": f"{len(reqs)} solves, exponential arrivals at {args.rate}/s (seed 4); "
                               + ("one object (the first request's: " + f"{reqs[0]['geo']} m={reqs[0]['m']} "
                                  f"p={reqs[0]['p']} kappa={reqs[0]['kappa']:.2f}), random plane waves; "
                                  if args.same_object else "")
                               + ("sphere" if args.sphere_only else "sphere or torus") + ", control-point jitter N(0, 0.01^2), m in 3..6, p in 1..2, kappa in [1, 20], "
                               f"q=8, eta={args.eta}, {args.waves} plane wave(s) per request, GMRES tol 1e-6, "
                               f"restart {restart}, maxit {args.maxit}",
                   "workers": args.workers, "refine": bool(args.refine), "waves_per_request": args.waves,
                   "max_merge": args.max_merge, "same_object": bool(args.same_object)},
        "merged_requests": int(sum(1 for st in stats if st["merged"] > 1)),
        "reused_operator": int(sum(1 for st in stats if st["reused"])),
        "requests_s": len(done) / span,
        "total_iters": int(sum(st["iters"] for st in stats)),
        "total_dof": int(sum(st["n_dof"] for st in stats)),
    }
    print(json.dumps(out), flush=True)
    for g in set(geoms):
        g.close()
    ctx.close()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU (one operator per device); "
                                   "sharding over several GPUs is not built"}))
        sys.exit(2)
    if args.mode == "serve":
        run_serving(args)
        return
    if args.mode == "solve":
        run_solve(args)
        return
    import numpy as np
    import torch

    from paper_1807_03097_amd import binding as B
    from paper_1807_03097_amd import workloads as W

    p, m, kappa, q, eta, d = 2, args.level, args.kappa, args.q, args.eta, args.leaf_depth
    pats = W.cube_sphere()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.copy_probe_mb > 0:
        src_buf = torch.empty(args.copy_probe_mb << 20, dtype=torch.uint8, device=dev)
        dst_buf = torch.empty_like(src_buf)
        dst_buf.copy_(src_buf)
        torch.cuda.synchronize()
        del src_buf, dst_buf
    ctx = B.Context(0, stream.cuda_stream)
    geom = B.Geometry(ctx, pats)
    q_level = None
    if args.q_level == "rule":
        plan = B.Operator(geom, p, m, kappa, q, eta, 5, 5, d, kappa_cap=args.kappa_cap, plan_only=True)
        q_level = B.degree_rule(plan.info, kappa, q, set(plan.partition()["far"][:, 0].tolist()))
        plan.close()
    elif args.q_level:
        q_level = [int(v) for v in args.q_level.split(",")]
    t0 = time.perf_counter()
    op = B.Operator(geom, p, m, kappa, q, eta, 5, 5, d, store_coupling=args.store_coupling,
                    kappa_cap=args.kappa_cap, q_level=q_level)
    t_asm = time.perf_counter() - t0
    info = op.info
    far_per_level = np.bincount(op.partition()["far"][:, 0], minlength=info.leaf_level + 1).tolist() \
        if info.far_pairs else [0] * (info.leaf_level + 1)
    q_used = op.q_levels()
    N = op.N
    log(f"assembled N={N} nnz={info.near_nnz} far={info.far_pairs} near_leaf={info.near_leaf_pairs} "
        f"L={info.leaf_level} in {t_asm:.2f} s")
    r = args.nrhs
    xh = W.random_coeffs(N, 0, nrhs=r)
    x = torch.from_numpy(xh).to(dev)
    y = torch.empty_like(x)
    for _ in range(args.warmup):
        op.apply(x, y, prec=args.prec)
    torch.cuda.synchronize()
    tuned = None
    if args.autotune:
        tuned = op.autotune(r, args.prec)
        log(f"autotuned {tuned}")
        for _ in range(args.warmup):
            op.apply(x, y, prec=args.prec)
        torch.cuda.synchronize()

    # timed region: the boundaries of the block pass and of the coupling kernel only
    # (four timing events per apply); the full stage breakdown comes from the
    # isolated pass below
    op.set_profiling(2)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    w0 = time.perf_counter()
    for _ in range(args.steps):
        op.apply(x, y, prec=args.prec)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = ev0.elapsed_time(ev1) / args.steps
    stages = op.stage_times()
    names = ["p2m", "m2m", "m2l", "m2l_reduce", "l2l", "near_spmv", "l2p", "near_blk", "m2l_kernel"]
    st = {n: float(stages[names.index(n)]) for n in ("near_blk", "m2l_kernel")}
    log("timed kernels ms: " + " ".join(f"{k}={v:.4f}" for k, v in st.items())
        + f"  step={ms_step:.4f} ms wall/step={1e3 * wall / args.steps:.4f}")

    # roofline of the dominant kernel (durations from the timed region)
    near_once = r == 1 and info.near_distinct > 0 and os.environ.get("IGE_NEAR_COMPACT", "1") != "0"
    traffic_ref = load_traffic(r, "k_near_cmp" if near_once else "k_near_blk")

    Qc = (q + 1) ** 2
    Qpc = 32 * ((Qc + 31) // 32)
    # FP64 applies of 8 or more columns: coupling on the FP64 matrix cores (stored blocks)
    f64mx = (args.prec == 0 and r >= 8 and Qpc <= 128 and info.far_pairs > 0
             and os.environ.get("IGE_M2L_F64") != "generate")

    def roofline_coupling(stage_ms):
        """Matrix-core coupling (r > 1, BF16 precisions; FP64 with 8 or more columns):
        issued matrix-core operations of the real product [[Gr,-Gi],[Gi,Gr]] . [Re V; Im V]
        over padded 2Qp x 2Qp blocks and column chunks, over the kernel's own time."""
        if not (f64mx or (args.prec in (2, 3, 4) and r > 1)):
            return None
        Q, Qp = Qc, Qpc
        MT = Qp // 16
        if f64mx:
            split, cap, kern, peak = 1, 128, "k_m2l_md", FP64_MFMA_PEAK_TFLOPS
        else:
            split = 1 if args.prec == 2 else 3
            cap = (64 if split == 3 else 128) if MT >= 8 else (128 if MT >= 6 else 256)
            kern, peak = "k_m2l_mx", BF16_MFMA_PEAK_TFLOPS
        ncol = 16
        while ncol < 4 * r and ncol < cap:
            ncol *= 2
        if not f64mx and ncol >= 128 and os.environ.get("IGE_M2L_RM", "1") != "0":
            kern = "k_m2l_mxr"   # wide chunks: real and imaginary row tiles in one wave
        nchunk = -(-r // (ncol // 4))
        issued = info.far_pairs * nchunk * 2.0 * (2 * Qp) * (2 * Qp) * ncol * split
        useful = info.far_pairs * 8.0 * Q * Q * 4 * r
        t_ms = stage_ms["m2l_kernel"]
        ach = issued / (t_ms * 1e-3) / 1e12
        return {"kernel": kern, "bound": "mfma", "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak, "traffic": None,
                "useful_tflops": useful / (t_ms * 1e-3) / 1e12, "issued_flop": issued, "avg_ms": t_ms}

    def roofline(stage_ms, dom=None):
        # the dominant kernel: the near-field block pass or the coupling kernel
        if dom is None:
            dom = "near_spmv" if stage_ms["near_blk"] >= stage_ms["m2l_kernel"] else "m2l"
        if dom == "m2l" and (f64mx or (args.prec in (2, 3, 4) and r > 1)):
            return roofline_coupling(stage_ms)   # the matrix-core coupling kernel
        Q = (q + 1) ** 2
        if dom == "near_spmv" and r > 1:
            # many columns: matrix-core products over every ordered leaf pair (block and
            # transposed block), the whole near-field stage timed (operands, product, sum)
            s_el = 2 ** (m - info.leaf_level)
            W_ = s_el + p
            nF = 2 * W_ * (W_ - 1)
            t_ms = stage_ms["near_blk"]
            if args.prec == 4:
                Qn = 32 * ((nF + 31) // 32)
                ncol = 64 if r > 32 else (32 if r > 16 else 16)
                issued = info.near_leaf_pairs * (-(-r // ncol)) * 12 * 2.0 * Qn * Qn * ncol
                ach = issued / (t_ms * 1e-3) / 1e12
                return {"kernel": "k_near_bx", "bound": "mfma", "achieved": ach, "peak": BF16_MFMA_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": ach / BF16_MFMA_PEAK_TFLOPS, "traffic": None,
                        "issued_flop": issued, "avg_ms": t_ms}
            flops = info.near_leaf_pairs * nF * nF * 8.0 * r
            ach = flops / (t_ms * 1e-3) / 1e12
            out = {"kernel": "k_near_md" if r >= 56 else "k_near_mfma", "bound": "mfma", "achieved": ach,
                   "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP64_MFMA_PEAK_TFLOPS,
                   "traffic": None, "flop": flops, "avg_ms": t_ms}
            if r >= 56:
                # real products over the padded blocks: (2 Qn) x (2 Qn) by 64 columns per chunk
                Qn = 32 * ((nF + 31) // 32)
                out["issued_flop"] = info.near_leaf_pairs * (-(-r // 64)) * 2.0 * (2 * Qn) ** 2 * 64
            return out
        if dom == "near_spmv" and near_once:
            # the method's bytes: every distinct entry of the symmetric near-field matrix
            # (16 B) once, x read and y written once
            alg = info.near_distinct * 16 + 2 * N * 16
            t_ms = stage_ms["near_blk"]
            achieved = alg / (t_ms * 1e-3) / 1e9
            kname = "k_near_cmp1" if os.environ.get("IGE_NEAR_ONE", "1") != "0" else "k_near_cmp"
            return {"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_ref,
                    "traffic_over_algorithmic": None if traffic_ref is None else traffic_ref / alg,
                    "algorithmic_bytes": int(alg), "near_distinct_entries": int(info.near_distinct),
                    "avg_ms": t_ms}
        if dom == "near_spmv":
            # the block pass: stored block entries (16 B each) streamed once per pass
            # of up to 4 columns, x read once per column
            passes = 1 if r == 1 else (r + 3) // 4
            traffic_alg = info.near_nnz * 16 * passes + N * 16 * r
            t_ms = stage_ms["near_blk"]
            achieved = traffic_alg / (t_ms * 1e-3) / 1e9
            return {"kernel": "k_near_blk", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_ref,
                    "algorithmic_bytes": int(traffic_alg), "avg_ms": t_ms}
        # M2L: per interpolation-node pair the kernel G(|x - x'|) (distance 8,
        # sqrt/rcp/sin/cos 4, scaling 2 FP64 operations) and four complex
        # multiply-adds per right-hand side (32 operations each)
        entries = sum(nf * (ql + 1) ** 4 for nf, ql in zip(far_per_level, q_used))
        flops = entries * (14.0 + 32.0 * r)
        t_ms = stage_ms["m2l_kernel"]
        achieved = flops / (t_ms * 1e-3) / 1e12
        return {"kernel": "k_m2l", "bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                "node_pairs": int(entries), "avg_ms": t_ms}

    roof = roofline(st)
    roof_cpl = roofline_coupling(st)

    def measured(rf):
        """the same fraction against the device's achievable peak (the library's probes)"""
        if rf is None:
            return rf
        m = None
        if rf["bound"] == "hbm":
            m = peaks["hbm_GBps"]
        elif rf["bound"] == "mfma":
            m = peaks["f64_mfma_TFLOPs"] if rf["kernel"] in ("k_m2l_md", "k_near_md", "k_near_mfma") \
                else peaks["bf16_mfma_TFLOPs"]
        rf["peak_measured"] = m
        rf["frac_of_measured"] = None if m is None else rf["achieved"] / m
        return rf

    # error of a reduced-precision apply against the FP64 apply of the same columns
    err_fp64 = None
    if args.prec != 0:
        y64 = torch.empty_like(x)
        op.apply(x, y64, prec=0)
        torch.cuda.synchronize()
        err_fp64 = float(torch.linalg.vector_norm(y - y64) / torch.linalg.vector_norm(y64))
        log(f"relative error vs the FP64 apply: {err_fp64:.2e}")
    # the same kernels timed in isolation (stages in order on one stream)
    op.set_overlap(False)
    op.set_profiling(True)
    for _ in range(min(args.steps, 20)):
        op.apply(x, y, prec=args.prec)
    torch.cuda.synchronize()
    st_iso = {n: float(v) for n, v in zip(names, op.stage_times())}
    op.set_profiling(False)
    op.set_overlap(True)
    # achievable peaks of this device (the library's own copy and matrix-core probes),
    # taken after the timed and the isolated passes so that they cannot disturb them
    peaks = {"hbm_GBps": B.ige_peak_probe(ctx.h, B.IGE_PROBE_HBM),
             "bf16_mfma_TFLOPs": B.ige_peak_probe(ctx.h, B.IGE_PROBE_MFMA_BF16),
             "f64_mfma_TFLOPs": B.ige_peak_probe(ctx.h, B.IGE_PROBE_MFMA_F64)}
    log("measured peaks: " + " ".join(f"{k}={v:.1f}" for k, v in peaks.items()))
    roof, roof_cpl = measured(roof), measured(roof_cpl)
    roof_iso = measured(roofline(st_iso))
    # the near-field product alone on the device (stages in order on one stream)
    roof_near_iso = measured(roofline(st_iso, dom="near_spmv"))
    log("isolated stage ms: " + " ".join(f"{k}={v:.4f}" for k, v in st_iso.items()))

    # parity spot check against the oracle (sampled rows) + CPU baseline
    yh = y.cpu().numpy() if r == 1 else y[0].cpu().numpy()
    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        cpu, sel, yo = cpu_baseline(pats, p, m, kappa, q, eta, d, xh if r == 1 else xh[0], args.cpu_rows)
        parity = float(np.linalg.norm(yh[sel] - yo) / np.linalg.norm(yo))
        log(f"cpu baseline {cpu['value']:.1f} DOF/s on {cpu['cores']} threads; sampled rel.err vs oracle {parity:.2e}")

    solve = None
    if not args.no_solve and args.level == 5 and r == 1 and args.prec == 0:
        op.close()
        geom.close()
        ctx.close()
        op = geom = ctx = None
        solve = solve_leg()
    out = {
        "metric": "EFIE FMM matvec DOF/s",
        "value": N * r / (ms_step * 1e-3),
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ["f64", "f64 (f32 coupling)", "f64 (bf16 matrix-core coupling)",
                  "f64 (split-bf16 matrix-core coupling)",
                  "f64 moments/transfers (split-bf16 coupling and near field)"][args.prec],
        "data": "synthetic",
        "config": {"workload": f"FMM matvec: 6-patch NURBS sphere, level {m}, p={p}, kappa={kappa}, q={q}, "
                               f"5x5 Gauss near field, x ~ N(0,1)+iN(0,1) seed 0",
                   "n_dof": N, "nrhs": r, "eta": eta, "leaf_depth": d, "near_nnz": int(info.near_nnz),
                   "store_coupling": args.store_coupling, "kappa_cap": args.kappa_cap, "q_level": q_used,
                   "far_pairs": int(info.far_pairs), "far_pairs_per_level": far_per_level,
                   "parallelism": "single GPU"},
        "timed_kernel_ms": st,
        "assemble_s": t_asm,
        "superspace_dof_per_s": 2 * len(pats) * ((1 << m) + p) * ((1 << m) + p - 1) * r / (ms_step * 1e-3),
        "peaks_measured": peaks,
        "roofline": roof,
        "roofline_isolated": roof_iso,
        "roofline_near_isolated": roof_near_iso,
        "roofline_coupling": roof_cpl,
        "rel_err_vs_fp64": err_fp64,
        "autotuned": tuned,
        "stage_ms_isolated": st_iso,
        "cpu_baseline": cpu,
        "parity_sampled_rel_err": parity,
        "solve_c3": solve,
    }
    print(json.dumps(out), flush=True)
    for h in (op, geom, ctx):
        if h is not None:
            h.close()


if __name__ == "__main__":
    main()
