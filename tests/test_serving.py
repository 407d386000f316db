"""Serving loop: many independent scattering solves on one device.

Each request is a full solve (assembly, plane-wave right-hand side, GMRES); the
server runs several at once on separate streams and admits them by their planned
device footprint.  Checks: results equal direct solves bit for bit, admission never exceeds the
budget, an oversized request is refused, and a request's solution does not depend
on what else runs beside it (bit for bit).
"""
import numpy as np
import pytest

from paper_1807_03097_amd import workloads as W

# (geometry, p, m, kappa, q, eta, leaf depth, plane-wave seed)
REQS = [
    ("sphere", 1, 2, 2.0, 6, 1.0, 0, 11),
    ("torus", 1, 2, 3.0, 6, 1.0, 0, 12),
    ("sphere", 2, 3, 5.0, 6, 1.0, 1, 13),
    ("jittered", 1, 3, 4.0, 6, 1.0, 1, 14),
    ("torus", 2, 2, 6.0, 6, 1.0, 1, 15),
    ("sphere", 1, 3, 1.5, 5, 1.0, 1, 16),
]
TOL = 1e-10


def _same(x, ref):
    """Two solves of the same request give the same bits: assembly, applies and
    GMRES sum in fixed orders, whatever else shares the device."""
    return x.shape == ref.shape and np.array_equal(x.view(np.uint64), ref.view(np.uint64))


def _geom(B, ctx, name):
    pats = {"sphere": W.cube_sphere, "torus": W.torus,
            "jittered": lambda: W.jitter(W.cube_sphere(), 0.01, 3)}[name]()
    return B.Geometry(ctx, pats)


def _wave(seed):
    d, pol = W.random_plane_waves(1, seed)
    return d[0], pol[0]


def test_server_refuses_host_context():
    from paper_1807_03097_amd import binding as B
    c = B.Context(-1)
    with pytest.raises(B.IgeError):
        B.Server(c, 2)
    c.close()


@pytest.mark.gpu
def test_server_matches_direct_solves_and_budget():
    from paper_1807_03097_amd import binding as B
    ctx = B.Context(0)
    geoms = {n: _geom(B, ctx, n) for n in ("sphere", "torus", "jittered")}
    # direct solves on the caller's context
    ref, fps = [], []
    for (n, p, m, kap, q, eta, d, seed) in REQS:
        op = B.Operator(geoms[n], p, m, kap, q, eta, 5, 5, d)
        di, pol = _wave(seed)
        f = op.rhs_plane_wave(di, pol)[0]
        x, st, rc = op.solve(f, tol=TOL, restart=300, maxit=3000)
        assert rc == 0
        ref.append(x)
        op.close()
    # the server, with a budget that holds about two requests at a time
    probe = B.Server(ctx, 1)
    fps = []
    for (n, p, m, kap, q, eta, d, seed) in REQS:
        di, pol = _wave(seed)
        t = probe.submit(geoms[n], p, m, kap, di, pol, q=q, eta=eta, leaf_depth=d, tol=TOL, restart=300, maxit=3000)
        fps.append(probe.wait(t)["footprint"])
    probe.close()
    budget = int(max(fps) * 2.2)
    srv = B.Server(ctx, 4, budget)
    tickets = []
    for (n, p, m, kap, q, eta, d, seed) in REQS:
        di, pol = _wave(seed)
        tickets.append(srv.submit(geoms[n], p, m, kap, di, pol, q=q, eta=eta, leaf_depth=d, tol=TOL,
                                  restart=300, maxit=3000))
    stats = []
    for k, t in enumerate(tickets):
        x, st = srv.result(t)
        stats.append(st)
        err = np.linalg.norm(x - ref[k]) / np.linalg.norm(ref[k])
        print(f"request {k}: N={st['n_dof']} iters={st['iters']} relres={st['relres']:.1e} "
              f"fp={st['footprint'] / 2**20:.1f} MiB vs direct {err:.1e}", flush=True)
        assert st["rc"] == 0 and st["relres"] <= TOL * 1.05
        assert _same(x, ref[k]), err
    # admission: requests running at the same time fit the budget together
    for i in range(len(stats)):
        live = [j for j in range(len(stats))
                if stats[j]["t_start"] < stats[i]["t_done"] and stats[i]["t_start"] < stats[j]["t_done"]]
        # every set of overlapping requests at the start of request i
        at = [j for j in live if stats[j]["t_start"] <= stats[i]["t_start"] < stats[j]["t_done"]]
        assert sum(stats[j]["footprint"] for j in at) <= budget
    assert max(st["t_start"] for st in stats) > 0.0
    srv.close()
    # a request larger than the budget is refused at submission
    tiny = B.Server(ctx, 1, 1 << 20)
    n, p, m, kap, q, eta, d, seed = REQS[2]
    di, pol = _wave(seed)
    with pytest.raises(B.IgeError):
        tiny.submit(geoms[n], p, m, kap, di, pol, q=q, eta=eta, leaf_depth=d)
    tiny.close()
    for g in geoms.values():
        g.close()
    ctx.close()


@pytest.mark.gpu
def test_solution_alone_equals_solution_in_mix():
    """The same request solved alone and among five others (four workers)."""
    from paper_1807_03097_amd import binding as B
    ctx = B.Context(0)
    geoms = {n: _geom(B, ctx, n) for n in ("sphere", "torus", "jittered")}
    n, p, m, kap, q, eta, d, seed = REQS[2]
    di, pol = _wave(seed)
    alone = B.Server(ctx, 1)
    t = alone.submit(geoms[n], p, m, kap, di, pol, q=q, eta=eta, leaf_depth=d, tol=1e-8, restart=200)
    xa, sa = alone.result(t)
    alone.close()
    mix = B.Server(ctx, 4)
    ts = []
    for k, (n2, p2, m2, kap2, q2, eta2, d2, seed2) in enumerate(REQS):
        dd, pp = _wave(seed2)
        ts.append(mix.submit(geoms[n2], p2, m2, kap2, dd, pp, q=q2, eta=eta2, leaf_depth=d2, tol=1e-8, restart=200))
    xm, sm = mix.result(ts[2])
    for t2 in ts:
        mix.wait(t2)
    mix.close()
    err = np.linalg.norm(xm - xa) / np.linalg.norm(xa)
    print(f"alone iters={sa['iters']} mix iters={sm['iters']} difference {err:.1e}", flush=True)
    assert sa["rc"] == 0 and sm["rc"] == 0
    assert sa["iters"] == sm["iters"] and _same(xm, xa), err
    for g in geoms.values():
        g.close()
    ctx.close()


@pytest.mark.gpu
@pytest.mark.parametrize("inner", [3, 4], ids=["split-coupling", "split-coupling-and-near"])
def test_refined_requests_meet_the_fp64_tolerance(inner):
    """Requests solved by FP64 refinement around lower-precision inner solves (several
    at once) reach the tolerance on the FP64 operator and the FP64 solution."""
    from paper_1807_03097_amd import binding as B
    ctx = B.Context(0)
    geoms = {n: _geom(B, ctx, n) for n in ("sphere", "torus", "jittered")}
    reqs = REQS[:4]
    ref = []
    for (n, p, m, kap, q, eta, d, seed) in reqs:
        op = B.Operator(geoms[n], p, m, kap, q, eta, 5, 5, d)
        di, pol = _wave(seed)
        x, st, rc = op.solve(op.rhs_plane_wave(di, pol)[0], tol=TOL, restart=300, maxit=3000)
        assert rc == 0
        ref.append(x)
        op.close()
    srv = B.Server(ctx, 3)
    ts = []
    for (n, p, m, kap, q, eta, d, seed) in reqs:
        di, pol = _wave(seed)
        ts.append(srv.submit(geoms[n], p, m, kap, di, pol, q=q, eta=eta, leaf_depth=d, tol=TOL, restart=300,
                             maxit=6000, refine=True, inner_tol=1e-4, inner_prec=inner))
    for k, t in enumerate(ts):
        x, st = srv.result(t)
        err = np.linalg.norm(x - ref[k]) / np.linalg.norm(ref[k])
        print(f"request {k}: inner {inner} iters={st['iters']} relres={st['relres']:.1e} vs FP64 {err:.1e}",
              flush=True)
        assert st["rc"] == 0 and st["relres"] <= TOL * 1.05
        assert err <= 1e-6
    srv.close()
    for g in geoms.values():
        g.close()
    ctx.close()


@pytest.mark.gpu
def test_multi_wave_requests_match_direct_solves():
    """Requests of several plane waves (one operator, all waves solved together, the
    batched kernels from two waves and the matrix-core ones from eight) equal direct
    solves of the same columns, beside single-wave requests; a refined nine-wave
    request (split-BF16 coupling and near field inside) reaches the FP64 tolerance and
    the FP64 solution; the planned footprint grows with the waves."""
    from paper_1807_03097_amd import binding as B
    ctx = B.Context(0)
    geoms = {n: _geom(B, ctx, n) for n in ("sphere", "torus", "jittered")}
    cases = [(REQS[2], 3, False), (REQS[3], 9, False), (REQS[4], 2, False), (REQS[2], 9, True)]
    ref = []
    for (n, p, m, kap, q, eta, d, seed), nw, _ in cases:
        op = B.Operator(geoms[n], p, m, kap, q, eta, 5, 5, d)
        dirs, pols = W.random_plane_waves(nw, seed)
        X, st, rc = op.solve(op.rhs_plane_wave(dirs, pols), tol=TOL, restart=300, maxit=3000)
        assert rc == 0
        ref.append(X)
        op.close()
    srv = B.Server(ctx, 3)
    ts, singles = [], []
    for ((n, p, m, kap, q, eta, d, seed), nw, refine) in cases:
        dirs, pols = W.random_plane_waves(nw, seed)
        ts.append(srv.submit(geoms[n], p, m, kap, dirs, pols, q=q, eta=eta, leaf_depth=d, tol=TOL, restart=300,
                             maxit=6000, refine=refine, inner_tol=1e-4, inner_prec=B.IGE_BF16X3_ALL))
        di, pol = _wave(seed)
        singles.append(srv.submit(geoms[n], p, m, kap, di, pol, q=q, eta=eta, leaf_depth=d, tol=TOL, restart=300))
    fp = {}
    for k, (t, (rq, nw, refine)) in enumerate(zip(ts, cases)):
        X, st = srv.result(t)
        assert st["n_waves"] == nw and X.shape == (nw, st["n_dof"])
        err = max(np.linalg.norm(X[c] - ref[k][c]) / np.linalg.norm(ref[k][c]) for c in range(nw))
        print(f"request {k}: {nw} waves refine={refine} iters={st['iters']} relres={st['relres']:.1e} "
              f"vs direct {err:.1e} footprint {st['footprint'] / 2**20:.0f} MiB", flush=True)
        assert st["rc"] == 0 and st["relres"] <= TOL * 1.05
        assert err <= 1e-6 if refine else _same(X, ref[k]), err
        fp[(rq[0], rq[2], nw, refine)] = st["footprint"]
    for t in singles:
        x1, s1 = srv.result(t)
        assert s1["rc"] == 0 and s1["n_waves"] == 1 and x1.shape == (s1["n_dof"],)
    srv.close()
    assert fp[("sphere", 3, 9, True)] > fp[("sphere", 3, 3, False)]
    for g in geoms.values():
        g.close()
    ctx.close()


@pytest.mark.gpu
def test_waiting_requests_on_one_operator_are_merged_and_the_operator_stays_resident():
    """Continuous batching: single-wave requests on the same object that wait behind a
    running one are solved together as one many-column system; each meets the FP64
    tolerance and agrees with its direct solve within the tolerance-aware bound (the
    residual of the difference is at most the sum of the two residuals).  A later
    request on the same object runs on the resident operator (no assembly) and equals
    its direct solve bit for bit."""
    from paper_1807_03097_amd import binding as B
    ctx = B.Context(0)
    geoms = {n: _geom(B, ctx, n) for n in ("sphere", "torus")}
    n, p, m, kap, q, eta, d, _ = REQS[2]
    seeds = [21, 22, 23, 24, 25]
    op = B.Operator(geoms[n], p, m, kap, q, eta, 5, 5, d)
    direct = {}
    for sd in seeds:
        di, pol = _wave(sd)
        f = op.rhs_plane_wave(di, pol)[0]
        x, st, rc = op.solve(f, tol=TOL, restart=300, maxit=3000)
        assert rc == 0
        direct[sd] = (x, f)
    srv = B.Server(ctx, 1, max_merge=8)
    # a blocker on another object keeps the single worker busy while the others queue
    nb, pb, mb, kb, qb, eb, db, sb = REQS[4]
    db_, pol_ = _wave(sb)
    tb = srv.submit(geoms[nb], pb, mb, kb, db_, pol_, q=qb, eta=eb, leaf_depth=db, tol=TOL, restart=300, maxit=3000)
    ts = []
    for sd in seeds[:4]:
        di, pol = _wave(sd)
        ts.append(srv.submit(geoms[n], p, m, kap, di, pol, q=q, eta=eta, leaf_depth=d, tol=TOL, restart=300,
                             maxit=3000))
    srv.wait(tb)
    for sd, t in zip(seeds[:4], ts):
        x, st = srv.result(t)
        xd, f = direct[sd]
        dx = x - xd
        res_diff = np.linalg.norm(op.apply(dx)) / np.linalg.norm(f)
        print(f"seed {sd}: merged {st['merged']} reused {st['reused']} iters {st['iters']} relres {st['relres']:.1e} "
              f"vs direct {np.linalg.norm(dx) / np.linalg.norm(xd):.1e}, residual of the difference {res_diff:.1e}",
              flush=True)
        assert st["rc"] == 0 and st["relres"] <= TOL * 1.05
        assert res_diff <= 2.1 * TOL
    stats = [srv.wait(t) for t in ts]
    assert max(s["merged"] for s in stats) >= 2
    # the same object again, alone: resident operator, same bits as the direct solve
    di, pol = _wave(seeds[4])
    t5 = srv.submit(geoms[n], p, m, kap, di, pol, q=q, eta=eta, leaf_depth=d, tol=TOL, restart=300, maxit=3000)
    x5, s5 = srv.result(t5)
    print(f"resident: reused {s5['reused']} assemble {s5['assemble_s']:.3f} s merged {s5['merged']}", flush=True)
    assert s5["reused"] == 1 and s5["assemble_s"] == 0.0 and s5["merged"] == 1
    assert _same(x5, direct[seeds[4]][0])
    srv.close()
    op.close()
    for g in geoms.values():
        g.close()
    ctx.close()
