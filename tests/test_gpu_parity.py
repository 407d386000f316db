"""Parity of the HIP path with the CPU oracle (FP64).

Every test builds the operator through the C ABI on device 0 and compares its
output with the oracle on the same seeded inputs.  Bar: relative 2-norm error
<= 1e-12 for the FP64 operator (matvec), the right-hand side and the element-pair
quadrature; GMRES solutions within tol * cond(A) of LAPACK / the oracle.
"""
import sys

import numpy as np
import pytest

from paper_1807_03097_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1807_03097_amd import binding as B
    c = B.Context(0)
    yield c
    c.close()


def _geom(name):
    return {"sphere": W.cube_sphere, "torus": W.torus, "cube": W.flat_cube,
            "jittered": lambda: W.jitter(W.cube_sphere(), 0.01, 3),
            "multispan": lambda: [W.refine_patch_knots(pt, 2, 2) for pt in W.cube_sphere()]}[name]()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = [
    # geometry, p, m, kappa, q, eta, leaf depth, g, gs
    ("sphere", 1, 2, 1.0, 8, 0.0, -1, 5, 5),      # dense: everything near field
    ("sphere", 1, 0, 2.0, 4, 0.0, -1, 4, 4),      # one element per patch
    ("sphere", 2, 3, 8.0, 8, 1.6, 1, 5, 5),       # three far levels, ragged leaf blocks
    ("sphere", 2, 4, 8.0, 8, 1.0, 2, 5, 5),
    ("torus", 2, 3, 4.0, 6, 1.0, 1, 5, 4),
    ("cube", 1, 3, 3.0, 5, 1.0, 1, 4, 5),         # flat patches, sharp edges and corners
    ("jittered", 2, 3, 6.0, 7, 1.0, 1, 5, 5),
    ("multispan", 2, 3, 5.0, 6, 1.0, 1, 5, 5),    # NURBS input with interior knots
    ("sphere", 1, 3, 2.0, 3, 1.0, 0, 3, 6),       # leaf = element, low q
    ("sphere", 2, 3, 8.0, 8, 1.6, 3, 5, 5),       # leaf = patch: far field only between patches
    ("sphere", 3, 3, 6.0, 6, 1.0, 1, 5, 5),       # cubic splines (24 local functions per element)
    ("sphere", 4, 2, 4.0, 8, 1.0, 1, 5, 5),       # quartic splines (40 local functions per element)
    ("jittered", 4, 3, 6.0, 8, 1.6, 1, 5, 5),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-p{c[1]}-m{c[2]}-eta{c[5]}-d{c[6]}" for c in CASES])
def test_apply_matches_oracle(oracle_mod, ctx, case):
    from paper_1807_03097_amd import binding as B
    name, p, m, kappa, q, eta, d, g, gs = case
    _say(f"case {case}")
    pats = _geom(name)
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, p, m, kappa, q, eta, g, gs, d)
    x = W.random_coeffs(op.N, 0)
    y = op.apply(x)
    o = oracle_mod.Oracle(pats, p, m, kappa, g=g, gs=gs)
    dd = d if d >= 0 else int(np.ceil(np.log2((q + 1) / (p + 1)) - 1e-12))
    yo = o.fmm_apply(x, q, eta, dd)
    err = _rel(y, yo)
    _say(f"  N={op.N} far={op.info.far_pairs} near={op.info.near_leaf_pairs} sing={op.info.singular_pairs} err={err:.2e}")
    assert err <= TOL
    # several right-hand sides in one call (batched kernels, column chunks of up
    # to 8 with a ragged last chunk) equal single calls up to summation order
    X = np.stack([x] + [W.random_coeffs(op.N, s) for s in range(1, 11)])
    Y = op.apply(X)
    for c in (0, 5, 10):
        yc = y if c == 0 else op.apply(X[c].copy())
        assert _rel(Y[c], yc) <= 1e-14


@pytest.mark.parametrize("case", [CASES[2], CASES[4], CASES[8]], ids=["sphere-d1", "torus-d1", "sphere-d0"])
def test_stored_and_generated_coupling_match_oracle(oracle_mod, ctx, case):
    """The stored coupling blocks (one per unordered pair, applied with their
    transposes) and the per-apply evaluation give the same operator."""
    from paper_1807_03097_amd import binding as B
    name, p, m, kappa, q, eta, d, g, gs = case
    _say(f"case {case}")
    pats = _geom(name)
    geom = B.Geometry(ctx, pats)
    o = oracle_mod.Oracle(pats, p, m, kappa, g=g, gs=gs)
    x = W.random_coeffs(op_n := B.Operator(geom, p, m, kappa, q, eta, g, gs, d, plan_only=True).N, 0)
    yo = o.fmm_apply(x, q, eta, d)
    X = np.stack([x] + [W.random_coeffs(op_n, s) for s in range(1, 7)])
    res = {}
    for store in (1, 0):
        op = B.Operator(geom, p, m, kappa, q, eta, g, gs, d, store_coupling=store)
        y = op.apply(x)
        err = _rel(y, yo)
        Y = op.apply(X)
        errb = _rel(Y[0], yo)
        y32 = op.apply(x, prec=B.IGE_F32)
        err32 = _rel(y32, yo)
        _say(f"  store={store}: err={err:.2e} batched={errb:.2e} fp32={err32:.2e}")
        assert err <= TOL and errb <= TOL
        assert 1e-12 < err32 <= 1e-5
        res[store] = (y, Y)
        op.close()
    assert _rel(res[1][1], res[0][1]) <= 1e-13


def test_coupling_kernel_evaluation_accuracy(ctx):
    """The coupling stage's own evaluation of e^{ikr}/(4 pi r) (eq:HelmholtzGreen)
    against numpy's exp over r in [1e-3, 30] and kappa up to 40."""
    from paper_1807_03097_amd import binding as B
    r = np.r_[np.linspace(1e-3, 30.0, 200001), np.geomspace(1e-6, 1e-3, 1000)]
    for kappa in (0.5, 8.0, 40.0):
        got = B.ige_helmholtz_eval(ctx.h, kappa, r * r)
        ref = np.exp(1j * kappa * r) / (4 * np.pi * r)
        err = np.max(np.abs(got - ref) / np.abs(ref))
        _say(f"  kappa={kappa} max rel err {err:.2e}")
        assert err <= 5e-15 * max(1.0, kappa * 30.0)


def test_dense_matrix_columns_match_oracle(oracle_mod, ctx):
    """eta = 0: the library's operator is the dense Galerkin matrix; compare all
    columns (unit vectors) with the oracle's matrix."""
    from paper_1807_03097_amd import binding as B
    pats = W.cube_sphere()
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, 1, 1, 3.0, 4, 0.0, 5, 5, -1)
    A = oracle_mod.Oracle(pats, 1, 1, 3.0).dense_matrix()
    I = np.eye(op.N, dtype=np.complex128)
    Ag = op.apply(I).T            # column c = A e_c
    assert np.max(np.abs(Ag - A)) <= TOL * np.max(np.abs(A))


def test_device_pointers_match_host_pointers(ctx):
    import torch
    from paper_1807_03097_amd import binding as B
    geom = B.Geometry(ctx, W.cube_sphere())
    op = B.Operator(geom, 2, 3, 8.0, 8, 1.0, 5, 5, 1)
    x = W.random_coeffs(op.N, 7)
    yh = op.apply(x)
    xd = torch.from_numpy(x).to("cuda:0")
    yd = op.apply(xd)
    torch.cuda.synchronize()
    assert np.array_equal(yd.cpu().numpy(), yh)


def test_batched_apply_device_pointers(ctx):
    """64 right-hand sides on device memory through the batched kernels equal the
    single-column path column by column."""
    import torch
    from paper_1807_03097_amd import binding as B
    geom = B.Geometry(ctx, W.cube_sphere())
    op = B.Operator(geom, 2, 4, 8.0, 8, 1.6, 5, 5, 3)
    X = W.random_coeffs(op.N, 3, nrhs=64)
    Yd = op.apply(torch.from_numpy(X).to("cuda:0"))
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy()
    for c in (0, 17, 63):
        assert _rel(Y[c], op.apply(X[c].copy())) <= 1e-14


def test_rhs_plane_wave_matches_oracle(oracle_mod, ctx):
    from paper_1807_03097_amd import binding as B
    pats = W.torus()
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, 2, 2, 5.0, 6, 1.0, 5, 5, 1)
    o = oracle_mod.Oracle(pats, 2, 2, 5.0)
    dirs, pols = W.fibonacci_plane_waves(3)
    F = op.rhs_plane_wave(dirs, pols)
    for k in range(3):
        fo = o.rhs_plane_wave(dirs[k], pols[k])
        assert _rel(F[k], fo) <= TOL


def test_gmres_dense_c1_matches_lapack(oracle_mod, ctx):
    """Small dense problem: sphere, level 2, p = 1, kappa = 1, x-polarised plane wave
    along +z, GMRES relative tolerance 1e-8 (restart 1500)."""
    from paper_1807_03097_amd import binding as B
    pats = W.cube_sphere()
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, 1, 2, 1.0, 8, 0.0, 5, 5, -1)
    f = op.rhs_plane_wave([[0.0, 0.0, 1.0]], [[1.0, 0.0, 0.0]])[0]
    x, stats, rc = op.solve(f, tol=1e-8, restart=1500, maxit=2000)
    assert rc == 0
    it, _, relres, _ = stats[0]
    o = oracle_mod.Oracle(pats, 1, 2, 1.0)
    A = o.dense_matrix()
    fo = o.rhs_plane_wave([0, 0, 1], [1, 0, 0])
    assert _rel(f, fo) <= TOL
    xl = np.linalg.solve(A, fo)
    _say(f"  GMRES iterations {it}, relres {relres:.2e}")
    assert relres <= 1e-8
    assert np.linalg.norm(fo - A @ x) / np.linalg.norm(fo) <= 1.01e-8
    assert _rel(x, xl) <= 1e-8 * np.linalg.cond(A)
    # restarted GMRES reaches the same solution
    x2, stats2, rc2 = op.solve(f, tol=1e-8, restart=15, maxit=4000)
    assert rc2 == 0 and _rel(x2, xl) <= 1e-8 * np.linalg.cond(A)
    # maxit too small: not converged, reported as such
    x3, stats3, rc3 = op.solve(f, tol=1e-12, restart=5, maxit=3)
    assert rc3 == B.IGE_ENOTCONV and stats3[0][0] == 3
    # three right-hand sides solved together: each column matches LAPACK
    dirs, pols = W.fibonacci_plane_waves(3)
    F = op.rhs_plane_wave(dirs, pols)
    X, st, rc4 = op.solve(F, tol=1e-8, restart=40, maxit=2000)
    assert rc4 == 0
    for c in range(3):
        xl = np.linalg.solve(A, o.rhs_plane_wave(dirs[c], pols[c]))
        assert st[c][2] <= 1.05e-8
        assert _rel(X[c], xl) <= 1e-8 * np.linalg.cond(A)


def test_fp32_coupling_apply_and_refined_solve(oracle_mod, ctx):
    """Mixed precision: the FP32 coupling stage stays within its derived error
    (kappa * diam * 2^-23 per kernel value) of the oracle, and GMRES with FP64
    iterative refinement around FP32-coupling inner solves reaches the FP64
    tolerance and the FP64 solution within 1e-6."""
    from paper_1807_03097_amd import binding as B
    pats = W.cube_sphere()
    geom = B.Geometry(ctx, pats)
    kappa = 8.0
    op = B.Operator(geom, 2, 3, kappa, 8, 1.6, 5, 5, 1)
    x = W.random_coeffs(op.N, 0)
    yo = oracle_mod.Oracle(pats, 2, 3, kappa).fmm_apply(x, 8, 1.6, 1)
    y32 = op.apply(x, prec=B.IGE_F32)
    err32 = _rel(y32, yo)
    _say(f"  FP32 coupling rel.err {err32:.2e}")
    assert 1e-12 < err32 <= 1e-5
    r = np.geomspace(1e-3, 4.0, 20001)
    g32 = B.ige_helmholtz_eval(ctx.h, kappa, r * r, B.IGE_F32)
    ref = np.exp(1j * kappa * r) / (4 * np.pi * r)
    assert np.max(np.abs(g32 - ref) / np.abs(ref)) <= 4 * kappa * 4.0 * 2.0 ** -23 + 1e-6
    dirs, pols = W.fibonacci_plane_waves(2)
    F = op.rhs_plane_wave(dirs, pols)
    X64, st64, rc = op.solve(F, tol=1e-10, restart=100, maxit=3000)
    assert rc == 0
    Xir, stir, rc2 = op.solve(F, tol=1e-10, restart=100, maxit=3000, refine=True, inner_tol=1e-4,
                              inner_prec=B.IGE_F32)
    assert rc2 == 0
    for c in range(2):
        _say(f"  col {c}: FP64 iters {st64[c][0]}, IR iters {stir[c][0]} outer {stir[c][1]} relres {stir[c][2]:.2e}")
        assert stir[c][2] <= 1.05e-10 and stir[c][1] >= 2
        assert _rel(Xir[c], X64[c]) <= 1e-6


@pytest.mark.parametrize("case", [CASES[2], CASES[3], CASES[4], CASES[10], CASES[12]],
                         ids=["sphere-m3-d1", "sphere-m4-d2", "torus-m3", "sphere-p3", "jittered-p4"])
def test_bf16_matrix_core_coupling(oracle_mod, ctx, case):
    """Coupling on the BF16 matrix cores: plain BF16 within 2^-9-level error of the
    oracle, split BF16 (three products) within 2^-16-level error, one and several
    columns (ragged column chunk) alike; FP64 refinement around split-BF16 inner solves
    reaches the FP64 tolerance and the FP64 solution."""
    from paper_1807_03097_amd import binding as B
    name, p, m, kappa, q, eta, d, g, gs = case
    _say(f"case {case}")
    pats = _geom(name)
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, p, m, kappa, q, eta, g, gs, d)
    x = W.random_coeffs(op.N, 0)
    yo = oracle_mod.Oracle(pats, p, m, kappa, g=g, gs=gs).fmm_apply(x, q, eta, d)
    X = np.stack([x] + [W.random_coeffs(op.N, s) for s in range(1, 11)])
    y64 = op.apply(X)
    # 70 columns: several column chunks with a ragged last one
    X70 = np.stack([W.random_coeffs(op.N, 100 + s) for s in range(70)])
    y70 = op.apply(X70)
    for prec, lo, hi in ((B.IGE_BF16, 1e-6, 1e-2), (B.IGE_BF16X3, 1e-12, 2e-4), (B.IGE_BF16X3_ALL, 1e-12, 2e-4)):
        y1 = op.apply(x, prec=prec)
        Y = op.apply(X, prec=prec)
        Y70 = op.apply(X70, prec=prec)
        e1, eb = _rel(y1, yo), _rel(Y[0], yo)
        eall = max(_rel(Y[c], y64[c]) for c in range(len(X)))
        e70 = max(_rel(Y70[c], y70[c]) for c in range(len(X70)))
        _say(f"  prec {prec}: 1 column {e1:.2e}, 11 columns {eb:.2e}, worst column vs FP64 {eall:.2e}, "
             f"worst of 70 {e70:.2e}")
        assert lo < e1 <= hi and lo < eb <= hi and eall <= hi and e70 <= hi
    if op.N > 1000:   # the unpreconditioned FP64 reference solve needs thousands of iterations
        op.close()
        return
    dirs, pols = W.fibonacci_plane_waves(2)
    F = op.rhs_plane_wave(dirs, pols)
    X64, st64, rc = op.solve(F, tol=1e-10, restart=100, maxit=4000)
    assert rc == 0
    # the split near field (about 4e-6 on the whole product) needs more refinement steps
    for iprec, cap in ((B.IGE_BF16X3, 4000), (B.IGE_BF16X3_ALL, 12000)):
        Xir, stir, rc2 = op.solve(F, tol=1e-10, restart=100, maxit=cap, refine=True, inner_tol=1e-4,
                                  inner_prec=iprec)
        assert rc2 == 0
        for c in range(2):
            _say(f"  col {c}: FP64 iters {st64[c][0]}, inner prec {iprec} IR iters {stir[c][0]} "
                 f"outer {stir[c][1]} relres {stir[c][2]:.2e}")
            assert stir[c][2] <= 1.05e-10
            assert _rel(Xir[c], X64[c]) <= 1e-6
    op.close()


@pytest.mark.parametrize("case", [CASES[2], CASES[4], CASES[8], CASES[9]],
                         ids=["sphere-d1", "torus-d1", "sphere-d0", "sphere-d3"])
def test_fp64_matrix_core_coupling(oracle_mod, ctx, monkeypatch, case):
    """FP64 applies of 8 or more columns take the coupling on the FP64 matrix cores
    (stored FP64 blocks): equal to the oracle to the FP64 tolerance, and to single
    columns and to the per-apply evaluated coupling up to summation order, for 8, 9
    and 70 columns (one, one ragged, and several column chunks with a ragged last)."""
    from paper_1807_03097_amd import binding as B
    name, p, m, kappa, q, eta, d, g, gs = case
    _say(f"case {case}")
    pats = _geom(name)
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, p, m, kappa, q, eta, g, gs, d)
    monkeypatch.setenv("IGE_M2L_F64", "generate")
    opg = B.Operator(geom, p, m, kappa, q, eta, g, gs, d)
    monkeypatch.delenv("IGE_M2L_F64")
    o = oracle_mod.Oracle(pats, p, m, kappa, g=g, gs=gs)
    X70 = np.stack([W.random_coeffs(op.N, 300 + s) for s in range(70)])
    for nc in (8, 9, 70):
        X = X70[:nc].copy()
        Y = op.apply(X)
        Yg = opg.apply(X)
        eg = max(_rel(Y[c], Yg[c]) for c in range(nc))
        e1 = max(_rel(Y[c], op.apply(X[c].copy())) for c in (0, nc // 2, nc - 1))
        eo = _rel(Y[nc - 1], o.fmm_apply(X[nc - 1], q, eta, d)) if nc < 70 else 0.0
        _say(f"  {nc} columns: vs generated {eg:.2e}, vs single columns {e1:.2e}, last column vs oracle {eo:.2e}")
        assert eg <= 1e-13 and e1 <= 1e-13 and eo <= TOL
    opg.close()
    op.close()


@pytest.mark.parametrize("case", [CASES[2], CASES[4], CASES[8], CASES[10]],
                         ids=["sphere-m3-d1", "torus-m3", "sphere-d0", "sphere-p3"])
def test_fp64_matrix_core_near_field(oracle_mod, ctx, monkeypatch, case):
    """FP64 applies of 56 or more columns take the near field as FP64 matrix-core
    products over ordered leaf pairs: equal to the unordered-block kernel and to
    single columns up to summation order, and the first column to the oracle, for 56,
    64 and 130 columns (one ragged chunk of 64, one full, three with a ragged last)."""
    from paper_1807_03097_amd import binding as B
    name, p, m, kappa, q, eta, d, g, gs = case
    _say(f"case {case}")
    pats = _geom(name)
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, p, m, kappa, q, eta, g, gs, d)
    monkeypatch.setenv("IGE_NEAR_F64", "blocks")
    opb = B.Operator(geom, p, m, kappa, q, eta, g, gs, d)
    monkeypatch.delenv("IGE_NEAR_F64")
    o = oracle_mod.Oracle(pats, p, m, kappa, g=g, gs=gs)
    XA = np.stack([W.random_coeffs(op.N, 500 + s) for s in range(130)])
    yo = o.fmm_apply(XA[0], q, eta, d)
    for nc in (56, 64, 130):
        X = XA[:nc].copy()
        Y = op.apply(X)
        Yb = opb.apply(X)
        eb = max(_rel(Y[c], Yb[c]) for c in range(nc))
        e1 = max(_rel(Y[c], op.apply(X[c].copy())) for c in (0, nc // 2, nc - 1))
        eo = _rel(Y[0], yo)
        _say(f"  {nc} columns: vs unordered blocks {eb:.2e}, vs single columns {e1:.2e}, "
             f"first column vs oracle {eo:.2e}")
        assert eb <= 1e-13 and e1 <= 1e-13 and eo <= TOL
    opb.close()
    op.close()


def test_stage_profiling_levels(ctx):
    """Level 1 times every stage of a single-column apply (and of a batched one); level
    2 only the block pass and the coupling kernel, the other stages reading 0; neither
    changes the result."""
    from paper_1807_03097_amd import binding as B
    geom = B.Geometry(ctx, _geom("sphere"))
    op = B.Operator(geom, 2, 3, 8.0, 8, 1.6, 5, 5, 1)
    x = W.random_coeffs(op.N, 7)
    y0 = op.apply(x)
    X = np.stack([W.random_coeffs(op.N, 70 + s) for s in range(9)])
    for level in (1, 2):
        for xx in (x, X):
            op.set_profiling(level)
            y = op.apply(xx)
            st = np.asarray(op.stage_times())
            op.set_profiling(0)
            _say(f"  level {level}, {xx.ndim} dims: {np.round(st * 1e3, 1)} us")
            assert st[7] > 0 and st[8] > 0
            if level == 1:
                assert np.all(st[[0, 1, 2, 4, 5, 6]] > 0)
            else:
                assert np.all(st[:7] == 0)
            if xx.ndim == 1:
                assert _rel(y, y0) == 0.0
    with pytest.raises(B.IgeError):
        op.set_profiling(3)
    op.close()


@pytest.mark.parametrize("nrhs, prec", [(1, 0), (3, 0), (3, 3)], ids=["1col-f64", "3col-f64", "3col-splitbf16"])
def test_solve_graph_replays_equal_eager(ctx, monkeypatch, nrhs, prec):
    """GMRES with the apply captured as a HIP graph and replayed every iteration gives
    bitwise the same iterates as the eager launches (every replay feeds the next)."""
    from paper_1807_03097_amd import binding as B
    geom = B.Geometry(ctx, _geom("sphere"))
    op = B.Operator(geom, 2, 3, 8.0, 8, 1.6, 5, 5, 1)
    dirs, pols = W.fibonacci_plane_waves(nrhs)
    F = op.rhs_plane_wave(dirs, pols)
    if nrhs == 1:
        F = F[0]
    kw = dict(tol=1e-8, restart=60, maxit=300)
    if prec:
        kw.update(refine=True, inner_prec=prec, inner_tol=1e-3)
    monkeypatch.setenv("IGE_GRAPH", "0")
    Xe, ste, rce = op.solve(F, **kw)
    monkeypatch.setenv("IGE_GRAPH", "1")
    Xg, stg, rcg = op.solve(F, **kw)
    _say(f"  eager {[s[:3] for s in ste]}, graph {[s[:3] for s in stg]}")
    assert rce == rcg and [s[:3] for s in ste] == [s[:3] for s in stg]
    assert np.array_equal(Xe, Xg)
    op.close()


@pytest.mark.parametrize("prec", [0, 3, 4], ids=["f64", "splitbf16", "splitbf16-near"])
def test_autotune_keeps_results(ctx, prec):
    """The autotuner only changes tile shapes (column chunking), launch order and, for
    FP64, which of two FP64 evaluations of the coupling runs; applies before and after
    tuning agree to rounding (checked to 1e-13)."""
    from paper_1807_03097_amd import binding as B
    geom = B.Geometry(ctx, _geom("sphere"))
    op = B.Operator(geom, 2, 3, 8.0, 8, 1.6, 5, 5, 1)
    X = np.stack([W.random_coeffs(op.N, 200 + s) for s in range(20)])
    y0 = op.apply(X, prec=prec)
    ch = op.autotune(20, prec)
    y1 = op.apply(X, prec=prec)
    err = max(_rel(y1[c], y0[c]) for c in range(len(X)))
    _say(f"  prec {prec}: chosen {ch}, max rel change {err:.1e}")
    assert ch and err <= 1e-13
    op.close()


def test_refinement_escalates_inner_precision(ctx):
    """Plain BF16 inner solves cannot reach 1e-10 alone (the inner operator's error
    times the condition number is too large); the refined solve of two waves moves the
    inner precision towards FP64 and meets the tolerance on the FP64 operator."""
    from paper_1807_03097_amd import binding as B
    geom = B.Geometry(ctx, _geom("sphere"))
    op = B.Operator(geom, 2, 3, 8.0, 8, 1.6, 5, 5, 1)
    dirs, pols = W.fibonacci_plane_waves(2)
    F = op.rhs_plane_wave(dirs, pols)
    X64, st64, rc = op.solve(F, tol=1e-10, restart=100, maxit=4000)
    assert rc == 0
    Xr, st, rc2 = op.solve(F, tol=1e-10, restart=100, maxit=12000, refine=True, inner_tol=1e-4,
                           inner_prec=B.IGE_BF16)
    for c in range(2):
        _say(f"  FP64 iters {st64[c][0]}, BF16-start refined iters {st[c][0]} outer {st[c][1]} relres {st[c][2]:.2e}")
        assert st[c][2] <= 1.05e-10
        assert _rel(Xr[c], X64[c]) <= 1e-6
    assert rc2 == 0
    op.close()


def test_single_wave_inner_solves_run_in_fp32(ctx, monkeypatch):
    """One right-hand side: refinement with a BF16 inner precision runs its inner solves
    as FP32 (the same iterations and bits as inner_prec = FP32); IGE_SINGLE_INNER=asked
    keeps the BF16 inner operator (different iterates); all meet the FP64 tolerance."""
    from paper_1807_03097_amd import binding as B
    geom = B.Geometry(ctx, _geom("sphere"))
    op = B.Operator(geom, 2, 3, 8.0, 8, 1.6, 5, 5, 1)
    dirs, pols = W.fibonacci_plane_waves(1)
    f = op.rhs_plane_wave(dirs, pols)[0]
    x32, s32, rc32 = op.solve(f, tol=1e-8, restart=200, maxit=4000, refine=True, inner_prec=B.IGE_F32)
    xb, sb, rcb = op.solve(f, tol=1e-8, restart=200, maxit=4000, refine=True, inner_prec=B.IGE_BF16X3)
    monkeypatch.setenv("IGE_SINGLE_INNER", "asked")
    xa, sa, rca = op.solve(f, tol=1e-8, restart=200, maxit=4000, refine=True, inner_prec=B.IGE_BF16X3)
    monkeypatch.delenv("IGE_SINGLE_INNER")
    _say(f"  FP32 inner {s32[0][0]} iterations, BF16X3 asked {sb[0][0]}, BF16X3 kept {sa[0][0]}")
    assert rc32 == 0 and rcb == 0 and rca == 0
    assert np.array_equal(xb, x32) and sb[0][0] == s32[0][0]
    assert not np.array_equal(xa, x32)
    for st in (s32, sb, sa):
        assert st[0][2] <= 1.05e-8
    op.close()


@pytest.mark.parametrize("inner_tol", [1e-4, 1e-6], ids=["fp32-basis", "fp64-basis"])
def test_inner_krylov_basis_precision(ctx, monkeypatch, inner_tol):
    """Refined solves of 3 waves with the inner Krylov basis in FP32 (default for
    inner_tol >= 1e-5) and in FP64 (IGE_INNER_BASIS=fp64, or a tighter inner_tol) both
    meet the FP64 tolerance and agree with the FP64 solve to 1e-6."""
    from paper_1807_03097_amd import binding as B
    geom = B.Geometry(ctx, _geom("sphere"))
    op = B.Operator(geom, 2, 3, 8.0, 8, 1.6, 5, 5, 1)
    dirs, pols = W.fibonacci_plane_waves(3)
    F = op.rhs_plane_wave(dirs, pols)
    X64, st64, rc = op.solve(F, tol=1e-10, restart=100, maxit=4000)
    assert rc == 0
    res = {}
    for basis in ("default", "fp64"):
        if basis == "fp64":
            monkeypatch.setenv("IGE_INNER_BASIS", "fp64")
        Xr, st, rc2 = op.solve(F, tol=1e-10, restart=100, maxit=6000, refine=True, inner_tol=inner_tol,
                               inner_prec=B.IGE_BF16X3)
        monkeypatch.delenv("IGE_INNER_BASIS", raising=False)
        assert rc2 == 0
        for c in range(3):
            _say(f"  {basis} basis, inner_tol {inner_tol}: col {c} iters {st[c][0]} outer {st[c][1]} "
                 f"relres {st[c][2]:.2e}")
            assert st[c][2] <= 1.05e-10
            assert _rel(Xr[c], X64[c]) <= 1e-6
        res[basis] = Xr
    if inner_tol < 1e-5:   # both runs used the FP64 basis: identical
        assert max(_rel(res["default"][c], res["fp64"][c]) for c in range(3)) == 0.0
    op.close()


@pytest.mark.parametrize("name, p, m, kappa", [("sphere", 2, 3, 8.0), ("torus", 1, 3, 3.0), ("jittered", 2, 2, 5.0)])
def test_potential_matches_oracle(oracle_mod, ctx, name, p, m, kappa):
    """Scattered field e_s = V~ w at points off the surface (two columns)."""
    from paper_1807_03097_amd import binding as B
    pats = _geom(name)
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, p, m, kappa, 6, 1.0, 5, 5, 1)
    o = oracle_mod.Oracle(pats, p, m, kappa, g=5, gs=5)
    w = np.stack([W.random_coeffs(op.N, 3), W.random_coeffs(op.N, 4)])
    pts = oracle_mod.fibonacci_sphere(24, 2.5)
    E = op.potential(w, pts)
    for c in range(2):
        Eo = o.potential(w[c], pts)
        err = _rel(E[c], Eo)
        _say(f"  {name}: column {c} rel.err {err:.2e}")
        assert err <= TOL
    op.close()


def test_plane_wave_scattering_against_mie(ctx):
    """End to end on the device: solve the plane-wave problem on the NURBS sphere and
    evaluate the scattered field at radius 3 against the Mie series.  The NURBS sphere
    deviates radially by up to 0.02 from the unit sphere, which bounds the agreement."""
    from paper_1807_03097_amd import binding as B
    from oracle import mie
    geom = B.Geometry(ctx, W.cube_sphere())
    kappa = 1.0
    op = B.Operator(geom, 2, 3, kappa, 8, 1.6, 5, 5, 1)
    f = op.rhs_plane_wave(np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0], complex))[0]
    x, st, rc = op.solve(f, tol=1e-10, restart=300, maxit=3000)
    assert rc == 0
    rng = np.random.default_rng(5)
    pts = rng.standard_normal((40, 3))
    pts = 3.0 * pts / np.linalg.norm(pts, axis=1, keepdims=True)
    E = op.potential(x, pts)
    Em = mie.fields(pts, kappa, "E_s")
    err = np.linalg.norm(E - Em) / np.linalg.norm(Em)
    _say(f"  scattered field vs Mie at r=3: rel.err {err:.2e} ({st[0][0]} iterations)")
    assert err <= 0.05
    op.close()


def test_c2_full_size_sampled_rows(oracle_mod, ctx):
    """Matvec configuration as the benchmark times it: sphere, level 5, p = 2,
    kappa = 8, q = 8, eta = 1.6, leaf depth 3, 5x5 Gauss, x seed 0.  On the 48 rows of
    tests/golden/c2_dense_rows.json: the HIP FMM equals the oracle's FMM (computed row
    by row) to 1e-12 and the stored dense Galerkin rows to 1e-6."""
    import json
    import os
    from paper_1807_03097_amd import binding as B
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c2_dense_rows.json")))
    rows = np.array(g["rows"])
    yd = np.array(g["re"]) + 1j * np.array(g["im"])
    pats = W.cube_sphere()
    geom = B.Geometry(ctx, pats)
    eta, d = 1.6, 3
    op = B.Operator(geom, 2, 5, 8.0, 8, eta, 5, 5, d)
    x = W.random_coeffs(op.N, 0)
    y = op.apply(x)
    o = oracle_mod.Oracle(pats, 2, 5, 8.0, g=5, gs=5)
    yo = o.fmm_apply(x, 8, eta, d, rows=rows)
    err = _rel(y[rows], yo)
    errd = _rel(y[rows], yd)
    _say(f"  C2 N={op.N} distinct near entries={op.info.near_distinct} far={op.info.far_pairs} "
         f"vs oracle FMM {err:.2e}, vs dense rows {errd:.2e}")
    assert err <= TOL and errd <= 1e-6
    op.close()


HIGHQ_CASES = [
    # geometry, p, m, kappa, q, eta, leaf depth, g, gs: q = 10 (121 nodes, matrix-core
    # tiles of 128) at kappa 16 and 40
    ("sphere", 2, 4, 16.0, 10, 1.6, 2, 5, 5),
    ("sphere", 2, 4, 40.0, 10, 1.6, 2, 5, 5),
    ("jittered", 2, 3, 16.0, 10, 1.0, 1, 5, 5),
]


@pytest.mark.parametrize("case", HIGHQ_CASES, ids=[f"{c[0]}-m{c[2]}-k{int(c[3])}-q{c[4]}" for c in HIGHQ_CASES])
def test_high_q_and_kappa_match_oracle(oracle_mod, ctx, case):
    """q = 10 and kappa = 16, 40 against the oracle: FP64 one column and batched
    (generated coupling) to 1e-12, the FP64 matrix-core coupling of 16 columns to
    1e-12, BF16 within (1e-6, 1e-2] and split BF16 within (1e-12, 2e-4]."""
    from paper_1807_03097_amd import binding as B
    name, p, m, kappa, q, eta, d, g, gs = case
    _say(f"case {case}")
    pats = _geom(name)
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, p, m, kappa, q, eta, g, gs, d)
    x = W.random_coeffs(op.N, 0)
    yo = oracle_mod.Oracle(pats, p, m, kappa, g=g, gs=gs).fmm_apply(x, q, eta, d)
    y1 = op.apply(x)
    X = np.stack([x] + [W.random_coeffs(op.N, s) for s in range(1, 16)])
    Y4 = op.apply(X[:4].copy())
    Y16 = op.apply(X)
    e1, e4, e16 = _rel(y1, yo), _rel(Y4[0], yo), _rel(Y16[0], yo)
    e16c = max(_rel(Y16[c], Y4[c]) for c in range(4))
    _say(f"  N={op.N} far={op.info.far_pairs}: 1 column {e1:.1e}, 4 columns {e4:.1e}, 16 columns (matrix cores) "
         f"{e16:.1e} (vs 4 columns {e16c:.1e})")
    assert e1 <= TOL and e4 <= TOL and e16 <= TOL and e16c <= 1e-13
    for prec, lo, hi in ((B.IGE_BF16, 1e-6, 1e-2), (B.IGE_BF16X3, 1e-12, 2e-4)):
        Yp = op.apply(X, prec=prec)
        ep = _rel(Yp[0], yo)
        _say(f"  prec {prec}: {ep:.1e}")
        assert lo < ep <= hi
    op.close()


# Assembly cases for the colour launches of the near-field quadrature: trial squares
# smaller than the leaf (p = 3 with 8 x 8-element leaves: squares of 2 x 2, three
# apart; p = 2 with 16 x 16-element leaves: squares of 8 x 8, two apart), and the
# single-square cases of every degree.
ASSEMBLY_CASES = [
    ("sphere", 1, 3, 3.0, 6, 1.0, 1, 5, 5),
    ("sphere", 2, 3, 5.0, 6, 1.0, 1, 5, 5),
    ("torus", 2, 2, 6.0, 6, 1.0, 1, 5, 5),
    ("sphere", 3, 3, 6.0, 6, 1.6, 3, 5, 4),
    ("sphere", 2, 4, 8.0, 8, 1.6, 4, 5, 5),
    ("sphere", 4, 3, 6.0, 8, 1.6, 2, 5, 4),
]


@pytest.mark.parametrize("case", ASSEMBLY_CASES,
                         ids=[f"{c[0]}-p{c[1]}-m{c[2]}-d{c[6]}" for c in ASSEMBLY_CASES])
def test_assembly_is_bitwise_reproducible(oracle_mod, ctx, case):
    """Two assemblies of the same operator give the same near-field blocks bit for
    bit (every element-pair contribution is summed in a fixed order), hence the same
    applies; the operator matches the oracle (Sec. 4.1 quadrature, Sec. 4.2 FMM)."""
    from paper_1807_03097_amd import binding as B
    name, p, m, kappa, q, eta, d, g, gs = case
    _say(f"case {case}")
    pats = _geom(name)
    geom = B.Geometry(ctx, pats)
    op1 = B.Operator(geom, p, m, kappa, q, eta, g, gs, d)
    op2 = B.Operator(geom, p, m, kappa, q, eta, g, gs, d)
    b1, b2 = op1.near_blocks(), op2.near_blocks()
    assert b1.shape == b2.shape and np.count_nonzero(b1) > 0
    assert np.array_equal(b1.view(np.uint64), b2.view(np.uint64))
    x = W.random_coeffs(op1.N, 0)
    y1, y2 = op1.apply(x), op2.apply(x)
    assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))
    X = np.stack([W.random_coeffs(op1.N, s) for s in range(1, 10)])
    assert np.array_equal(op1.apply(X).view(np.uint64), op2.apply(X).view(np.uint64))
    o = oracle_mod.Oracle(pats, p, m, kappa, g=g, gs=gs)
    yo = o.fmm_apply(x, q, eta, d)
    err = _rel(y1, yo)
    _say(f"  N={op1.N} blocks={op1.info.near_leaf_pairs} sing={op1.info.singular_pairs} err={err:.2e}")
    assert err <= TOL
    op1.close()
    op2.close()


NEAR_ONCE_CASES = [CASES[0], CASES[2], CASES[4], CASES[5], CASES[7], CASES[9], CASES[10], CASES[12],
                   ASSEMBLY_CASES[3], ASSEMBLY_CASES[5]]


@pytest.mark.parametrize("case", NEAR_ONCE_CASES,
                         ids=[f"{c[0]}-p{c[1]}-m{c[2]}-eta{c[5]}-d{c[6]}" for c in NEAR_ONCE_CASES])
def test_near_once_per_entry_equals_leaf_pair_blocks(oracle_mod, ctx, case, monkeypatch):
    """The one-column near-field product over the distinct entries of the symmetric
    matrix (owner blocks, upper triangles of the diagonal squares), in one launch and in
    two (IGE_NEAR_ONE=0), equals the product over the leaf-pair blocks and their
    transposes up to summation order, and the whole apply matches the oracle."""
    from paper_1807_03097_amd import binding as B
    name, p, m, kappa, q, eta, d, g, gs = case
    _say(f"case {case}")
    pats = _geom(name)
    geom = B.Geometry(ctx, pats)
    monkeypatch.setenv("IGE_NEAR_COMPACT", "0")
    op0 = B.Operator(geom, p, m, kappa, q, eta, g, gs, d)
    monkeypatch.delenv("IGE_NEAR_COMPACT")
    op1 = B.Operator(geom, p, m, kappa, q, eta, g, gs, d)
    monkeypatch.setenv("IGE_NEAR_ONE", "0")
    op2 = B.Operator(geom, p, m, kappa, q, eta, g, gs, d)
    monkeypatch.delenv("IGE_NEAR_ONE")
    ys0, ys1, ys2 = [], [], []
    for seed in range(3):
        x = W.random_coeffs(op1.N, seed)
        ys0.append(op0.apply(x))
        ys1.append(op1.apply(x))
        ys2.append(op2.apply(x))
    err = max(max(_rel(a, b) for a, b in zip(ys1, ys0)), max(_rel(a, b) for a, b in zip(ys2, ys0)))
    op2.close()
    x = W.random_coeffs(op1.N, 0)
    dd = d if d >= 0 else int(np.ceil(np.log2((q + 1) / (p + 1)) - 1e-12))
    yo = oracle_mod.Oracle(pats, p, m, kappa, g=g, gs=gs).fmm_apply(x, q, eta, dd)
    erro = _rel(ys1[0], yo)
    _say(f"  distinct {op1.info.near_distinct} of {op1.info.near_nnz} block entries; vs blocks {err:.1e}, "
         f"vs oracle {erro:.1e}")
    assert err <= 1e-14 and erro <= TOL
    op0.close()
    op1.close()


SYM_CASES = [CASES[2], CASES[3], CASES[4], CASES[6], CASES[7], CASES[8], CASES[10], CASES[12],
             ("sphere", 2, 3, 8.0, 10, 1.6, 1, 5, 5)]


@pytest.mark.parametrize("case", SYM_CASES, ids=[f"{c[0]}-p{c[1]}-m{c[2]}-q{c[4]}-d{c[6]}" for c in SYM_CASES])
def test_unordered_pair_coupling_equals_ordered(oracle_mod, ctx, case, monkeypatch):
    """The one-column FP64 coupling over unordered far pairs (IGE_M2L_SYM=1: each kernel
    value used for both clusters, the kernel being symmetric) equals the coupling over
    ordered pairs (default) up to summation order, for one, four and eight partners per
    work item and for the scalar single layer; degree 10 keeps the ordered form; the
    apply matches the oracle."""
    from paper_1807_03097_amd import binding as B
    name, p, m, kappa, q, eta, d, g, gs = case
    _say(f"case {case}")
    pats = _geom(name)
    geom = B.Geometry(ctx, pats)
    for kind in (B.IGE_OP_EFIE, B.IGE_OP_SCALAR):
        op0 = B.Operator(geom, p, m, kappa, q, eta, g, gs, d, kind=kind)
        monkeypatch.setenv("IGE_M2L_SYM", "1")
        ops = []
        for ch in ("1", "8", None):
            if ch is not None:
                monkeypatch.setenv("IGE_M2L_SYM_CHUNK", ch)
            ops.append(B.Operator(geom, p, m, kappa, q, eta, g, gs, d, kind=kind))
            monkeypatch.delenv("IGE_M2L_SYM_CHUNK", raising=False)
        monkeypatch.delenv("IGE_M2L_SYM")
        assert op0.info.m2l_unordered == 0
        assert all(o.info.m2l_unordered == (1 if (q <= 8 and op0.info.far_pairs > 0) else 0) for o in ops)
        err = 0.0
        for seed in range(2):
            x = W.random_coeffs(op0.N, seed)
            y0 = op0.apply(x)
            for o in ops:
                err = max(err, _rel(o.apply(x), y0))
        if kind == B.IGE_OP_EFIE:
            x = W.random_coeffs(op0.N, 0)
            dd = d if d >= 0 else int(np.ceil(np.log2((q + 1) / (p + 1)) - 1e-12))
            yo = oracle_mod.Oracle(pats, p, m, kappa, g=g, gs=gs).fmm_apply(x, q, eta, dd)
            erro = _rel(ops[-1].apply(x), yo)
        else:
            erro = 0.0
        _say(f"  kind {kind}: far pairs {op0.info.far_pairs}, unordered {ops[-1].info.m2l_unordered}; "
             f"vs ordered {err:.1e}, vs oracle {erro:.1e}")
        assert err <= 1e-14 and erro <= TOL
        for o in [op0] + ops:
            o.close()


def test_quartic_dense_solve_matches_lapack(oracle_mod, ctx):
    """p = 4 (the paper's Table 1, last column: N = 300 at level 1): the dense operator
    (eta = 0) against the oracle's matrix, and a plane-wave GMRES solve against LAPACK
    within tol * cond(A)."""
    from paper_1807_03097_amd import binding as B
    pats = W.cube_sphere()
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, 4, 1, 1.0, 8, 0.0, 5, 5, -1)
    assert op.N == 300
    o = oracle_mod.Oracle(pats, 4, 1, 1.0)
    A = o.dense_matrix()
    Ag = op.apply(np.eye(op.N, dtype=np.complex128)).T
    assert np.max(np.abs(Ag - A)) <= TOL * np.max(np.abs(A))
    f = op.rhs_plane_wave([[0.0, 0.0, 1.0]], [[1.0, 0.0, 0.0]])[0]
    fo = o.rhs_plane_wave([0, 0, 1], [1, 0, 0])
    assert _rel(f, fo) <= TOL
    x, st, rc = op.solve(f, tol=1e-10, restart=400, maxit=4000)
    assert rc == 0
    xl = np.linalg.solve(A, fo)
    _say(f"  p=4 N={op.N}: GMRES iterations {st[0][0]}, relres {st[0][2]:.1e}, vs LAPACK {_rel(x, xl):.1e}")
    assert _rel(x, xl) <= 1e-10 * np.linalg.cond(A)


def test_kappa_cap_operator_matches_oracle(oracle_mod, ctx):
    """The wavenumber cap of the admissibility condition (kappa * diam <= 8): same
    partition as the oracle's and the same operator to 1e-12, one and four columns."""
    from paper_1807_03097_amd import binding as B
    pats = W.cube_sphere()
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, 2, 4, 16.0, 8, 1.6, 5, 5, 1, kappa_cap=8.0)
    o = oracle_mod.Oracle(pats, 2, 4, 16.0, g=5, gs=5)
    tr = o.block_tree(1.6, 1, kappa_cap=8.0)
    pt = op.partition()
    assert np.array_equal(pt["far"], tr["far"]) and np.array_equal(pt["near"], tr["near"])
    assert op.info.far_pairs > 0 and op.info.far_pairs > len(o.block_tree(1.6, 1)["far"])
    X = np.stack([W.random_coeffs(op.N, s) for s in range(4)])
    yo = o.fmm_apply(X[0], 8, 1.6, 1, tree=tr)
    e1, e4 = _rel(op.apply(X[0].copy()), yo), _rel(op.apply(X)[0], yo)
    _say(f"  far {op.info.far_pairs}: {e1:.1e} (1 column), {e4:.1e} (4 columns)")
    assert e1 <= TOL and e4 <= TOL
    op.close()


@pytest.mark.parametrize("name", ["c3", "c5"])
def test_high_kappa_rows_match_dense_with_kappa_cap(oracle_mod, ctx, name):
    """Level 6, kappa = 16, q = 8 and the jittered level-7 sphere at kappa = 40, q = 11,
    both with the wavenumber cap (kappa * diam <= 8 and <= 12): the HIP FMM equals the
    oracle's FMM to 1e-12 and the dense Galerkin rows of tests/golden to 1e-6."""
    import json
    import os
    from paper_1807_03097_amd import binding as B
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", f"{name}_dense_rows.json")))
    rows = np.array(g["rows"])
    yd = np.array(g["re"]) + 1j * np.array(g["im"])
    cf = g["config"]
    q, cap = (8, 8.0) if name == "c3" else (11, 12.0)
    pats = W.cube_sphere() if name == "c3" else W.jitter(W.cube_sphere(), 0.02, 7)
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, 2, cf["level"], cf["kappa"], q, 1.6, 5, 5, 3, kappa_cap=cap)
    assert op.N == cf["n_dof"]
    x = W.random_coeffs(op.N, 0)
    y = op.apply(x)
    o = oracle_mod.Oracle(pats, 2, cf["level"], cf["kappa"], g=5, gs=5)
    yo = o.fmm_apply(x, q, 1.6, 3, rows=rows, tree=o.block_tree(1.6, 3, kappa_cap=cap))
    err, errd = _rel(y[rows], yo), _rel(y[rows], yd)
    _say(f"  {name}: N={op.N} far={op.info.far_pairs} vs oracle FMM {err:.1e}, vs dense {errd:.1e}")
    assert err <= TOL and errd <= 1e-6
    op.close()


LQ_CASES = [
    # geometry, p, m, kappa, eta, leaf depth, degree per level, scalar
    ("sphere", 2, 4, 8.0, 1.0, 1, [8, 10, 9, 6], False),    # larger and smaller than the leaf degree
    ("torus", 1, 3, 4.0, 1.0, 1, [4, 13, 5], False),       # degree 13: transfer kernels above 64 KB of LDS
    ("jittered", 3, 3, 6.0, 1.0, 1, [6, 7, 9], False),
    ("sphere", 2, 3, 8.0, 1.0, 1, [6, 9, 7], True),         # scalar single layer
]


@pytest.mark.parametrize("case", LQ_CASES, ids=[f"{c[0]}-p{c[1]}-m{c[2]}-q{'.'.join(map(str, c[6]))}"
                                                + ("-scalar" if c[7] else "") for c in LQ_CASES])
def test_level_degrees_match_oracle(oracle_mod, ctx, case):
    """A degree per cluster-tree level: the restriction of the largest degree's moments
    to each level's nodes and the lift of its local expansions give the oracle's
    operator (moments taken directly per level) to 1e-12; several columns (3, 11 and 70:
    the many-column kernels with coupling blocks of each level's size in one launch, a
    ragged column chunk) equal single columns to 1e-13 and the oracle to 1e-12; FP32
    stays within 1e-5 on one and on several columns."""
    from paper_1807_03097_amd import binding as B
    name, p, m, kappa, eta, d, ql, scalar = case
    _say(f"case {case}")
    pats = _geom(name)
    geom = B.Geometry(ctx, pats)
    kind = B.IGE_OP_SCALAR if scalar else B.IGE_OP_EFIE
    op = B.Operator(geom, p, m, kappa, 8, eta, 5, 5, d, kind=kind, q_level=ql)
    assert op.q_levels() == ql
    o = oracle_mod.Oracle(pats, p, m, kappa, g=5, gs=5, scalar=scalar)
    x = W.random_coeffs(op.N, 0)
    y = op.apply(x)
    yo = o.fmm_apply(x, ql, eta, d)
    err = _rel(y, yo)
    nfar = np.bincount(op.partition()["far"][:, 0], minlength=len(ql)).tolist()
    _say(f"  N={op.N} far per level {nfar} err={err:.2e}")
    assert err <= TOL
    X = np.stack([x, W.random_coeffs(op.N, 1), W.random_coeffs(op.N, 2)])
    Y = op.apply(X)
    assert _rel(Y[0], y) <= 1e-13 and _rel(Y[2], o.fmm_apply(X[2], ql, eta, d)) <= TOL
    X70 = np.stack([x] + [W.random_coeffs(op.N, 10 + c) for c in range(69)])
    y69 = op.apply(X70[69].copy())
    for nc in (11, 70):
        Y = op.apply(X70[:nc].copy())
        e1 = max(_rel(Y[0], y), _rel(Y[nc - 1], op.apply(X70[nc - 1].copy())))
        _say(f"  {nc} columns: vs single columns {e1:.1e}")
        assert e1 <= 1e-13 and _rel(Y[0], yo) <= TOL
    assert _rel(Y[69], y69) <= 1e-13
    e32 = _rel(op.apply(x, prec=B.IGE_F32), yo)
    Y32 = op.apply(X70[:11].copy(), prec=B.IGE_F32)
    e32b = max(_rel(Y32[c], op.apply(X70[c].copy())) for c in (0, 5, 10))
    _say(f"  FP32: one column {e32:.1e}, 11 columns {e32b:.1e}")
    assert 1e-12 < e32 <= 1e-5 and e32b <= 1e-5
    op.close()


def test_level_degrees_refusals_and_refined_solve(oracle_mod, ctx):
    """Operators with a degree above 10 on a level with far pairs (one degree, or a
    degree per level) refuse the BF16 couplings (applies, autotuning, refinement inner
    solves); a degree per level refuses stored coupling blocks; FP64 autotuning keeps
    the results to 1e-13; FP64 refinement around FP32 inner solves of one and of three
    waves reaches the tolerance on the FP64 operator."""
    from paper_1807_03097_amd import binding as B
    pats = W.cube_sphere()
    geom = B.Geometry(ctx, pats)
    ql = [8, 10, 9, 6]
    with pytest.raises(B.IgeError):
        B.Operator(geom, 2, 4, 8.0, 8, 1.0, 5, 5, 1, store_coupling=1, q_level=ql)
    with pytest.raises(B.IgeError):
        B.Operator(geom, 2, 4, 8.0, 8, 1.0, 5, 5, 1, q_level=[8, 16])
    op = B.Operator(geom, 2, 4, 8.0, 8, 1.0, 5, 5, 1, q_level=ql)
    x = W.random_coeffs(op.N, 0)
    q11 = B.Operator(geom, 2, 3, 8.0, 11, 1.0, 5, 5, 1)
    tgeom = B.Geometry(ctx, W.torus())
    q13 = B.Operator(tgeom, 1, 3, 4.0, 8, 1.0, 5, 5, 1, q_level=[4, 13, 5])   # degree 13 on a far level
    for o_ in (q11, q13):
        for prec in (B.IGE_BF16, B.IGE_BF16X3, B.IGE_BF16X3_ALL):
            with pytest.raises(B.IgeError) as e:
                o_.apply(W.random_coeffs(o_.N, 0), prec=prec)
            assert e.value.code == B.IGE_EINVAL
        with pytest.raises(B.IgeError):
            o_.autotune(4, B.IGE_BF16X3)
    with pytest.raises(B.IgeError):
        q13.solve(W.random_coeffs(q13.N, 1), refine=True, inner_prec=B.IGE_BF16X3)
    q11.close()
    q13.close()
    X = np.stack([W.random_coeffs(op.N, 40 + c) for c in range(8)])
    y0 = op.apply(X)
    ch = op.autotune(8)
    d = max(_rel(a, b) for a, b in zip(op.apply(X), y0))
    _say(f"  autotune FP64: {ch}, max change {d:.1e}")
    assert d <= 1e-13
    F = op.rhs_plane_wave([[0.0, 0.0, 1.0], [0.0, 1.0, 0.0], [1.0, 0.0, 0.0]],
                          [[1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, 1.0, 0.0]])
    f = F[0]
    xs, st, rc = op.solve(f, tol=1e-8, restart=300, maxit=3000)
    xr, sr, rcr = op.solve(f, tol=1e-8, restart=300, maxit=3000, refine=True, inner_prec=B.IGE_F32)
    _say(f"  FP64 iters {st[0][0]} relres {st[0][2]:.1e}; refined iters {sr[0][0]} relres {sr[0][2]:.1e}")
    assert rc == 0 and rcr == 0 and sr[0][2] <= 1e-8 * 1.05
    # the refined solution's true residual on the FP64 operator; the two solutions differ
    # by at most about tol * cond(A)
    assert _rel(op.apply(xr), f) <= 1.05e-8
    assert _rel(xr, xs) <= 1e-4
    # three waves: the many-column kernels inside the FP64 and FP32 Krylov iterations
    X3, s3, rc3 = op.solve(F, tol=1e-8, restart=300, maxit=3000, refine=True, inner_prec=B.IGE_F32)
    assert rc3 == 0
    R = op.apply(X3)
    for c in range(3):
        _say(f"  wave {c}: refined iters {s3[c][0]} relres {s3[c][2]:.1e}")
        assert _rel(R[c], F[c]) <= 1.05e-8
    assert _rel(X3[0], xs) <= 1e-4
    op.close()


MQ_CASES = [LQ_CASES[0], LQ_CASES[2], LQ_CASES[3]]


@pytest.mark.parametrize("case", MQ_CASES, ids=[f"{c[0]}-q{'.'.join(map(str, c[6]))}" + ("-scalar" if c[7] else "")
                                                for c in MQ_CASES])
def test_level_degrees_matrix_core_coupling(oracle_mod, ctx, case):
    """Degrees per level on the BF16 matrix cores, one launch per level with that
    level's padded block size (and its own column chunking): plain BF16 within
    2^-9-level error of the oracle, split BF16 within 2^-16-level error, on 1, 11 and 70
    columns (a ragged chunk) against the FP64 product; FP64 refinement around
    split-BF16 inner solves reaches the FP64 tolerance and the FP64 solution."""
    from paper_1807_03097_amd import binding as B
    name, p, m, kappa, eta, d, ql, scalar = case
    _say(f"case {case}")
    pats = _geom(name)
    geom = B.Geometry(ctx, pats)
    kind = B.IGE_OP_SCALAR if scalar else B.IGE_OP_EFIE
    op = B.Operator(geom, p, m, kappa, 8, eta, 5, 5, d, kind=kind, q_level=ql)
    o = oracle_mod.Oracle(pats, p, m, kappa, g=5, gs=5, scalar=scalar)
    X = np.stack([W.random_coeffs(op.N, 600 + c) for c in range(70)])
    yo = o.fmm_apply(X[0], ql, eta, d)
    Y11, Y70 = op.apply(X[:11].copy()), op.apply(X)
    assert _rel(Y11[0], yo) <= TOL
    for prec, lo, hi in ((B.IGE_BF16, 1e-6, 1e-2), (B.IGE_BF16X3, 1e-12, 2e-4), (B.IGE_BF16X3_ALL, 1e-12, 2e-4)):
        e1 = _rel(op.apply(X[0].copy(), prec=prec), yo)
        Y = op.apply(X[:11].copy(), prec=prec)
        eb = max(_rel(Y[c], Y11[c]) for c in range(11))
        Z = op.apply(X, prec=prec)
        e70 = max(_rel(Z[c], Y70[c]) for c in range(70))
        _say(f"  prec {prec}: 1 column {e1:.2e}, worst of 11 {eb:.2e}, worst of 70 {e70:.2e}")
        assert lo < e1 <= hi and eb <= hi and e70 <= hi
    if scalar:
        F = op.rhs_scalar(B.IGE_RHS_POINT, [[0.1, 0.2, -0.15], [0.3, -0.1, 0.2]])
    else:
        dirs, pols = W.fibonacci_plane_waves(2)
        F = op.rhs_plane_wave(dirs, pols)
    X64, st64, rc = op.solve(F, tol=1e-8, restart=300, maxit=4000)
    assert rc == 0
    Xr, st, rc2 = op.solve(F, tol=1e-8, restart=300, maxit=8000, refine=True, inner_tol=1e-4,
                           inner_prec=B.IGE_BF16X3)
    assert rc2 == 0
    R = op.apply(Xr)
    for c in range(2):
        _say(f"  wave {c}: FP64 iters {st64[c][0]}, refined iters {st[c][0]} outer {st[c][1]} relres {st[c][2]:.1e}")
        assert st[c][2] <= 1.05e-8 and _rel(R[c], F[c]) <= 1.05e-8
        assert _rel(Xr[c], X64[c]) <= 1e-4
    op.close()


@pytest.mark.parametrize("name", ["c3", "c5"])
def test_high_kappa_rows_match_dense_with_level_degrees(oracle_mod, ctx, name):
    """Level 6, kappa = 16 on the paper's partition and the jittered level-7 sphere at
    kappa = 40 with kappa_cap = 20, both with degrees from the kappa * diam rule of the
    binding (degree_rule, levels with far blocks only): the HIP FMM equals the oracle's
    FMM with the same degrees to 1e-12 and the dense Galerkin rows of tests/golden to
    1e-6."""
    import json
    import os
    from paper_1807_03097_amd import binding as B
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", f"{name}_dense_rows.json")))
    rows = np.array(g["rows"])
    yd = np.array(g["re"]) + 1j * np.array(g["im"])
    cf = g["config"]
    q, cap = (8, 0.0) if name == "c3" else (10, 20.0)
    pats = W.cube_sphere() if name == "c3" else W.jitter(W.cube_sphere(), 0.02, 7)
    geom = B.Geometry(ctx, pats)
    plan = B.Operator(geom, 2, cf["level"], cf["kappa"], q, 1.6, 5, 5, 3, kappa_cap=cap, plan_only=True)
    far_levels = set(plan.partition()["far"][:, 0].tolist())
    ql = B.degree_rule(plan.info, cf["kappa"], q, far_levels)
    plan.close()
    op = B.Operator(geom, 2, cf["level"], cf["kappa"], q, 1.6, 5, 5, 3, kappa_cap=cap, q_level=ql)
    assert op.N == cf["n_dof"]
    x = W.random_coeffs(op.N, 0)
    y = op.apply(x)
    o = oracle_mod.Oracle(pats, 2, cf["level"], cf["kappa"], g=5, gs=5)
    yo = o.fmm_apply(x, ql, 1.6, 3, rows=rows, tree=o.block_tree(1.6, 3, kappa_cap=cap))
    err, errd = _rel(y[rows], yo), _rel(y[rows], yd)
    # the same product among 4 columns of the many-column kernels (the full-size shape)
    Y = op.apply(np.stack([x] + [W.random_coeffs(op.N, c) for c in (1, 2, 3)]))
    eb = _rel(Y[0], y)
    _say(f"  {name}: degrees {ql} far={op.info.far_pairs} vs oracle FMM {err:.1e}, vs dense {errd:.1e}, "
         f"4 columns vs one {eb:.1e}")
    assert err <= TOL and errd <= 1e-6 and eb <= 1e-13
    op.close()


@pytest.mark.parametrize("case", [("sphere", 1, 3, 4.0, 6, 0.3, 0, 4, 4), ("sphere", 2, 3, 4.0, 8, 0.5, 1, 4, 4),
                                  ("sphere", 1, 3, 4.0, 6, 0.5, 0, 4, 4)],
                         ids=["far-on-leaves-only-d0", "far-on-leaves-only-d1", "far-on-two-finest"])
def test_far_pairs_on_fine_levels_only(oracle_mod, ctx, case):
    """Partitions whose coarse levels have no far pairs (small eta): the upward pass
    stops at the coarsest level with far pairs and the downward pass starts there (no
    M2M or L2L at all when only the leaves have far pairs); one and 11 columns in FP64
    and split BF16 match the oracle."""
    from paper_1807_03097_amd import binding as B
    name, p, m, kappa, q, eta, d, g, gs = case
    _say(f"case {case}")
    pats = _geom(name)
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, p, m, kappa, q, eta, g, gs, d)
    far = op.partition()["far"]
    levels = sorted(set(far[:, 0].tolist()))
    assert levels[0] > 0
    o = oracle_mod.Oracle(pats, p, m, kappa, g=g, gs=gs)
    X = np.stack([W.random_coeffs(op.N, 700 + c) for c in range(11)])
    yo = o.fmm_apply(X[0], q, eta, d)
    y1 = op.apply(X[0].copy())
    Y = op.apply(X)
    e1, eb = _rel(y1, yo), max(_rel(Y[c], op.apply(X[c].copy())) for c in (0, 5, 10))
    es = _rel(op.apply(X, prec=B.IGE_BF16X3)[0], yo)
    _say(f"  far levels {levels}, N={op.N}: 1 column {e1:.1e}, 11 columns vs single {eb:.1e}, split BF16 {es:.1e}")
    assert e1 <= TOL and _rel(Y[0], yo) <= TOL and eb <= 1e-13 and 1e-12 < es <= 2e-4
    op.close()


def test_edge_and_degenerate_cases(oracle_mod, ctx):
    """Degenerate inputs through the C ABI: zero columns are refused; a zero density
    gives exactly zero (product, right-hand side of zero polarisation, solve, potential);
    an empty point set is accepted; the scalar operator with one element per patch and
    an operator whose only far level is level 0 (leaf = patch) with its own degree match
    the oracle; a leaf level below a level of larger degree keeps parity."""
    from paper_1807_03097_amd import binding as B
    pats = W.cube_sphere()
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, 2, 3, 6.0, 6, 1.0, 5, 5, 1)
    with pytest.raises(B.IgeError) as e:
        op.apply(np.zeros((0, op.N), np.complex128))
    assert e.value.code == B.IGE_EINVAL
    z = np.zeros(op.N, np.complex128)
    assert np.array_equal(op.apply(z), z)
    f0 = op.rhs_plane_wave([[0.0, 0.0, 1.0]], [[0.0, 0.0, 0.0]])[0]
    assert np.array_equal(f0, z)
    x0, st, rc = op.solve(f0, tol=1e-8)
    assert rc == 0 and st[0][0] == 0 and np.array_equal(x0, z)
    assert op.potential(W.random_coeffs(op.N, 0), np.zeros((0, 3))).shape == (0, 3)
    assert np.array_equal(op.potential(z, [[0.0, 0.0, 3.0]]), np.zeros((1, 3), np.complex128))
    op.close()
    # scalar single layer with one element per patch
    sc = B.Operator(geom, 2, 0, 2.0, 4, 1.0, 5, 5, 0, kind=B.IGE_OP_SCALAR)
    o = oracle_mod.Oracle(pats, 2, 0, 2.0, g=5, gs=5, scalar=True)
    x = W.random_coeffs(sc.N, 1)
    assert sc.N == 6 * 9 and _rel(sc.apply(x), o.fmm_apply(x, 4, 1.0, 0)) <= TOL
    sc.close()
    # leaf = patch (leaf depth 3 at level 3): far blocks between opposite patches only
    # (eta = 12: their balls are 0.16 apart), on level 0, with a degree of its own
    ol = oracle_mod.Oracle(pats, 2, 3, 8.0, g=5, gs=5)
    for ql in ([9], [9, 0, 0, 0]):
        lq = B.Operator(geom, 2, 3, 8.0, 6, 12.0, 5, 5, 3, q_level=ql)
        assert lq.info.leaf_level == 0 and lq.q_levels() == [9] and lq.info.far_pairs == 6
        x = W.random_coeffs(lq.N, 2)
        assert _rel(lq.apply(x), ol.fmm_apply(x, [9], 12.0, 3)) <= TOL
        lq.close()


def test_peak_probes_are_plausible(ctx):
    """The library's own probes of the device's achievable peaks lie below the published
    figures (HBM 8 TB/s, dense BF16 2.5 PFLOP/s, FP64 matrix cores 78.6 TFLOP/s, with 10 %
    allowance for clocks above the nominal one) and well above a tenth of them."""
    from paper_1807_03097_amd import binding as B
    hbm = B.ige_peak_probe(ctx.h, B.IGE_PROBE_HBM)
    bf16 = B.ige_peak_probe(ctx.h, B.IGE_PROBE_MFMA_BF16)
    f64 = B.ige_peak_probe(ctx.h, B.IGE_PROBE_MFMA_F64)
    _say(f"  measured peaks: HBM {hbm:.0f} GB/s, BF16 {bf16:.0f} TFLOP/s, FP64 matrix cores {f64:.1f} TFLOP/s")
    assert 800.0 < hbm <= 8000.0 * 1.1
    assert 250.0 < bf16 <= 2500.0 * 1.1
    assert 7.86 < f64 <= 78.6 * 1.1
    with pytest.raises(B.IgeError):
        B.ige_peak_probe(ctx.h, 7)
