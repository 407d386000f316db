"""Parity of the HIP scalar single layer operator with the CPU oracle (FP64).

The scalar Helmholtz single layer on patchwise tensor B-splines, compressed with the
K_2 block alone (Sec. 4.2, eq. (eq:FMMlr) with the surface elements inside the
localized kernel eq. (eq:lockernel)).  Same bar as the EFIE operator: relative 2-norm
error <= 1e-12 against the oracle's compressed operator on the same partition, the
right-hand side and the single layer potential; GMRES solutions within tol * cond(A)
of LAPACK.
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
            "jittered": lambda: W.jitter(W.cube_sphere(), 0.01, 3)}[name]()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


SCASES = [
    # geometry, p, m, kappa, q, eta, leaf depth, g, gs
    ("sphere", 1, 2, 2.0, 6, 0.0, -1, 5, 5),       # dense: everything near field
    ("sphere", 2, 3, 8.0, 8, 1.0, 1, 5, 5),        # far field on three levels
    ("sphere", 2, 4, 8.0, 8, 1.0, 2, 5, 5),        # 16 x 16 elements per patch, 4 x 4 leaves
    ("torus", 2, 3, 4.0, 6, 1.0, 1, 5, 4),
    ("cube", 1, 3, 3.0, 5, 1.0, 1, 4, 5),          # flat patches, edges and corners
    ("jittered", 3, 3, 6.0, 7, 1.0, 1, 5, 5),      # cubic (16 local functions)
    ("sphere", 4, 2, 4.0, 8, 1.0, 1, 5, 5),        # quartic (25 local functions)
    ("sphere", 1, 3, 2.0, 3, 1.0, 0, 3, 6),        # leaf = element, low q
]


@pytest.mark.parametrize("case", SCASES, ids=[f"{c[0]}-p{c[1]}-m{c[2]}-eta{c[5]}-d{c[6]}" for c in SCASES])
def test_scalar_apply_matches_oracle(oracle_mod, ctx, case):
    from paper_1807_03097_amd import binding as B
    name, p, m, kappa, q, eta, d, g, gs = case
    _say(f"scalar case {case}")
    pats = _geom(name)
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, p, m, kappa, q, eta, g, gs, d, kind=B.IGE_OP_SCALAR)
    o = oracle_mod.Oracle(pats, p, m, kappa, g=g, gs=gs, scalar=True)
    assert op.N == o.N == len(pats) * ((1 << m) + p) ** 2
    dof, _ = op.dofmap()
    assert np.array_equal(dof, o.dof)
    x = W.random_coeffs(op.N, 0)
    y = op.apply(x)
    dd = d if d >= 0 else int(np.ceil(np.log2((q + 1) / (p + 1)) - 1e-12))
    yo = o.fmm_apply(x, q, eta, dd)
    err = _rel(y, yo)
    _say(f"  N={op.N} far={op.info.far_pairs} near={op.info.near_leaf_pairs} err={err:.2e}")
    assert err <= TOL
    # several columns in one call: the many-column kernels with the scalar branch
    X = np.stack([x, W.random_coeffs(op.N, 1), W.random_coeffs(op.N, 2)])
    Y = op.apply(X)
    assert _rel(Y[0], y) <= 1e-13
    assert _rel(Y[2], o.fmm_apply(X[2], q, eta, dd)) <= TOL


def test_scalar_dense_columns_match_oracle(oracle_mod, ctx):
    """eta = 0: every column of the library's scalar matrix against the oracle's dense
    matrix; the matrix is complex symmetric."""
    from paper_1807_03097_amd import binding as B
    pats = W.cube_sphere()
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, 2, 1, 3.0, 4, 0.0, 5, 5, -1, kind=B.IGE_OP_SCALAR)
    A = oracle_mod.Oracle(pats, 2, 1, 3.0, scalar=True).dense_matrix()
    Ag = op.apply(np.eye(op.N, dtype=np.complex128)).T
    assert np.max(np.abs(Ag - A)) <= TOL * np.max(np.abs(A))
    assert np.max(np.abs(Ag - Ag.T)) <= 1e-13 * np.max(np.abs(Ag))


def test_scalar_near_assembly_is_reproducible(ctx):
    """Assembly of the scalar near field is deterministic: two assemblies give the same
    bits, and so do two applies."""
    from paper_1807_03097_amd import binding as B
    geom = B.Geometry(ctx, _geom("jittered"))
    ops = [B.Operator(geom, 2, 3, 6.0, 7, 1.0, 5, 5, 1, kind=B.IGE_OP_SCALAR) for _ in range(2)]
    assert np.array_equal(ops[0].near_blocks(), ops[1].near_blocks())
    x = W.random_coeffs(ops[0].N, 3)
    assert np.array_equal(ops[0].apply(x), ops[1].apply(x))


@pytest.mark.parametrize("kind", ["point", "plane"])
def test_scalar_rhs_matches_oracle(oracle_mod, ctx, kind):
    from paper_1807_03097_amd import binding as B
    pats = _geom("torus")
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, 2, 2, 3.0, 6, 1.0, 4, 4, 1, kind=B.IGE_OP_SCALAR)
    o = oracle_mod.Oracle(pats, 2, 2, 3.0, g=4, gs=4, scalar=True)
    a = [[0.1, 0.2, -0.15], [2.5, 0.3, 0.4]] if kind == "point" else [[0.0, 0.6, 0.8], [1.0, 0.0, 0.0]]
    code = B.IGE_RHS_POINT if kind == "point" else B.IGE_RHS_PLANE
    F = op.rhs_scalar(code, a)
    for c in range(2):
        assert _rel(F[c], o.rhs_scalar(kind, a[c])) <= TOL


def test_scalar_solve_and_potential(oracle_mod, ctx):
    """Exterior Dirichlet problem with the data of a point source inside the sphere:
    GMRES on the compressed scalar operator, then the single layer potential at
    r = 3.  The density matches the oracle's dense LAPACK solve within tol * cond, and
    the potential reproduces G(x - x0) to the discretisation error the oracle itself
    reaches (p = 2, m = 3)."""
    from paper_1807_03097_amd import binding as B
    pats = W.cube_sphere()
    geom = B.Geometry(ctx, pats)
    x0, kappa = np.array([0.1, 0.2, -0.15]), 2.0
    op = B.Operator(geom, 2, 3, kappa, 10, 1.0, 5, 5, 1, kind=B.IGE_OP_SCALAR)
    f = op.rhs_scalar(B.IGE_RHS_POINT, x0)[0]
    w, st, rc = op.solve(f, tol=1e-11, restart=200, maxit=2000)
    assert rc == B.IGE_OK, st
    _say(f"  N={op.N} iters={st[0][0]} relres={st[0][2]:.2e}")
    o = oracle_mod.Oracle(pats, 2, 3, kappa, g=5, gs=5, scalar=True)
    A = o.dense_matrix()
    wd = np.linalg.solve(A, o.rhs_scalar("point", x0))
    cond = np.linalg.cond(A)
    assert _rel(w, wd) <= 1e-11 * cond + 1e-8, (_rel(w, wd), cond)
    pts = np.array([[3.0, 0, 0], [0, -3.0, 0], [0, 0, 3.0], [1.7, 1.7, 1.7], [-2.0, 1.0, -2.0]])
    u = op.potential(w, pts)
    assert np.all(u[:, 1:] == 0)
    uo = o.potential_scalar(w, pts)
    assert _rel(u[:, 0], uo) <= TOL
    d = np.linalg.norm(pts - x0, axis=1)
    ref = np.exp(1j * kappa * d) / (4 * np.pi * d)
    err = np.abs(u[:, 0] - ref).max() / np.abs(ref).max()
    _say(f"  potential error vs point source {err:.2e}")
    assert err <= 1e-5


MCASES = [SCASES[2], SCASES[5], SCASES[6], SCASES[7]]


@pytest.mark.parametrize("case", MCASES, ids=[f"{c[0]}-p{c[1]}-m{c[2]}-d{c[6]}" for c in MCASES])
def test_scalar_many_columns_and_precisions(oracle_mod, ctx, case):
    """The scalar operator on the many-column kernels (the scalar branches of the
    batched P2M, M2M, coupling reduction, L2P and gather) and in every apply
    precision.  FP64: 11 columns, 64 (the FP64 matrix-core coupling and near field)
    and 70 (a ragged column chunk) against single columns to 1e-13 and the oracle to
    1e-12; FP32 coupling within its 2^-23-level bound; plain BF16 coupling within
    2^-9-level error; split BF16 (coupling, and coupling and near field) within
    2^-16-level error; an operator with stored coupling blocks equal to the generated
    one."""
    from paper_1807_03097_amd import binding as B
    name, p, m, kappa, q, eta, d, g, gs = case
    _say(f"scalar many-column case {case}")
    pats = _geom(name)
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, p, m, kappa, q, eta, g, gs, d, kind=B.IGE_OP_SCALAR)
    o = oracle_mod.Oracle(pats, p, m, kappa, g=g, gs=gs, scalar=True)
    XA = np.stack([W.random_coeffs(op.N, 300 + s) for s in range(70)])
    cols = (0, 10, 35, 63, 69)
    Y1 = {c: op.apply(XA[c].copy()) for c in cols}
    yo0, yo69 = o.fmm_apply(XA[0], q, eta, d), o.fmm_apply(XA[69], q, eta, d)
    assert _rel(Y1[0], yo0) <= TOL
    for nc in (11, 64, 70):
        Y = op.apply(XA[:nc].copy())
        e1 = max(_rel(Y[c], Y1[c]) for c in cols if c < nc)
        eo = _rel(Y[0], yo0)
        _say(f"  N={op.N} {nc} columns: vs single columns {e1:.2e}, first vs oracle {eo:.2e}")
        assert e1 <= 1e-13 and eo <= TOL
    assert _rel(Y[69], yo69) <= TOL
    X11 = XA[:11].copy()
    Y64 = op.apply(X11)
    for prec, lo, hi in ((B.IGE_F32, 1e-12, 1e-5), (B.IGE_BF16, 1e-6, 1e-2), (B.IGE_BF16X3, 1e-12, 2e-4),
                         (B.IGE_BF16X3_ALL, 1e-12, 2e-4)):
        y1 = op.apply(XA[0].copy(), prec=prec)
        Y = op.apply(X11, prec=prec)
        e1, eb = _rel(y1, yo0), max(_rel(Y[c], Y64[c]) for c in range(11))
        _say(f"  prec {prec}: 1 column vs oracle {e1:.2e}, worst of 11 vs FP64 {eb:.2e}")
        if op.info.far_pairs > 0 or prec == B.IGE_BF16X3_ALL:
            assert lo < e1
        assert e1 <= hi and eb <= hi
    st = B.Operator(geom, p, m, kappa, q, eta, g, gs, d, store_coupling=1, kind=B.IGE_OP_SCALAR)
    es1, esb = _rel(st.apply(XA[0].copy()), yo0), max(_rel(a, b) for a, b in zip(st.apply(X11), Y64))
    _say(f"  stored coupling: 1 column vs oracle {es1:.2e}, 11 columns vs generated {esb:.2e}")
    assert es1 <= TOL and esb <= 1e-13
    st.close()
    op.close()


def test_scalar_refined_solve_and_autotune(oracle_mod, ctx):
    """FP64 refinement around FP32, split-BF16 and split-BF16-near-field inner solves of
    the scalar operator meets the FP64 tolerance, and the solutions agree with the FP64
    solve within the tolerance times the condition number; autotuning keeps the
    results to rounding."""
    from paper_1807_03097_amd import binding as B
    pats = W.cube_sphere()
    geom = B.Geometry(ctx, pats)
    op = B.Operator(geom, 2, 3, 2.0, 10, 1.0, 5, 5, 1, kind=B.IGE_OP_SCALAR)
    F = op.rhs_scalar(B.IGE_RHS_POINT, [[0.1, 0.2, -0.15], [0.3, -0.1, 0.2]])
    X64, st64, rc = op.solve(F, tol=1e-10, restart=200, maxit=3000)
    assert rc == B.IGE_OK, st64
    cond = np.linalg.cond(oracle_mod.Oracle(pats, 2, 3, 2.0, g=5, gs=5, scalar=True).dense_matrix())
    for iprec in (B.IGE_F32, B.IGE_BF16X3, B.IGE_BF16X3_ALL):
        Xr, st, rc2 = op.solve(F, tol=1e-10, restart=200, maxit=6000, refine=True, inner_tol=1e-4,
                               inner_prec=iprec)
        assert rc2 == B.IGE_OK, st
        for c in range(2):
            d = _rel(Xr[c], X64[c])
            _say(f"  inner prec {iprec} col {c}: FP64 iters {st64[c][0]}, refined iters {st[c][0]} outer "
                 f"{st[c][1]} relres {st[c][2]:.2e}, vs FP64 {d:.2e} (cond {cond:.1e})")
            assert st[c][2] <= 1.05e-10 and d <= 2.1e-10 * cond
    X = np.stack([W.random_coeffs(op.N, 400 + s) for s in range(20)])
    for prec in (B.IGE_F64, B.IGE_BF16X3):
        y0 = op.apply(X, prec=prec)
        ch = op.autotune(20, prec)
        y1 = op.apply(X, prec=prec)
        err = max(_rel(y1[c], y0[c]) for c in range(len(X)))
        _say(f"  autotune prec {prec}: chosen {ch}, max rel change {err:.1e}")
        assert ch and err <= 1e-13
    op.close()


def test_scalar_refusals(ctx):
    """Plane-wave EFIE data, a scalar right-hand side on the EFIE operator, an unknown
    data kind and serving of the scalar operator are refused with IGE_EINVAL."""
    from paper_1807_03097_amd import binding as B
    geom = B.Geometry(ctx, W.cube_sphere())
    op = B.Operator(geom, 1, 2, 2.0, 6, 1.0, 4, 4, 1, kind=B.IGE_OP_SCALAR)
    with pytest.raises(B.IgeError) as e:
        op.rhs_plane_wave([0, 0, 1.0], [1.0, 0, 0])
    assert e.value.code == B.IGE_EINVAL
    efie = B.Operator(geom, 1, 2, 2.0, 6, 1.0, 4, 4, 1)
    with pytest.raises(B.IgeError):
        efie.rhs_scalar(B.IGE_RHS_POINT, [0, 0, 0])
    with pytest.raises(B.IgeError):
        op.rhs_scalar(5, [0, 0, 0])
    srv = B.Server(ctx, 1)
    try:
        with pytest.raises(B.IgeError):
            srv.submit(geom, 1, 2, 2.0, [0, 0, 1.0], [1.0, 0, 0], kind=B.IGE_OP_SCALAR)
    finally:
        srv.close()
