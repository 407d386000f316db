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
    # several columns in one call: column by column on the same kernels, same bits
    X = np.stack([x, W.random_coeffs(op.N, 1), W.random_coeffs(op.N, 2)])
    Y = op.apply(X)
    assert np.array_equal(Y[0], y)
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


def test_scalar_refusals(ctx):
    """The scalar operator runs in FP64 only: lower-precision couplings, refinement,
    autotuning, plane-wave EFIE data and serving are refused with IGE_EINVAL."""
    from paper_1807_03097_amd import binding as B
    geom = B.Geometry(ctx, W.cube_sphere())
    op = B.Operator(geom, 1, 2, 2.0, 6, 1.0, 4, 4, 1, kind=B.IGE_OP_SCALAR)
    x = W.random_coeffs(op.N, 0)
    for prec in (B.IGE_F32, B.IGE_BF16X3):
        with pytest.raises(B.IgeError) as e:
            op.apply(x, prec=prec)
        assert e.value.code == B.IGE_EINVAL
    with pytest.raises(B.IgeError):
        op.solve(x, refine=True)
    with pytest.raises(B.IgeError):
        op.autotune(2)
    with pytest.raises(B.IgeError):
        op.rhs_plane_wave([0, 0, 1.0], [1.0, 0, 0])
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
