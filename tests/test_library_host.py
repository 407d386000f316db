"""CPU checks of the HIP library: the shared object loads, exports every entry
point the header declares, and its host-side planning (glued unknowns, cluster
and block-cluster trees) equals the oracle's bit for bit.  No device calls."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1807_03097_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(ige_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    from paper_1807_03097_amd import binding
    lib = ctypes.CDLL(binding.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert binding.ige_version().startswith("igaefie")


def test_invalid_geometry_is_rejected():
    from paper_1807_03097_amd import binding as B
    ctx = B.Context(-1)
    pats = W.cube_sphere()
    bad = [dict(p) for p in pats]
    bad[0] = dict(bad[0], ctrl=bad[0]["ctrl"].copy())
    bad[0]["ctrl"][1, 1, 3] = -1.0          # negative weight
    with pytest.raises(B.IgeError) as e:
        B.Geometry(ctx, bad)
    assert e.value.code == B.IGE_EINVAL
    with pytest.raises(B.IgeError):
        B.Geometry(ctx, pats[:5])           # open surface: an edge without partner
    moved = [dict(p) for p in pats]
    moved[2] = dict(moved[2], ctrl=moved[2]["ctrl"] + np.array([0, 0, 1e-3, 0]))
    with pytest.raises(B.IgeError):
        B.Geometry(ctx, moved)              # interfaces do not coincide
    g = B.Geometry(ctx, pats)
    with pytest.raises(B.IgeError):
        B.Operator(g, 0, 2, 1.0, plan_only=True)     # p < 1
    with pytest.raises(B.IgeError):
        B.Operator(g, 1, 2, -1.0, plan_only=True)    # kappa <= 0
    op = B.Operator(g, 1, 1, 1.0, plan_only=True)
    with pytest.raises(B.IgeError):
        op.apply(np.zeros(op.N, np.complex128))      # planned, not assembled
    with pytest.raises(B.IgeError) as e:
        op.autotune(4, B.IGE_BF16X3)                 # planned, not assembled
    assert e.value.code == B.IGE_EINVAL
    with pytest.raises(B.IgeError):
        op.apply(np.zeros(op.N, np.complex128), prec=6)   # no such precision


def test_plan_with_kappa_cap_matches_oracle(oracle_mod):
    """The wavenumber cap of the admissibility condition gives the oracle's partition."""
    from paper_1807_03097_amd import binding as B
    pats = W.cube_sphere()
    ctx = B.Context(-1)
    g = B.Geometry(ctx, pats)
    o = oracle_mod.Oracle(pats, 2, 4, 16.0, g=2)
    for cap in (6.0, 8.0, 12.0):
        op = B.Operator(g, 2, 4, 16.0, 8, 1.6, leaf_depth=2, plan_only=True, kappa_cap=cap)
        tr = o.block_tree(1.6, 2, kappa_cap=cap)
        pt = op.partition()
        assert np.array_equal(pt["far"], tr["far"]) and np.array_equal(pt["near"], tr["near"])
    with pytest.raises(B.IgeError):
        B.Operator(g, 2, 4, 16.0, 8, 1.6, leaf_depth=2, plan_only=True, kappa_cap=-1.0)


@pytest.mark.parametrize("geom,p,m,eta,d,q", [
    ("sphere", 1, 2, 0.0, -1, 8), ("sphere", 2, 3, 1.6, 1, 8), ("sphere", 2, 5, 1.0, 2, 8),
    ("torus", 2, 4, 1.0, 2, 6), ("cube", 1, 4, 0.7, 1, 4), ("jittered", 2, 4, 1.0, 2, 8),
    ("multispan", 2, 3, 1.0, 1, 6),
])
def test_plan_matches_oracle(oracle_mod, geom, p, m, eta, d, q):
    from paper_1807_03097_amd import binding as B
    pats = {"sphere": W.cube_sphere, "torus": W.torus, "cube": W.flat_cube,
            "jittered": lambda: W.jitter(W.cube_sphere(), 0.01, 3),
            "multispan": lambda: [W.refine_patch_knots(pt, 2, 2) for pt in W.cube_sphere()]}[geom]()
    ctx = B.Context(-1)
    g = B.Geometry(ctx, pats)
    op = B.Operator(g, p, m, 8.0, q, eta, leaf_depth=d, plan_only=True)
    o = oracle_mod.Oracle(pats, p, m, 8.0, g=2)
    assert op.N == o.N
    dof, sgn = op.dofmap()
    assert np.array_equal(dof, o.dof) and np.array_equal(sgn, o.sgn)
    dd = d if d >= 0 else int(np.ceil(np.log2((q + 1) / (p + 1)) - 1e-12))
    tr = o.block_tree(eta if eta > 0 else 0.0, dd)
    pt = op.partition()
    assert pt["L"] == tr["L"]
    assert np.array_equal(pt["far"], tr["far"])
    assert np.array_equal(pt["near"], tr["near"])


@pytest.mark.parametrize("geom,p,m,eta,d", [
    ("sphere", 2, 3, 1.6, 1), ("torus", 1, 3, 1.0, 1), ("sphere", 3, 3, 1.0, 2), ("sphere", 1, 2, 0.0, -1),
])
def test_near_distinct_entries_match_oracle_pattern(oracle_mod, geom, p, m, eta, d):
    """The near field stored once per entry holds exactly the distinct entries
    (i <= j) of the near-field pattern: glued unknowns i, j whose supports meet the
    leaves of a near leaf pair, counted here from the oracle's own unknown table and
    block tree (Sec. 4.2, eq. (eq::superspace) supports)."""
    from paper_1807_03097_amd import binding as B
    pats = {"sphere": W.cube_sphere, "torus": W.torus}[geom]()
    ctx = B.Context(-1)
    g = B.Geometry(ctx, pats)
    op = B.Operator(g, p, m, 4.0, 6, eta, leaf_depth=d, plan_only=True)
    o = oracle_mod.Oracle(pats, p, m, 4.0, g=2)
    dd = d if d >= 0 else int(np.ceil(np.log2(7 / (p + 1)) - 1e-12))
    tr = o.block_tree(eta, dd)
    L, n = tr["L"], 1 << m
    s, SL = n >> L, 1 << L
    # unknowns whose support meets each leaf
    sets = [set() for _ in range(o.P * SL * SL)]
    J, A, I2, I1 = np.nonzero(o.dof >= 0)
    for j, a, i2, i1 in zip(J, A, I2, I1):
        pu, pv = (p, p - 1) if a == 0 else (p - 1, p)
        for e2 in range(max(0, i2 - pv), min(n, i2 + 1)):
            for e1 in range(max(0, i1 - pu), min(n, i1 + 1)):
                sets[(j * SL + e2 // s) * SL + e1 // s].add(int(o.dof[j, a, i2, i1]))
    keys = set()
    for t, u in tr["near"]:
        I = np.array(sorted(sets[t])); Jv = np.array(sorted(sets[u]))
        ii, jj = np.meshgrid(I, Jv, indexing="ij")
        keys.update((np.minimum(ii, jj).ravel() * o.N + np.maximum(ii, jj).ravel()).tolist())
    assert op.info.near_distinct == len(keys)
    assert op.info.near_distinct < op.info.near_nnz or eta == 0.0


@pytest.mark.parametrize("p,m,eta,d", [(1, 3, 1.0, 1), (2, 3, 1.6, 1), (4, 2, 1.0, 1)])
def test_scalar_plan_matches_oracle(oracle_mod, p, m, eta, d):
    """The scalar single layer (kind IGE_OP_SCALAR): unknown table, partition and the
    count of distinct near-field entries equal the oracle's (tensor B-splines of degree
    p on every patch, supports of p + 1 elements per direction)."""
    from paper_1807_03097_amd import binding as B
    pats = W.cube_sphere()
    ctx = B.Context(-1)
    g = B.Geometry(ctx, pats)
    op = B.Operator(g, p, m, 4.0, 6, eta, leaf_depth=d, plan_only=True, kind=B.IGE_OP_SCALAR)
    o = oracle_mod.Oracle(pats, p, m, 4.0, g=2, scalar=True)
    assert op.N == o.N == len(pats) * ((1 << m) + p) ** 2
    dof, sgn = op.dofmap()
    assert np.array_equal(dof, o.dof) and np.array_equal(sgn, o.sgn)
    tr = o.block_tree(eta, d)
    pt = op.partition()
    assert np.array_equal(pt["far"], tr["far"]) and np.array_equal(pt["near"], tr["near"])
    L, n = tr["L"], 1 << m
    s, SL = n >> L, 1 << L
    sets = [set() for _ in range(o.P * SL * SL)]
    J, _, I2, I1 = np.nonzero(o.dof >= 0)
    for j, i2, i1 in zip(J, I2, I1):
        for e2 in range(max(0, i2 - p), min(n, i2 + 1)):
            for e1 in range(max(0, i1 - p), min(n, i1 + 1)):
                sets[(j * SL + e2 // s) * SL + e1 // s].add(int(o.dof[j, 0, i2, i1]))
    keys = set()
    for t, u in tr["near"]:
        I = np.array(sorted(sets[t])); Jv = np.array(sorted(sets[u]))
        ii, jj = np.meshgrid(I, Jv, indexing="ij")
        keys.update((np.minimum(ii, jj).ravel() * o.N + np.maximum(ii, jj).ravel()).tolist())
    assert op.info.near_distinct == len(keys)
    with pytest.raises(B.IgeError):
        B.Operator(g, p, m, 4.0, 6, eta, leaf_depth=d, plan_only=True, kind=2)


def test_level_degrees_plan_and_diameters_match_oracle(oracle_mod):
    """q_level: the partition does not depend on the degrees, the info reports each
    level's degree and the largest bounding-ball diameter of its clusters (the
    oracle's balls, to rounding), the binding's degree rule gives the oracle-pinned
    degrees at level 6 / kappa 16, and out-of-range degrees are refused."""
    from paper_1807_03097_amd import binding as B
    pats = W.cube_sphere()
    ctx = B.Context(-1)
    g = B.Geometry(ctx, pats)
    op0 = B.Operator(g, 2, 4, 8.0, 8, 1.0, leaf_depth=1, plan_only=True)
    op = B.Operator(g, 2, 4, 8.0, 8, 1.0, leaf_depth=1, plan_only=True, q_level=[8, 10, 0, 6])
    assert op.q_levels() == [8, 10, 8, 6] and op.info.q == 10 and op0.q_levels() == [8, 8, 8, 8]
    p0, p1 = op0.partition(), op.partition()
    assert np.array_equal(p0["far"], p1["far"]) and np.array_equal(p0["near"], p1["near"])
    o = oracle_mod.Oracle(pats, 2, 4, 8.0, g=2)
    for lvl, dm in enumerate(op.level_diameters()):
        _, rad = o.bounding_balls(lvl)
        assert abs(dm - 2 * rad.max()) <= 1e-12 * dm
    c3 = B.Operator(g, 2, 6, 16.0, 8, 1.6, leaf_depth=3, plan_only=True)
    far_levels = set(c3.partition()["far"][:, 0].tolist())
    assert B.degree_rule(c3.info, 16.0, 8, far_levels) == [8, 14, 10, 8]
    for bad in ([16], [-1], [0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 20]):
        with pytest.raises(B.IgeError):
            B.Operator(g, 2, 4, 8.0, 8, 1.0, leaf_depth=1, plan_only=True, q_level=bad)
