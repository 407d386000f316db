"""Seeded synthetic inputs shared by the library tests, the benchmark and the oracle.

This module only *builds inputs*: NURBS patch descriptions of closed surfaces,
random coefficient vectors and incident plane-wave directions.  It holds none
of the boundary-element arithmetic (no basis functions, no quadrature, no
kernel), so both the HIP library and the CPU oracle may take their inputs from
here without sharing any of the method's code.

A patch is a dict with keys
    deg   (pu, pv)                polynomial degrees of the NURBS map F_j
    ku,kv open knot vectors       (nu+pu+1,), (nv+pv+1,)
    ctrl  (nv, nu, 4) float64     Euclidean control point (x, y, z) and weight w>0,
                                  u index fastest (ctrl[j2, j1] multiplies b_j1(u) b_j2(v))
which is the rational tensor-product map of Section 3.1 (definition of the
parametrisation F_j : [0,1]^2 -> Gamma_j).  Every generator orients its patches so
that d_u F x d_v F points out of the enclosed domain.
"""
from __future__ import annotations

import math
import numpy as np

__all__ = [
    "cube_sphere", "torus", "flat_cube", "jitter", "pack", "random_coeffs",
    "fibonacci_plane_waves", "random_plane_waves", "refine_patch_knots",
]


def _patch(ctrl, deg=(2, 2), ku=None, kv=None):
    ctrl = np.ascontiguousarray(ctrl, dtype=np.float64)
    pu, pv = deg
    nv, nu = ctrl.shape[:2]
    if ku is None:
        ku = np.r_[np.zeros(pu + 1), np.ones(pu + 1)]
    if kv is None:
        kv = np.r_[np.zeros(pv + 1), np.ones(pv + 1)]
    return {"deg": (int(pu), int(pv)), "ku": np.asarray(ku, float),
            "kv": np.asarray(kv, float), "ctrl": ctrl}


# --------------------------------------------------------------------------
# cube-sphere: six biquadratic rational patches approximating the unit sphere
# --------------------------------------------------------------------------
def _face_frames():
    """(normal, e_u, e_v) of the six cube faces with e_u x e_v = normal."""
    I = np.eye(3)
    frames = []
    for axis in range(3):
        for sgn in (1.0, -1.0):
            n = sgn * I[axis]
            a, b = I[(axis + 1) % 3], I[(axis + 2) % 3]
            if sgn < 0:
                a, b = b, a
            assert np.allclose(np.cross(a, b), n)
            frames.append((n, a, b))
    return frames


def cube_sphere(radius: float = 1.0):
    """Six biquadratic rational Bezier patches covering a sphere-like closed surface.

    The four boundary curves of every patch are exact great-circle arcs between
    the projected cube corners (rational quadratic arc: middle weight cos(theta/2),
    theta = arccos(1/3)), shared verbatim with the neighbouring patch, so the
    interfaces coincide exactly.  The interior control point lies on the face axis
    with the tensor weight cos^2(theta/2) and is placed so that F(1/2,1/2) is on the
    sphere.  Away from the arcs and the face centre the surface deviates from the
    sphere by about 1e-2 of the radius (`cube_sphere_radial_deviation`).
    """
    s3 = 1.0 / math.sqrt(3.0)
    wa = math.sqrt(2.0 / 3.0)              # cos(theta/2) with cos(theta) = 1/3
    patches = []
    for n, a, b in _face_frames():
        P = np.zeros((3, 3, 4))
        W = np.zeros((3, 3))
        for j2, y in enumerate((-1.0, 0.0, 1.0)):
            for j1, x in enumerate((-1.0, 0.0, 1.0)):
                c = n + x * a + y * b
                if x != 0.0 and y != 0.0:           # cube corner projected to the sphere
                    pt, w = c * s3, 1.0
                elif x == 0.0 and y == 0.0:
                    pt, w = None, wa * wa
                else:                                # arc middle point: midpoint direction / cos(theta/2)
                    pt, w = c / np.linalg.norm(c) / wa, wa
                if pt is not None:
                    P[j2, j1, :3] = pt
                W[j2, j1] = w
        # place the centre point on the axis so that F(1/2,1/2) = n
        B = np.array([0.25, 0.5, 0.25])
        BB = np.outer(B, B)
        den = np.sum(BB * W)
        num = np.einsum("ij,ij,ijk->k", BB, W, P[:, :, :3])
        # num + BB[1,1]*W[1,1]*c*n = den*n  (centre contribution along n only)
        cz = (den - num @ n) / (BB[1, 1] * W[1, 1])
        P[1, 1, :3] = cz * n
        P[:, :, :3] *= radius
        P[:, :, 3] = W
        patches.append(_patch(P))
    return patches


def flat_cube(half: float = 0.5):
    """Six bilinear (degree (1,1)) flat patches bounding the cube [-half, half]^3."""
    patches = []
    for n, a, b in _face_frames():
        P = np.zeros((2, 2, 4))
        for j2, y in enumerate((-1.0, 1.0)):
            for j1, x in enumerate((-1.0, 1.0)):
                P[j2, j1, :3] = half * (n + x * a + y * b)
                P[j2, j1, 3] = 1.0
        patches.append(_patch(P, deg=(1, 1)))
    return patches


def torus(R: float = 1.0, r: float = 0.3):
    """Sixteen exact rational biquadratic patches of the torus (major R, minor r).

    Tensor product of two circles, each split into four quarter arcs with
    weights (1, sqrt(2)/2, 1); u runs along the major circle, v along the minor
    one, which orients d_u F x d_v F outwards.
    """
    h = math.sqrt(0.5)
    quarter = [((1, 0), (1, 1), (0, 1)), ((0, 1), (-1, 1), (-1, 0)),
               ((-1, 0), (-1, -1), (0, -1)), ((0, -1), (1, -1), (1, 0))]
    wq = (1.0, h, 1.0)
    patches = []
    for qi in range(4):            # major circle quarter (u)
        for qj in range(4):        # minor circle quarter (v)
            P = np.zeros((3, 3, 4))
            for j2 in range(3):
                cx, cz = quarter[qj][j2]
                X, Z = R + r * cx, r * cz          # profile control point in the (rho, z) half plane
                for j1 in range(3):
                    ax, ay = quarter[qi][j1]
                    P[j2, j1, :3] = (X * ax, X * ay, Z)
                    P[j2, j1, 3] = wq[j1] * wq[j2]
            patches.append(_patch(P))
    return patches


def refine_patch_knots(patch, nu_spans: int, nv_spans: int):
    """Re-express a single-span rational Bezier patch on uniform knot vectors with
    `nu_spans` x `nv_spans` C^0 spans (knot multiplicity = degree), by rational
    Bezier subdivision.  Produces genuine multi-span NURBS inputs describing the
    same surface (used to exercise Bezier extraction of general knot vectors)."""
    pu, pv = patch["deg"]
    ctrl = patch["ctrl"]
    assert ctrl.shape[:2] == (pv + 1, pu + 1), "single Bezier span expected"
    hom = ctrl.copy()
    hom[..., :3] *= hom[..., 3:4]

    def sub1d(cp, a, b, p):
        # control points of the restriction of a degree-p Bezier curve to [a,b] (blossoming
        # via repeated de Casteljau), cp shape (p+1, k)
        # split at b -> keep left part, then split that at a/b -> keep right part
        def split(c, t):
            left = [c[0].copy()]
            right = [c[-1].copy()]
            cc = c.copy()
            for r in range(1, p + 1):
                cc = (1 - t) * cc[:-1] + t * cc[1:]
                left.append(cc[0].copy())
                right.append(cc[-1].copy())
            return np.array(left), np.array(right[::-1])
        left, _ = split(cp, b)
        if b == 0:
            return left
        _, right = split(left, a / b)
        return right

    nu_c = nu_spans * pu + 1
    nv_c = nv_spans * pv + 1
    out = np.zeros((nv_c, nu_c, 4))
    # subdivide in u for each row, then in v for each column
    tmp = np.zeros((pv + 1, nu_c, 4))
    for j2 in range(pv + 1):
        for s in range(nu_spans):
            seg = sub1d(hom[j2], s / nu_spans, (s + 1) / nu_spans, pu)
            tmp[j2, s * pu: s * pu + pu + 1] = seg
    for j1 in range(nu_c):
        for s in range(nv_spans):
            seg = sub1d(tmp[:, j1], s / nv_spans, (s + 1) / nv_spans, pv)
            out[s * pv: s * pv + pv + 1, j1] = seg
    out[..., :3] /= out[..., 3:4]
    ku = np.r_[np.zeros(pu + 1), np.repeat(np.arange(1, nu_spans) / nu_spans, pu), np.ones(pu + 1)]
    kv = np.r_[np.zeros(pv + 1), np.repeat(np.arange(1, nv_spans) / nv_spans, pv), np.ones(pv + 1)]
    return _patch(out, deg=(pu, pv), ku=ku, kv=kv)


def jitter(patches, sigma: float, seed: int, tol: float = 1e-12):
    """Perturb every *distinct* control point once by i.i.d. N(0, sigma^2) per
    coordinate (points shared by several patches move together, so interfaces stay
    conforming); weights are unchanged."""
    rng = np.random.default_rng(seed)
    out = [dict(p, ctrl=p["ctrl"].copy()) for p in patches]
    reps, moves = [], []
    for p in out:
        c = p["ctrl"]
        for j2 in range(c.shape[0]):
            for j1 in range(c.shape[1]):
                x = c[j2, j1, :3]
                hit = None
                for k, r in enumerate(reps):
                    if np.max(np.abs(r - x)) <= tol:
                        hit = k
                        break
                if hit is None:
                    reps.append(x.copy())
                    moves.append(rng.standard_normal(3) * sigma)
                    hit = len(reps) - 1
                c[j2, j1, :3] = x + moves[hit]
    return out


def pack(patches):
    """Flatten patches into the C-ABI arrays: degree[2P], n_ctrl[2P], knots (u then v
    per patch, concatenated), ctrl [sum nu*nv][4] (x,y,z,w), u fastest."""
    deg = np.array([d for p in patches for d in p["deg"]], dtype=np.int32)
    nctrl = np.array([s for p in patches for s in (p["ctrl"].shape[1], p["ctrl"].shape[0])], dtype=np.int32)
    knots = np.concatenate([np.r_[p["ku"], p["kv"]] for p in patches]).astype(np.float64)
    ctrl = np.concatenate([p["ctrl"].reshape(-1, 4) for p in patches]).astype(np.float64)
    return deg, nctrl, np.ascontiguousarray(knots), np.ascontiguousarray(ctrl)


def random_coeffs(n: int, seed: int = 0, nrhs: int = 1):
    """x = N(0,1) + i N(0,1) per entry; all real parts are drawn first, then all
    imaginary parts; column-major for nrhs > 1 (shape (nrhs, n) row = one RHS)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(n * nrhs)
    im = rng.standard_normal(n * nrhs)
    x = (re + 1j * im).reshape(nrhs, n)
    return x[0] if nrhs == 1 else x


def fibonacci_plane_waves(n: int):
    """n directions on a Fibonacci lattice of S^2 with theta-hat polarisations.
    Returns (dirs (n,3), pols (n,3) complex)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    d = np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)
    pol = np.stack([z * np.cos(phi), z * np.sin(phi), -rho], axis=1)
    return d, pol.astype(np.complex128)


def random_plane_waves(n: int, seed: int):
    """n random unit directions with a random unit polarisation orthogonal to each."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    g = rng.standard_normal((n, 3))
    g -= np.sum(g * d, axis=1, keepdims=True) * d
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return d, g.astype(np.complex128)
