"""The allocation-free potential entry point (ige_potential_noalloc) against the
allocating one (ige_potential): same kernels, so the same bits, on two calls in a row
(the second with a smaller operator and fewer points and columns, so the fixed scratch
holds the first call's data when the second starts), and a clear refusal of an
operator whose source data exceed the fixed scratch."""
import numpy as np
import pytest

from paper_1807_03097_amd import workloads as W

pytestmark = pytest.mark.gpu


def _points(n, radius, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    return radius * v / np.linalg.norm(v, axis=1, keepdims=True)


def test_potential_noalloc_equals_potential():
    import torch
    from paper_1807_03097_amd import binding as B
    ctx = B.Context(0)
    geom = B.Geometry(ctx, W.cube_sphere())
    # (p, level, kappa, columns, points): the second call is smaller in every size
    for (p, m, kappa, r, npts) in ((2, 4, 6.0, 3, 150), (1, 2, 2.0, 1, 17)):
        print(f"noalloc potential: sphere p={p} m={m} kappa={kappa} r={r} npts={npts}", flush=True)
        op = B.Operator(geom, p, m, kappa, 8, 1.0, 5, 5, 1)
        w = np.stack([W.random_coeffs(op.N, s) for s in range(r)])
        pts = _points(npts, 3.0, p + m)
        ref = op.potential(w, pts)                       # [r][npts][3], host
        wd = torch.from_numpy(w).to("cuda:0")
        pd = torch.from_numpy(pts).to("cuda:0")
        Ed = torch.full((r, npts, 3), complex("nan"), dtype=torch.complex128, device="cuda:0")
        op.potential_noalloc(wd, pd, Ed)
        torch.cuda.synchronize()
        got = Ed.cpu().numpy()
        assert np.all(np.isfinite(got))
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"  rel. difference {err:.1e}", flush=True)
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
        op.close()
    # elements * g^2 * 88 bytes > 64 MiB: refused before any device work
    big = B.Operator(geom, 1, 6, 2.0, 8, 1.6, 6, 4, 3)
    w = torch.zeros((big.N,), dtype=torch.complex128, device="cuda:0")
    pd = torch.zeros((4, 3), dtype=torch.float64, device="cuda:0")
    Ed = torch.zeros((4, 3), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(B.IgeError, match="fixed potential scratch"):
        big.potential_noalloc(w, pd, Ed)
    big.close()
    geom.close()
    ctx.close()
