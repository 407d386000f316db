"""Writes tests/golden/<name>_dense_rows.json: sampled rows of the dense Galerkin
matrix-vector product A x (no compression: every element pair by the quadrature of
Sec. 4.1, i.e. the plain definition of eq. (eq:MSLtested)), computed by the CPU oracle
alone, for x = N(0,1) + i N(0,1) from seed 0 in the canonical unknown order.

  c2  six-patch NURBS sphere, level 5, p = 2, kappa = 8, 48 rows
  c3  the same sphere, level 6, p = 2, kappa = 16, 24 rows
  c5  the sphere with control points jittered N(0, 0.02^2) (seed 7), level 7, p = 2,
      kappa = 40, 12 rows

Disjoint element pairs take the 5 x 5 Gauss rule, the singular sub-rules 5 points per
variable.  The FMM rows of the same configurations are compared with these (Theorem
(thm::mutlipole): the compression error decays exponentially in q).

Run from the repository root:  python tests/golden/make_dense_rows.py c2|c3|c5
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O                         # noqa: E402
from paper_1807_03097_amd import workloads as W        # noqa: E402  (seeded inputs only)

CONFIGS = {
    "c2": dict(level=5, kappa=8.0, rows=48, jitter=None),
    "c3": dict(level=6, kappa=16.0, rows=24, jitter=None),
    "c5": dict(level=7, kappa=40.0, rows=12, jitter=(0.02, 7)),
}


def main(name):
    cf = CONFIGS[name]
    pats = W.cube_sphere()
    if cf["jitter"]:
        pats = W.jitter(pats, *cf["jitter"])
    o = O.Oracle(pats, 2, cf["level"], cf["kappa"], g=5, gs=5)
    x = W.random_coeffs(o.N, 0)
    rows = np.unique(np.linspace(0, o.N - 1, cf["rows"]).astype(int))
    t0 = time.perf_counter()
    y = o.dense_apply(x, rows=rows)
    dt = time.perf_counter() - t0
    out = {
        "what": "rows of the dense Galerkin product A x (eq. MSLtested, every element pair by the "
                "near-field quadrature), oracle only",
        "config": {"geometry": "six-patch NURBS cube-sphere"
                               + (f", control points jittered N(0, {cf['jitter'][0]}^2) seed {cf['jitter'][1]}"
                                  if cf["jitter"] else ""),
                   "level": cf["level"], "p": 2, "kappa": cf["kappa"], "gauss_near": 5, "gauss_singular": 5,
                   "x": "N(0,1)+iN(0,1), seed 0, canonical unknown order", "n_dof": int(o.N)},
        "rows": rows.tolist(),
        "re": y.real.tolist(),
        "im": y.imag.tolist(),
        "oracle_threads": int(O.lib().or_num_threads()),
        "seconds": dt,
    }
    path = os.path.join(ROOT, "tests", "golden", f"{name}_dense_rows.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {path}: {len(rows)} rows in {dt:.1f} s")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c2")
