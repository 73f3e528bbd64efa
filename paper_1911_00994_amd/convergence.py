"""Convergence factor of the multigrid iteration on its own (Sect. 5.3, eq. (convfact)) on the HIP path.

The factor is measured on the homogeneous problem (zero right-hand side and boundary data) from a seeded random
initial iterate: cycles x <- x + B'(b - M x) (gp_mg_vcycle, no Krylov acceleration), rho = geometric mean of the
last six ratios of successive max-norm residuals.  The paper's setting: the rotating five-petal flower of
eq. (domains), Re = 100, W(2,1) cycles (two pre- and one post-relaxation), reference factor 0.119; the colour order
(i + 2j) mod 5 of the box sweep replaces the lexicographic order, which the paper allows.

Command line (one GPU):  python -m paper_1911_00994_amd.convergence --N 128 256 512 1024
"""
from __future__ import annotations

import argparse
import math
import sys

import numpy as np

from . import gpmg
from . import workloads as wl


def factor(N, shape, omega=0.0, t=0.0, Re=100.0, cycles=24, seed=0, **params):
    """(rho, residual history) of the plain cycle; rho is inf when the iteration diverges"""
    p = dict(krylov=0)
    p.update(params)
    s = gpmg.Solver(N, Re=Re, **p)
    try:
        mo = np.array([0.0, 0.0, 0.0, 0.0, omega])
        s.set_levelset_analytic(shape.kind, shape.params, t, mo)
        h = 2.0 / N
        s.set_alpha(h / (2.0 * Re))  # dt = h
        W = N + 2
        z = np.zeros((W, W))
        s.set_rhs(z, z, z)
        s.set_boundary_values(z, z, z)
        cls = s.classes()
        rng = np.random.default_rng(seed)
        s.set_x(*[rng.standard_normal((W, W)) * (cls[g] != 3) for g in range(3)], 0.0)
        hist = [s.residual()[1]]
        for _ in range(cycles):
            r = s.cycle()
            hist.append(r)
            if not (r == r) or r > 1e8 * hist[0] or r < 1e-280:
                break
    finally:
        s.close()
    h = np.array(hist)
    if not np.all(np.isfinite(h)) or h[-1] > h[0]:
        return math.inf, h
    rat = h[1:] / h[:-1]
    return float(np.exp(np.mean(np.log(rat[-6:])))), h


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, nargs="+", default=[128, 256, 512, 1024])
    ap.add_argument("--times", type=float, nargs="+", default=[0.0, 0.37, 0.81])
    a = ap.parse_args()
    sh = wl.paper_flower()
    om = 2.0 * math.pi / 5.0
    cases = [("W(2,1), coupled boxes on the finest level", dict(gamma=2, nu1=2, nu2=1, ghost_box_levels=1)),
             ("W(2,1), coupled boxes on every level", dict(gamma=2, nu1=2, nu2=1, ghost_box_levels=99)),
             ("V(2,2), coupled boxes on the finest level", dict(gamma=1, nu1=2, nu2=2, ghost_box_levels=1))]
    print("| cycle | N | " + " | ".join(f"t = {t}" for t in a.times) + " |")
    print("|---|---|" + "---|" * len(a.times))
    for name, prm in cases:
        for N in a.N:
            rhos = [factor(N, sh, om, t, **prm)[0] for t in a.times]
            print(f"| {name} | {N} | " + " | ".join("diverges" if not math.isfinite(r) else f"{r:.3f}" for r in rhos)
                  + " |", flush=True)


if __name__ == "__main__":
    sys.exit(main())
