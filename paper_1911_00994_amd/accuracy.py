"""Accuracy runs of Sect. 5.1 on the HIP path: the manufactured solution of eq. (sol:exa) on the three bodies of
eq. (domains) (circle, ellipse, five-petal flower), at rest or rotating about the origin with omega = 2 pi / 5,
Re = 100, from the exact fields at t = 0 to a final time T (the paper's tables use T = 10), with the paper's step
bound dt <= min(h, h / max |u|): |u_exa| <= sqrt(2), so dt = T / ceil(sqrt(2) T / h).

Reported per run: the max-norm and L1 errors (L1 = mean over the internal points, reading c19) of u and v at T
against the exact fields, and the divergence error |div_h u - g| = |xi| (the continuity rows make div_h u - g the
constant xi, so its L1 and max norms agree).  The observed order between successive N is log2 of the error
ratio.  Every step runs in the library (geometry, right-hand side, solve); this module only supplies the
manufactured forcing and boundary data, which depend on the boundary points of the current geometry.

Command line (one GPU):  python -m paper_1911_00994_amd.accuracy --T 10 --N 64 128 256
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import gpmg
from . import workloads as wl

WALL_DIRICHLET = 3


def _boundary_points(s):
    """boundary point of every boundary row of the finest level; wall Dirichlet rows use the node itself"""
    g = s.boundary_geometry()
    cls = s.classes()
    B = [b.copy() for b in g["B"]]
    for k in range(3):
        x, y = wl.node_coords(s.N, k)
        m = cls[k] == WALL_DIRICHLET
        B[k][m, 0] = x[m]
        B[k][m, 1] = y[m]
    return dict(B=tuple(B), nB=g["nB"])


def run(N: int, shape: wl.Shape, omega: float, T: float, Re: float = 100.0, tol: float = 1e-10,
        log=None) -> dict:
    """One run; returns the errors at the final time and the step count."""
    m = wl.PaperMMS()
    h = 2.0 / N
    steps = int(math.ceil(math.sqrt(2.0) * T / h - 1e-9))
    dt = T / steps
    mo = np.array([0.0, 0.0, 0.0, 0.0, omega])
    moving = omega != 0.0
    s = gpmg.Solver(N, Re=Re)
    t0 = time.perf_counter()
    n, t1 = 0, 0.0
    try:
        s.set_levelset_analytic(shape.kind, shape.params, 0.0, mo)
        u0, v0, p0 = wl.mms_fields(m, N, 0.0)
        s.set_state(u0, v0, dt * p0, 0.0)
        xu, yu = wl.node_coords(N, 0)
        xv, yv = wl.node_coords(N, 1)
        xp, yp = wl.node_coords(N, 2)
        geom = None
        cycles = 0
        t = 0.0
        for n in range(steps):
            t1 = (n + 1) * dt
            if moving:
                s.set_levelset_analytic(shape.kind, shape.params, t1, mo)
                if n + 1 < steps:  # the motion is prescribed: the next geometry builds during this step
                    s.prepare_levelset_analytic(shape.kind, shape.params, t1 + dt, mo)
            if geom is None or moving:
                geom = _boundary_points(s)
            th = t + 0.5 * dt
            bu, bv, bp = wl.boundary_values_from(m, geom, t1, th, p_scale=dt)
            s.set_boundary_values(bu, bv, bp)
            fu, _ = m.forcing(xu, yu, th, Re)
            _, fv = m.forcing(xv, yv, th, Re)
            st, info = s.cn_step(dt, fu, fv, m.div(xp, yp, t1), tol=tol, max_cycles=200, picard_eps=1e-10,
                                 picard_max=40, check=False)
            if st != gpmg.GP_OK:
                return {"N": N, "steps": steps, "failed_step": n, "T": t1, "status": st, "info": info}
            cycles += info["cycles"]
            t = t1
            if log and (n + 1) % max(1, steps // 4) == 0:
                log(f"    N={N} step {n + 1}/{steps} ({time.perf_counter() - t0:.1f} s)")
        u, v, _, xi = s.get_x()
        cls = s.classes()
        eu = np.abs(u - m.u(xu, yu, t))[cls[0] == 1]
        ev = np.abs(v - m.v(xv, yv, t))[cls[1] == 1]
    except gpmg.GpmgError as e:  # a geometry the library rejects (a body too thin for the grid)
        return {"N": N, "steps": steps, "failed_step": n, "T": t1, "status": e.status, "info": str(e)}
    finally:
        s.close()
    return {"N": N, "steps": steps, "T": t, "cycles": cycles, "seconds": time.perf_counter() - t0,
            "Linf_u": float(eu.max()), "Linf_v": float(ev.max()), "L1_u": float(eu.mean()), "L1_v": float(ev.mean()),
            "div": float(abs(xi))}


def bodies():
    return {"circle": wl.paper_circle(), "ellipse": wl.paper_ellipse(), "flower": wl.paper_flower()}


def summary(q) -> str:
    if "failed_step" in q:
        return f"N={q['N']}: status {q['status']} at step {q['failed_step']} (t = {q['T']:.3f})"
    return (f"N={q['N']}: L1 u {q['L1_u']:.3e} v {q['L1_v']:.3e}  Linf u {q['Linf_u']:.3e} v {q['Linf_v']:.3e}  "
            f"div {q['div']:.3e}  {q['cycles'] / q['steps']:.1f} cycles/step, {q['seconds']:.1f} s")


def table(Ns, T, body_names=("circle", "ellipse", "flower"), omegas=(0.0, 2.0 * math.pi / 5.0), log=None):
    out = []
    for name in body_names:
        sh = bodies()[name]
        for om in omegas:
            runs = []
            for N in Ns:
                if log:
                    log(f"[accuracy] {name} omega={om:.4f} N={N} T={T}")
                runs.append(run(N, sh, om, T, log=log))
                if log:
                    log("  " + summary(runs[-1]))
            for a, b in zip(runs, runs[1:]):
                if "failed_step" in a or "failed_step" in b:
                    continue
                for k in ("Linf_u", "Linf_v", "L1_u", "L1_v", "div"):
                    b["order_" + k] = math.log2(a[k] / b[k]) if b[k] > 0 and a[k] > 0 else None
            out.append({"body": name, "omega": om, "runs": runs})
    return out


def markdown(rows) -> str:
    lines = ["| body | omega | N | L1 u | L1 v | Linf u | Linf v | div | order L1 u / v | order Linf u / v | cycles/step |",
             "|---|---|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        for q in r["runs"]:
            if "failed_step" in q:
                lines.append(f"| {r['body']} | {r['omega']:.4f} | {q['N']} | status {q['status']} at step "
                             f"{q['failed_step']} (t = {q['T']:.3f}) | | | | | | | |")
                continue
            o1 = f"{q['order_L1_u']:.2f} / {q['order_L1_v']:.2f}" if "order_L1_u" in q else ""
            o2 = f"{q['order_Linf_u']:.2f} / {q['order_Linf_v']:.2f}" if "order_Linf_u" in q else ""
            lines.append(f"| {r['body']} | {r['omega']:.4f} | {q['N']} | {q['L1_u']:.2e} | {q['L1_v']:.2e} | "
                         f"{q['Linf_u']:.2e} | {q['Linf_v']:.2e} | {q['div']:.2e} | {o1} | {o2} | "
                         f"{q['cycles'] / q['steps']:.1f} |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--T", type=float, default=10.0)
    ap.add_argument("--N", type=int, nargs="+", default=[64, 128, 256])
    ap.add_argument("--bodies", nargs="+", default=["circle", "ellipse", "flower"])
    ap.add_argument("--motion", choices=["both", "steady", "moving"], default="both")
    ap.add_argument("--json", default=None)
    a = ap.parse_args()
    om = {"both": (0.0, 2.0 * math.pi / 5.0), "steady": (0.0,), "moving": (2.0 * math.pi / 5.0,)}[a.motion]

    def log(msg):
        print(msg, flush=True)

    rows = table(a.N, a.T, a.bodies, om, log=log)
    print(markdown(rows), flush=True)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
