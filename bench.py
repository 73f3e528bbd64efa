"""Benchmark of the hot path: Crank-Nicolson steps of the rotating-flower workload on one MI355X.

Workload (N = 1024): 1024 x 1024-cell MAC grid on (-1, 1)^2, five-petal body r = 0.35 (1 + 0.2 cos 5 theta)
rotating at omega = 1, Re = 400, dt = h, seeded random smooth forcing (10 Fourier modes, amplitude 1), each step
solved to a max-norm residual of 1e-8 (relative to max(1, ||b||)).  One step = device level-set sampling +
geometry + CN right-hand side + multigrid solve (all of it in the HIP library).

Prints one JSON line: MG unknowns/s = (unknowns of the system) x (V-cycles) / (wall time), whole job.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# HBM bytes per launch of the finest-level five-colour box kernel from the two rocprofv3 counter runs (FETCH_SIZE
# and WRITE_SIZE, each scaled by what it reads for a 64 MiB device copy); None until taken for the current kernel
BOX_TRAFFIC_BYTES = 89.43e6
BOX_TRAFFIC_SOURCE = "profiles/k_box5_flower1024_hbm_traffic.md"
# the launch probe times every 5th finest box sweep (5 is prime to the 4 finest sweeps of a V(2,2) cycle, so all
# four positions are sampled in turn); each timed dispatch leaves the device idle for several microseconds
PROBE_EVERY = 5


def box_sweep_bytes(cls, N, elem=8):
    """Algorithmic bytes of one launch of the five-colour box sweep: the distinct array elements that the five
    colours read or write together, each counted once.  Reads: the class bytes of the box unknowns, and for every
    internal unknown of a box its row's stencil values and its right-hand side; writes: the internal unknowns.
    (A u row takes the 5-point u stencil and the two pressures beside the face, a v row likewise, a continuity
    row the four velocities of its cell.)  Boxes with no internal unknown are skipped by the kernel."""
    import numpy as np
    W = N + 2
    I, J = np.meshgrid(np.arange(N), np.arange(N))
    c = ((J + 1) * W + (I + 1)).ravel()
    u, v, p = cls[0].ravel(), cls[1].ravel(), cls[2].ravel()
    act = (u[c] == 1) | (u[c + 1] == 1) | (v[c] == 1) | (v[c + W] == 1) | (p[c] == 1)
    c = c[act]
    seen = {f: np.zeros(W * W, dtype=bool) for f in "uvp"}
    total = 0
    box = {"u": [0, 1], "v": [0, W], "p": [0]}
    for f, cf in zip("uvp", (u, v, p)):
        m = np.zeros(W * W, dtype=bool)
        for o in box[f]:
            m[c + o] = True
        total += int(m.sum())  # class bytes
        k = np.flatnonzero(m & (cf == 1))  # internal unknowns of the boxes
        total += k.size * 2 * elem  # right-hand side read, value written
        if f == "u":
            for o in (-1, 0, 1, -W, W):
                seen["u"][k + o] = True
            seen["p"][k - 1] = seen["p"][k] = True
        elif f == "v":
            for o in (-1, 0, 1, -W, W):
                seen["v"][k + o] = True
            seen["p"][k - W] = seen["p"][k] = True
        else:
            seen["u"][k] = seen["u"][k + 1] = True
            seen["v"][k] = seen["v"][k + W] = True
    return total + sum(int(x.sum()) for x in seen.values()) * elem


def cpu_baseline(wk, sizes=((256, 8), (512, 4), (1024, 2)), tol=1e-8):
    """The oracle (plain C) on the same system, built for this host (-O3 -march=native), one thread and OpenMP
    over all host threads (the boxes of a colour, the ghost rows, the rows of the residual and transfers): per
    size N the geometry at t = 0, then timed cycles (the first, which also factorises the coarsest system, is not
    timed); at N = 1024 also the time of a solve to tol from x = 0 (GCR around the cycle, as on the GPU)."""
    import platform
    import subprocess
    import tempfile

    import numpy as np
    import oracle as O
    from paper_1911_00994_amd import workloads as wl
    tmp = tempfile.mkdtemp(prefix="oracle_native_")
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        model = next((ln.split(":", 1)[1].strip() for ln in out.splitlines() if ln.startswith("Model name")), "")
    except OSError:
        pass
    res = {"host": platform.node(), "cpu_model": model, "nproc": os.cpu_count(), "runs": []}
    mo = wk.motion.as_array()
    for threads in ("1", "all"):
        path = O.build_native(os.path.join(tmp, f"liboracle_{threads}.so"), openmp=threads == "all")
        O.lib(path)
        nth = O.lib().or_threads()
        for N, cyc in sizes:
            h = 2.0 / N
            o = O.Oracle(N, Re=wk.Re)
            phi = O.levelset_analytic(wk.shape.kind, wk.shape.padded(), mo, 0.0, N)
            assert o.set_levelset(phi, 0.0, mo) == O.OK
            o.set_alpha(h / (2.0 * wk.Re))
            fu, fv = wl.fourier_forcing(N, seed=0)
            o.set_rhs(fu, fv, None)
            o.cycle()
            cls = o.classes(0)
            n_unk = int(((cls == 1) | (cls == 2) | (cls == 4) | (cls == 7)).sum()) + 1
            t0 = time.perf_counter()
            for _ in range(cyc):
                o.cycle()
            sec = time.perf_counter() - t0
            run = {"threads": nth, "N": N, "cycles": cyc, "seconds": sec, "unknowns_per_s": n_unk * cyc / sec}
            if N == 1024 and threads == "all":
                W = N + 2
                z = np.zeros((W, W))
                o.set_x(z, z, z, 0.0)
                t0 = time.perf_counter()
                st, info = o.solve(tol, 100)
                run["time_to_tol_s"] = time.perf_counter() - t0
                run["time_to_tol_cycles"] = info["cycles"]
                run["time_to_tol_status"] = st
            res["runs"].append(run)
            del o
    O.lib(O.build_oracle())
    best = [r for r in res["runs"] if r["N"] == 1024 and r["threads"] > 1] or [r for r in res["runs"] if r["N"] == 1024]
    b = best[-1]
    res.update({"value": b["unknowns_per_s"], "unit": "unknowns/s", "cores": b["threads"], "kind": "oracle",
                "sample": "cycles of the rotating-petal system (Re = 400, dt = h, t = 0) at N = 256, 512, 1024 "
                          "(8, 4, 2 timed cycles), one thread and all threads; value: N = 1024, all threads"})
    return res


def cavity_time_to_tol(gpmg, wl, np, torch, warm_steps=5, tol=1e-8):
    """Time to tol from x = 0, FP64 against mixed precision, on the N = 2048 lid-driven cavity around the fixed
    circle (Re = 1000, dt = h) after a few steps (its FP64 working set, about 0.4 GB, is larger than the MALL)."""
    wk = wl.config_cavity2048()
    N = wk.N
    s = gpmg.Solver(N, Re=wk.Re, stream=torch.cuda.current_stream().cuda_stream)
    s.set_walls(wk.walls)
    s.set_levelset_analytic(wk.shape.kind, wk.shape.params, 0.0, None)
    W = N + 2
    z = np.zeros((W, W))
    s.set_state(z, z, z, 0.0)
    dt = 2.0 / N
    for _ in range(warm_steps):
        s.cn_step(dt, None, None, None, tol=tol, max_cycles=200, picard_eps=1e-8, picard_max=40)
    out = {"workload": wk.name, "N": N, "tol": tol, "after_steps": warm_steps}
    sols = {}
    for name, pr in (("fp64", gpmg.GP_FP64), ("mixed", gpmg.GP_MIXED), ("fp64_again", gpmg.GP_FP64),
                     ("mixed_again", gpmg.GP_MIXED)):
        s.set_x(z, z, z, 0.0)
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        st, info = s.solve(tol, 400, precision=pr, check=False)
        out[name] = {"ms": 1000 * (time.perf_counter() - a0), "cycles": info["cycles"], "res": info["res"],
                     "status": st, "bytes_alg": info["bytes_alg"]}
        sols[name] = np.concatenate([a.ravel() for a in s.get_x()[:3]])
    cls = s.classes().ravel()
    act = (cls == 1) | (cls == 2) | (cls == 4) | (cls == 7)
    out["max_rel_diff_mixed_vs_fp64"] = float(np.abs(sols["fp64"] - sols["mixed"])[act].max() /
                                             max(1.0, np.abs(sols["fp64"][act]).max()))
    out["speedup"] = out["fp64_again"]["ms"] / out["mixed_again"]["ms"]
    s.close()
    return out


def adjoint_run(gpmg, wl, N=512, steps=40, K=8, tol=1e-8):
    """Reverse mode of the moving-circle run (N = 512, r = 0.25 translating at (0.5, 0), Re = 100, 40 steps of
    dt = h, stream-function forcing of 64 modes): J = h^2 sum of the internal u^2 + v^2 at the end, gradients with
    respect to the 64 forcing coefficients and the boundary-velocity offset, checkpoints every 8 steps."""
    import numpy as np
    import torch
    wk = wl.config_circle512_adjoint()
    h = 2.0 / N
    s = gpmg.Solver(N, Re=wk.Re, stream=torch.cuda.current_stream().cuda_stream)
    mo = wk.motion.as_array()
    s.set_levelset_analytic(wk.shape.kind, wk.shape.params, 0.0, mo[:5])
    W = N + 2
    z = np.zeros((W, W))
    s.set_state(z, z, z, 0.0)
    coeffs = wl.adjoint_coeffs(seed=1)
    fu, fv = wl.streamfunction_forcing(N, coeffs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fwd = s.tape_forward(wk.shape.kind, wk.shape.params, mo, 0.0, h, steps, fu, fv, tol=tol, max_cycles=200,
                         picard_eps=1e-10, picard_max=40, checkpoint_every=K)
    t1 = time.perf_counter()
    u, v, _, _ = s.get_x()
    cls = s.classes()
    J = h * h * (float((u[cls[0] == 1] ** 2).sum()) + float((v[cls[1] == 1] ** 2).sum()))
    seed_u = np.where(cls[0] == 1, 2 * h * h * u, 0.0)
    seed_v = np.where(cls[1] == 1, 2 * h * h * v, 0.0)
    t2 = time.perf_counter()
    out = s.tape_backward(seed_u, seed_v, tol=tol, max_cycles=300)
    t3 = time.perf_counter()
    gpath, unmatched = s.tape_path_gradient()
    return {"workload": wk.name, "N": N, "steps": steps, "checkpoint_every": K, "tol": tol, "J": J,
            "forward_ms": 1000 * (t1 - t0), "forward_cycles": fwd["cycles"], "backward_ms": 1000 * (t3 - t2),
            "adjoint_cycles": out["stats"]["cycles"], "adjoint_solves": out["stats"]["outer"],
            "backward_over_forward": (t3 - t2) / (t1 - t0), "dJdU": [float(x) for x in out["dU"]],
            "dJdU_path": [float(x) for x in gpath], "dJdU_total": [float(a + b) for a, b in zip(out["dU"], gpath)],
            "path_rows_unmatched": unmatched,
            "grad_forcing_inf": float(max(np.abs(out["dfu"]).max(), np.abs(out["dfv"]).max()))}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--no-prepare", action="store_true",
                    help="build each step's geometry when the step starts (by default the next step's geometry is "
                         "built in the background during the current step)")
    ap.add_argument("--graphs", action="store_true",
                    help="replay each solver iteration from a HIP graph (by default the launches are issued from the "
                         "host, with the next cycle's first sweep queued ahead of the convergence test)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-cavity", action="store_true", help="skip the N = 2048 cavity time-to-tolerance comparison")
    ap.add_argument("--krylov", type=int, default=None,
                    help="GCR restart length of the solver (library default when not given; 0: the plain cycle)")
    ap.add_argument("--cycle", default=None,
                    help="nu1,nu2,gamma of the solver's cycle (library default V(2,2) when not given)")
    ap.add_argument("--profile-kernel", action="store_true",
                    help="set up the N=1024 system, run a plain 64 MiB device copy (counter calibration) and 10 "
                         "launches of the five-colour box sweep on the finest level, then exit (for rocprofv3 "
                         "--pmc runs)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the solver has no multi-GPU "
              f"decomposition", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1911_00994_amd import gpmg
    from paper_1911_00994_amd import workloads as wl

    wk = wl.config_flower1024()
    N = args.N
    Re = wk.Re
    h = 2.0 / N
    dt = h
    prec = gpmg.GP_MIXED if args.precision == "mixed" else gpmg.GP_FP64
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    extra = {} if args.krylov is None else {"krylov": args.krylov}
    if args.cycle:
        extra.update(zip(("nu1", "nu2", "gamma"), (int(v) for v in args.cycle.split(","))))
    solver = gpmg.Solver(N, Re=Re, stream=stream.cuda_stream, graph_iterations=1 if args.graphs else 0, **extra)
    cyc = f"{'W' if solver._p.gamma == 2 else 'V'}({solver._p.nu1},{solver._p.nu2})"
    fu, fv = wl.fourier_forcing(N, seed=0)
    fu_d = torch.from_numpy(fu).to(dev)
    fv_d = torch.from_numpy(fv).to(dev)
    motion = wk.motion.as_array()[:5]
    shape = wk.shape
    W = N + 2
    z = np.zeros((W, W))
    solver.set_levelset_analytic(shape.kind, shape.params, 0.0, motion)
    solver.set_state(z, z, z, 0.0)
    t = 0.0

    def step():
        nonlocal t
        t1 = t + dt
        solver.set_levelset_analytic(shape.kind, shape.params, t1, motion)
        if not args.no_prepare:  # the body's motion is prescribed: the next geometry builds during this step
            solver.prepare_levelset_analytic(shape.kind, shape.params, t1 + dt, motion)
        st, info = solver.cn_step(dt, fu_d.data_ptr(), fv_d.data_ptr(), None, on_device=True, precision=prec,
                                  tol=args.tol, max_cycles=200, check=False)
        if st != 0:
            raise RuntimeError(f"cn_step status {st} at t={t1}: {info}")
        t = t1
        return info

    if args.profile_kernel:
        src = torch.ones(8 << 20, dtype=torch.float64, device=dev)  # 64 MiB
        dst = torch.empty_like(src)
        flush = torch.empty(64 << 20, dtype=torch.float64, device=dev)  # 512 MiB: evicts L2 and MALL
        for _ in range(3):
            flush.fill_(1.0)
            dst.copy_(src)
        torch.cuda.synchronize()
        del flush
        solver.set_alpha(dt / (2.0 * Re))
        solver.set_rhs(fu, fv, None)
        us = solver.time_kernel(5, level=0, reps=10)
        print(json.dumps({"profile_kernel": "k_box5<double, 32> finest", "launches": 10, "avg_launch_us": us,
                          "copy_bytes": 2 * (64 << 20)}))
        return
    for _ in range(args.warmup):
        step()
    cls = solver.classes(0)
    n_unk = int(((cls == 1) | (cls == 2) | (cls == 4) | (cls == 7)).sum()) + 1
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    cycles = 0
    picard = 0
    if not args.no_kernel_timing:
        solver.probe_start(4096, every=PROBE_EVERY)
    t_wall0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        info = step()
        cycles += info["cycles"]
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall0
    ms = e0.elapsed_time(e1)
    sec = ms / 1000.0
    value = n_unk * cycles / sec
    # algorithmic bytes of one V(2,2) cycle on the FP64 hierarchy: about 417 B per fine cell
    cyc_bytes = 417.0 * N * N
    cyc_gbs = cyc_bytes * cycles / sec / 1e9
    roofline = None
    if not args.no_kernel_timing:
        # dominant kernel: the finest-level box relaxation, all five colours per launch; its launches inside the
        # timed steps were bracketed by HIP events on the solver's stream
        avg_us, nprobe = solver.probe_stop()
        iso_us = solver.time_kernel(5, level=0, reps=10)
        nbytes = box_sweep_bytes(cls, N)
        achieved = nbytes / (avg_us * 1e-6) / 1e9
        traffic = BOX_TRAFFIC_BYTES if N == 1024 else None
        roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                    "kernel": "k_box5<double, 32> finest level (five colours per launch)", "bytes_per_launch": nbytes,
                    "avg_launch_us": avg_us, "launches_timed": nprobe, "probe_every": PROBE_EVERY,
                    "isolated_launch_us": iso_us,
                    "traffic_gbs": traffic / (avg_us * 1e-6) / 1e9 if traffic else None,
                    "traffic_source": BOX_TRAFFIC_SOURCE if traffic else None}
    # time to 1e-8 from x = 0 on the last step's system: FP64 cycles against FP32 cycles in FP64 refinement
    u, v, p, xi = solver.get_x()
    z = np.zeros((W, W))
    ttt = {}
    sols = {}
    # each precision twice, the second timed (the first mixed solve allocates the FP32 hierarchy)
    for name, pr in (("fp64", gpmg.GP_FP64), ("mixed", gpmg.GP_MIXED), ("fp64", gpmg.GP_FP64),
                     ("mixed", gpmg.GP_MIXED)):
        solver.set_x(z, z, z, 0.0)
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        st, info = solver.solve(args.tol, 400, precision=pr, check=False)
        ttt[name] = {"ms": 1000 * (time.perf_counter() - a0), "cycles": info["cycles"], "outer": info["outer"],
                     "res": info["res"], "status": st, "bytes_alg": info["bytes_alg"]}
        sols[name] = np.concatenate([a.ravel() for a in solver.get_x()[:3]])
    act = ((cls == 1) | (cls == 2) | (cls == 4) | (cls == 7)).ravel()
    diff = float(np.abs(sols["fp64"] - sols["mixed"])[act].max() / max(1.0, np.abs(sols["fp64"][act]).max()))
    solver.set_x(u, v, p, xi)
    mixed_vs_fp64 = {"tol": args.tol, "fp64": ttt["fp64"], "mixed": ttt["mixed"],
                     "speedup": ttt["fp64"]["ms"] / ttt["mixed"]["ms"], "max_rel_diff_mixed_vs_fp64": diff}
    cavity = None if args.no_cavity else cavity_time_to_tol(gpmg, wl, np, torch)
    adjoint = None if args.no_adjoint else adjoint_run(gpmg, wl)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wk)
    out = {
        "metric": "MG unknowns/s at N=1024 (% HBM peak); mixed vs FP64 time-to-1e-8 residual",
        "value": value,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == gpmg.GP_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wk.name, "N": N, "Re": Re, "dt": "h", "tol": args.tol,
                   "solver": (f"GCR({solver._p.krylov}) around {cyc} cycles" if solver._p.krylov > 0 else
                              f"{cyc} cycles") + " (coupled ghost boxes on the finest level)",
                   "precision": args.precision, "unknowns": n_unk, "cycles": cycles,
                   "cycles_per_step": cycles / args.steps, "wall_s": wall,
                   "cycle_level_hbm_fraction": cyc_gbs / PEAK_HBM_GBS},
        "roofline": roofline,
        "mixed_vs_fp64_time_to_tol": mixed_vs_fp64,
        "mixed_vs_fp64_time_to_tol_cavity2048": cavity,
        "adjoint": adjoint,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    del picard


if __name__ == "__main__":
    main()
