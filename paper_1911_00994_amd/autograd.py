"""torch.autograd interface to a recorded run of Crank-Nicolson steps.

`cn_run(solver, fu, fv, ub_offset, run)` advances the solver's current state (geometry and state set beforehand,
as for gp_tape_forward) by run["nsteps"] steps with constant forcing (fu, fv) and an offset of the rigid boundary
velocity of the body, and returns the final velocity grids (u, v).  Backpropagating a scalar built from them calls
the library's reverse mode (gp_tape_backward): the gradients with respect to fu, fv (W*W grids) and ub_offset (2)
come from the transposed solves of every step, replayed from checkpoints.  All arithmetic runs in the library;
this module only hands device buffers across.  One backward pass per forward (the tape holds the last run of the
solver).

`cn_run_body(solver, fu, fv, U, run)` is the same run with the body's velocity U (2) as the differentiable input in
place of the offset: the motion is X(t) = X0 + U t, and the gradient with respect to U is the direct part (u_b
depends on U as on the offset) plus the part through the body path (gp_tape_path_gradient: the boundary rows of every
step move with the body, their discrete decisions held fixed).
"""
from __future__ import annotations

import torch

from . import gpmg


def _f64(t, device):
    return t.detach().to(device=device, dtype=torch.float64).contiguous()


class CNRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, fu, fv, ub_offset, solver, run):
        dev = fu.device
        if dev.type != "cuda":
            raise ValueError("cn_run: fu, fv must be device tensors")
        fu_d, fv_d = _f64(fu, dev), _f64(fv, dev)
        off = [float(v) for v in ub_offset.detach().cpu().to(torch.float64)]
        torch.cuda.current_stream(dev).synchronize()
        solver.tape_forward(run["kind"], run["params"], run["motion"], run.get("t0", 0.0), run["dt"], run["nsteps"],
                            fu=fu_d.data_ptr(), fv=fv_d.data_ptr(), ub_offset=off, tol=run.get("tol", 1e-10),
                            max_cycles=run.get("max_cycles", 200), picard_eps=run.get("picard_eps", 1e-10),
                            picard_max=run.get("picard_max", 40), checkpoint_every=run.get("checkpoint_every", 8),
                            on_device=True)
        u = torch.empty_like(fu_d)
        v = torch.empty_like(fu_d)
        p = torch.empty_like(fu_d)
        solver.get_x(device_out=(u.data_ptr(), v.data_ptr(), p.data_ptr()))
        ctx.solver, ctx.run, ctx.dev = solver, run, dev
        ctx.off_dtype, ctx.off_device = ub_offset.dtype, ub_offset.device
        return u, v

    @staticmethod
    def backward(ctx, gu, gv):
        dev = ctx.dev
        zero = None
        if gu is None or gv is None:
            zero = torch.zeros((ctx.solver.W, ctx.solver.W), dtype=torch.float64, device=dev)
        su = _f64(gu, dev) if gu is not None else zero
        sv = _f64(gv, dev) if gv is not None else zero
        dfu = torch.empty_like(su)
        dfv = torch.empty_like(su)
        torch.cuda.current_stream(dev).synchronize()
        out = ctx.solver.tape_backward(su.data_ptr(), sv.data_ptr(), tol=ctx.run.get("tol", 1e-10),
                                       max_cycles=ctx.run.get("adjoint_max_cycles", 300),
                                       device_out=(dfu.data_ptr(), dfv.data_ptr(), None, None))
        dU = torch.tensor(out["dU"], dtype=ctx.off_dtype, device=ctx.off_device)
        return dfu, dfv, dU, None, None


class CNRunBody(torch.autograd.Function):
    @staticmethod
    def forward(ctx, fu, fv, U, solver, run):
        motion = [float(v) for v in run["motion"]]
        motion[2], motion[3] = [float(v) for v in U.detach().cpu().to(torch.float64)]
        body_run = dict(run, motion=motion)
        off = torch.zeros(2, dtype=torch.float64)
        u, v = CNRun.forward(ctx, fu, fv, off, solver, body_run)
        ctx.u_dtype, ctx.u_device = U.dtype, U.device
        return u, v

    @staticmethod
    def backward(ctx, gu, gv):
        dfu, dfv, d_off, _, _ = CNRun.backward(ctx, gu, gv)
        path, unmatched = ctx.solver.tape_path_gradient()
        if unmatched:
            raise RuntimeError(f"cn_run_body: {unmatched} boundary rows did not reproduce their Alg. 1 path")
        dU = d_off.to(torch.float64).cpu() + torch.tensor(path, dtype=torch.float64)
        return dfu, dfv, dU.to(dtype=ctx.u_dtype, device=ctx.u_device), None, None


def cn_run_body(solver: "gpmg.Solver", fu: torch.Tensor, fv: torch.Tensor, U: torch.Tensor, run: dict):
    """(u, v) at the end of the run with the body moving at velocity U, differentiable with respect to fu, fv and U"""
    return CNRunBody.apply(fu, fv, U, solver, run)


def cn_run(solver: "gpmg.Solver", fu: torch.Tensor, fv: torch.Tensor, ub_offset: torch.Tensor, run: dict):
    """(u, v) at the end of the run, differentiable with respect to fu, fv and ub_offset (see the module doc)"""
    return CNRun.apply(fu, fv, ub_offset, solver, run)
