"""torch.autograd.Function over the exact closure: particle velocities -> coefficients.

Forward runs fp_moments and fp_closure_solve; backward runs fp_closure_solve_backward
(adjoint solve and the transposed system assembly, with the theta and tau chain) and
fp_moments_backward (per-particle gradients recomputed from the velocities).  The saved
state is the moment and update records only: O(cells), not O(particles x moments).
"""
import torch

from . import fpgpu as F


class ExactClosure(torch.autograd.Function):
    """coefficients = ExactClosure.apply(vx, vy, vz, ctx, offsets)

    vx, vy, vz: 1-D device tensors (float64 or float32, the context's precision),
    particles grouped by cell as given by offsets.  Returns [ncell][9] float64
    (Ct11 Ct12 Ct13 Ct22 Ct23 Ct33, Gamma1..3); cells whose status is not OK carry no
    gradient."""

    @staticmethod
    def forward(fctx, vx, vy, vz, ctx: F.Context, offsets):
        n = vx.shape[0]
        p = _view(ctx, vx, vy, vz, n)
        nc = ctx.ncell
        mom = torch.zeros((nc, F.MOM_STRIDE), dtype=torch.float64, device=vx.device)
        rec = torch.zeros((nc, F.REC_STRIDE), dtype=torch.float64, device=vx.device)
        st = torch.zeros(nc, dtype=torch.int32, device=vx.device)
        ctx.moments(p, offsets, mom)
        ctx.closure_solve(mom, rec, st)
        fctx.ctx = ctx
        fctx.save_for_backward(vx, vy, vz, offsets, mom, rec)
        return rec[:, :9].clone()

    @staticmethod
    def backward(fctx, gy):
        vx, vy, vz, offsets, mom, rec = fctx.saved_tensors
        ctx = fctx.ctx
        nc = ctx.ncell
        ybar = torch.zeros((nc, F.REC_STRIDE), dtype=torch.float64, device=vx.device)
        ybar[:, :9] = gy
        mombar = torch.zeros((nc, F.MOM_STRIDE), dtype=torch.float64, device=vx.device)
        ctx.closure_solve_backward(mom, rec, ybar, mombar)
        n = vx.shape[0]
        gx = torch.zeros(n, dtype=torch.float64, device=vx.device)
        gyy = torch.zeros_like(gx)
        gz = torch.zeros_like(gx)
        ctx.moments_backward(_view(ctx, vx, vy, vz, n), offsets, mom, mombar, gx, gyy, gz)
        return gx.to(vx.dtype), gyy.to(vy.dtype), gz.to(vz.dtype), None, None


def _view(ctx, vx, vy, vz, n):
    p = F.Particles.__new__(F.Particles)
    p.n = n
    p.n_dev = None
    p.capacity = n
    p.x = vx            # positions are not read by the moment kernels
    p.y = None
    p.vx, p.vy, p.vz = vx, vy, vz
    p.pid = torch.zeros(1, dtype=torch.int32, device=vx.device)
    p.key = p.pid
    return p
