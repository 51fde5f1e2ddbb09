"""torch.autograd.Function over the adjoint form (argument marshalling only:
the forward run and the reverse sweep are lbm_adjoint's kernels).

J(theta) is the time-averaged settling velocity U_z^{n+1/2} over nsteps of a
fresh run whose body force g (three components), Shan-Chen coupling G and
wetting offset Delta rho are theta = (g_x, g_y, g_z, G, Delta rho); every
other run parameter comes from `params`.  Sec. 2 and 3 of Xue, Biferale,
Sbragaglia, Toschi (eq. lbe, eq. sc-force, wetting layer; eq. fp).
"""
import numpy as np
import torch

from . import workloads
from .sim import Simulation


class SettlingVelocity(torch.autograd.Function):
    """forward runs the steps once (lbm_adjoint_forward: checkpoints and the
    recorded last segment) and keeps the run; backward runs the reverse sweep
    over it (lbm_adjoint_backward) and releases it."""

    @staticmethod
    def forward(ctx, theta, params, nsteps, precision="fp32", segment=0):
        th = theta.detach().to("cpu", torch.float64).numpy()
        p = workloads.full(dict(params))
        p["g"] = (float(th[0]), float(th[1]), float(th[2]))
        p["G"] = float(th[3])
        p["wet_drho"] = float(th[4])
        sim = Simulation(p, precision)
        try:
            J = sim.adjoint_forward(int(nsteps), int(segment))
        except Exception:
            sim.close()
            raise
        ctx.sim = sim
        ctx.theta_dtype = theta.dtype
        return theta.new_tensor(J)

    @staticmethod
    def backward(ctx, gJ):
        sim = ctx.sim
        ctx.sim = None
        try:
            grad = sim.adjoint_backward()
        finally:
            sim.close()
        g = torch.as_tensor(np.asarray(grad), dtype=ctx.theta_dtype)
        return gJ.to("cpu") * g, None, None, None, None


def settling_velocity(theta, params, nsteps, precision="fp32", segment=0):
    """J(theta) with an adjoint backward; theta is a CPU tensor of 5 values."""
    return SettlingVelocity.apply(theta, params, nsteps, precision, segment)
