"""torch.autograd.Function around the RK4 forward and its discrete adjoint.

Forward: theta(T) after nsteps classical RK4 steps from theta0 (kur_step_rk4). Backward:
kur_adjoint_rk4 with the incoming dL/dtheta(T), returning dL/dtheta0, dL/domega and dL/dK. Any
loss built from theta(T) with torch operations (for example on the order parameter r(T)) thus
differentiates through the integrator. Only argument marshalling happens here; every step runs
in the HIP kernels of libkur.so.
"""
from __future__ import annotations

import numpy as np
import torch

from .kur import Kuramoto


def _host(t) -> np.ndarray:
    return t.detach().to("cpu", torch.float64).contiguous().numpy()


class KuramotoRK4(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta0, omega, K, model: Kuramoto, dt: float, nsteps: int, ckpt_every: int = 32,
                record_stages: bool = False):
        th0 = _host(theta0)
        om = _host(omega)
        k = float(K)
        model.set_params(om, k)
        model.set_phases(th0)
        model.set_option("checkpoint_every", ckpt_every)  # keep checkpoints for the backward pass
        model.set_option("record_stages", 1 if record_stages else 0)  # and every stage state
        model.step_rk4(dt, nsteps)
        model.set_option("checkpoint_every", 0)
        model.set_option("record_stages", 0)
        ctx.rec = model.recorded_run()[0]
        thT = model.get_phases(wrapped=False)
        ctx.model, ctx.dt, ctx.nsteps, ctx.ckpt = model, dt, nsteps, ckpt_every
        ctx.th0, ctx.om, ctx.k = th0, om, k
        ctx.dev, ctx.dtype = theta0.device, theta0.dtype
        ctx.k_is_tensor = torch.is_tensor(K)
        return torch.from_numpy(thT).to(theta0.device, theta0.dtype)

    @staticmethod
    def backward(ctx, grad_thetaT):
        m = ctx.model
        seed = _host(grad_thetaT)
        if ctx.rec and m.recorded_run()[0] == ctx.rec:  # this forward run's own checkpoints
            gt, gw, gk = m.adjoint_recorded(seed)
        else:  # the model ran or changed since: repeat the forward pass inside the adjoint
            m.set_params(ctx.om, ctx.k)
            gt, gw, gk = m.adjoint_rk4(ctx.dt, ctx.nsteps, seed, theta0=ctx.th0, ckpt_every=ctx.ckpt)
        to = dict(device=ctx.dev, dtype=ctx.dtype)
        g_k = torch.tensor(gk, **to) if ctx.k_is_tensor else None
        return torch.from_numpy(gt).to(**to), torch.from_numpy(gw).to(**to), g_k, None, None, None, None, None


def integrate(model: Kuramoto, theta0, omega, K, dt: float, nsteps: int, ckpt_every: int = 32,
              record_stages: bool = False):
    """theta(T) as a differentiable function of (theta0, omega, K). record_stages: the forward
    run keeps every stage state (16 n reals per step of device memory) and the backward pass
    recomputes nothing."""
    return KuramotoRK4.apply(theta0, omega, K, model, dt, nsteps, ckpt_every, record_stages)


def order_parameter(theta):
    """r of (1/N) sum e^{i theta} as a torch expression (differentiable)."""
    return torch.sqrt(torch.cos(theta).mean() ** 2 + torch.sin(theta).mean() ** 2)
