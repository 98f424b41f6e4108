"""torch.autograd.Functions around the RK4 forward, its discrete adjoint, and the order parameter.

KuramotoRK4: forward = theta(T) after nsteps classical RK4 steps from theta0 (kur_set_params_dev,
kur_set_phases_dev, kur_step_rk4, kur_get_phases_dev); backward = the discrete adjoint with the
incoming dL/dtheta(T) (kur_adjoint_rk4_recorded_dev, or kur_adjoint_rk4_dev when the recording
no longer belongs to this forward run), returning dL/dtheta0, dL/domega and dL/dK.

OrderParameter: (r, psi) of a phase vector (Sec. 2, eq. OrderParameter) by
kur_order_parameter_dev, differentiated by kur_order_parameter_vjp_dev. A loss on r(T) and on
the terminal phases thus differentiates through the integrator with every step on the device:
this module only marshals tensors (dtype, device, contiguity) and hands data pointers to the
library. K enters the library as a host value; a K tensor is read once per forward call.
"""
from __future__ import annotations

import torch

from .kur import Kuramoto


def _real(model: Kuramoto):
    return torch.float32 if model.dtype in ("f32", "float32") else torch.float64


def _dev(model: Kuramoto, t):
    """t as a contiguous tensor of the model's dtype on the model's device."""
    return t.detach().to(device=torch.device("cuda", model.device), dtype=_real(model)).contiguous()


class KuramotoRK4(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta0, omega, K, model: Kuramoto, dt: float, nsteps: int, ckpt_every: int = 32,
                record_stages: bool = False):
        th0 = _dev(model, theta0)
        om = _dev(model, omega)
        k = float(K)
        model.set_params_dev(om, k)
        model.set_phases_dev(th0)
        model.set_option("checkpoint_every", ckpt_every)  # keep checkpoints for the backward pass
        model.set_option("record_stages", 1 if record_stages else 0)  # and every stage state
        model.step_rk4(dt, nsteps, want_r=False)
        model.set_option("checkpoint_every", 0)
        model.set_option("record_stages", 0)
        ctx.rec = model.recorded_run()[0]
        thT = torch.empty_like(th0)
        model.get_phases_dev(thT, wrapped=False)
        ctx.save_for_backward(th0, om)
        ctx.model, ctx.dt, ctx.nsteps, ctx.ckpt, ctx.k = model, dt, nsteps, ckpt_every, k
        ctx.out = (theta0.device, theta0.dtype, omega.device, omega.dtype)
        ctx.k_like = K if torch.is_tensor(K) else None
        return thT.to(device=theta0.device, dtype=theta0.dtype)

    @staticmethod
    def backward(ctx, grad_thetaT):
        m = ctx.model
        th0, om = ctx.saved_tensors
        seed = _dev(m, grad_thetaT)
        gt = torch.empty_like(seed)
        gw = torch.empty_like(seed)
        gk = torch.empty(1, dtype=seed.dtype, device=seed.device)
        if ctx.rec and m.recorded_run()[0] == ctx.rec:  # this forward run's own checkpoints
            m.adjoint_recorded_dev(seed, gt, gw, gk)
        else:  # the model ran or changed since: repeat the forward pass inside the adjoint
            m.set_params_dev(om, ctx.k)
            m.adjoint_rk4_dev(ctx.dt, ctx.nsteps, seed, gt, gw, gk, theta0_t=th0, ckpt_every=ctx.ckpt)
        d0, t0, d1, t1 = ctx.out
        g_k = None
        if ctx.k_like is not None:
            g_k = gk.reshape(()).to(device=ctx.k_like.device, dtype=ctx.k_like.dtype)
        return (gt.to(device=d0, dtype=t0), gw.to(device=d1, dtype=t1), g_k, None, None, None, None, None)


class OrderParameter(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, model: Kuramoto):
        th = _dev(model, theta)
        rpsi = torch.empty(2, dtype=th.dtype, device=th.device)
        model.order_parameter_dev(th, rpsi)
        ctx.save_for_backward(th, rpsi)
        ctx.model = model
        ctx.out = (theta.device, theta.dtype)
        return rpsi.to(device=theta.device, dtype=theta.dtype)

    @staticmethod
    def backward(ctx, grad_rpsi):
        th, rpsi = ctx.saved_tensors
        grad = _dev(ctx.model, grad_rpsi)
        out = torch.empty_like(th)
        ctx.model.order_parameter_vjp_dev(th, rpsi, grad, out)
        d, t = ctx.out
        return out.to(device=d, dtype=t), None


def integrate(model: Kuramoto, theta0, omega, K, dt: float, nsteps: int, ckpt_every: int = 32,
              record_stages: bool = False):
    """theta(T) as a differentiable function of (theta0, omega, K). record_stages: the forward
    run keeps every stage state (16 n reals per step of device memory) and the backward pass
    recomputes nothing."""
    return KuramotoRK4.apply(theta0, omega, K, model, dt, nsteps, ckpt_every, record_stages)


def order_parameter(model: Kuramoto, theta):
    """(r, psi) of (1/N) sum e^{i theta}, differentiable in theta (computed by the library)."""
    rpsi = OrderParameter.apply(theta, model)
    return rpsi[0], rpsi[1]
