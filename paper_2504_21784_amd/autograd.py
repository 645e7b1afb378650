"""Differentiable objectives of a run of time steps: a ``torch.autograd.Function``
over the library's adjoint (the reverse sweeps and the pointwise temperature
adjoint run in the HIP library; this module only moves the parameter vectors
and the gradients between torch and the C ABI).

``objective(log_sigma0, log_cv, ctx, T0, n_steps, dt, kind)`` sets the
per-region opacity coefficients and heat capacities of the context to
``exp(log_sigma0)``, ``exp(log_cv)``, resets its state to the temperature
``T0`` (equilibrium radiation), runs ``n_steps`` time steps and returns, as a
0-d float64 tensor, the time-integrated outflow through the x+ boundary
(``kind`` 0, also ``outflow(...)``) or the material energy sum_n w_n c_v T_n
at the last step (``kind`` 1, also ``material_energy(...)``); ``backward``
returns the adjoint gradient with respect to both vectors.
"""
import numpy as np
import torch


class ObjectiveFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, log_sigma0, log_cv, ctx, T0, n_steps, dt, kind):
        s0 = np.exp(log_sigma0.detach().cpu().double().numpy())
        cv = np.exp(log_cv.detach().cpu().double().numpy())
        ctx.set_materials(s0, cv)
        ctx.set_state(T0)
        J, gs, gc, _ = ctx.adjoint(n_steps, dt, objective=kind)
        # gradients live where the parameters live (CPU or GPU tensors alike)
        fctx.save_for_backward(torch.from_numpy(gs).to(device=log_sigma0.device, dtype=log_sigma0.dtype),
                               torch.from_numpy(gc).to(device=log_cv.device, dtype=log_cv.dtype))
        return torch.tensor(J, dtype=torch.float64, device=log_sigma0.device)

    @staticmethod
    def backward(fctx, gJ):
        gs, gc = fctx.saved_tensors
        return (gJ.to(device=gs.device, dtype=gs.dtype) * gs, gJ.to(device=gc.device, dtype=gc.dtype) * gc,
                None, None, None, None, None)


def objective(log_sigma0, log_cv, ctx, T0, n_steps, dt, kind=0):
    return ObjectiveFunction.apply(log_sigma0, log_cv, ctx, T0, n_steps, dt, int(kind))


def outflow(log_sigma0, log_cv, ctx, T0, n_steps, dt):
    return objective(log_sigma0, log_cv, ctx, T0, n_steps, dt, 0)


def material_energy(log_sigma0, log_cv, ctx, T0, n_steps, dt):
    return objective(log_sigma0, log_cv, ctx, T0, n_steps, dt, 1)
