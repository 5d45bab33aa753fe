"""Sensitivities of the time-averaged wall Nusselt number of a boiling run.

J(theta) is the mean of Nu over the states average_from .. steps-1 of a run (Nu as defined for the
heated cylinder, Sec. IV B), theta = (dTr_wall, u_in, acentric, tau).  The tangent precision of
liblbm (LBM_F64_TANGENT) carries the derivatives of every value of the FP64 step along the four
parameter directions (forward-mode dual numbers through the same kernels), so one run gives J and
its exact discrete gradient.  ``NuTimeAverage`` exposes that as a torch.autograd.Function.

The coexistence densities rho_l, rho_v (the initial liquid, the gravity and wall densities and the
Nu normalisation use them) are held fixed: ``hold_coexistence`` writes the values the library
derives for a configuration into it, so that runs at perturbed parameters keep them.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lbm
from .config import F64_TANGENT, TANGENT_PARAMS, LBMConfig

__all__ = ["TANGENT_PARAMS", "params_of", "with_params", "hold_coexistence",
           "nu_average_and_gradient", "NuTimeAverage"]


def params_of(cfg: LBMConfig) -> np.ndarray:
    """theta = (dTr_wall, u_in, acentric, tau) of a configuration; tau = nu / cs^2 + 1/2."""
    return np.array([cfg.dTr_wall, cfg.u_in, cfg.acentric, 3.0 * cfg.nu + 0.5])


def with_params(base: LBMConfig, theta) -> LBMConfig:
    """``base`` at parameters theta; alpha_T follows nu so that nu / alpha_T is held."""
    dtr, u_in, acentric, tau = (float(t) for t in theta)
    nu = (tau - 0.5) / 3.0
    pr = base.nu / base.alpha_T
    return base.replace(dTr_wall=dtr, u_in=u_in, acentric=acentric, nu=nu, alpha_T=nu / pr)


def hold_coexistence(cfg: LBMConfig) -> LBMConfig:
    """``cfg`` with explicit rho_l, rho_v: the Maxwell densities the library derives for it (a host
    computation, no device needed)."""
    if cfg.rho_l > 0 and cfg.rho_v > 0:
        return cfg
    sat = lbm.saturation(cfg)
    return cfg.replace(rho_l=sat["rho_l"], rho_v=sat["rho_v"])


def nu_average_and_gradient(cfg: LBMConfig, steps: int, average_from: int = 0):
    """(J, dJ/dtheta) of one run stepped ``steps`` times from its default state, J the mean Nu of
    the states average_from .. steps-1."""
    if not 0 <= average_from < steps:
        raise ValueError("need 0 <= average_from < steps")
    sim = lbm.Simulation(cfg.replace(precision=F64_TANGENT, diag_every=1))
    try:
        sim.step(average_from)
        sim.reset_time_average()
        sim.step(steps - average_from)
        _, _, J = sim.wall_heat_flux()
        _, dJ = sim.nu_tangent()
    finally:
        sim.close()
    return J, dJ


class NuTimeAverage(torch.autograd.Function):
    """J = NuTimeAverage.apply(theta, base_cfg, steps, average_from) for a float64 tensor theta of
    the four parameters; backward returns grad_J * dJ/dtheta from the tangent run."""

    @staticmethod
    def forward(ctx, theta, base: LBMConfig, steps: int, average_from: int):
        cfg = with_params(base, theta.detach().cpu().numpy())
        J, g = nu_average_and_gradient(cfg, steps, average_from)
        ctx.save_for_backward(torch.as_tensor(g, dtype=theta.dtype, device=theta.device))
        return theta.new_tensor(J)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None, None, None
