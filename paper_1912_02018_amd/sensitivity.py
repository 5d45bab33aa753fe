"""Sensitivities of the time-averaged wall Nusselt number of a boiling run.

J(theta) is the mean of Nu over the states average_from .. steps-1 of a run (Nu as defined for the
heated cylinder, Sec. IV B), theta = (dTr_wall, u_in, acentric, tau).  Two exact routes to the
discrete gradient of the FP64 step:
  * reverse mode (``nu_average_and_gradient_adjoint``): liblbm's hand-written adjoint of the step run
    backwards over the trajectory, which is recomputed segment by segment from checkpoints taken
    every K steps (lbm_nu_gradient); its cost does not grow with the number of parameters;
  * forward mode (``nu_average_and_gradient``): the tangent precision LBM_F64_TANGENT carries the
    four derivatives of every value through the same kernels in one run.
``NuTimeAverage`` is the torch.autograd.Function: forward runs the FP64 step for J, backward the
reverse sweep (or, with mode="tangent", the tangent run).

The coexistence densities rho_l, rho_v (the initial liquid, the gravity and wall densities and the
Nu normalisation use them) are held fixed: ``hold_coexistence`` writes the values the library
derives for a configuration into it, so that runs at perturbed parameters keep them.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lbm
from .config import F64_TANGENT, FP64, TANGENT_PARAMS, LBMConfig

__all__ = ["TANGENT_PARAMS", "params_of", "with_params", "hold_coexistence", "nu_average",
           "nu_average_and_gradient", "nu_average_and_gradient_adjoint", "NuTimeAverage"]


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


def nu_average(cfg: LBMConfig, steps: int, average_from: int = 0) -> float:
    """J of the FP64 (or the configuration's) step: the mean Nu of the states average_from .. steps-1."""
    if not 0 <= average_from < steps:
        raise ValueError("need 0 <= average_from < steps")
    sim = lbm.Simulation(cfg.replace(diag_every=1))
    try:
        sim.step(average_from)
        sim.reset_time_average()
        sim.step(steps - average_from)
        return sim.wall_heat_flux()[2]
    finally:
        sim.close()


def nu_average_and_gradient_adjoint(cfg: LBMConfig, steps: int, average_from: int = 0,
                                    checkpoint_every: int = 200):
    """(J, dJ/dtheta) of one FP64 run from its default state by the reverse sweep with
    checkpoint-and-recompute every checkpoint_every steps."""
    if not 0 <= average_from < steps:
        raise ValueError("need 0 <= average_from < steps")
    sim = lbm.Simulation(cfg.replace(precision=FP64, diag_every=1))
    try:
        return sim.nu_gradient(steps, average_from, checkpoint_every)
    finally:
        sim.close()


class NuTimeAverage(torch.autograd.Function):
    """J = NuTimeAverage.apply(theta, base_cfg, steps, average_from, checkpoint_every, mode) for a
    float64 tensor theta of the four parameters.  Forward: the FP64 run for J.  Backward:
    grad_J * dJ/dtheta from the reverse sweep with checkpoints every checkpoint_every steps
    (mode "adjoint", the default), or from the tangent run (mode "tangent")."""

    @staticmethod
    def forward(ctx, theta, base: LBMConfig, steps: int, average_from: int, checkpoint_every: int = 200,
                mode: str = "adjoint"):
        if mode not in ("adjoint", "tangent"):
            raise ValueError("mode is 'adjoint' or 'tangent'")
        cfg = with_params(base, theta.detach().cpu().numpy()).replace(precision=FP64)
        ctx.args = (cfg, steps, average_from, checkpoint_every, mode)
        ctx.meta = (theta.dtype, theta.device)
        return theta.new_tensor(nu_average(cfg, steps, average_from))

    @staticmethod
    def backward(ctx, grad_out):
        cfg, steps, average_from, every, mode = ctx.args
        if mode == "adjoint":
            _, g = nu_average_and_gradient_adjoint(cfg, steps, average_from, every)
        else:
            _, g = nu_average_and_gradient(cfg, steps, average_from)
        dtype, device = ctx.meta
        return grad_out * torch.as_tensor(g, dtype=dtype, device=device), None, None, None, None, None
