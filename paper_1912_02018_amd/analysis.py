"""Post-processing of boiling runs: the dimensionless groups of film boiling, the heat-transfer
correlations the paper compares its Nu against (Sec. I, Sec. V on the Nu-Ja diagram, and the
appendix on film-boiling correlations), the interface law of the Stefan problem (Sec. III E) and
the Plesset-Zwick bubble growth (appendix on bubble growth).

Nu = h D / lambda_v with h = q / dT (the wall heat flux of lbm_wall_heat_flux); the groups are
gamma = rho_l / rho_v, eta = nu_l / nu_v, Re = u_l D / nu_l, Pr = nu_v / alpha_v and
Ja = c_p,v dT / h_fg.  With one kinematic viscosity for both phases (the configurations here),
eta = 1; c_p = c_v (ratio of specific heats 1, Sec. IV A).
"""
from __future__ import annotations

import math

from .config import LBMConfig

__all__ = ["groups", "jakob", "bromley", "epstein_hauser", "ito", "correlations", "stefan_beta",
           "stefan_interface", "plesset_zwick_radius", "cylinder_bubble_beta"]

# constants of the correlations as the paper uses them
BROMLEY_C = 2.7
EPSTEIN_HAUSER_C = (0.537, 1.13)   # theory for a cylinder; fit to subcooled experiments
ITO_C = (0.46, 0.48, 0.51)         # water, ethanol, hexane


def jakob(cp_v: float, dT: float, h_fg: float) -> float:
    """Ja = c_p,v dT / h_fg."""
    return cp_v * dT / h_fg


def groups(cfg: LBMConfig, sat: dict | None = None) -> dict:
    """Dimensionless groups of a cylinder run.  ``sat`` is the saturation state of the fluid
    (``lbm.saturation(cfg)``: T_c, rho_l, rho_v, h_fg); D = 2R, dT = dTr_wall T_c."""
    if sat is None:
        from . import lbm
        sat = lbm.saturation(cfg)
    D = 2.0 * cfg.cyl_r
    dT = cfg.dTr_wall * sat["Tc"]
    return {"gamma": sat["rho_l"] / sat["rho_v"], "eta": 1.0, "Re": cfg.u_in * D / cfg.nu,
            "Pr": cfg.nu / cfg.alpha_T, "Ja": jakob(cfg.cv, dT, sat["h_fg"]), "D": D, "dT": dT}


def bromley(eta: float, Re: float, Pr: float, Ja: float, C: float = BROMLEY_C) -> float:
    """Mode 1 (Bromley et al., high-flow form): Nu = C eta^1/2 Re^1/2 Pr^1/2 (c_p dT / h_fg')^-1/2
    with the effective latent heat h_fg' = h_fg (1 + 0.4 Ja)^2."""
    ja_eff = Ja / (1.0 + 0.4 * Ja) ** 2
    return C * math.sqrt(eta * Re * Pr / ja_eff)


def epstein_hauser(gamma: float, eta: float, Re: float, Pr: float, Ja: float,
                   C: float = EPSTEIN_HAUSER_C[0]) -> float:
    """Mode 2 (Epstein-Hauser, saturated limit): Nu = C gamma^1/4 eta^1/2 Re^1/2 Pr^1/4 Ja^-1/4."""
    return C * gamma ** 0.25 * math.sqrt(eta * Re) * (Pr / Ja) ** 0.25


def ito(gamma: float, eta: float, Re: float, Pr: float, Ja: float, C: float = ITO_C[0]) -> float:
    """Ito et al. (forced-convection dominated): the Mode 2 form with C = 0.46 (water)."""
    return epstein_hauser(gamma, eta, Re, Pr, Ja, C)


def correlations(g: dict) -> dict:
    """Nu predicted by the six correlations of the Nu-Ja comparison for groups ``g``."""
    out = {"bromley": bromley(g["eta"], g["Re"], g["Pr"], g["Ja"])}
    for c in EPSTEIN_HAUSER_C:
        out[f"epstein_hauser_C{c}"] = epstein_hauser(g["gamma"], g["eta"], g["Re"], g["Pr"], g["Ja"], c)
    for c in ITO_C:
        out[f"ito_C{c}"] = ito(g["gamma"], g["eta"], g["Re"], g["Pr"], g["Ja"], c)
    return out


def stefan_beta(cp_v: float, dT: float, h_fg: float) -> float:
    """Root of beta exp(beta^2) erf(beta) = c_p,v dT / (h_fg sqrt(pi)) (Stefan problem): the left
    side increases monotonically from 0, so the root is bracketed and bisected to machine precision."""
    rhs = cp_v * dT / (h_fg * math.sqrt(math.pi))
    if rhs <= 0.0:
        return 0.0
    f = lambda b: b * math.exp(b * b) * math.erf(b) - rhs
    lo, hi = 0.0, 1.0
    while f(hi) < 0.0:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) < 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def stefan_interface(t, beta: float, alpha_v: float):
    """Interface position y_i(t) = 2 beta sqrt(alpha_v t) of the Stefan problem."""
    return 2.0 * beta * (alpha_v * t) ** 0.5


def plesset_zwick_radius(t, alpha_l: float, rho_l: float, rho_v: float, cp_l: float, dT: float,
                         h_fg: float):
    """R(t) = (12 alpha_l / pi)^1/2 rho_l c_p,l dT / (rho_v h_fg) t^1/2: bubble growth in a uniformly
    superheated liquid (Plesset-Zwick)."""
    return math.sqrt(12.0 * alpha_l / math.pi) * rho_l * cp_l * dT / (rho_v * h_fg) * t ** 0.5


def cylinder_bubble_beta(ja: float, eps: float) -> float:
    """Growth constant of a cylindrical (2-D) vapour bubble in a uniformly superheated liquid, from the
    similarity solution R(t) = 2 beta sqrt(alpha_l t): with eta = r / (2 sqrt(alpha_l t)) and the liquid's
    radial outflow u = eps R dR/dt / r (eps = 1 - rho_v / rho_l), the liquid temperature obeys
    T'' + (1/eta + 2 eta - 2 eps beta^2 / eta) T' = 0, so T' is proportional to
    eta^(2 eps beta^2 - 1) exp(-eta^2); T = T_sat at eta = beta, T -> T_sat + dT far away, and the
    interface balance rho_v h_fg dR/dt = k dT/dr gives
        Ja = 2 beta int_beta^inf (s / beta)^(2 eps beta^2 - 1) exp(-(s^2 - beta^2)) ds,
    Ja = rho_l c_p,l dT / (rho_v h_fg).  The right side increases with beta from 0, so the root is
    bracketed and bisected.  For eps = 1 and large Ja it tends to the thin-layer law
    beta = sqrt(2 / pi) Ja, the cylindrical counterpart of Plesset-Zwick's sqrt(3 / pi) Ja."""
    if ja <= 0.0:
        return 0.0

    def rhs(beta):
        p = 2.0 * eps * beta * beta - 1.0
        # composite Simpson on [beta, beta + L]; the integrand is 1 at s = beta and decays at least
        # like exp(-(1 + eps) x^2 - 2 beta (1 - eps) x) beyond it
        L = 12.0 / (1.0 + beta * (1.0 - eps)) + 12.0
        n = 20000
        h = L / n
        tot = 0.0
        for i in range(n + 1):
            s = beta + i * h
            w = 1.0 if i in (0, n) else (4.0 if i % 2 else 2.0)
            tot += w * math.exp(p * math.log(s / beta) - (s * s - beta * beta))
        return 2.0 * beta * tot * h / 3.0

    lo, hi = 1e-9, 1.0
    while rhs(hi) < ja:
        hi *= 2.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if rhs(mid) < ja:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)
