"""Bubble growth in a superheated liquid (appendix on bubble growth), reduced: a vapour bubble of
radius 15 at T_sat in liquid superheated by 0.04 T_c, alpha_l = 5.8e-2 (the appendix's resolved case),
nu = 1.5 alpha_l, T_r = 0.86, FP32, on a 512 x 384 channel: the liquid displaced by the growing bubble
leaves through a convective outlet at the local outflow speed (x = nx - 1) opposite a closed inlet
(u_in = 0) -- a closed periodic box would stop the growth, since the liquid cannot be compressed.  The
superheated liquid starts at the density of the liquid branch at T_sat + dT and p_sat (the oracle's
Peng-Robinson pressure, Newton), the bubble at rho_v, T_sat.

The appendix compares with the Plesset-Zwick law, R = (12 alpha_l / pi)^1/2 Ja t^1/2 for a sphere;
a two-dimensional run grows a cylinder, whose exact similarity solution is
analysis.cylinder_bubble_beta (pinned on the CPU).  Checks:
  * R grows as sqrt(t): R^2 linear in t over the last 80 % of 30000 steps (correlation > 0.9999);
  * its coefficient lies within [0.5, 1] of the exact cylindrical value (0.62 measured on MI355X;
    0.64 of the spherical Plesset-Zwick value, Ja taken with the superheated liquid's density) -- the
    model grows more slowly than the sharp-interface
    theory, and part of the gap is the diffuse interface's conduction: with one diffusivity the
    conductivity rho c_v alpha falls 15-fold across the interface,
  * so a vapour diffusivity raising the vapour's conductivity (alpha_vapor 0.6: lambda_v = 0.68 lambda_l)
    grows the bubble faster (0.72 of the exact value measured).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1912_02018_amd import analysis
from paper_1912_02018_amd.config import BC_INLET_OUTLET, FP32, OUTLET_LOCAL, LBMConfig

pytestmark = pytest.mark.gpu

NX, NY, R0, STEPS, SAMPLES = 512, 384, 15.0, 30000, 40
ALPHA, DT_R = 5.8e-2, 0.04


@pytest.fixture(scope="module")
def lbm_mod():
    import torch
    assert torch.cuda.is_available()
    from paper_1912_02018_amd import lbm
    return lbm


def grow(lbm, alpha_v):
    sat = lbm.saturation(LBMConfig(Tr_sat=0.86))
    nu = 1.5 * ALPHA
    cfg = LBMConfig(nx=NX, ny=NY, bc_x=BC_INLET_OUTLET, rk_stages=4, nu=nu, alpha_T=ALPHA, Tr_sat=0.86,
                    dTr_wall=DT_R, rho_l=sat["rho_l"], rho_v=sat["rho_v"], u_in=0.0, precision=FP32,
                    outlet_kind=OUTLET_LOCAL, diag_every=0, alpha_vapor=alpha_v,
                    nu_vapor=nu if alpha_v > 0 else 0.0)
    dT = DT_R * sat["Tc"]
    Th = sat["T_sat"] + dT
    rl = sat["rho_l"]
    for _ in range(60):   # liquid branch at T_sat + dT and p_sat
        rl -= (oracle.eos_p(cfg, rl, Th) - sat["p_sat"]) / oracle.eos_dpdrho(cfg, rl, Th)
    rv = sat["rho_v"]
    x, y = np.arange(NX)[None, :], np.arange(NY)[:, None]
    r = np.hypot(x - NX // 2, y - NY // 2)
    rho = 0.5 * (rl + rv) + 0.5 * (rl - rv) * np.tanh((r - R0) / 2.0)
    T = np.where(r < R0, sat["T_sat"], Th)
    sim = lbm.Simulation(cfg)
    sim.set_fields(rho, np.zeros_like(rho), np.zeros_like(rho), T)
    mid = 0.5 * (sat["rho_l"] + rv)
    ts, rs = [], []
    for _ in range(SAMPLES):
        sim.step(STEPS // SAMPLES)
        ts.append(sim.step_count)
        rs.append(math.sqrt(float((sim.fields()["rho"] < mid).sum()) / math.pi))
    sim.close()
    ts, rs = np.array(ts, float), np.array(rs)
    assert np.all(np.diff(rs) > 0), rs
    sel = ts >= 0.2 * STEPS
    slope = np.polyfit(ts[sel], rs[sel] ** 2, 1)[0]
    corr = np.corrcoef(ts[sel], rs[sel] ** 2)[0, 1]
    ja = rl * cfg.cv * dT / (rv * sat["h_fg"])
    exact = 2.0 * analysis.cylinder_bubble_beta(ja, 1.0 - rv / rl) * math.sqrt(ALPHA)
    pz = analysis.plesset_zwick_radius(1.0, ALPHA, rl, rv, cfg.cv, dT, sat["h_fg"])
    c = math.sqrt(slope)
    print(f"bubble growth alpha_v {alpha_v}: R {rs[0]:.1f} -> {rs[-1]:.1f}, R^2 = {slope:.5f} t + c (corr {corr:.6f}); "
          f"coefficient {c:.4f}: {c / exact:.3f} of the cylinder's similarity solution {exact:.4f}, "
          f"{c / pz:.3f} of Plesset-Zwick {pz:.4f} (Ja {ja:.3f})", flush=True)
    return c / exact, corr


def test_bubble_grows_as_sqrt_t(lbm_mod):
    ratio, corr = grow(lbm_mod, 0.0)
    assert corr > 0.9999
    assert 0.5 <= ratio <= 1.0


def test_vapour_conduction_speeds_growth(lbm_mod):
    base, _ = grow(lbm_mod, 0.0)
    hi, corr = grow(lbm_mod, 0.6)
    assert corr > 0.9999
    assert base < hi <= 1.0
