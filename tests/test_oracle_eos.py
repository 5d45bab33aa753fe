"""Pins of the oracle's Peng-Robinson thermodynamics (Sec. II C, Sec. III D, Sec. IV A of
Saito et al., arXiv:1912.02018) against printed constants and independent numerics."""
import json
import os

import numpy as np
import pytest
from scipy import integrate, optimize

import oracle
from paper_1912_02018_amd.config import LBMConfig

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PAPER = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
CFG = LBMConfig()


def close_to_printed(value, printed, digits):
    """Agreement to the number of significant digits the paper prints."""
    scale = 10.0 ** (np.floor(np.log10(abs(printed))) - digits + 1)
    return abs(value - printed) <= 0.5 * scale + 1e-15


def test_critical_point_matches_printed():
    Tc, pc = oracle.Tc(CFG), oracle.pc(CFG)
    assert close_to_printed(Tc, PAPER["critical_temperature"]["value"], 4)
    assert close_to_printed(pc, PAPER["critical_pressure"]["value"], 4)
    # critical density: where dp/drho and d2p/drho2 vanish at T_c (inflection of the isotherm)
    rc = optimize.minimize_scalar(lambda r: oracle.eos_dpdrho(CFG, r, Tc), bounds=(1.5, 4.0),
                                  method="bounded", options={"xatol": 1e-10}).x
    assert close_to_printed(rc, PAPER["critical_density"]["value"], 4)
    assert abs(oracle.eos_dpdrho(CFG, rc, Tc)) < 1e-3
    assert np.isclose(oracle.eos_p(CFG, rc, Tc), pc, rtol=2e-3)


def test_derivatives_match_finite_differences():
    Tc = oracle.Tc(CFG)
    for rho in (0.3, 2.0, 6.5):
        for T in (0.8 * Tc, 0.86 * Tc, 1.1 * Tc):
            h = 1e-6 * T
            fd = (oracle.eos_p(CFG, rho, T + h) - oracle.eos_p(CFG, rho, T - h)) / (2 * h)
            assert np.isclose(oracle.eos_dpdT(CFG, rho, T), fd, rtol=1e-7)
            hr = 1e-6 * rho
            fdr = (oracle.eos_p(CFG, rho + hr, T) - oracle.eos_p(CFG, rho - hr, T)) / (2 * hr)
            assert np.isclose(oracle.eos_dpdrho(CFG, rho, T), fdr, rtol=1e-6, atol=1e-9)


def test_pseudopotential_recovers_eos_pressure():
    """The interaction force's bulk pressure rho cs^2 + G cs^2 psi^2 / 2 equals p_EOS (eq. potential)."""
    Tc = oracle.Tc(CFG)
    for rho in (0.2, 1.0, 3.0, 6.5, 8.0):
        T = 0.86 * Tc
        psi = oracle.psi(CFG, rho, T)
        assert np.isfinite(psi)
        assert np.isclose(rho / 3 + CFG.G / 3 * psi * psi / 2, oracle.eos_p(CFG, rho, T), rtol=1e-12)


@pytest.mark.parametrize("Tr", [0.86, 0.90, 0.95])
def test_maxwell_construction_independent_check(Tr):
    """Equal pressures and equal chemical potentials, the latter by quadrature of dp/rho."""
    T = Tr * oracle.Tc(CFG)
    rv, rl, ps = oracle.maxwell(CFG, T)
    assert rv < rl
    assert np.isclose(oracle.eos_p(CFG, rv, T), ps, rtol=1e-10)
    assert np.isclose(oracle.eos_p(CFG, rl, T), ps, rtol=1e-10)
    # mu_l - mu_v = int_{rho_v}^{rho_l} (dp/drho)/rho drho = 0 at coexistence
    dmu, err = integrate.quad(lambda r: oracle.eos_dpdrho(CFG, r, T) / r, rv, rl, limit=400,
                              epsabs=1e-13, epsrel=1e-12)
    assert abs(dmu) < 1e-9
    # mechanical stability of both phases
    assert oracle.eos_dpdrho(CFG, rv, T) > 0 and oracle.eos_dpdrho(CFG, rl, T) > 0


def test_density_ratio_and_latent_heat_match_printed():
    T = 0.86 * oracle.Tc(CFG)
    rv, rl, _ = oracle.maxwell(CFG, T)
    assert abs(rl / rv - PAPER["density_ratio_Tr086"]["value"]) < 0.5
    assert close_to_printed(oracle.hfg(CFG, T), PAPER["latent_heat_Tr086"]["value"], 3)

