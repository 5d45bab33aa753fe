"""Saturation state of the library's host thermodynamics and the post-processing of boiling runs
(no device needed).

Pins: the printed critical temperature (4 digits), latent heat at T_r = 0.86 (3 digits) and density
ratio ~17 (Sec. II C, Sec. IV A); the oracle's Maxwell densities and pressure (a different
implementation, bisection on the equal-area condition in the oracle, tabulated in the golden file)
and its finite-difference Clausius-Clapeyron latent heat (agreement to the 1e-9 of that difference,
the library integrates the Maxwell relation instead); the Stefan root against its small-St
asymptote and a brute-force scan; the correlation forms through their exponents and constants; the
growth constant of a cylindrical bubble against a time-dependent moving-boundary solution and its
thin-layer limit.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1912_02018_amd import analysis, lbm
from paper_1912_02018_amd.config import LBMConfig, config2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PAPER = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
COEX = json.load(open(os.path.join(GOLDEN, "maxwell_coexistence.json")))["coexistence"]


def test_saturation_matches_printed_values():
    s = lbm.saturation(LBMConfig(Tr_sat=0.86))
    assert round(s["Tc"], 4) == PAPER["critical_temperature"]["value"]
    assert round(s["h_fg"], 3) == PAPER["latent_heat_Tr086"]["value"]
    assert round(s["rho_l"] / s["rho_v"]) == PAPER["density_ratio_Tr086"]["value"]


@pytest.mark.parametrize("tr", ["0.80", "0.86", "0.90", "0.95"])
def test_saturation_matches_oracle_maxwell(tr):
    s = lbm.saturation(LBMConfig(Tr_sat=float(tr)))
    o = COEX[tr]
    for k in ("rho_l", "rho_v", "p_sat"):
        assert abs(s[k] / o[k] - 1.0) < 1e-12, k
    assert abs(s["h_fg"] / o["h_fg"] - 1.0) < 2e-9


def test_saturation_rejects_supercritical():
    with pytest.raises(lbm.LBMError):
        lbm.saturation(LBMConfig(Tr_sat=1.2))


def test_groups_of_the_boiling_channel():
    cfg = config2()
    s = lbm.saturation(cfg)
    g = analysis.groups(cfg, s)
    assert abs(g["Re"] - 300.0) < 1e-9 and abs(g["Pr"] - 1.5) < 1e-12 and g["eta"] == 1.0
    assert abs(g["gamma"] - s["rho_l"] / s["rho_v"]) < 1e-12
    assert abs(g["Ja"] - 11.0 * 0.1 * s["Tc"] / s["h_fg"]) < 1e-15


def test_stefan_root():
    for st in (1e-4, 1e-3, 0.05, 0.2, 1.0, 5.0):
        b = analysis.stefan_beta(st, 1.0, 1.0)
        assert abs(b * math.exp(b * b) * math.erf(b) - st / math.sqrt(math.pi)) < 1e-14 * max(1.0, st)
        # brute force: the sign change on a fine grid brackets the same root
        grid = np.linspace(0.0, 3.0, 300001)
        f = grid * np.exp(grid ** 2) * np.vectorize(math.erf)(grid) - st / math.sqrt(math.pi)
        k = int(np.argmax(f >= 0))
        assert grid[k - 1] <= b <= grid[k]
    # small St: beta exp(beta^2) erf(beta) ~ 2 beta^2 / sqrt(pi), so beta ~ sqrt(St / 2)
    st = 1e-6
    assert abs(analysis.stefan_beta(st, 1.0, 1.0) / math.sqrt(st / 2) - 1.0) < 1e-5
    assert analysis.stefan_beta(1.0, 0.0, 1.0) == 0.0


def test_stefan_cases_of_the_paper():
    """The three Stefan runs (T_r, dT) = (0.86, 0.010), (0.86, 0.023), (0.90, 0.010), c_p = 11:
    beta from the library's latent heat equals beta from the oracle's (golden) latent heat."""
    for tr, dT in (("0.86", 0.010), ("0.86", 0.023), ("0.90", 0.010)):
        h = lbm.saturation(LBMConfig(Tr_sat=float(tr)))["h_fg"]
        b = analysis.stefan_beta(11.0, dT, h)
        b0 = analysis.stefan_beta(11.0, dT, COEX[tr]["h_fg"])
        assert abs(b / b0 - 1.0) < 1e-8
        assert 0.2 < b < 0.6


def test_correlation_forms():
    g = {"gamma": 17.1, "eta": 1.0, "Re": 300.0, "Pr": 1.5, "Ja": 0.21}
    c = analysis.correlations(g)
    assert len(c) == 6
    # Mode 2: Nu ~ Ja^-1/4, gamma^1/4, Pr^1/4, Re^1/2; constants in the ratio of the C values
    for k, e in (("Ja", -0.25), ("gamma", 0.25), ("Pr", 0.25), ("Re", 0.5), ("eta", 0.5)):
        g2 = dict(g, **{k: g[k] * 1.5})
        r = analysis.correlations(g2)["epstein_hauser_C0.537"] / c["epstein_hauser_C0.537"]
        assert abs(r - 1.5 ** e) < 1e-12, k
    assert abs(c["ito_C0.46"] / c["epstein_hauser_C0.537"] - 0.46 / 0.537) < 1e-14
    assert abs(c["epstein_hauser_C1.13"] / c["epstein_hauser_C0.537"] - 1.13 / 0.537) < 1e-14
    # Mode 1: Nu ~ (eta Re Pr)^1/2 (Ja / (1 + 0.4 Ja)^2)^-1/2, so Ja^-1/2 as Ja -> 0
    b = analysis.bromley(1.0, 300.0, 1.5, 0.21)
    assert abs(b - 2.7 * math.sqrt(300.0 * 1.5) * (1 + 0.4 * 0.21) / math.sqrt(0.21)) < 1e-12 * b
    lo = analysis.bromley(1.0, 300.0, 1.5, 1e-8) / analysis.bromley(1.0, 300.0, 1.5, 4e-8)
    assert abs(lo - 2.0) < 1e-6


def test_plesset_zwick():
    r1 = analysis.plesset_zwick_radius(100.0, 5.8e-2, 6.5, 0.38, 11.0, 0.0044, 0.572)
    assert abs(analysis.plesset_zwick_radius(400.0, 5.8e-2, 6.5, 0.38, 11.0, 0.0044, 0.572) / r1 - 2.0) < 1e-14
    assert abs(r1 - math.sqrt(12 * 5.8e-2 / math.pi) * 6.5 * 11.0 * 0.0044 / (0.38 * 0.572) * 10.0) < 1e-14


def _front_fixing_beta(ja, eps, xi_max=8.0, n=700, r_end=40.0):
    """The cylindrical bubble solved as an initial-value problem, independently of the similarity
    reduction: the liquid temperature in xi = r / R(t) on [1, xi_max] (explicit finite differences;
    alpha = 1, rho_l c_p = 1, T = 0 at the interface, 1 at xi_max), the liquid moving outward with
    eps R R' / r, and R' = Ja dT/dr at the interface, from R = 1 and a step profile.  Returns
    sqrt(d(R^2)/dt) / 2 over the second half of the growth to R = r_end."""
    xi = np.linspace(1.0, xi_max, n)
    h = xi[1] - xi[0]
    T = np.ones(n)
    T[0] = 0.0
    R, t, rec = 1.0, 0.0, []
    x = xi[1:-1]
    while R < r_end:
        Tx = (T[2:] - T[:-2]) / (2 * h)
        Txx = (T[2:] - 2 * T[1:-1] + T[:-2]) / (h * h)
        Rd = ja * (-3 * T[0] + 4 * T[1] - T[2]) / (2 * h) / R
        dt = 0.2 * h * h * R * R
        T[1:-1] += dt * ((Txx + Tx / x) / (R * R) + (Rd / R) * (x - eps / x) * Tx)
        R += dt * Rd
        t += dt
        rec.append((t, R))
    rec = np.array(rec[len(rec) // 2:])
    return math.sqrt(np.polyfit(rec[:, 0], rec[:, 1] ** 2, 1)[0]) / 2.0


@pytest.mark.parametrize("ja,eps", [(1.288, 0.934), (0.5, 1.0), (3.0, 0.9)])
def test_cylinder_bubble_growth_constant_against_front_fixing_solution(ja, eps):
    """The similarity root against the time-dependent moving-boundary problem (0.1-0.3 % observed;
    the finite-difference solution carries its grid and start-up errors)."""
    b = analysis.cylinder_bubble_beta(ja, eps)
    fd = _front_fixing_beta(ja, eps)
    assert abs(fd / b - 1.0) < 5e-3, (ja, eps, b, fd)


def test_cylinder_bubble_thin_layer_limit():
    """For eps = 1 and large Ja the growth constant tends to the thin-layer law beta = sqrt(2/pi) Ja
    (the heat flux of a planar layer after the effective time t/2 of a cylinder's stretching)."""
    r50 = analysis.cylinder_bubble_beta(50.0, 1.0) / (math.sqrt(2 / math.pi) * 50.0)
    r200 = analysis.cylinder_bubble_beta(200.0, 1.0) / (math.sqrt(2 / math.pi) * 200.0)
    assert abs(r200 - 1.0) < 3e-3 and abs(r200 - 1.0) < abs(r50 - 1.0)
    assert analysis.cylinder_bubble_beta(0.0, 1.0) == 0.0
