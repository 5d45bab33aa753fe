"""Pins of the oracle's isotropic stencils and temperature equation (Sec. II B-C of Saito et al.,
arXiv:1912.02018) against isotropy conditions, polynomial exactness and the exact discrete
Fourier symbol of the scheme."""
import numpy as np
import pytest

import oracle
from paper_1912_02018_amd import inputs
from paper_1912_02018_amd.config import LBMConfig, BC_PERIODIC

VECS = [(ex, ey) for ey in range(-2, 3) for ex in range(-2, 3) if (ex, ey) != (0, 0)]


def w(e):
    return oracle.stencil_weight(e[0] ** 2 + e[1] ** 2)


def test_stencil_isotropy_sixth_order():
    """Weights with w(0) = 247/140 sum to 3 = 1/cs^2; second moment is the identity; 4th and
    6th moments are isotropic (the 6th-order isotropic gradient of the interaction force)."""
    s0 = sum(w(e) for e in VECS) + 247.0 / 140.0
    assert np.isclose(s0, 3.0, rtol=1e-15)
    m = lambda a, b: sum(w(e) * e[0] ** a * e[1] ** b for e in VECS)
    assert np.isclose(m(2, 0), 1.0) and np.isclose(m(0, 2), 1.0) and abs(m(1, 1)) < 1e-16
    assert np.isclose(m(4, 0), 3 * m(2, 2))
    assert np.isclose(m(6, 0), 5 * m(4, 2))
    assert abs(m(1, 0)) < 1e-16 and abs(m(3, 0)) < 1e-16 and abs(m(2, 1)) < 1e-16


def _poly_field(n, coef, deg):
    y, x = np.mgrid[0:n, 0:n].astype(float)
    a = np.zeros((n, n))
    k = 0
    for i in range(deg + 1):
        for j in range(deg + 1 - i):
            a += coef[k] * x**i * y**j
            k += 1
    return a, x, y


def test_gradient_exact_on_quadratics_laplacian_exact_on_cubics():
    rng = np.random.default_rng(7)
    n = 16
    c = rng.normal(size=10)
    a, x, y = _poly_field(n, c, 3)
    # cubic a = sum c_k x^i y^j ; analytic derivatives
    dx = np.zeros_like(a); dy = np.zeros_like(a); lap = np.zeros_like(a)
    k = 0
    for i in range(4):
        for j in range(4 - i):
            if i >= 1: dx += c[k] * i * x**(i - 1) * y**j
            if j >= 1: dy += c[k] * j * x**i * y**(j - 1)
            if i >= 2: lap += c[k] * i * (i - 1) * x**(i - 2) * y**j
            if j >= 2: lap += c[k] * j * (j - 1) * x**i * y**(j - 2)
            k += 1
    inner = (slice(2, n - 2), slice(2, n - 2))
    L = oracle.iso_lap_periodic(a)
    assert np.allclose(L[inner], lap[inner], rtol=1e-10, atol=1e-9)
    q, _, _ = _poly_field(n, c[:6], 2)
    gx, gy = oracle.iso_grad_periodic(q)
    # analytic gradient of the quadratic with the same coefficient ordering
    dqx = np.zeros_like(q); dqy = np.zeros_like(q)
    k = 0
    for i in range(3):
        for j in range(3 - i):
            if i >= 1: dqx += c[k] * i * x**(i - 1) * y**j
            if j >= 1: dqy += c[k] * j * x**i * y**(j - 1)
            k += 1
    assert np.allclose(gx[inner], dqx[inner], rtol=1e-11, atol=1e-11)
    assert np.allclose(gy[inner], dqy[inner], rtol=1e-11, atol=1e-11)


def uniform_flow_sim(U, V, alpha, rk, nx=32, ny=16, upwind_kind=0):
    cfg = LBMConfig(nx=nx, ny=ny, bc_x=BC_PERIODIC, rk_stages=rk, nu=0.1, alpha_T=alpha,
                    upwind_kind=upwind_kind)
    s = oracle.Sim(cfg)
    d = s.derived()
    r, ux, uy = inputs.uniform(nx, ny, d["rho_l"], U, V)
    s.set_fields(r, ux, uy)
    return s, d


def symbol(kx, ky, U, V, alpha, cd):
    conv = 0j
    for u, k in ((U, kx), (V, ky)):
        conv += 1j * u * (8 * np.sin(k) - np.sin(2 * k)) / 6 + abs(u) * cd * (2 * np.cos(2 * k) - 8 * np.cos(k) + 6)
    lap = sum(2 * w(e) * (np.cos(kx * e[0] + ky * e[1]) - 1) for e in VECS)
    return -conv + alpha * lap


@pytest.mark.parametrize("upwind_kind,cd", [(0, 1 / 12), (1, 1 / 4)])
@pytest.mark.parametrize("U,V", [(0.04, 0.0), (-0.03, 0.02)])
def test_thermal_operator_fourier_symbol(upwind_kind, cd, U, V):
    """L(e^{ik.x}) = lambda(k) e^{ik.x} in a uniform stream: third-order upwind convection plus
    isotropic diffusion; the pressure-work source vanishes because div u = 0."""
    nx, ny = 32, 16
    alpha = 0.03
    s, d = uniform_flow_sim(U, V, alpha, 4, nx, ny, upwind_kind)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    for mx, my in ((1, 0), (3, 2), (5, -1)):
        kx, ky = 2 * np.pi * mx / nx, 2 * np.pi * my / ny
        delta = 1e-3
        mode = np.exp(1j * (kx * x + ky * y))
        Y = d["T_sat"] + delta * mode.imag
        L = s.thermal_rhs(Y)
        lam = symbol(kx, ky, U, V, alpha, cd)
        assert np.allclose(L, delta * (lam * mode).imag, rtol=0, atol=1e-15)


@pytest.mark.parametrize("rk", [2, 4])
def test_runge_kutta_amplification(rk):
    """One step multiplies a Fourier mode by the RK stability polynomial of lambda."""
    nx, ny = 32, 16
    U, V, alpha = 0.05, -0.01, 0.04
    s, d = uniform_flow_sim(U, V, alpha, rk, nx, ny)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    kx, ky = 2 * np.pi * 2 / nx, 2 * np.pi * 1 / ny
    mode = np.exp(1j * (kx * x + ky * y))
    delta = 1e-3
    Y = d["T_sat"] + delta * mode.imag
    out = s.thermal_advance(Y)
    lam = symbol(kx, ky, U, V, alpha, 1 / 12)
    G = 1 + lam + lam**2 / 2 if rk == 2 else 1 + lam + lam**2 / 2 + lam**3 / 6 + lam**4 / 24
    assert np.allclose(out - d["T_sat"], delta * (G * mode).imag, rtol=0, atol=1e-15)


def test_thermal_operator_assembly_with_density_and_divergence():
    """With non-uniform rho and u the right-hand side combines upwind convection, isotropic
    diffusion alpha (lap T + grad rho . grad T / rho) and -T (dp/dT)_rho div u / (rho c_v)."""
    nx, ny = 24, 16
    cfg = LBMConfig(nx=nx, ny=ny, bc_x=BC_PERIODIC, rk_stages=4, nu=0.1, alpha_T=0.02)
    s = oracle.Sim(cfg)
    d = s.derived()
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    rho = d["rho_l"] * (1 + 0.01 * np.sin(2 * np.pi * x / nx) * np.cos(2 * np.pi * y / ny))
    ux = 0.02 * np.sin(2 * np.pi * 2 * x / nx)
    uy = 0.01 * np.cos(2 * np.pi * y / ny)
    s.set_fields(rho, ux, uy)
    F = s.fields()
    Y = d["T_sat"] * (1 + 0.02 * np.cos(2 * np.pi * (x / nx + 2 * y / ny)))
    L = s.thermal_rhs(Y)

    def up(a, u, axis):
        p1, p2 = np.roll(a, -1, axis), np.roll(a, -2, axis)
        m1, m2 = np.roll(a, 1, axis), np.roll(a, 2, axis)
        return u * (-p2 + 8 * p1 - 8 * m1 + m2) / 12 + np.abs(u) * (p2 - 4 * p1 + 6 * a - 4 * m1 + m2) / 12

    conv = up(Y, F["ux"], 1) + up(Y, F["uy"], 0)
    gTx, gTy = oracle.iso_grad_periodic(Y)
    grx, gry = oracle.iso_grad_periodic(F["rho"])
    div = oracle.iso_grad_periodic(F["ux"])[0] + oracle.iso_grad_periodic(F["uy"])[1]
    lap = oracle.iso_lap_periodic(Y)
    dpdT = np.vectorize(lambda r, t: oracle.eos_dpdT(cfg, r, t))(F["rho"], Y)
    expect = -conv + cfg.alpha_T * (lap + (grx * gTx + gry * gTy) / F["rho"]) - Y * dpdT * div / (F["rho"] * cfg.cv)
    assert np.allclose(L, expect, rtol=1e-12, atol=1e-16)
    assert np.abs(div).max() > 1e-4  # the source term is exercised
