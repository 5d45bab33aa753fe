"""Pins of the oracle's central-moment algebra against matrices and moments printed in the paper
(Saito et al., arXiv:1912.02018, Sec. II A and Appendix A) and against library routines."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CX = np.array([0, 1, -1, 0, 0, 1, -1, 1, -1], dtype=float)
CY = np.array([0, 0, 0, 1, -1, 1, -1, -1, 1], dtype=float)


def printed_M():
    return np.loadtxt(os.path.join(GOLDEN, "transform_M.txt"))


def printed_N(ux, uy):
    """Shift matrix N(u) as printed in Appendix A (eq. shiftD2Q9)."""
    return np.array([
        [1, 0, 0, 0, 0, 0, 0, 0, 0],
        [-ux, 1, 0, 0, 0, 0, 0, 0, 0],
        [-uy, 0, 1, 0, 0, 0, 0, 0, 0],
        [ux**2 + uy**2, -2 * ux, -2 * uy, 1, 0, 0, 0, 0, 0],
        [ux**2 - uy**2, -2 * ux, 2 * uy, 0, 1, 0, 0, 0, 0],
        [ux * uy, -uy, -ux, 0, 0, 1, 0, 0, 0],
        [-ux**2 * uy, 2 * ux * uy, ux**2, -uy / 2, -uy / 2, -2 * ux, 1, 0, 0],
        [-ux * uy**2, uy**2, 2 * ux * uy, -ux / 2, ux / 2, -2 * uy, 0, 1, 0],
        [ux**2 * uy**2, -2 * ux * uy**2, -2 * ux**2 * uy, (ux**2 + uy**2) / 2,
         -(ux**2 - uy**2) / 2, 4 * ux * uy, -2 * uy, -2 * ux, 1],
    ], dtype=float)


RNG = np.random.default_rng(20191204)
VELOCITIES = [(0.0, 0.0), (0.05, -0.02), (-0.11, 0.07), (0.3, 0.25)]


def test_T_at_rest_is_printed_M():
    assert np.array_equal(oracle.T_matrix(0.0, 0.0), printed_M())


def test_det_M_and_invertibility():
    M = printed_M()
    assert np.isclose(np.linalg.det(M), -128.0)
    for ux, uy in VELOCITIES:
        T = oracle.T_matrix(ux, uy)
        # T = N M with N unit lower-triangular, so det T = det M for every u
        assert np.isclose(np.linalg.det(T), -128.0, rtol=1e-12)
        assert np.allclose(np.linalg.inv(T) @ T, np.eye(9), atol=1e-13)


@pytest.mark.parametrize("u", VELOCITIES)
def test_T_factorises_into_printed_N_and_M(u):
    T = oracle.T_matrix(*u)
    assert np.allclose(T, printed_N(*u) @ printed_M(), atol=1e-14)
    # N(u)^-1 = N(-u): the moments shift back
    assert np.allclose(printed_N(*u) @ printed_N(-u[0], -u[1]), np.eye(9), atol=1e-14)


def test_lu_solver_matches_numpy():
    for _ in range(20):
        A = RNG.normal(size=(9, 9))
        b = RNG.normal(size=9)
        assert np.allclose(oracle.lu_solve9(A, b), np.linalg.solve(A, b), rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("u", VELOCITIES)
def test_equilibrium_central_moments_printed(u):
    """k^eq = T f^eq = [rho, 0, 0, 2 rho/3, 0, 0, 0, 0, rho/9] (Sec. II A)."""
    rho = 1.7
    keq = oracle.T_matrix(*u) @ oracle.feq(rho, *u)
    assert np.allclose(keq, [rho, 0, 0, 2 * rho / 3, 0, 0, 0, 0, rho / 9], atol=1e-14)


@pytest.mark.parametrize("u", VELOCITIES)
def test_equilibrium_raw_moments(u):
    rho = 0.9
    f = oracle.feq(rho, *u)
    ux, uy = u
    assert np.isclose(f.sum(), rho)
    assert np.allclose([f @ CX, f @ CY], [rho * ux, rho * uy], atol=1e-15)
    # second moments of the Hermite equilibrium: rho (u u + cs^2 I)
    assert np.isclose(f @ (CX * CX), rho * (ux * ux + 1 / 3))
    assert np.isclose(f @ (CX * CY), rho * ux * uy)


@pytest.mark.parametrize("u", VELOCITIES)
def test_force_central_moments_printed(u):
    """R = T F = [0, Fx, Fy, 0, 0, 0, Fy/3, Fx/3, 0] (eq. force1)."""
    Fx, Fy = 3e-3, -1.1e-3
    R = oracle.T_matrix(*u) @ oracle.force_pop(Fx, Fy, *u)
    assert np.allclose(R, [0, Fx, Fy, 0, 0, 0, Fy / 3, Fx / 3, 0], atol=1e-17)


@pytest.mark.parametrize("u", VELOCITIES)
def test_force_raw_moments(u):
    """Hermite forcing: zeroth moment 0, first F, second F u + u F."""
    Fx, Fy = 2e-3, 5e-4
    F = oracle.force_pop(Fx, Fy, *u)
    ux, uy = u
    assert abs(F.sum()) < 1e-17
    assert np.allclose([F @ CX, F @ CY], [Fx, Fy], atol=1e-17)
    assert np.isclose(F @ (CX * CX), 2 * Fx * ux, atol=1e-17)
    assert np.isclose(F @ (CX * CY), Fx * uy + Fy * ux, atol=1e-17)


@pytest.mark.parametrize("u", VELOCITIES)
@pytest.mark.parametrize("omega", [0.8, 1.25, 1.95])
def test_equilibrium_is_fixed_point(u, omega):
    """With no force the equilibrium of any velocity is reproduced by the collision."""
    rho = 2.3
    f = oracle.feq(rho, *u)
    fs = oracle.collide_node(omega, 0.38, f, rho, u[0], u[1], 0.0, 0.0, 0.0)
    assert np.allclose(fs, f, atol=1e-15)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_collision_matches_closed_form_two_step_reconstruction(seed):
    """f* = M^-1 N(-u) k* with k* from eq. postColl2, using the printed M and N."""
    rng = np.random.default_rng(seed)
    omega, sigma = 1.6, 0.38
    rho = 1.0 + rng.random()
    f = oracle.feq(rho, 0.03, -0.01) + 1e-3 * rng.normal(size=9)
    rho = f.sum()
    F = 1e-3 * rng.normal(size=2)
    Fm2p = abs(1e-4 * rng.normal())
    u = (np.array([f @ CX, f @ CY]) + F / 2) / rho
    fs = oracle.collide_node(omega, sigma, f, rho, u[0], u[1], F[0], F[1], Fm2p)
    M = printed_M()
    k = printed_N(*u) @ M @ f
    A = 2 * sigma * Fm2p
    kstar = np.array([rho, F[0] / 2, F[1] / 2, 2 * rho / 3 + A, (1 - omega) * k[4],
                      (1 - omega) * k[5], F[1] / 6, F[0] / 6, rho / 9 + A / 3])
    expect = np.linalg.solve(M, printed_N(-u[0], -u[1]) @ kstar)
    assert np.allclose(fs, expect, rtol=0, atol=1e-15)
    # conservation: mass, and momentum gains the full force
    assert np.isclose(fs.sum(), rho, rtol=1e-15)
    assert np.allclose([fs @ CX, fs @ CY], [f @ CX + F[0], f @ CY + F[1]], atol=1e-15)
