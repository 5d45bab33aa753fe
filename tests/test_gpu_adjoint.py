"""Reverse-mode adjoint of the step (lbm_adjoint_step, lbm_nu_gradient): the reverse sweep with
checkpoint-and-recompute against the forward-mode tangents, which are the exact derivatives of the
same discrete FP64 step (the two differ only by rounding).

J(theta) = mean Nu of the states average_from .. steps-1, theta = (dTr_wall, u_in, acentric, tau).
Cases (FP64, no heated wall): the boiling channel of the tangent tests (96x48, R 6, Re 30, RK4) with
checkpoint intervals that do and do not divide the run; RK2; no temperature update; a warm-up that
ends inside the run; a channel periodic in x.  Bound: 1e-9 of max |dJ/dtheta| per component (the
tangent run's value part rounds differently from the FP64 run, and the difference grows over the
run), J to 1e-12."""
import json
import os

import numpy as np
import pytest

from paper_1912_02018_amd.config import BC_PERIODIC, F64_TANGENT, FP64, cylinder_config

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
_C = json.load(open(os.path.join(GOLDEN, "maxwell_coexistence.json")))["coexistence"]["0.86"]


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available()
    from paper_1912_02018_amd import lbm, sensitivity
    return lbm, sensitivity


def base_case(**kw):
    c = cylinder_config(96, 48, 6, 24, re=30.0, u_in=0.02, dTr_wall=0.1, precision=FP64, warmup=0,
                        rk_stages=4, diag_every=1)
    return c.replace(rho_l=_C["rho_l"], rho_v=_C["rho_v"], **kw)


def compare(lbm, sens, cfg, steps, avg_from, every, label, tol=1e-9):
    Jt, gt = sens.nu_average_and_gradient(cfg, steps, avg_from)
    sim = lbm.Simulation(cfg)
    Ja, ga = sim.nu_gradient(steps, avg_from, every)
    scale = np.abs(gt).max()
    err = np.abs(ga - gt) / scale
    print(f"[adjoint] {label}: J {Ja:.12e} (tangent {Jt:.12e}); dJ/dtheta adjoint {ga} tangent {gt}; "
          f"max rel diff {err.max():.2e}", flush=True)
    assert abs(Ja - Jt) <= 1e-12 * abs(Jt)
    assert err.max() <= tol, (label, err)
    # the handle ends in the forward run's final state
    assert sim.step_count == steps
    ref = lbm.Simulation(cfg)
    ref.step(steps)
    fa, fr = sim.fields(), ref.fields()
    for k in ("rho", "ux", "uy", "T"):
        assert np.array_equal(fa[k], fr[k]), k
    return ga


@pytest.mark.parametrize("every", [64, 100, 300])
def test_adjoint_matches_tangent_rk4(mods, every):
    lbm, sens = mods
    compare(lbm, sens, base_case(), 300, 100, every, f"96x48 RK4, checkpoints every {every}")


def test_adjoint_matches_tangent_rk2(mods):
    lbm, sens = mods
    compare(lbm, sens, base_case(rk_stages=2), 200, 50, 40, "96x48 RK2")


def test_adjoint_matches_tangent_flow_only(mods):
    """No temperature update: Nu follows the density at the probes (streaming, boundary conditions,
    collision, interaction force and pseudopotential in reverse)."""
    lbm, sens = mods
    compare(lbm, sens, base_case(rk_stages=0), 200, 50, 50, "96x48 no temperature update")


def test_adjoint_matches_tangent_warmup(mods):
    lbm, sens = mods
    compare(lbm, sens, base_case(warmup_steps=60), 200, 100, 50, "96x48 RK4, warm-up of 60 steps")


def test_adjoint_matches_tangent_periodic(mods):
    lbm, sens = mods
    cfg = base_case(bc_x=BC_PERIODIC, gx=-2e-5, upwind_kind=1)
    compare(lbm, sens, cfg, 200, 50, 70, "96x48 periodic in x, Kawamura-Kuwahara")


def test_adjoint_step_by_step_equals_driver(mods):
    """The reverse sweep driven from Python through lbm_adjoint_step (states set with lbm_set_state)
    gives the driver's gradient bit for bit in the components without an initial-state term (the
    acentric factor and tau); the driver adds the initial state's dependence on the superheat (solid
    nodes at T_w) and, from lbm_create's default state, on u_in."""
    import torch
    lbm, sens = mods
    cfg = base_case()
    steps, avg_from = 40, 10
    sim = lbm.Simulation(cfg)
    states = []
    for s in range(steps):
        states.append(sim.get_state())
        sim.step(1)
    drv = lbm.Simulation(cfg)
    _, gd = drv.nu_gradient(steps, avg_from, 16)
    a0, a1, scr = sim.adjoint_buffers()
    bufs = [a0, a1]
    cur = 0
    for s in reversed(range(steps)):
        fs, hist, T, st = states[s]
        sim.set_state(fs, hist, T, st)
        w = 1.0 / (steps - avg_from) if s >= avg_from else 0.0
        g = sim.adjoint_step(bufs[cur], bufs[cur ^ 1], scr, w)
        cur ^= 1
    print(f"[adjoint] step by step {g} driver {gd}", flush=True)
    assert np.array_equal(g[[2, 3]], gd[[2, 3]])
