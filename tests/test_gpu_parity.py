"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

FP64: max-norm relative error ||a_gpu - a_ref||_inf / ||a_ref||_inf <= 1e-12 per 1000 steps for
rho, T and the post-collision populations, and for the velocity vector relative to
max(||u||_inf, u_ref).  The two sides differ only by rounding order (closed-form reconstruction
versus LU solve, tree versus serial sums, FMA contraction).  FP32 runs are compared with the
oracle stepped one step from the same state, within bounds set by FP32 rounding of one step
(unit roundoff 6e-8 times a dependent chain of ~30 operations: 2e-6; 2e-5 for the velocity, a
difference of populations), and after 1000 steps with the accumulated bound stated in the test.
Sizes span several tiles and ragged tails.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1912_02018_amd import inputs
from paper_1912_02018_amd.config import (LBMConfig, FP64, FP32, BC_PERIODIC, BC_INLET_OUTLET,
                                         config1, config2, cylinder_config)

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
COEX = json.load(open(os.path.join(GOLDEN, "maxwell_coexistence.json")))["coexistence"]
TOL64 = 1e-12


def coex(tr=0.86):
    c = COEX[f"{tr:.2f}"]
    return c["rho_l"], c["rho_v"]


@pytest.fixture(scope="module")
def lbm_mod():
    import torch
    assert torch.cuda.is_available()
    from paper_1912_02018_amd import lbm
    return lbm


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def compare(sim, ref, label, tol=TOL64, tol_u=None, u_ref=0.01, run=0):
    """Relative max-norm differences of rho, T and the populations f*; velocity as a vector,
    relative to max(||u||_inf, u_ref) so that a flow decaying towards rest is not measured against
    its own vanishing scale (u_ref = inlet velocity for channels, 0.01 otherwise)."""
    g, o = sim.fields(run), ref.fields()
    assert np.array_equal(g["mask"], o["mask"])
    fluid = o["mask"] == 0
    errs = {k: rel(g[k][fluid], o[k][fluid]) for k in ("rho", "T")}
    du = np.hypot(g["ux"] - o["ux"], g["uy"] - o["uy"])[fluid].max()
    umax = np.hypot(o["ux"], o["uy"])[fluid].max()
    errs["u"] = float(du / max(umax, u_ref))
    fg, _, _, _ = sim.get_state(run)
    fo, _, _, _ = ref.get_state()
    errs["f*"] = max(rel(fg[i][fluid], fo[i][fluid]) for i in range(9))
    print(f"[parity] {label}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items())
          + f" (|u|max {umax:.3e})", flush=True)
    for k, v in errs.items():
        t = tol_u if (tol_u is not None and k == "u") else tol
        assert v <= t, (label, k, v)
    return errs


def run_pair(lbm, cfg, steps, fields=None):
    sim = lbm.Simulation(cfg)
    ref = oracle.Sim(cfg)
    if fields is not None:
        sim.set_fields(*fields)
        ref.set_fields(*fields)
    sim.step(steps)
    ref.step(steps)
    return sim, ref


@pytest.mark.parametrize("steps", [1000, 2000])
def test_flat_interface_fp64(lbm_mod, steps):
    rl, rv = coex()
    cfg = config1().replace(rho_l=rl, rho_v=rv)
    rho = inputs.slab(128, 64, 32, 96, rl, rv, 1e-3, 1912)
    sim, ref = run_pair(lbm_mod, cfg, steps, (rho, 0.0, 0.0))
    # rounding-order differences accumulate about linearly: 1e-12 per 1000 steps
    compare(sim, ref, f"flat interface 128x64 {steps} steps", tol=TOL64 * steps / 1000)
    # the GPU step closes the mass balance node by node: its total mass is constant to rounding;
    # the oracle's own drift (LU rounding, pinned at < 1e-12 over 2000 steps) bounds the gap
    m_g, m_o = sim.total_mass(), ref.total_mass()
    assert abs(m_g / rho.sum() - 1) < 1e-13
    assert abs(m_g / m_o - 1) < 1e-12


def cylinder_case(nx=128, ny=64, r=8, cx=40, re=100.0, rk=4, precision=FP64, **kw):
    rl, rv = coex()
    cfg = cylinder_config(nx, ny, r, cx, re=re, u_in=0.02, dTr_wall=0.1, precision=precision,
                          warmup=0, rk_stages=rk, diag_every=10)
    return cfg.replace(rho_l=rl, rho_v=rv, **kw)


def test_heated_cylinder_channel_fp64(lbm_mod):
    cfg = cylinder_case()
    sim, ref = run_pair(lbm_mod, cfg, 1000)
    compare(sim, ref, "cylinder 128x64 R8 RK4 1000 steps", u_ref=cfg.u_in)
    qg, nug, nuag = sim.wall_heat_flux()
    qo, nuo, nuao = ref.wall_heat_flux()
    print(f"[parity] heat flux gpu {qg:.10e} {nug:.10e} {nuag:.10e} oracle {qo:.10e} {nuo:.10e} {nuao:.10e}", flush=True)
    assert abs(qg / qo - 1) < TOL64 and abs(nug / nuo - 1) < TOL64 and abs(nuag / nuao - 1) < TOL64
    assert abs(sim.total_mass() / ref.total_mass() - 1) < TOL64


def test_ragged_tiles_rk2_kawamura_kuwahara_fp64(lbm_mod):
    cfg = cylinder_case(nx=100, ny=50, r=6, cx=30, rk=2, upwind_kind=1)
    sim, ref = run_pair(lbm_mod, cfg, 300)
    compare(sim, ref, "cylinder 100x50 R6 RK2 KK 300 steps", u_ref=cfg.u_in)


@pytest.mark.parametrize("rk", [4, 2])
def test_odd_row_count_every_thermal_variant_fp64(lbm_mod, rk):
    """The temperature kernel updates positions in vertically adjacent pairs: with an odd number of
    rows the last pair of a tile column reaches one row past the domain (a periodic copy, computed and
    not stored).  Every temperature-kernel variant against the oracle, on a channel and on a tiny
    periodic box whose halo spans several periods."""
    cfg = cylinder_case(nx=90, ny=45, r=6, cx=28, rk=rk)
    ref = oracle.Sim(cfg)
    ref.step(150)
    rl, rv = coex()
    tiny = LBMConfig(nx=6, ny=5, bc_x=BC_PERIODIC, rk_stages=rk, nu=0.1, alpha_T=0.05, rho_l=rl, rho_v=rv,
                     precision=FP64)
    fields = inputs.random_fields(6, 5, rl, 1e-3, 1e-3, seed=21)
    T = np.full((5, 6), 0.86 * COEX_TC()) * (1 + inputs.uniform_noise(22, (5, 6), 1e-3))
    tiny_ref = oracle.Sim(tiny)
    tiny_ref.set_fields(*fields, T)
    tiny_ref.step(100)
    for vt in range(len(lbm_mod.Simulation(cfg).variants(1))):
        sim = lbm_mod.Simulation(cfg)
        sim.set_variant(1, vt)
        sim.step(150)
        compare(sim, ref, f"channel 90x45 RK{rk} thermal variant {vt}", u_ref=cfg.u_in)
        t = lbm_mod.Simulation(tiny)
        t.set_variant(1, vt)
        t.set_fields(*fields, T)
        t.step(100)
        compare(t, tiny_ref, f"periodic 6x5 RK{rk} thermal variant {vt}")


def test_periodic_array_with_gravity_fp64(lbm_mod):
    rl, rv = coex()
    cfg = LBMConfig(nx=72, ny=40, bc_x=BC_PERIODIC, cyl_x=36, cyl_y=20, cyl_r=7, rk_stages=4,
                    nu=0.05, alpha_T=0.03, dTr_wall=0.05, gx=1e-5, gy=-2e-6, rho_gref=0.0,
                    rho_l=rl, rho_v=rv, precision=FP64)
    sim, ref = run_pair(lbm_mod, cfg, 300)
    compare(sim, ref, "periodic cylinder array 72x40 300 steps")


def test_tiny_grid_random_fields_fp64(lbm_mod):
    rl, rv = coex()
    cfg = LBMConfig(nx=5, ny=4, bc_x=BC_PERIODIC, rk_stages=4, nu=0.1, alpha_T=0.05,
                    rho_l=rl, rho_v=rv, precision=FP64)
    rho, ux, uy = inputs.random_fields(5, 4, rl, 1e-3, 1e-3, seed=11)
    T = np.full((4, 5), 0.86 * COEX_TC()) * (1 + inputs.uniform_noise(12, (4, 5), 1e-3))
    sim, ref = run_pair(lbm_mod, cfg, 200, (rho, ux, uy, T))
    compare(sim, ref, "tiny 5x4 random 200 steps")


def COEX_TC():
    return json.load(open(os.path.join(GOLDEN, "maxwell_coexistence.json")))["Tc"]


def test_warmup_switch_fp64(lbm_mod):
    cfg = cylinder_case(nx=96, ny=48, r=6, cx=30).replace(warmup_steps=40)
    sim, ref = run_pair(lbm_mod, cfg, 100)
    compare(sim, ref, "warm-up 40 then 60 coupled steps", u_ref=cfg.u_in)


def test_state_roundtrip_and_reproducibility(lbm_mod):
    cfg = cylinder_case(nx=96, ny=48, r=6, cx=30)
    a = lbm_mod.Simulation(cfg)
    a.step(50)
    fs, hist, T, step = a.get_state()
    b = lbm_mod.Simulation(cfg)
    b.set_state(fs, hist, T, step)
    a.step(50)
    b.step(50)
    sa, sb = a.get_state(), b.get_state()
    assert all(np.array_equal(x, y) for x, y in zip(sa[:3], sb[:3]))


def developed_state(lbm, cfg, steps):
    sim = lbm.Simulation(cfg)
    sim.step(steps)
    return sim


@pytest.mark.parametrize("precision,tol,tol_u,rk", [(FP64, TOL64, TOL64, 4), (FP32, 2e-6, 2e-5, 4),
                                                     (FP32, 2e-6, 2e-5, 2)])
def test_full_size_one_step(lbm_mod, precision, tol, tol_u, rk):
    """1024x512 boiling channel (bench launch configuration; RK2 too, the paper's scheme): after 200
    coupled steps on the GPU the oracle takes the GPU state and both advance one step."""
    rl, rv = coex()
    cfg = config2(precision).replace(warmup_steps=0, rho_l=rl, rho_v=rv, rk_stages=rk)
    sim = lbm_mod.Simulation(cfg)
    sim.autotune(5)  # the launch variants the bench would time
    sim.step(200)
    fs, hist, T, step = sim.get_state()
    ref = oracle.Sim(cfg.replace(precision=FP64))
    ref.set_state(fs, hist, T, step)
    sim.step(1)
    ref.step(1)
    compare(sim, ref, f"1024x512 RK{rk} one step from GPU state ({'fp64' if precision == FP64 else 'fp32'})",
            tol=tol, tol_u=tol_u, u_ref=cfg.u_in)


def storage_half_ulp(v, pname):
    """Half the spacing of the 16-bit storage format at |v| (FP16: 10 fraction bits, subnormal below
    2^-14; BF16: 7 fraction bits)."""
    a = np.abs(v)
    if pname == "f16":
        e = np.floor(np.log2(np.maximum(a, 2.0 ** -14)))
        return 0.5 * 2.0 ** (e - 10)
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -126)))
    return 0.5 * 2.0 ** (e - 7)


@pytest.mark.parametrize("pname", ["f16", "bf16"])
def test_full_size_reduced_storage_one_step(lbm_mod, pname):
    """1024x512 channel at Re 30000 (u_in 0.05) with the populations stored in FP16 / BF16 as
    f - w_i rho_l: after 200 coupled steps on the GPU the oracle takes the GPU state (values the storage
    represents) and both advance one step.
      * every stored population differs from the oracle's by at most half a storage ulp of
        f - w_i rho_l plus the FP32 rounding of the step;
      * T (advanced with rho, u of the step, computed in FP32 from the shared state) to FP32 rounding;
      * rho, u of the new state (a macroscopic pass over the stored populations) against the oracle
        reading the same GPU state, to FP32 rounding."""
    from paper_1912_02018_amd.config import FP16S, BF16S, config3
    prec = FP16S if pname == "f16" else BF16S
    rl, rv = coex()
    cfg = config3(prec).replace(warmup_steps=0, rho_l=rl, rho_v=rv, rho_ref_shift=rl)
    sim = developed_state(lbm_mod, cfg, 200)
    fs, hist, T, step = sim.get_state()
    ref = oracle.Sim(cfg.replace(precision=FP64))
    ref.set_state(fs, hist, T, step)
    sim.step(1)
    ref.step(1)
    fluid = ref.fields()["mask"] == 0
    fg, hg, Tg, sg = sim.get_state()
    fo, _, To, _ = ref.get_state()
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    worst = 0.0
    for i in range(9):
        shift = float(np.float32(w[i] * rl))
        bound = storage_half_ulp(fo[i] - shift, pname) + 4e-6 * np.abs(fo[i][fluid]).max()
        worst = max(worst, float((np.abs(fg[i] - fo[i]) / bound)[fluid].max()))
    errT = rel(Tg[fluid], To[fluid])
    print(f"[parity] {pname} storage 1024x512 one step: f* at most {worst:.3f} of half a storage ulp + FP32, "
          f"T {errT:.2e}", flush=True)
    assert worst <= 1.0
    assert errT <= 2e-6
    now = oracle.Sim(cfg.replace(precision=FP64))
    now.set_state(fg, hg, Tg, sg)
    compare(sim, now, f"{pname} storage 1024x512 macroscopic pass of the stepped GPU state", tol=2e-6, tol_u=2e-5,
            u_ref=cfg.u_in)


def test_full_size_sweep_sampled_runs(lbm_mod):
    """The 64-run sweep at its full sizes (14.9 M nodes) in the bench's launch configuration (one
    handle, autotuned variants, 3 stream groups): after 100 steps three sampled runs (the largest,
    the smallest and one between) are handed to the oracle and both advance one step (FP32 vs FP64)."""
    from paper_1912_02018_amd.config import sweep_configs
    cfgs = [c.replace(warmup_steps=0) for c in sweep_configs(64, 2018, FP32)]
    sizes = [c.nx * c.ny for c in cfgs]
    picks = [int(np.argmax(sizes)), int(np.argmin(sizes)), len(cfgs) // 2]
    sim = lbm_mod.Simulation(cfgs)
    sim.step(10)
    sim.autotune(3)
    sim.set_stream_groups(3)
    sim.step(90)
    refs = {}
    for r in picks:
        fs, hist, T, step = sim.get_state(r)
        refs[r] = oracle.Sim(cfgs[r].replace(precision=FP64))
        refs[r].set_state(fs, hist, T, step)
    sim.step(1)
    for r in picks:
        refs[r].step(1)
        compare(sim, refs[r], f"sweep run {r} ({cfgs[r].nx}x{cfgs[r].ny}) one step from the batched GPU state",
                tol=2e-6, tol_u=2e-5, u_ref=cfgs[r].u_in, run=r)


def test_fp32_error_after_1000_steps(lbm_mod):
    """FP32 path against the FP64 oracle on the heated cylinder after 1000 steps."""
    cfg64 = cylinder_case()
    cfg32 = cfg64.replace(precision=FP32)
    sim = lbm_mod.Simulation(cfg32)
    ref = oracle.Sim(cfg64)
    sim.step(1000)
    ref.step(1000)
    compare(sim, ref, "fp32 vs oracle cylinder 1000 steps", tol=1e-4, tol_u=1e-3, u_ref=cfg32.u_in)


# Reduced-precision storage (FP32 compute, populations stored as f_i - w_i rho_ref in FP16 or BF16)
# after 1000 steps of a 256x128 channel (R 8, no warm-up) against the FP64 oracle.  Storage rounding
# has relative spacing 2^-11 (FP16) or 2^-8 (BF16) on f_i - w_i rho_ref; with rho_ref = rho_l the
# liquid's populations keep most of their bits, with rho_ref = 1 (f_i - w_i) they do not.
# Accuracy target of a usable reduced-storage run (max-norm relative over fluid nodes; u relative to
# max(|u|, u_in); Nu relative): rho and T within 1e-3, u within 1e-2, Nu within 1e-3.  FP16 storage
# shifted by w_i rho_l must meet it at both Reynolds numbers.  FP16 with the literal shift w_i and
# BF16 storage do not (measured on MI355X: FP16 / w_i rho 1.1e-2 and u 4.0e-2 at Re 30000; BF16 /
# w_i rho_l rho 6.1e-3 and u 4.4e-2 at Re 30000, 6.4e-3 and 3.7e-2 at Re 300): their errors are
# reported and only held below a sanity ceiling of 0.2.
STORAGE_TARGET = (1e-3, 1e-2, 1e-3, 1e-3)       # rho, u, T, Nu
STORAGE_CASES = [("f16", "rho_l"), ("f16", "one"), ("bf16", "rho_l")]


@pytest.mark.parametrize("re,u_in", [(30000.0, 0.05), (300.0, 0.02)])
def test_reduced_precision_storage_error_bounds(lbm_mod, re, u_in):
    from paper_1912_02018_amd.config import FP16S, BF16S
    rl, rv = coex()
    base = cylinder_config(256, 128, 8, 64, re=re, u_in=u_in, dTr_wall=0.1, precision=FP64, warmup=0,
                           diag_every=10).replace(rho_l=rl, rho_v=rv)
    ref = oracle.Sim(base)
    ref.step(1000)
    o = ref.fields()
    fl = o["mask"] == 0
    nu0 = ref.wall_heat_flux()[1]
    errs = {}
    for pname, shift in STORAGE_CASES:
        prec = FP16S if pname == "f16" else BF16S
        # the default shift (rho_ref_shift <= 0) is rho_l
        sim = lbm_mod.Simulation(base.replace(precision=prec, rho_ref_shift=0.0 if shift == "rho_l" else 1.0))
        sim.step(1000)
        g = sim.fields()
        du = np.hypot(g["ux"] - o["ux"], g["uy"] - o["uy"])[fl].max()
        e = (rel(g["rho"][fl], o["rho"][fl]), float(du / max(np.hypot(o["ux"], o["uy"])[fl].max(), u_in)),
             rel(g["T"][fl], o["T"][fl]), abs(sim.wall_heat_flux()[1] / nu0 - 1.0))
        errs[(pname, shift)] = e
        meets = all(v <= t for v, t in zip(e, STORAGE_TARGET))
        print(f"Re {re:g} {pname} shift {shift}: rho {e[0]:.2e} u {e[1]:.2e} T {e[2]:.2e} Nu {e[3]:.2e} "
              f"({'meets' if meets else 'misses'} the accuracy target)", flush=True)
        if (pname, shift) == ("f16", "rho_l"):
            for name, v, b in zip(("rho", "u", "T", "Nu"), e, STORAGE_TARGET):
                assert v <= b, (re, pname, shift, name, v, b)
        else:
            assert all(np.isfinite(v) and v <= 0.2 for v in e), (re, pname, shift, e)
    # shifting by w_i rho_l rather than w_i keeps the liquid's precision
    assert errs[("f16", "rho_l")][0] * 5 <= errs[("f16", "one")][0]


def test_graph_replay_matches_eager_bitwise(lbm_mod):
    """Steps replayed from captured HIP graphs equal directly launched steps bit for bit, over
    several replays separated by eager work (field read-back, heat-flux reductions)."""
    cfg = cylinder_case(nx=96, ny=48, r=6, cx=30, precision=FP32)
    a, b = lbm_mod.Simulation(cfg), lbm_mod.Simulation(cfg)
    b.set_graphs(False)
    for chunk in (7, 40, 25, 100, 3, 60):
        a.step(chunk)
        b.step(chunk)
        fa, fb = a.fields(), b.fields()
        assert all(np.array_equal(fa[k], fb[k]) for k in ("rho", "ux", "uy", "T")), chunk
        assert a.wall_heat_flux() == b.wall_heat_flux()
    assert all(np.array_equal(x, y) for x, y in zip(a.get_state()[:3], b.get_state()[:3]))


def test_profiled_steps_advance_like_steps(lbm_mod):
    """lbm_profile_steps advances the state exactly as lbm_step (bit for bit) and reports a
    positive mean duration for both kernels and for the diagnostic reductions (every 10 steps);
    out-of-range counts are rejected."""
    cfg = cylinder_case(nx=96, ny=48, r=6, cx=30, precision=FP32)
    a, b = lbm_mod.Simulation(cfg), lbm_mod.Simulation(cfg)
    a.step(10)
    b.step(10)
    ms = a.profile_steps(37)
    b.step(37)
    assert a.step_count == b.step_count == 47
    assert all(np.array_equal(x, y) for x, y in zip(a.get_state()[:3], b.get_state()[:3]))
    assert 0 < ms[0] < 100 and 0 < ms[1] < 100 and 0 < ms[2] < 100, ms
    for bad in (0, 4097):
        with pytest.raises(lbm_mod.LBMError):
            a.profile_steps(bad)


@pytest.mark.parametrize("precision,rk", [(FP32, 4), (FP64, 4), (FP32, 2)])
def test_launch_variants_agree(lbm_mod, precision, rk):
    """Every tile shape of both stencil kernels gives the same state bit for bit (the per-node
    arithmetic does not depend on the tile, nor on where a temperature slot keeps T^n and its
    accumulator); FP64 variants also match the oracle."""
    cfg = cylinder_case(nx=100, ny=50, r=6, cx=30, precision=precision, rk=rk)
    ref_state = None
    probe = lbm_mod.Simulation(cfg)
    nl, nt = len(probe.variants(0)), len(probe.variants(1))
    for vl in range(nl):
        for vt in range(nt):
            sim = lbm_mod.Simulation(cfg)
            sim.set_variant(0, vl)
            sim.set_variant(1, vt)
            sim.step(120)
            st = sim.get_state()[:3]
            if ref_state is None:
                ref_state = st
                if precision == FP64:
                    ref = oracle.Sim(cfg)
                    ref.step(120)
                    compare(sim, ref, f"variants lbm {vl} thermal {vt}", u_ref=cfg.u_in)
            else:
                assert all(np.array_equal(x, y) for x, y in zip(st, ref_state)), (vl, vt)


@pytest.mark.parametrize("case", ["channel", "periodic", "warmup", "wall", "f16", "bf16"])
def test_stream_collide_variants_agree_several_strips(lbm_mod, case):
    """Every launch variant of the stream-and-collide kernel (tiles, and strips marching down chunks of
    rows) gives the same state bit for bit on grids that take several strips and chunks with ragged
    last ones: a heated-cylinder channel (populations stored in FP32, FP16 and BF16), a periodic box
    with random fields, a warm-up that ends mid-run, and a heated wall with phase-dependent transport
    and the local outlet speed."""
    from paper_1912_02018_amd.config import BC_WALL_OUTLET, OUTLET_LOCAL
    rl, rv = coex()
    fields = None
    if case == "channel":
        cfg = cylinder_case(nx=300, ny=150, r=12, cx=90, precision=FP32)
    elif case in ("f16", "bf16"):
        from paper_1912_02018_amd.config import FP16S, BF16S
        cfg = cylinder_case(nx=300, ny=150, r=12, cx=90, precision=FP16S if case == "f16" else BF16S)
    elif case == "periodic":
        cfg = LBMConfig(nx=270, ny=133, bc_x=BC_PERIODIC, rk_stages=4, nu=0.05, alpha_T=0.02, dTr_wall=0.05,
                        rho_l=rl, rho_v=rv, precision=FP32, gy=-1e-5)
        fields = inputs.random_fields(270, 133, rl, 0.05, 0.01, seed=7)
    elif case == "warmup":
        cfg = cylinder_case(nx=260, ny=140, r=10, cx=70, precision=FP32, warmup_steps=25)
    else:
        cfg = LBMConfig(nx=300, ny=70, bc_x=BC_WALL_OUTLET, rk_stages=4, nu=0.05, nu_vapor=0.15, alpha_T=0.01,
                        alpha_vapor=0.1, rho_l=rl, rho_v=rv, rho_wall=rv, dTr_wall=0.09, precision=FP32,
                        outlet_kind=OUTLET_LOCAL)
        fields = (inputs.slab(300, 70, 20, 300, rl, rv), np.zeros((70, 300)), np.zeros((70, 300)))
    ref_state = None
    nl = len(lbm_mod.Simulation(cfg).variants(0))
    for vl in range(nl):
        sim = lbm_mod.Simulation(cfg)
        if fields is not None:
            sim.set_fields(*fields)
        sim.set_variant(0, vl)
        sim.step(60)
        st = sim.get_state()[:3]
        if ref_state is None:
            ref_state = st
        else:
            assert all(np.array_equal(x, y) for x, y in zip(st, ref_state)), (case, vl)


@pytest.mark.parametrize("case", ["channel", "periodic", "warmup", "wall", "rk2"])
def test_temperature_variants_agree_several_strips(lbm_mod, case):
    """Every launch variant of the temperature kernel (tiles, and strips marching down chunks of rows)
    gives the same state bit for bit on grids that take several strips and chunks with ragged last
    ones: a heated-cylinder channel whose cylinder spans two chunks, a periodic box with random
    fields, a warm-up that ends mid-run, a heated wall with phase-dependent transport, and RK2 with
    the Kawamura-Kuwahara upwind weight."""
    from paper_1912_02018_amd.config import BC_WALL_OUTLET, OUTLET_LOCAL
    rl, rv = coex()
    fields = None
    if case == "channel":
        cfg = cylinder_case(nx=600, ny=150, r=12, cx=250, precision=FP32).replace(cyl_y=64)
    elif case == "periodic":
        cfg = LBMConfig(nx=270, ny=133, bc_x=BC_PERIODIC, rk_stages=4, nu=0.05, alpha_T=0.02, dTr_wall=0.05,
                        rho_l=rl, rho_v=rv, precision=FP32, gy=-1e-5)
        fields = inputs.random_fields(270, 133, rl, 0.05, 0.01, seed=9)
    elif case == "warmup":
        cfg = cylinder_case(nx=500, ny=140, r=10, cx=70, precision=FP32, warmup_steps=25)
    elif case == "wall":
        cfg = LBMConfig(nx=300, ny=70, bc_x=BC_WALL_OUTLET, rk_stages=4, nu=0.05, nu_vapor=0.15, alpha_T=0.01,
                        alpha_vapor=0.1, rho_l=rl, rho_v=rv, rho_wall=rv, dTr_wall=0.09, precision=FP32,
                        outlet_kind=OUTLET_LOCAL)
        fields = (inputs.slab(300, 70, 20, 300, rl, rv), np.zeros((70, 300)), np.zeros((70, 300)))
    else:
        cfg = cylinder_case(nx=520, ny=150, r=10, cx=120, rk=2, upwind_kind=1, precision=FP32)
    ref_state = None
    nt = len(lbm_mod.Simulation(cfg).variants(1))
    for vt in range(nt):
        sim = lbm_mod.Simulation(cfg)
        if fields is not None:
            sim.set_fields(*fields)
        sim.set_variant(1, vt)
        sim.step(60)
        st = sim.get_state()[:3]
        if ref_state is None:
            ref_state = st
        else:
            assert all(np.array_equal(x, y) for x, y in zip(st, ref_state)), (case, vt)


def test_autotune_cache(lbm_mod):
    """A tuned choice is remembered per workload shape: cached=True on another handle of the same
    shape applies it without timing; a new shape is tuned on its first cached call."""
    cfg = cylinder_case(nx=96, ny=48, r=6, cx=30, precision=FP32)
    a = lbm_mod.Simulation(cfg)
    best = a.autotune(3)
    b = lbm_mod.Simulation(cfg)
    b.set_variant(0, (best[0] + 1) % len(b.variants(0)))
    assert b.autotune(cached=True) == best
    assert (b.get_variant(0), b.get_variant(1)) == best
    c = lbm_mod.Simulation(cfg.replace(nx=112))
    got = c.autotune(cached=True)
    assert 0 <= got[0] < len(c.variants(0)) and 0 <= got[1] < len(c.variants(1))
    assert c.autotune(cached=True) == got


def test_autotune_over_whole_steps_advances_the_state_as_stepping(lbm_mod):
    """With whole-step tuning the autotuner steps the handle (3 + launches steps per variant and round,
    two rounds over each kernel's variants); since every variant gives the same state bit for bit,
    the state then equals that of plain stepping by the same count."""
    cfg = cylinder_case(nx=96, ny=48, r=6, cx=30, precision=FP32)
    a = lbm_mod.Simulation(cfg)
    a.step(5)
    a.set_tune_steps(True)
    best = a.autotune(2)
    nv = len(a.variants(0)) + len(a.variants(1))
    assert a.step_count == 5 + 2 * (3 + 2) * nv
    assert (a.get_variant(0), a.get_variant(1)) == best
    b = lbm_mod.Simulation(cfg)
    b.step(a.step_count)
    assert all(np.array_equal(x, y) for x, y in zip(a.get_state()[:3], b.get_state()[:3]))
    assert a.wall_heat_flux() == b.wall_heat_flux()
    a.set_tune_steps(False)
    n = a.step_count
    a.autotune(2)
    assert a.step_count == n


def test_autotune_keeps_results(lbm_mod):
    cfg = cylinder_case(nx=128, ny=64, precision=FP32)
    a, b = lbm_mod.Simulation(cfg), lbm_mod.Simulation(cfg)
    best = a.autotune(5)
    assert a.get_variant(0) == best[0] and a.get_variant(1) == best[1]
    a.step(50)
    b.step(50)
    assert all(np.array_equal(x, y) for x, y in zip(a.get_state()[:3], b.get_state()[:3]))


def test_degenerate_cases(lbm_mod):
    """Uniform saturated liquid at rest in a periodic box stays at rest (equilibrium is a fixed
    point of the collision, psi is uniform so the force vanishes, and T_sat is a steady state of
    the temperature equation); with zero superheat the cylinder reports Nu = 0 (no division by
    the zero temperature difference)."""
    rl, rv = coex()
    cfg = LBMConfig(nx=48, ny=40, bc_x=BC_PERIODIC, rk_stages=4, nu=0.1, alpha_T=0.05, rho_l=rl, rho_v=rv,
                    precision=FP64)
    sim = lbm_mod.Simulation(cfg)
    sim.step(100)
    f = sim.fields()
    assert np.abs(f["rho"] - rl).max() <= 1e-13 * rl
    assert np.hypot(f["ux"], f["uy"]).max() <= 1e-14
    Tsat = sim.derived()["T_sat"]
    assert np.abs(f["T"] - Tsat).max() <= 1e-15
    cyl = cylinder_config(96, 48, 6, 24, re=30.0, u_in=0.02, dTr_wall=0.0, precision=FP64, warmup=0,
                          diag_every=1).replace(rho_l=rl, rho_v=rv)
    sim = lbm_mod.Simulation(cyl)
    sim.step(20)
    q, nu, nua = sim.wall_heat_flux()
    assert nu == 0.0 and nua == 0.0
    assert np.isfinite(q)


def test_unstable_state_is_reported_and_checkpoint_recovers(lbm_mod):
    """Failure detection, forced from the host (the kernels only compute non-finite values and exit):
    a NaN density injected at one node makes lbm_step report LBM_EUNSTABLE at its next check;
    restoring the last checkpoint recovers, and the run then equals the uninterrupted one bit for bit.
    A wall superheat far beyond the range where the pseudopotential is real (negative radicand at the
    solid nodes' density and wall temperature, reported as non-finite rather than clamped) fails the same
    way."""
    cfg = cylinder_case(nx=96, ny=48, r=6, cx=30, precision=FP64, check_every=10, diag_every=5)
    ref = lbm_mod.Simulation(cfg)
    ref.step(100)
    sim = lbm_mod.Simulation(cfg)
    sim.step(50)
    blob = sim.save()
    f = sim.fields()
    rho = f["rho"].copy()
    rho[20, 40] = np.nan
    sim.set_fields(rho, f["ux"], f["uy"], f["T"])
    with pytest.raises(lbm_mod.LBMError) as err:
        sim.step(20)
    assert err.value.code == lbm_mod.LBM_EUNSTABLE
    sim.load(blob)
    sim.step(50)
    assert all(np.array_equal(x, y) for x, y in zip(sim.get_state()[:3], ref.get_state()[:3]))
    assert sim.wall_heat_flux() == ref.wall_heat_flux()
    hot = lbm_mod.Simulation(cylinder_case(nx=96, ny=48, r=6, cx=30, precision=FP64, check_every=1, dTr_wall=1.0))
    with pytest.raises(lbm_mod.LBMError) as err:
        hot.step(5)
    assert err.value.code == lbm_mod.LBM_EUNSTABLE


@pytest.mark.parametrize("pname", ["f64", "f16", "tangent"])
def test_checkpoint_resume_bitwise(lbm_mod, pname):
    """A checkpoint taken mid-run and loaded into another handle (which had stepped elsewhere) resumes
    the uninterrupted run bit for bit: populations, outlet history, temperature, step counter, the Nu
    time average and, in the tangent precision, its derivatives; a checkpoint of other runs is refused."""
    from paper_1912_02018_amd.config import F64_TANGENT, FP16S
    rl, _ = coex()
    prec = {"f64": FP64, "f16": FP16S, "tangent": F64_TANGENT}[pname]
    a_cfg = cylinder_case(nx=96, ny=48, r=6, cx=30, precision=prec, diag_every=3)
    b_cfg = cylinder_case(nx=80, ny=40, r=5, cx=25, precision=prec, diag_every=4, dTr_wall=0.15)
    if prec == FP16S:
        a_cfg, b_cfg = a_cfg.replace(rho_ref_shift=rl), b_cfg.replace(rho_ref_shift=rl)
    cfgs = [a_cfg, b_cfg] if prec != F64_TANGENT else [a_cfg]
    ref = lbm_mod.Simulation(cfgs)
    ref.step(240)
    first = lbm_mod.Simulation(cfgs)
    first.step(110)
    blob = first.save()
    first.step(9)
    other = lbm_mod.Simulation(cfgs)
    other.step(17)
    other.load(blob)
    assert other.step_count == 110
    other.step(130)
    for r in range(len(cfgs)):
        assert all(np.array_equal(x, y) for x, y in zip(other.get_state(r)[:3], ref.get_state(r)[:3])), (pname, r)
        assert other.wall_heat_flux(r) == ref.wall_heat_flux(r), (pname, r)
    if prec == F64_TANGENT:
        ga, gb = other.nu_tangent(), ref.nu_tangent()
        assert all(np.array_equal(np.asarray(x), np.asarray(y)) for x, y in zip(ga, gb))
    wrong = lbm_mod.Simulation([a_cfg.replace(nx=100)] + cfgs[1:])
    with pytest.raises(lbm_mod.LBMError):
        wrong.load(blob)


def test_stream_groups_graph_replay_bitwise(lbm_mod):
    """Stream groups captured into one graph per window (fork, the groups' launches as parallel
    branches, join) and replayed many times, with direct launches, reads and synchronisation between
    the calls: every read equals the same runs stepped on one stream without graphs."""
    cfgs = [cylinder_case(nx=96, ny=48, r=6, cx=30, precision=FP32, warmup_steps=12, diag_every=5),
            cylinder_case(nx=130, ny=70, r=8, cx=40, precision=FP32, dTr_wall=0.2, diag_every=5),
            cylinder_case(nx=64, ny=40, r=5, cx=20, precision=FP32, diag_every=10),
            cylinder_case(nx=160, ny=64, r=6, cx=40, precision=FP32, diag_every=5)]
    ref = lbm_mod.Simulation(cfgs)
    ref.set_graphs(False)
    sim = lbm_mod.Simulation(cfgs)
    sim.set_stream_groups(3)
    for n in (7, 40, 13, 60, 20, 3, 57):
        ref.step(n)
        sim.step(n)
        for r in range(len(cfgs)):
            assert all(np.array_equal(x, y) for x, y in zip(sim.get_state(r)[:3], ref.get_state(r)[:3])), (n, r)
            assert sim.wall_heat_flux(r) == ref.wall_heat_flux(r), (n, r)
    sim.close()
    ref.close()


def test_stream_groups_bitwise(lbm_mod):
    """Runs stepped as stream groups (contiguous ranges of runs on streams of their own) end in the
    same states, fields and heat fluxes as the same handle on one stream, through warm-ups that end at
    different steps, heat-flux accumulation and NaN checks; out-of-range group counts are rejected."""
    cfgs = [cylinder_case(nx=96, ny=48, r=6, cx=30, precision=FP32, warmup_steps=30),
            cylinder_case(nx=130, ny=70, r=8, cx=40, precision=FP32, dTr_wall=0.2, upwind_kind=1),
            cylinder_case(nx=64, ny=40, r=5, cx=20, precision=FP32, warmup_steps=55, check_every=25),
            cylinder_case(nx=160, ny=64, r=6, cx=40, precision=FP32, diag_every=7),
            cylinder_case(nx=80, ny=48, r=6, cx=25, precision=FP32)]
    ref = lbm_mod.Simulation(cfgs)
    ref.step(61)
    ref.step(89)
    for groups in (2, 3, 5):
        sim = lbm_mod.Simulation(cfgs)
        sim.set_stream_groups(groups)
        parts = sim.stream_groups()
        assert len(parts) == groups and parts[0][0] == 0 and parts[-1][1] == len(cfgs)
        assert all(a < b for a, b in parts) and all(parts[i][1] == parts[i + 1][0] for i in range(groups - 1))
        sim.step(61)
        sim.step(89)
        for r in range(len(cfgs)):
            assert all(np.array_equal(x, y) for x, y in zip(sim.get_state(r)[:3], ref.get_state(r)[:3])), (groups, r)
            assert sim.wall_heat_flux(r) == ref.wall_heat_flux(r), (groups, r)
        for bad in (0, 6, 9):
            with pytest.raises(lbm_mod.LBMError):
                sim.set_stream_groups(bad)
        sim.set_stream_groups(1)
        assert sim.stream_groups() == [(0, len(cfgs))]
        sim.close()


def test_batched_runs_equal_single_runs_bitwise(lbm_mod):
    """Runs stepped together in one handle (one launch per kernel over all their tiles) end in
    bit-identical states to the same runs stepped alone: tiles never mix runs and a run's arithmetic
    does not depend on which other runs share the launch.  A batch that holds a run with a heated
    wall and phase-dependent transport switches its launches to the kernels that carry those
    features: that run is bit-identical to itself alone, and the other runs (whose values are the
    same arithmetic, but compiled into a different kernel, so FMA contraction may differ) agree with
    their single runs to FP32 rounding."""
    from paper_1912_02018_amd.config import BC_WALL_OUTLET
    rl, rv = coex()
    a = cylinder_case(nx=96, ny=48, r=6, cx=30, precision=FP32)
    b = cylinder_case(nx=130, ny=70, r=8, cx=40, precision=FP32, dTr_wall=0.2, upwind_kind=1)
    c = LBMConfig(nx=100, ny=5, bc_x=BC_WALL_OUTLET, rk_stages=4, nu=0.05, nu_vapor=0.15, alpha_T=0.01,
                  alpha_vapor=0.1, rho_l=rl, rho_v=rv, rho_wall=rv, dTr_wall=0.09, precision=FP32)
    singles = {}
    for k, cfg in enumerate((a, b, c)):
        one = lbm_mod.Simulation(cfg)
        one.step(150)
        singles[k] = (one.fields(), one.get_state()[0], one.wall_heat_flux())
    for batch in ((0, 1), (0, 1, 2)):
        sim = lbm_mod.Simulation([(a, b, c)[k] for k in batch])
        sim.step(150)
        for r, k in enumerate(batch):
            f, fs, q = sim.fields(r), sim.get_state(r)[0], sim.wall_heat_flux(r)
            f1, fs1, q1 = singles[k]
            same_kernels = batch == (0, 1) or k == 2
            for name in ("rho", "ux", "uy", "T"):
                if same_kernels:
                    assert np.array_equal(f[name], f1[name]), (batch, k, name)
                else:
                    # FP32 rounding differences grown over 150 steps (u: relative to u_in)
                    tol = 1e-4 * 0.02 if name in ("ux", "uy") else 1e-5 * np.abs(f1[name]).max()
                    assert np.abs(f[name] - f1[name]).max() <= tol, (batch, k, name)
            if same_kernels:
                assert np.array_equal(fs, fs1), (batch, k)
                assert q == q1, (batch, k)



@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_hbm_resident_grid_launch_agrees_with_tiles(lbm_mod, storage):
    """The 8192x4096 channel (R 256) in the launch the bench times there (the stream-and-collide tile
    or strip it picks, the temperature strips with chunks sized to the resident workgroups: 35 strips)
    gives the plain tile variants' state bit for bit after a few coupled steps; the tiles are the ones
    pinned to the oracle on the smaller grids."""
    from paper_1912_02018_amd.config import FP16S
    prec = FP32 if storage == "f32" else FP16S
    cfg = cylinder_config(8192, 4096, 256, 2048, re=300.0, u_in=0.02, dTr_wall=0.1, precision=prec, warmup=0)
    if prec == FP16S:
        cfg = cfg.replace(rho_ref_shift=lbm_mod.saturation(cfg)["rho_l"])
    states = []
    for vl, vt in (((6 if storage == "f32" else 10), 6), (3, 0)):
        sim = lbm_mod.Simulation(cfg)
        sim.set_variant(0, vl)
        sim.set_variant(1, vt)
        sim.step(3)
        states.append(sim.get_state()[:3])
        print(f"[full-size] {storage} variants ({vl}, {vt}) stepped", flush=True)
        sim.close()
        del sim
    assert all(np.array_equal(x, y) for x, y in zip(*states))
