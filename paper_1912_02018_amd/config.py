"""Run configuration of one boiling / two-phase simulation, and the workload presets.

The field list mirrors ``lbm_config`` in ``include/lbm.h``.  The presets describe the synthetic
workloads (grid, cylinder, flow and thermal parameters); they contain no step arithmetic: the
relaxation rate, the critical temperature, the coexistence densities and every other derived
quantity are computed by the library that receives the configuration.

Workload shapes follow the boiling set-up of Saito et al. (arXiv:1912.02018, Sec. IV A): saturated
liquid at T_r = 0.86 flowing past a heated cylinder, Peng-Robinson EOS with a = 3/49, b = 2/21,
R = 1, acentric factor 0.344 (Sec. II C), sigma = 0.38 (Sec. III D), c_v = 11, Pr = 1.5.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

FP64, FP32, FP16S, BF16S, F64_TANGENT = 0, 1, 2, 3, 4
PRECISION_NAMES = {FP64: "f64", FP32: "f32", FP16S: "f16-store", BF16S: "bf16-store",
                   F64_TANGENT: "f64+tangents"}
# parameter directions of the tangent precision (order of lbm_nu_tangent)
TANGENT_PARAMS = ("dTr_wall", "u_in", "acentric", "tau")
BC_PERIODIC, BC_INLET_OUTLET, BC_WALL_OUTLET = 0, 1, 2
OUTLET_U_IN, OUTLET_LOCAL = 0, 1


@dataclass
class LBMConfig:
    nx: int = 128
    ny: int = 64
    bc_x: int = BC_INLET_OUTLET
    rk_stages: int = 4           # 0 isothermal, 2 Heun, 4 classical RK4
    warmup_steps: int = 0
    cyl_x: int = 0
    cyl_y: int = 0
    cyl_r: int = 0               # <= 0: no cylinder
    upwind_kind: int = 0         # 0 third-order upwind, 1 Kawamura-Kuwahara
    diag_every: int = 0          # accumulate Nu every diag_every steps
    nu: float = 0.1              # kinematic viscosity (lattice units)
    eos_a: float = 3.0 / 49.0
    eos_b: float = 2.0 / 21.0
    eos_R: float = 1.0
    acentric: float = 0.344
    Tr_sat: float = 0.86         # T_sat / T_c
    dTr_wall: float = 0.0        # (T_w - T_sat) / T_c
    G: float = -2.0
    sigma: float = 0.38
    gx: float = 0.0
    gy: float = 0.0
    rho_gref: float = -1.0       # F_g = (rho - rho_gref) g; < 0 selects rho_l
    rho_l: float = 0.0           # <= 0 (with rho_v <= 0): Maxwell construction
    rho_v: float = 0.0
    rho_wall: float = 0.0        # <= 0 selects rho_l
    u_in: float = 0.0
    alpha_T: float = 0.0
    cv: float = 11.0
    precision: int = FP64
    check_every: int = 0         # > 0: lbm_step reports non-finite state
    rho_ref_shift: float = 0.0   # reduced-precision storage holds f_i - w_i * rho_ref_shift; <= 0: rho_l
    nu_vapor: float = 0.0        # > 0: vapour viscosity (nu is then the liquid's), linear in density between
    alpha_vapor: float = 0.0     # > 0: vapour thermal diffusivity (alpha_T the liquid's), same interpolation
    outlet_kind: int = 0         # convective-outlet speed: 0 u_in, 1 local outflow velocity of the outlet node
    pad_: int = 0

    def replace(self, **kw) -> "LBMConfig":
        return dataclasses.replace(self, **kw)

    @property
    def nodes(self) -> int:
        return self.nx * self.ny


def viscosity_from_re(u_in: float, diameter: float, re: float) -> float:
    """Re = u_l D / nu_l (Sec. I, definition of the liquid Reynolds number)."""
    return u_in * diameter / re


def config1(precision: int = FP64) -> LBMConfig:
    """Flat liquid-vapour interface: 128x64 periodic, T_r = 0.86, nu = 0.1, isothermal."""
    return LBMConfig(nx=128, ny=64, bc_x=BC_PERIODIC, rk_stages=0, warmup_steps=0, nu=0.1,
                     Tr_sat=0.86, sigma=0.38, precision=precision)


def cylinder_config(nx: int, ny: int, radius: int, cx: int, re: float, u_in: float,
                    dTr_wall: float, precision: int = FP32, warmup: int = 3000,
                    rk_stages: int = 4, pr: float = 1.5, gx: float = -1e-5,
                    diag_every: int = 100) -> LBMConfig:
    nu = viscosity_from_re(u_in, 2.0 * radius, re)
    return LBMConfig(nx=nx, ny=ny, bc_x=BC_INLET_OUTLET, rk_stages=rk_stages, warmup_steps=warmup,
                     cyl_x=cx, cyl_y=ny // 2, cyl_r=radius, nu=nu, Tr_sat=0.86, dTr_wall=dTr_wall,
                     gx=gx, u_in=u_in, alpha_T=nu / pr, cv=11.0, precision=precision,
                     diag_every=diag_every)


def config2(precision: int = FP32) -> LBMConfig:
    """Forced-convection boiling: 1024x512 channel, R = 32 at x = 256, u_in = 0.02, Re = 300,
    superheat 0.1 T_c, gravity -1e-5 along x, RK4, 3000 warm-up steps, wall Nu logged every 20
    steps."""
    return cylinder_config(1024, 512, 32, 256, re=300.0, u_in=0.02, dTr_wall=0.1,
                           precision=precision, diag_every=20)


def config3(precision: int = FP16S) -> LBMConfig:
    """config2 at Re = 30000 with u_in = 0.05."""
    return cylinder_config(1024, 512, 32, 256, re=30000.0, u_in=0.05, dTr_wall=0.1,
                           precision=precision, diag_every=20)


def config5(precision: int = FP32) -> LBMConfig:
    """Sensitivity run: 512x256, R = 16 at x = 128, Re = 300, superheat 0.1 T_c, no warm-up."""
    return cylinder_config(512, 256, 16, 128, re=300.0, u_in=0.02, dTr_wall=0.1,
                           precision=precision, warmup=0)


def sweep_configs(n_runs: int = 64, seed: int = 2018, precision: int = FP32) -> list:
    """Boiling-curve sweep of uneven runs: nx in 64*{4..16}, ny = nx/2, radius uniform in
    8..min(32, ny/8), centre (nx/4, ny/2), superheat uniform in 0.02..0.30 T_c, Re log-uniform
    in 30..3000, u_in = 0.02.  Draws come from the seeded SplitMix64 stream of ``inputs``."""
    from .inputs import uniform01
    u = uniform01(seed, 4 * n_runs).reshape(n_runs, 4)
    out = []
    for k in range(n_runs):
        nx = 64 * (4 + min(12, int(u[k, 0] * 13)))
        ny = nx // 2
        rmax = min(32, ny // 8)
        radius = 8 + min(rmax - 8, int(u[k, 1] * (rmax - 8 + 1)))
        dtr = 0.02 + 0.28 * u[k, 2]
        re = math.exp(math.log(30.0) + (math.log(3000.0) - math.log(30.0)) * u[k, 3])
        out.append(cylinder_config(nx, ny, radius, nx // 4, re=re, u_in=0.02, dTr_wall=dtr,
                                   precision=precision))
    return out
