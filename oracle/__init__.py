"""FP64 CPU oracle of the central-moment pseudopotential LBM step (test infrastructure only).

Only the test-suite, the package smoke check and the CPU-baseline leg of the benchmark may
import this package.  It is a ctypes binding to ``lbm_oracle.c`` (plain C, FP64, OpenMP over
nodes) and shares no code with the HIP implementation.

Citations name sections and equations of Saito et al., arXiv:1912.02018.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

PARAM_FIELDS = [
    ("nx", C.c_int32), ("ny", C.c_int32), ("bc_x", C.c_int32), ("rk_stages", C.c_int32),
    ("warmup_steps", C.c_int32), ("cyl_x", C.c_int32), ("cyl_y", C.c_int32), ("cyl_r", C.c_int32),
    ("upwind_kind", C.c_int32), ("diag_every", C.c_int32),
    ("nu", C.c_double), ("eos_a", C.c_double), ("eos_b", C.c_double), ("eos_R", C.c_double),
    ("acentric", C.c_double), ("Tr_sat", C.c_double), ("dTr_wall", C.c_double),
    ("G", C.c_double), ("sigma", C.c_double), ("gx", C.c_double), ("gy", C.c_double),
    ("rho_gref", C.c_double), ("rho_l", C.c_double), ("rho_v", C.c_double),
    ("rho_wall", C.c_double), ("u_in", C.c_double), ("alpha_T", C.c_double), ("cv", C.c_double),
    ("nu_vapor", C.c_double), ("alpha_vapor", C.c_double), ("outlet_kind", C.c_int32),
]


class OrcParams(C.Structure):
    _fields_ = PARAM_FIELDS


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (no FMA contraction, OpenMP over nodes)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fopenmp", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        d, i, p = C.c_double, C.c_int, C.c_void_p
        P = C.POINTER(OrcParams)
        dp = C.POINTER(C.c_double)
        L.orc_create.restype = p
        L.orc_create.argtypes = [P]
        L.orc_destroy.argtypes = [p]
        L.orc_set_fields.argtypes = [p, dp, dp, dp, dp]
        L.orc_set_state.argtypes = [p, dp, dp, dp, C.c_long]
        L.orc_get_state.argtypes = [p, dp, dp, dp, C.POINTER(C.c_long)]
        L.orc_step.argtypes = [p, i]
        L.orc_step.restype = i
        L.orc_fields.argtypes = [p, dp, dp, dp, dp, C.POINTER(C.c_uint8)]
        L.orc_populations.argtypes = [p, dp]
        L.orc_forces.argtypes = [p, dp, dp, dp]
        L.orc_total_mass.argtypes = [p]
        L.orc_total_mass.restype = d
        L.orc_wall_heat_flux.argtypes = [p, dp, dp, dp]
        L.orc_derived.argtypes = [p, dp]
        L.orc_probes.argtypes = [p, dp, dp]
        L.orc_probes.restype = i
        L.orc_step_count.argtypes = [p]
        L.orc_step_count.restype = C.c_long
        L.orc_thermal_rhs.argtypes = [p, dp, dp]
        L.orc_thermal_advance.argtypes = [p, dp, dp]
        L.orc_is_solid.argtypes = [p, i, i]
        L.orc_is_solid.restype = i
        L.orc_link_q.argtypes = [p, i, i, i]
        L.orc_link_q.restype = d
        for name in ("orc_Tc", "orc_pc"):
            getattr(L, name).argtypes = [P]
            getattr(L, name).restype = d
        for name in ("orc_phi", "orc_dphi_dT"):
            getattr(L, name).argtypes = [P, d]
            getattr(L, name).restype = d
        for name in ("orc_eos_p", "orc_eos_dpdT", "orc_eos_dpdrho", "orc_psi"):
            getattr(L, name).argtypes = [P, d, d]
            getattr(L, name).restype = d
        L.orc_maxwell.argtypes = [P, d, dp, dp, dp]
        L.orc_maxwell.restype = i
        L.orc_hfg.argtypes = [P, d]
        L.orc_hfg.restype = d
        L.orc_feq.argtypes = [d, d, d, dp]
        L.orc_force_pop.argtypes = [d, d, d, d, dp]
        L.orc_T_matrix.argtypes = [d, d, dp]
        L.orc_lu_solve9.argtypes = [dp, dp, dp]
        L.orc_lu_solve9.restype = i
        L.orc_collide_node.argtypes = [d, d, dp, d, d, d, d, d, d, dp]
        L.orc_zou_he.argtypes = [d, dp]
        L.orc_convective.argtypes = [d, d, d]
        L.orc_convective.restype = d
        L.orc_iso_grad_periodic.argtypes = [i, i, dp, dp, dp]
        L.orc_iso_lap_periodic.argtypes = [i, i, dp, dp]
        L.orc_stencil_weight.argtypes = [i]
        L.orc_stencil_weight.restype = d
        L.orc_threads.argtypes = []
        L.orc_threads.restype = i
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def params(cfg) -> OrcParams:
    """Copy the attributes of a run configuration into the oracle's parameter struct."""
    p = OrcParams()
    for name, _ in PARAM_FIELDS:
        setattr(p, name, getattr(cfg, name))
    return p


# ---- building blocks (each follows one equation of the paper) --------------------------------
def Tc(cfg) -> float:
    """Critical temperature from the PR relations (Sec. II C)."""
    return lib().orc_Tc(C.byref(params(cfg)))


def pc(cfg) -> float:
    return lib().orc_pc(C.byref(params(cfg)))


def eos_p(cfg, rho, T) -> float:
    """Peng-Robinson pressure (eq. eos)."""
    return lib().orc_eos_p(C.byref(params(cfg)), float(rho), float(T))


def eos_dpdT(cfg, rho, T) -> float:
    return lib().orc_eos_dpdT(C.byref(params(cfg)), float(rho), float(T))


def eos_dpdrho(cfg, rho, T) -> float:
    return lib().orc_eos_dpdrho(C.byref(params(cfg)), float(rho), float(T))


def psi(cfg, rho, T) -> float:
    """EOS-consistent pseudopotential (eq. potential)."""
    return lib().orc_psi(C.byref(params(cfg)), float(rho), float(T))


def maxwell(cfg, T):
    """Maxwell equal-area coexistence (rho_v, rho_l, p_sat) at temperature T (Sec. III D)."""
    rv, rl, ps = C.c_double(), C.c_double(), C.c_double()
    rc = lib().orc_maxwell(C.byref(params(cfg)), float(T), C.byref(rv), C.byref(rl), C.byref(ps))
    if rc != 0:
        raise ValueError("no coexistence at this temperature")
    return rv.value, rl.value, ps.value


def hfg(cfg, T) -> float:
    return lib().orc_hfg(C.byref(params(cfg)), float(T))


def feq(rho, ux, uy) -> np.ndarray:
    """Full-Hermite equilibrium (eq. equi)."""
    out = np.zeros(9)
    lib().orc_feq(rho, ux, uy, _dptr(out))
    return out


def force_pop(Fx, Fy, ux, uy) -> np.ndarray:
    """Hermite forcing term F_i (eq. forcingTerm)."""
    out = np.zeros(9)
    lib().orc_force_pop(Fx, Fy, ux, uy, _dptr(out))
    return out


def T_matrix(ux, uy) -> np.ndarray:
    """Central-moment transform T(u) (eq. matrix)."""
    out = np.zeros(81)
    lib().orc_T_matrix(ux, uy, _dptr(out))
    return out.reshape(9, 9)


def lu_solve9(A, b) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float64).reshape(81).copy()
    b = np.ascontiguousarray(b, dtype=np.float64).copy()
    x = np.zeros(9)
    if lib().orc_lu_solve9(_dptr(A), _dptr(b), _dptr(x)) != 0:
        raise ValueError("singular")
    return x


def collide_node(omega, sigma, f, rho, ux, uy, Fx, Fy, Fm2_over_psi2) -> np.ndarray:
    """One-node collision (eq. posColl0 with eq. force2)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(9)
    lib().orc_collide_node(omega, sigma, _dptr(f), rho, ux, uy, Fx, Fy, Fm2_over_psi2, _dptr(out))
    return out


def zou_he(u_in, f) -> np.ndarray:
    f = np.array(f, dtype=np.float64)
    lib().orc_zou_he(u_in, _dptr(f))
    return f


def convective(U, f_old_last, f_new_prev) -> float:
    return lib().orc_convective(U, f_old_last, f_new_prev)


def iso_grad_periodic(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    ny, nx = a.shape
    gx, gy = np.zeros_like(a), np.zeros_like(a)
    lib().orc_iso_grad_periodic(nx, ny, _dptr(a), _dptr(gx), _dptr(gy))
    return gx, gy


def iso_lap_periodic(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    ny, nx = a.shape
    out = np.zeros_like(a)
    lib().orc_iso_lap_periodic(nx, ny, _dptr(a), _dptr(out))
    return out


def threads() -> int:
    """Threads of the oracle's OpenMP loops over nodes."""
    return int(lib().orc_threads())


def stencil_weight(e2: int) -> float:
    return lib().orc_stencil_weight(e2)


class Sim:
    """One oracle simulation (post-collision populations, outlet history, temperature)."""

    def __init__(self, cfg):
        self.cfg = cfg
        self._p = params(cfg)
        self.h = lib().orc_create(C.byref(self._p))
        if not self.h:
            raise ValueError("oracle: invalid configuration")
        self.nx, self.ny = cfg.nx, cfg.ny

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            try:
                _lib.orc_destroy(h)
            except Exception:
                pass
            self.h = None

    def set_fields(self, rho, ux, uy, T=None):
        shp = (self.ny, self.nx)
        rho = np.ascontiguousarray(np.broadcast_to(rho, shp), dtype=np.float64)
        ux = np.ascontiguousarray(np.broadcast_to(ux, shp), dtype=np.float64)
        uy = np.ascontiguousarray(np.broadcast_to(uy, shp), dtype=np.float64)
        if T is None:
            T = np.full(shp, self.derived()["T_sat"])
        T = np.ascontiguousarray(np.broadcast_to(T, shp), dtype=np.float64)
        lib().orc_set_fields(self.h, _dptr(rho), _dptr(ux), _dptr(uy), _dptr(T))

    def set_state(self, fstar, hist, T, step):
        fstar = np.ascontiguousarray(fstar, dtype=np.float64).reshape(9, self.ny, self.nx)
        hist = np.ascontiguousarray(hist, dtype=np.float64).reshape(3, self.ny)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(self.ny, self.nx)
        lib().orc_set_state(self.h, _dptr(fstar), _dptr(hist), _dptr(T), int(step))

    def get_state(self):
        fstar = np.zeros((9, self.ny, self.nx))
        hist = np.zeros((3, self.ny))
        T = np.zeros((self.ny, self.nx))
        st = C.c_long()
        lib().orc_get_state(self.h, _dptr(fstar), _dptr(hist), _dptr(T), C.byref(st))
        return fstar, hist, T, st.value

    def step(self, n: int = 1) -> int:
        return lib().orc_step(self.h, int(n))

    @property
    def step_count(self) -> int:
        return lib().orc_step_count(self.h)

    def fields(self):
        shp = (self.ny, self.nx)
        rho, ux, uy, T = (np.zeros(shp) for _ in range(4))
        mask = np.zeros(shp, dtype=np.uint8)
        lib().orc_fields(self.h, _dptr(rho), _dptr(ux), _dptr(uy), _dptr(T),
                         mask.ctypes.data_as(C.POINTER(C.c_uint8)))
        return {"rho": rho, "ux": ux, "uy": uy, "T": T, "mask": mask}

    def populations(self):
        f = np.zeros((9, self.ny, self.nx))
        lib().orc_populations(self.h, _dptr(f))
        return f

    def forces(self):
        shp = (self.ny, self.nx)
        Fx, Fy, ps = np.zeros(shp), np.zeros(shp), np.zeros(shp)
        lib().orc_forces(self.h, _dptr(Fx), _dptr(Fy), _dptr(ps))
        return Fx, Fy, ps

    def total_mass(self) -> float:
        return lib().orc_total_mass(self.h)

    def wall_heat_flux(self):
        q, nu, nua = C.c_double(), C.c_double(), C.c_double()
        lib().orc_wall_heat_flux(self.h, C.byref(q), C.byref(nu), C.byref(nua))
        return q.value, nu.value, nua.value

    def derived(self):
        out = np.zeros(8)
        lib().orc_derived(self.h, _dptr(out))
        keys = ["Tc", "T_sat", "T_w", "rho_l", "rho_v", "rho_w", "rho_gref", "omega"]
        return dict(zip(keys, out.tolist()))

    def probes(self):
        n = lib().orc_probes(self.h, None, None)
        px, py = np.zeros(max(n, 1)), np.zeros(max(n, 1))
        lib().orc_probes(self.h, _dptr(px), _dptr(py))
        return px[:n], py[:n]

    def thermal_rhs(self, Y):
        Y = np.ascontiguousarray(Y, dtype=np.float64).reshape(self.ny, self.nx)
        L = np.zeros_like(Y)
        lib().orc_thermal_rhs(self.h, _dptr(Y), _dptr(L))
        return L

    def thermal_advance(self, Y):
        Y = np.ascontiguousarray(Y, dtype=np.float64).reshape(self.ny, self.nx)
        out = np.zeros_like(Y)
        lib().orc_thermal_advance(self.h, _dptr(Y), _dptr(out))
        return out

    def is_solid(self, x, y) -> bool:
        return bool(lib().orc_is_solid(self.h, int(x), int(y)))

    def link_q(self, x, y, i) -> float:
        return lib().orc_link_q(self.h, int(x), int(y), int(i))
