"""Thin ctypes binding of liblbm (include/lbm.h); argument marshalling only.

Every step of the method runs in the HIP kernels of liblbm.so.  PyTorch provides the device
workspace (a uint8 tensor) and the stream.  If the library is missing this module raises: there is
no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Sequence

import numpy as np

from .config import LBMConfig

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5

_CONFIG_FIELDS = [
    ("nx", C.c_int32), ("ny", C.c_int32), ("bc_x", C.c_int32), ("rk_stages", C.c_int32),
    ("warmup_steps", C.c_int32), ("cyl_x", C.c_int32), ("cyl_y", C.c_int32), ("cyl_r", C.c_int32),
    ("upwind_kind", C.c_int32), ("diag_every", C.c_int32),
    ("nu", C.c_double), ("eos_a", C.c_double), ("eos_b", C.c_double), ("eos_R", C.c_double),
    ("acentric", C.c_double), ("Tr_sat", C.c_double), ("dTr_wall", C.c_double),
    ("G", C.c_double), ("sigma", C.c_double), ("gx", C.c_double), ("gy", C.c_double),
    ("rho_gref", C.c_double), ("rho_l", C.c_double), ("rho_v", C.c_double),
    ("rho_wall", C.c_double), ("u_in", C.c_double), ("alpha_T", C.c_double), ("cv", C.c_double),
    ("precision", C.c_int32), ("check_every", C.c_int32), ("rho_ref_shift", C.c_double),
    ("nu_vapor", C.c_double), ("alpha_vapor", C.c_double), ("outlet_kind", C.c_int32), ("pad_", C.c_int32),
]

EXPORTED = [
    "lbm_workspace_bytes", "lbm_create", "lbm_step", "lbm_fields", "lbm_set_fields",
    "lbm_get_state", "lbm_set_state", "lbm_wall_heat_flux", "lbm_total_mass", "lbm_derived",
    "lbm_step_count", "lbm_last_error", "lbm_destroy", "lbm_time_kernel",
    "lbm_variant_count", "lbm_variant_shape", "lbm_set_variant", "lbm_get_variant", "lbm_autotune",
    "lbm_set_option", "lbm_nu_tangent", "lbm_reset_time_average", "lbm_saturation", "lbm_profile_steps",
    "lbm_get_option", "lbm_stream_group_runs", "lbm_checkpoint_bytes", "lbm_save", "lbm_load",
    "lbm_create_static", "lbm_adjoint_state_bytes", "lbm_adjoint_scratch_bytes", "lbm_adjoint_step",
    "lbm_nu_gradient_bytes", "lbm_nu_gradient",
]
STATIC_WORKSPACE_BYTES = 64 << 20
OPT_GRAPHS, OPT_STREAM_GROUPS, OPT_TUNE_STEPS = 0, 1, 2
KERNEL_STREAM_COLLIDE, KERNEL_THERMAL = 0, 1


class lbm_config(C.Structure):
    _fields_ = _CONFIG_FIELDS


class LBMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"liblbm error {code}: {msg}")
        self.code = code


_lib = None


def load_library():
    """Load liblbm.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "or python paper_1912_02018_amd/build.py")
    import torch  # noqa: F401  (loads the HIP runtime first)
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int, C.c_int64, C.POINTER(C.c_double)
    cfgp = C.POINTER(lbm_config)
    L.lbm_workspace_bytes.argtypes = [cfgp, i32]
    L.lbm_workspace_bytes.restype = C.c_size_t
    L.lbm_create.argtypes = [cfgp, i32, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.lbm_create_static.argtypes = [cfgp, i32, vp, C.POINTER(vp)]
    L.lbm_adjoint_state_bytes.argtypes = [vp, i32]
    L.lbm_adjoint_state_bytes.restype = C.c_size_t
    L.lbm_adjoint_scratch_bytes.argtypes = [vp, i32]
    L.lbm_adjoint_scratch_bytes.restype = C.c_size_t
    L.lbm_adjoint_step.argtypes = [vp, i32, C.c_double, vp, vp, vp, C.c_size_t, dp]
    L.lbm_nu_gradient_bytes.argtypes = [vp, i32, i32]
    L.lbm_nu_gradient_bytes.restype = C.c_size_t
    L.lbm_nu_gradient.argtypes = [vp, i32, i32, i32, vp, C.c_size_t, dp, dp]
    L.lbm_step.argtypes = [vp, i32]
    L.lbm_fields.argtypes = [vp, i32, dp, dp, dp, dp, C.POINTER(C.c_uint8)]
    L.lbm_set_fields.argtypes = [vp, i32, dp, dp, dp, dp]
    L.lbm_get_state.argtypes = [vp, i32, dp, dp, dp]
    L.lbm_set_state.argtypes = [vp, i32, dp, dp, dp, i64]
    L.lbm_wall_heat_flux.argtypes = [vp, i32, dp, dp, dp]
    L.lbm_total_mass.argtypes = [vp, i32, dp]
    L.lbm_derived.argtypes = [vp, i32, dp]
    L.lbm_nu_tangent.argtypes = [vp, i32, dp, dp]
    L.lbm_saturation.argtypes = [cfgp, dp]
    L.lbm_reset_time_average.argtypes = [vp, i32]
    L.lbm_time_kernel.argtypes = [vp, i32, i32]
    ip = C.POINTER(C.c_int)
    L.lbm_variant_count.argtypes = [i32, i32]
    L.lbm_variant_shape.argtypes = [i32, i32, i32, ip, ip, ip, ip]
    L.lbm_set_variant.argtypes = [vp, i32, i32]
    L.lbm_get_variant.argtypes = [vp, i32]
    L.lbm_autotune.argtypes = [vp, i32, ip]
    L.lbm_set_option.argtypes = [vp, i32, i32]
    L.lbm_get_option.argtypes = [vp, i32]
    L.lbm_checkpoint_bytes.argtypes = [vp]
    L.lbm_checkpoint_bytes.restype = C.c_size_t
    L.lbm_save.argtypes = [vp, vp, C.c_size_t]
    L.lbm_load.argtypes = [vp, vp, C.c_size_t]
    L.lbm_stream_group_runs.argtypes = [vp, i32, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.lbm_profile_steps.argtypes = [vp, i32, dp]
    L.lbm_step_count.argtypes = [vp]
    L.lbm_step_count.restype = i64
    L.lbm_last_error.argtypes = [vp]
    L.lbm_last_error.restype = C.c_char_p
    L.lbm_destroy.argtypes = [vp]
    L.lbm_destroy.restype = None
    _lib = L
    return L


def to_c_config(cfg: LBMConfig) -> lbm_config:
    c = lbm_config()
    for name, _ in _CONFIG_FIELDS:
        setattr(c, name, getattr(cfg, name))
    return c


def _dp(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def workspace_bytes(cfgs: Sequence[LBMConfig]) -> int:
    L = load_library()
    arr = (lbm_config * len(cfgs))(*[to_c_config(c) for c in cfgs])
    n = L.lbm_workspace_bytes(arr, len(cfgs))
    if n == 0:
        raise LBMError(LBM_EINVAL, L.lbm_last_error(None).decode())
    return n


def saturation(cfg: LBMConfig) -> dict:
    """Saturation state of the configuration's Peng-Robinson fluid at Tr_sat (host computation)."""
    L = load_library()
    out = np.zeros(6)
    c = to_c_config(cfg)
    if L.lbm_saturation(C.byref(c), _dp(out)) != LBM_OK:
        raise LBMError(LBM_EINVAL, L.lbm_last_error(None).decode())
    return dict(zip(["Tc", "T_sat", "p_sat", "rho_l", "rho_v", "h_fg"], out.tolist()))


class Simulation:
    """One handle stepping one or more runs on the current CUDA (HIP) device and stream."""

    def __init__(self, cfgs, device: str = "cuda", stream=None, static_workspace: bool = False):
        """static_workspace: create the handle on the library's static device array
        (lbm_create_static; no device allocation, the previous static handle of the device stops
        working) instead of a torch workspace."""
        import torch
        if isinstance(cfgs, LBMConfig):
            cfgs = [cfgs]
        self.cfgs = list(cfgs)
        L = load_library()
        self._L = L
        n = len(self.cfgs)
        arr = (lbm_config * n)(*[to_c_config(c) for c in self.cfgs])
        dev = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = C.c_void_p()
        if static_workspace:
            self.workspace = None
            rc = L.lbm_create_static(arr, n, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        else:
            nbytes = L.lbm_workspace_bytes(arr, n)
            if nbytes == 0:
                raise LBMError(LBM_EINVAL, L.lbm_last_error(None).decode())
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            rc = L.lbm_create(arr, n, C.c_void_p(self.workspace.data_ptr()), nbytes,
                              C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != LBM_OK:
            raise LBMError(rc, L.lbm_last_error(None).decode())
        self.h = h

    def _check(self, rc: int):
        if rc != LBM_OK:
            raise LBMError(rc, self._L.lbm_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self._L.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def step_count(self) -> int:
        return int(self._L.lbm_step_count(self.h))

    def step(self, n: int = 1):
        self._check(self._L.lbm_step(self.h, int(n)))

    def _shape(self, run):
        c = self.cfgs[run]
        return (c.ny, c.nx)

    def time_kernel(self, kernel: int, n: int):
        """Enqueue n launches of one kernel of the step without advancing the state."""
        self._check(self._L.lbm_time_kernel(self.h, int(kernel), int(n)))

    def profile_steps(self, n: int):
        """Advance n steps with each k_lbm / k_thermal dispatch timed by its own start / stop
        events; returns their mean durations in ms (k_lbm, k_thermal) and the diagnostic
        reductions' time per step (ms, averaged over the n steps)."""
        out = (C.c_double * 3)()
        self._check(self._L.lbm_profile_steps(self.h, int(n), out))
        return out[0], out[1], out[2]

    def variants(self, kernel: int):
        """(tx, ty, threads, min_waves) of every launch variant of a kernel (0 k_lbm, 1 k_thermal);
        min_waves > 0: compiled with a register budget for that many waves per SIMD."""
        prec = self.cfgs[0].precision
        out = []
        for v in range(self._L.lbm_variant_count(prec, kernel)):
            a, b, c, d = C.c_int(), C.c_int(), C.c_int(), C.c_int()
            self._L.lbm_variant_shape(prec, kernel, v, C.byref(a), C.byref(b), C.byref(c), C.byref(d))
            out.append((a.value, b.value, c.value, d.value))
        return out

    def set_variant(self, kernel: int, variant: int):
        self._check(self._L.lbm_set_variant(self.h, int(kernel), int(variant)))

    def get_variant(self, kernel: int) -> int:
        return int(self._L.lbm_get_variant(self.h, int(kernel)))

    def autotune(self, launches: int = 20, cached: bool = False):
        """Time every launch variant of both kernels on the current state; keep the fastest.
        cached: reuse this process's earlier choice for the same workload shape, if any."""
        best = (C.c_int * 2)()
        self._check(self._L.lbm_autotune(self.h, -1 if cached else int(launches), best))
        return best[0], best[1]

    def set_graphs(self, enabled: bool):
        self._check(self._L.lbm_set_option(self.h, OPT_GRAPHS, 1 if enabled else 0))

    def set_tune_steps(self, enabled: bool):
        """autotune() times whole steps (advancing the state) instead of pseudo-steps."""
        self._check(self._L.lbm_set_option(self.h, OPT_TUNE_STEPS, 1 if enabled else 0))

    def save(self) -> bytes:
        """Checkpoint of every run (raw device state, accumulators and step counter)."""
        n = self._L.lbm_checkpoint_bytes(self.h)
        buf = C.create_string_buffer(n)
        self._check(self._L.lbm_save(self.h, buf, n))
        return buf.raw

    def load(self, blob: bytes):
        """Restore a checkpoint written by save() of a handle with the same runs."""
        buf = C.create_string_buffer(bytes(blob), len(blob))
        self._check(self._L.lbm_load(self.h, buf, len(blob)))

    def set_stream_groups(self, groups: int):
        """Step the runs as `groups` contiguous ranges on streams of their own (1: one stream)."""
        self._check(self._L.lbm_set_option(self.h, OPT_STREAM_GROUPS, int(groups)))

    def stream_groups(self):
        """[(run0, run1), ...] of the current stream groups."""
        out = []
        for g in range(self._L.lbm_get_option(self.h, OPT_STREAM_GROUPS)):
            a, b = C.c_int(), C.c_int()
            self._check(self._L.lbm_stream_group_runs(self.h, g, C.byref(a), C.byref(b)))
            out.append((a.value, b.value))
        return out

    def set_fields(self, rho, ux, uy, T=None, run: int = 0):
        shp = self._shape(run)
        f = lambda a: None if a is None else np.ascontiguousarray(np.broadcast_to(a, shp), dtype=np.float64)
        rho, ux, uy, T = f(rho), f(ux), f(uy), f(T)
        self._check(self._L.lbm_set_fields(self.h, run, _dp(rho), _dp(ux), _dp(uy), _dp(T)))

    def fields(self, run: int = 0):
        shp = self._shape(run)
        rho, ux, uy, T = (np.zeros(shp) for _ in range(4))
        mask = np.zeros(shp, dtype=np.uint8)
        self._check(self._L.lbm_fields(self.h, run, _dp(rho), _dp(ux), _dp(uy), _dp(T),
                                       mask.ctypes.data_as(C.POINTER(C.c_uint8))))
        return {"rho": rho, "ux": ux, "uy": uy, "T": T, "mask": mask}

    def get_state(self, run: int = 0):
        ny, nx = self._shape(run)
        fstar, hist, T = np.zeros((9, ny, nx)), np.zeros((3, ny)), np.zeros((ny, nx))
        self._check(self._L.lbm_get_state(self.h, run, _dp(fstar), _dp(hist), _dp(T)))
        return fstar, hist, T, self.step_count

    def set_state(self, fstar, hist, T, step: int, run: int = 0):
        ny, nx = self._shape(run)
        fstar = np.ascontiguousarray(fstar, dtype=np.float64).reshape(9, ny, nx)
        hist = np.ascontiguousarray(hist, dtype=np.float64).reshape(3, ny)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(ny, nx)
        self._check(self._L.lbm_set_state(self.h, run, _dp(fstar), _dp(hist), _dp(T), int(step)))

    def wall_heat_flux(self, run: int = 0):
        q, nu, nua = C.c_double(), C.c_double(), C.c_double()
        self._check(self._L.lbm_wall_heat_flux(self.h, run, C.byref(q), C.byref(nu), C.byref(nua)))
        return q.value, nu.value, nua.value

    def total_mass(self, run: int = 0) -> float:
        m = C.c_double()
        self._check(self._L.lbm_total_mass(self.h, run, C.byref(m)))
        return m.value

    def derived(self, run: int = 0):
        out = np.zeros(8)
        self._check(self._L.lbm_derived(self.h, run, _dp(out)))
        keys = ["Tc", "T_sat", "T_w", "rho_l", "rho_v", "rho_w", "rho_gref", "omega"]
        return dict(zip(keys, out.tolist()))

    def nu_tangent(self, run: int = 0):
        """(dNu/dtheta, d<Nu>_t/dtheta) of a tangent-precision run, theta = (dTr_wall, u_in,
        acentric, tau), each a length-4 array."""
        d, da = np.zeros(4), np.zeros(4)
        self._check(self._L.lbm_nu_tangent(self.h, run, _dp(d), _dp(da)))
        return d, da

    def adjoint_buffers(self, run: int = 0):
        """(two adjoint-state buffers, scratch) as torch uint8 device tensors for adjoint_step."""
        import torch
        nb = self._L.lbm_adjoint_state_bytes(self.h, run)
        ns = self._L.lbm_adjoint_scratch_bytes(self.h, run)
        if nb == 0 or ns == 0:
            raise LBMError(LBM_EINVAL, self._L.lbm_last_error(self.h).decode())
        dev = torch.device("cuda", torch.cuda.current_device())
        return (torch.zeros(nb, dtype=torch.uint8, device=dev), torch.zeros(nb, dtype=torch.uint8, device=dev),
                torch.empty(ns, dtype=torch.uint8, device=dev))

    def adjoint_step(self, adj_in, adj_out, scratch, nu_weight: float = 0.0, run: int = 0):
        """Adjoint of one step from the current state (lbm_adjoint_step); returns the gradient
        accumulated in adj_out, dJ/dtheta (4)."""
        g = np.zeros(4)
        self._check(self._L.lbm_adjoint_step(self.h, run, float(nu_weight), C.c_void_p(adj_in.data_ptr()),
                                             C.c_void_p(adj_out.data_ptr()), C.c_void_p(scratch.data_ptr()),
                                             scratch.numel(), _dp(g)))
        return g

    def nu_gradient(self, steps: int, average_from: int, checkpoint_every: int = 200):
        """(J, dJ/dtheta) by the reverse sweep with checkpoints every checkpoint_every steps
        (lbm_nu_gradient); advances the handle by `steps` steps."""
        import torch
        nb = self._L.lbm_nu_gradient_bytes(self.h, int(steps), int(checkpoint_every))
        if nb == 0:
            raise LBMError(LBM_EINVAL, self._L.lbm_last_error(self.h).decode())
        ws = torch.empty(nb, dtype=torch.uint8, device=torch.device("cuda", torch.cuda.current_device()))
        J, g = C.c_double(), np.zeros(4)
        self._check(self._L.lbm_nu_gradient(self.h, int(steps), int(average_from), int(checkpoint_every),
                                            C.c_void_p(ws.data_ptr()), nb, C.byref(J), _dp(g)))
        del ws
        return J.value, g

    def reset_time_average(self, run: int = 0):
        self._check(self._L.lbm_reset_time_average(self.h, run))
