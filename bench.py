#!/usr/bin/env python3
"""Throughput of the coupled boiling step (flow + temperature) on one MI355X.

Workload: forced-convection boiling on a heated cylinder, 1024x512 channel, cylinder radius 32 at
x = 256, inlet velocity 0.02 at Re = 300, saturated liquid at T_r = 0.86, superheat 0.1 T_c,
gravity -1e-5 along x, RK4 temperature stages, FP32 (synthetic initial state: uniform saturated
liquid).  The configured 3000 warm-up steps (no forcing, no temperature update) run first and
untimed; the timed steps are full coupled steps.  One lattice update (LUP) = one node (fluid and
solid) advanced through one full step.

Prints one JSON line: MLUPS, per-step time, the roofline of the dominant kernel (HIP events over
isolated launches on the library's stream) and the FP64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP64_VECTOR_PEAK_TFLOPS = 78.6

# Algorithmic traffic / work per lattice update of each kernel of the step:
#   stream+collide: read 9 populations, write 9 populations, read T (psi)       -> 19 values
#   temperature:    read T^n, write T^{n+1}                                       ->  2 values
#   temperature useful flops: 4 stages x ~150 + ~130 stage-invariant             -> 730 flops
KERNEL_NAMES = {0: "k_lbm", 1: "k_thermal"}
THERMAL_FLOPS_PER_LUP = {4: 730.0, 2: 430.0}
PREC = {"f64": 0, "f32": 1, "f16s": 2, "bf16s": 3}
STORE_BYTES = {0: 8, 1: 4, 2: 2, 3: 2}
COMPUTE_BYTES = {0: 8, 1: 4, 2: 4, 3: 4}


def kernel_bytes_per_lup(kernel: int, prec: int) -> float:
    if kernel == 0:
        return 18 * STORE_BYTES[prec] + COMPUTE_BYTES[prec]
    return 2 * COMPUTE_BYTES[prec]


def source_digest() -> str:
    p = os.path.join(ROOT, "paper_1912_02018_amd", "csrc", "lbm_kernels.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def measured_traffic(variant: str, workload: str):
    """HBM-side bytes per launch of one launch variant (FETCH_SIZE and WRITE_SIZE of committed
    rocprofv3 counter runs, scaled by the same counters on a plain copy), if taken on this source."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p)).get(f"{variant}@{workload}")
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha") != source_digest():
        return None
    return rec.get("bytes_per_launch")


def cpu_model() -> str:
    """Model name of the host CPU (first entry of /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, budget_s: float):
    """FP64 oracle (OpenMP over nodes) on the same workload, timed on a bounded number of steps.
    cores: the OpenMP threads the oracle runs with (OMP_NUM_THREADS, else the cores of this
    process's affinity mask); the affinity mask's size is reported beside it."""
    import oracle
    from paper_1912_02018_amd.config import FP64
    c = cfg.replace(precision=FP64, warmup_steps=0)
    sim = oracle.Sim(c)
    t0 = time.perf_counter()
    sim.step(1)
    one = time.perf_counter() - t0
    n = max(1, min(200, int(budget_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    sim.step(n)
    dt = time.perf_counter() - t0
    affinity = len(os.sched_getaffinity(0))
    return {"value": round(c.nx * c.ny * n / dt / 1e6, 4), "unit": "MLUPS", "cores": oracle.threads(),
            "kind": "oracle", "cpu_model": cpu_model(), "affinity_cores": affinity,
            "sample": f"{n} coupled FP64 steps of the {c.nx}x{c.ny} workload after 1 untimed step "
                      f"({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--precision", default="f32", choices=sorted(PREC))
    ap.add_argument("--kernel-launches", type=int, default=200)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed windows of --steps steps each; the value is their median")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-physical-warmup", action="store_true",
                    help="start coupled steps at once (short profiler runs; same per-step work)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch variants")
    ap.add_argument("--stream-groups", type=int, default=3,
                    help="sweep: runs stepped as this many contiguous groups on streams of their own")
    ap.add_argument("--variants", default=None, metavar="L,T",
                    help="launch variant indices of k_lbm and k_thermal (instead of autotuning)")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "sweep", "big"],
                    help="c2: 1024x512 boiling channel (default); c3: the same at Re 30000; sweep: 64 uneven runs; "
                         "big: the Re 300 channel scaled by 8 (8192x4096, R 256), a state no cache holds, "
                         "coupled from its first step")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates HBM byte counters)")
    ap.add_argument("--no-extras", action="store_true",
                    help="c2: skip the batched-sweep, reduced-storage and HBM-resident sub-reports")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: a boiling run is not split across GPUs (the step would "
              "shard as x-slabs with halo exchange, the sweep by runs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.rand(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "launches": 5}))
        return
    from paper_1912_02018_amd import lbm
    from paper_1912_02018_amd.config import config2, config3, sweep_configs, cylinder_config

    prec = PREC[args.precision]
    torch.cuda.set_device(0)
    if args.workload == "sweep":
        line = run_sweep(args, lbm, sweep_configs(64, 2018, prec), prec)
    else:
        if args.workload == "big":
            cfg = cylinder_config(8192, 4096, 256, 2048, re=300.0, u_in=0.02, dTr_wall=0.1, precision=prec, warmup=0)
            if prec >= 2:
                cfg = cfg.replace(rho_ref_shift=lbm.saturation(cfg)["rho_l"])
        else:
            cfg = config2(prec) if args.workload == "c2" else config3(prec)
        re = 30000 if args.workload == "c3" else 300
        if args.skip_physical_warmup:
            cfg = cfg.replace(warmup_steps=0)
        workload = f"boiling-cylinder-{cfg.nx}x{cfg.ny}-R{cfg.cyl_r}-Re{re}-rk{cfg.rk_stages}-{args.precision}"
        line = run_single(args, lbm, cfg, prec, workload, re)
        if args.workload == "c2" and not args.no_extras:
            progress("batched_vs_single")
            line["batched_vs_single"] = sweep_summary(args, lbm)
            progress("reduced_storage")
            line["reduced_storage"] = reduced_storage_report(lbm)
            progress("hbm_resident")
            line["hbm_resident"] = hbm_resident_run(lbm)
            progress("sensitivity")
            line["sensitivity"] = sensitivity_run(lbm)
    print(json.dumps(line), flush=True)


def progress(what: str):
    """One line per phase on stderr (stdout carries only the JSON result line)."""
    print(f"[bench] {what} {time.strftime('%H:%M:%S')}", file=sys.stderr, flush=True)


def sweep_summary(args, lbm):
    """Aggregate MLUPS of the 64-run superheat sweep stepped by one handle against the same runs
    stepped one after another (shorter timing than --workload sweep)."""
    from paper_1912_02018_amd.config import sweep_configs
    sub = argparse.Namespace(**vars(args))
    sub.steps, sub.warmup, sub.kernel_launches, sub.variants, sub.repeats = 1000, 100, 20, None, 3
    rec = run_sweep(sub, lbm, sweep_configs(64, 2018, PREC["f32"]), PREC["f32"])
    return {"workload": rec["config"]["workload"], "nodes": rec["config"]["nodes"], "mlups": rec["value"],
            "sequential_mlups": rec["sequential_mlups"], "ratio": rec["batched_over_sequential"],
            "steps": sub.steps, "timing": rec["timing"], "variants": rec["config"]["variants"],
            "sequential_distinct_shapes_tuned": len(rec["sequential_variants"])}


def reduced_storage_report(lbm, steps=1000):
    """The Re 30000 channel (u_in 0.05) with FP64, FP32, FP16 and BF16 population storage: each
    precision runs its own untimed 3000-step warm-up, then `steps` timed coupled steps; the final
    fields and Nu are compared with the FP64 run (max-norm relative errors over fluid nodes; u
    relative to max(|u|, u_in))."""
    import numpy as np
    import torch
    from paper_1912_02018_amd.config import config3
    ref, out = None, {}
    rho_l = None
    cases = (("f64", "f64", None), ("f32", "f32", None), ("f16s_shift_1", "f16s", 1.0),
             ("f16s_shift_rho_l", "f16s", "rho_l"), ("bf16s_shift_rho_l", "bf16s", "rho_l"))
    # (the storage shift defaults to rho_l; the literal f_i - w_i of rho_ref = 1 is the comparison)
    for label, pname, shift in cases:
        cfg = config3(PREC[pname])
        if shift == "rho_l":
            cfg = cfg.replace(rho_ref_shift=rho_l)
        elif shift is not None:
            cfg = cfg.replace(rho_ref_shift=shift)
        sim = lbm.Simulation(cfg)
        if rho_l is None:
            rho_l = sim.derived()["rho_l"]
        sim.step(cfg.warmup_steps)
        # pseudo-step tuning leaves the state where it is: every precision is compared at the same
        # step (whole-step tuning would advance each by its own number of variants)
        sim.autotune(10)
        ms, _ = timed_steps(torch, sim, steps)
        assert sim.step_count == cfg.warmup_steps + steps
        f = sim.fields()
        _, nu, _ = sim.wall_heat_flux()
        rec = {"mlups": round(cfg.nx * cfg.ny / (ms / steps * 1e-3) / 1e6, 1)}
        if shift is not None:
            rec["rho_ref_shift"] = round(float(cfg.rho_ref_shift), 6)
        if ref is None:
            ref = (f, nu)
        else:
            g, nu0 = ref
            fl = g["mask"] == 0
            rel = lambda a, b: float(np.abs(a - b)[fl].max() / np.abs(b)[fl].max())
            du = np.hypot(f["ux"] - g["ux"], f["uy"] - g["uy"])[fl].max()
            umax = max(float(np.hypot(g["ux"], g["uy"])[fl].max()), cfg.u_in)
            rec["err_vs_f64"] = {"rho": rel(f["rho"], g["rho"]), "u": float(du / umax),
                                 "T": rel(f["T"], g["T"]), "nu": abs(nu / nu0 - 1.0)}
        out[label] = rec
        sim.close()
    return {"workload": "boiling-cylinder-1024x512-R32-Re30000-rk4", "steps_after_warmup": steps, **out}


def sensitivity_run(lbm, steps=4000, average_from=2000, checkpoint_every=200):
    """Time-averaged Nu of the 512x256 channel (R 16, Re 300, superheat 0.1 T_c, no warm-up) over
    steps 2000..3999 and its gradient with respect to (superheat, u_in, acentric factor, tau), by the
    reverse sweep (hand-written adjoint, checkpoints every 200 steps and recompute) and by one run of
    the forward-mode tangent precision (FP64 values + 4 derivatives per value)."""
    import numpy as np
    import torch
    from paper_1912_02018_amd import sensitivity
    from paper_1912_02018_amd.config import config5
    cfg = sensitivity.hold_coexistence(config5(PREC["f64"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, g = sensitivity.nu_average_and_gradient(cfg, steps, average_from)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sim = lbm.Simulation(cfg.replace(diag_every=1))
    ws_bytes = sim._L.lbm_nu_gradient_bytes(sim.h, steps, checkpoint_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Ja, ga = sim.nu_gradient(steps, average_from, checkpoint_every)
    torch.cuda.synchronize()
    dta = time.perf_counter() - t0
    sim.close()
    rel = float(np.abs(np.asarray(ga) - np.asarray(g)).max() / np.abs(np.asarray(g)).max())
    return {"workload": "boiling-cylinder-512x256-R16-Re300-rk4-f64", "steps": steps,
            "average_from": average_from, "J_mean_nu": Ja,
            "dJ_dtheta": dict(zip(sensitivity.TANGENT_PARAMS, [float(x) for x in ga])),
            "adjoint": {"method": f"reverse sweep, checkpoints every {checkpoint_every} steps, segments recomputed",
                        "wall_s": round(dta, 3), "device_workspace_bytes": int(ws_bytes)},
            "tangent": {"method": "forward mode, FP64 + 4 derivatives per value", "J_mean_nu": J,
                        "dJ_dtheta": dict(zip(sensitivity.TANGENT_PARAMS, [float(x) for x in g])),
                        "wall_s": round(dt, 3), "mlups_incl_setup": round(cfg.nx * cfg.ny * steps / dt / 1e6, 1)},
            "adjoint_vs_tangent_max_rel": rel}


def hbm_resident_run(lbm, steps=200):
    """The Re 300 channel scaled by 8 (8192x4096, cylinder R 256 at x 2048): a state of ~3 GB that
    no cache holds, with FP32 populations and with FP16 storage (shift w_i rho_l).  Coupled steps
    from the initial liquid state (no physical warm-up; the same per-step work)."""
    import torch
    copy_gbs = copy_bandwidth(torch)
    out = _hbm_resident(lbm, PREC["f32"], steps, copy_gbs=copy_gbs)
    out["f16_store"] = _hbm_resident(lbm, PREC["f16s"], steps, copy_gbs=copy_gbs)
    out["rk2"] = _hbm_resident(lbm, PREC["f32"], steps, rk=2, copy_gbs=copy_gbs)
    out["copy_gbs"] = round(copy_gbs, 1)
    return out


def copy_bandwidth(torch, mib=1024, reps=20):
    """Achievable HBM bandwidth on this device: a plain device-to-device copy of `mib` MiB (torch's
    copy kernel), bytes read + written per second over `reps` back-to-back copies."""
    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    gbs = 2 * n * 4 * reps / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def _hbm_resident(lbm, prec, steps, rk=4, copy_gbs=None):
    import torch
    from paper_1912_02018_amd.config import cylinder_config
    cfg = cylinder_config(8192, 4096, 256, 2048, re=300.0, u_in=0.02, dTr_wall=0.1, precision=prec,
                          warmup=0, rk_stages=rk)
    if prec >= 2:
        cfg = cfg.replace(rho_ref_shift=lbm.saturation(cfg)["rho_l"])
    sim = lbm.Simulation(cfg)
    sim.step(10)
    tune(sim, 5)
    sim.step(10)
    ms, _ = timed_steps(torch, sim, steps)
    nodes = cfg.nx * cfg.ny
    mlups = nodes / (ms / steps * 1e-3) / 1e6
    kt = dict(zip(KERNEL_NAMES.values(), timed_region_kernel_ms(sim, 20, ms / steps)[0].values()))
    pname = {v: k for k, v in PREC.items()}[prec]
    step_bytes = (18 * STORE_BYTES[prec] + 2 * COMPUTE_BYTES[prec]) * nodes  # populations + T, read and written
    rec = {"workload": f"boiling-cylinder-8192x4096-R256-Re300-rk{rk}-{pname}", "nodes": nodes, "mlups": round(mlups, 1),
           "ms_per_step": round(ms / steps, 4),
           "step_hbm_frac": round(step_bytes / (ms / steps * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "step_copy_frac": round(step_bytes / (ms / steps * 1e-3) / 1e9 / copy_gbs, 4) if copy_gbs else None,
           "kernel_ms": {k: round(v, 4) for k, v in kt.items()},
           "kernel_hbm_gbs": {KERNEL_NAMES[k]: round(kernel_bytes_per_lup(k, prec) * nodes / (kt[KERNEL_NAMES[k]] * 1e-3) / 1e9, 1)
                              for k in (0, 1)},
           "tiles": {"k_lbm": sim.variants(0)[sim.get_variant(0)], "k_thermal": sim.variants(1)[sim.get_variant(1)]}}
    sim.close()
    return rec


def tune(sim, launches, cached=False):
    """The library's autotuner timing whole steps (the state advances through them, as the untimed
    steps before a timed region do): pseudo-steps on an unchanged state see other cache contents than
    stepping, which alternates the double buffers.  Returns the chosen variants."""
    sim.set_tune_steps(True)
    best = sim.autotune(launches, cached=cached)
    sim.set_tune_steps(False)
    return best


def choose_variants(args, sim, launches):
    """Given variants (--variants), the defaults (--no-autotune) or the autotuner's choice."""
    if args.variants:
        for k, v in enumerate(int(x) for x in args.variants.split(",")):
            sim.set_variant(k, v)
    elif not args.no_autotune:
        tune(sim, launches)


def timed_steps(torch, sim, steps):
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(sim.stream)
    sim.step(steps)
    ev1.record(sim.stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1), time.perf_counter() - t0


def launch_period(cfgs) -> int:
    """Period of the library's launch pattern once the runs are past warm-up: the buffers alternate
    every step, and the Nu accumulation recurs every diag_every steps (lcm of 2 and those periods)."""
    L = 2
    for c in cfgs:
        if c.diag_every > 0:
            L = L * c.diag_every // math.gcd(L, c.diag_every)
    return L


def align(sim, period: int):
    """Untimed steps up to the next multiple of the launch period, so that a timed window starts where
    the library replays its captured period (graph launches, diagnostics included)."""
    r = sim.step_count % period
    if r:
        sim.step(period - r)


def timed_windows(torch, sim, steps, repeats, period):
    """`repeats` windows of exactly `steps` steps, each starting at a multiple of the launch period and
    bracketed by device synchronisations, after one untimed window; returns the median window's
    milliseconds and wall-clock seconds, and every window's milliseconds."""
    reps, walls = [], []
    align(sim, period)
    sim.step(steps)      # untimed: captures the graph of the period if the library replays one
    for _ in range(max(1, repeats)):
        align(sim, period)
        ms, wall = timed_steps(torch, sim, steps)
        reps.append(ms)
        walls.append(wall)
    order = sorted(range(len(reps)), key=lambda k: reps[k])
    mid = order[len(order) // 2]
    return reps[mid], walls[mid], reps


def isolated_kernel_ms(torch, sim, launches):
    """Average duration of back-to-back launches of each kernel on an unchanging state (HIP events
    on the library's stream): the inputs stay cache-hot, so these run faster than in the step."""
    kt = {}
    for k in (0, 1):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        sim.time_kernel(k, 10)
        e0.record(sim.stream)
        sim.time_kernel(k, launches)
        e1.record(sim.stream)
        torch.cuda.synchronize()
        kt[k] = e0.elapsed_time(e1) / launches  # ms per launch
    return kt


def timed_region_kernel_ms(sim, launches, ms_step):
    """Average duration of each kernel in the timed region: the timed step time (HIP events around the
    graph-replayed steps, whose kernels run back to back) divided between k_lbm, k_thermal and the
    diagnostic reductions in the proportion of their dispatch durations, measured by `launches`
    further steps right after the timed region with every dispatch timed by its own start / stop HIP
    events (the reductions by events around them, per step).  Directly launched steps leave gaps
    between the kernels, so their raw dispatch durations differ by a few percent from the back-to-back
    ones; both are returned."""
    disp = sim.profile_steps(launches)
    share = ms_step / (disp[0] + disp[1] + disp[2])
    return {0: disp[0] * share, 1: disp[1] * share}, {0: disp[0], 1: disp[1], "diag": disp[2]}


def kernel_roofline(torch, sim, cfg, prec, nodes, launches, workload, ms_step):
    """Timed-region duration of each kernel (timed_region_kernel_ms) and the roofline of the
    dominant one."""
    kt, disp = timed_region_kernel_ms(sim, launches, ms_step)
    dom = max(kt, key=kt.get)
    name = KERNEL_NAMES[dom]
    variant = variant_name(dom, sim.variants(dom)[sim.get_variant(dom)], cfg.rk_stages)
    if dom == 0:
        per_launch = kernel_bytes_per_lup(0, prec) * nodes
        achieved = per_launch / (kt[dom] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(variant, workload)}
    else:
        flops = THERMAL_FLOPS_PER_LUP[cfg.rk_stages] * nodes
        achieved = flops / (kt[dom] * 1e-3) / 1e12
        peak = FP64_VECTOR_PEAK_TFLOPS if prec == 0 else FP32_VECTOR_PEAK_TFLOPS
        roof = {"bound": "alu", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": measured_traffic(variant, workload)}
    roof["kernel"] = variant
    roof["kernel_ms"] = {KERNEL_NAMES[k]: round(v, 5) for k, v in kt.items()}
    roof["timing"] = (f"timed-region step time split by the dispatch-event durations of {launches} further steps; "
                      "kernel_ms_dispatch: those raw durations (directly launched steps)")
    roof["kernel_ms_dispatch"] = {KERNEL_NAMES.get(k, k): round(v, 5) for k, v in disp.items()}
    roof["kernel_ms_isolated"] = {KERNEL_NAMES[k]: round(v, 5) for k, v in isolated_kernel_ms(torch, sim, launches).items()}
    roof["kernel_hbm_gbs"] = {KERNEL_NAMES[k]: round(kernel_bytes_per_lup(k, prec) * nodes / (v * 1e-3) / 1e9, 1)
                              for k, v in kt.items()}
    return roof


def variant_name(kernel: int, shape, rk: int) -> str:
    """Name of a launch variant, as the profile summaries key it: k_lbm<tx x ty x threads[,wN]>,
    k_thermal<tx x ty x threads,rkS> (wN: register budget for N waves per SIMD)."""
    tx, ty, nt, mw = shape
    budget = f",w{mw}" if mw else ""
    if kernel == 0:
        return f"k_lbm<{tx}x{ty}x{nt}{budget}>"
    return f"k_thermal<{tx}x{ty}x{nt}{budget},rk{rk}>"


def base_line(args, prec, value, ms_step, workload_cfg):
    return {
        "metric": "MLUPS (flow+thermal) & % HBM peak; batched vs single & FP16-store vs FP32 at error",
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {0: "f64", 1: "f32", 2: "f16-store/f32", 3: "bf16-store/f32"}[prec],
        "data": "synthetic",
        "config": workload_cfg,
    }


def run_single(args, lbm, cfg, prec, workload, re):
    import torch
    progress(f"{workload}: warm-up")
    sim = lbm.Simulation(cfg)
    sim.step(cfg.warmup_steps)          # physical warm-up of the configuration (untimed)
    # launch variants timed over coupled steps (untimed); small grids take more steps per variant,
    # which keeps the choice stable against run-to-run noise at little cost
    choose_variants(args, sim, 100 if cfg.nx * cfg.ny <= (1 << 20) else 20)
    sim.step(args.warmup)
    untimed = sim.step_count
    ms, wall, reps = timed_windows(torch, sim, args.steps, args.repeats, launch_period([cfg]))
    ms_step = ms / args.steps
    nodes = cfg.nx * cfg.ny
    mlups = nodes / (ms_step * 1e-3) / 1e6
    mass = sim.total_mass()
    q, nu, nu_avg = sim.wall_heat_flux()
    if not (mass == mass and nu == nu):
        print("non-finite state after the timed steps", file=sys.stderr)
        sys.exit(3)
    line = base_line(args, prec, mlups, ms_step, {
        "workload": workload, "nx": cfg.nx, "ny": cfg.ny, "cyl_r": cfg.cyl_r, "u_in": cfg.u_in, "Re": re,
        "rk_stages": cfg.rk_stages, "warmup_steps_untimed": untimed,
        "diag_every": cfg.diag_every, "parallelism": "single-gpu",
        "tiles": {"k_lbm": sim.variants(0)[sim.get_variant(0)], "k_thermal": sim.variants(1)[sim.get_variant(1)]},
        "variants": [sim.get_variant(0), sim.get_variant(1)]})
    line["roofline"] = kernel_roofline(torch, sim, cfg, prec, nodes, args.kernel_launches, workload, ms_step)
    line["wall_s"] = round(wall, 3)
    line["timing"] = {"repeats": len(reps), "ms_per_step_each": [round(r / args.steps, 6) for r in reps],
                      "statistic": "median", "window_aligned_to_launch_period": launch_period([cfg])}
    line["diagnostics"] = {"mass": mass, "q_mean": q, "nu": nu}
    if not args.no_cpu_baseline:
        progress("cpu_baseline")
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_budget)
    return line


def run_sweep(args, lbm, cfgs, prec):
    """64 uneven boiling runs (superheat sweep) stepped together by one handle, against the same
    runs stepped one after another through their own handles."""
    import torch
    nodes = sum(c.nx * c.ny for c in cfgs)
    sim = lbm.Simulation(cfgs)
    sim.step(max(c.warmup_steps for c in cfgs))
    choose_variants(args, sim, 10)
    groups = max(1, min(args.stream_groups, len(cfgs)))
    sim.set_stream_groups(groups)
    sim.step(args.warmup)
    period = launch_period(cfgs)
    ms, wall, reps = timed_windows(torch, sim, args.steps, args.repeats, period)
    ms_step = ms / args.steps
    batched = nodes / (ms_step * 1e-3) / 1e6
    # sequential: each run alone on its own handle (same configuration, warm-up already passed), with
    # launch variants tuned for its own shape (remembered per shape) and timed over one whole launch
    # period (graph replay and its diagnostic step included), as the batched windows are
    seq_ms = 0.0
    seq_var = {}
    for c in cfgs:
        one = lbm.Simulation(c.replace(warmup_steps=0))
        one.step(20)
        if not args.no_autotune:
            seq_var[f"{c.nx}x{c.ny}r{c.cyl_r}"] = list(tune(one, 10, cached=True))
        align(one, period)
        t_ms, _ = timed_steps(torch, one, period)
        seq_ms += t_ms / period
        one.close()
        del one
    sequential = nodes / (seq_ms * 1e-3) / 1e6
    line = base_line(args, prec, batched, ms_step, {
        "workload": f"boiling-sweep-{len(cfgs)}-runs", "runs": len(cfgs), "nodes": nodes,
        "grids": "64*{4..16} x half, R 8..32, superheat 0.02..0.30 Tc, Re 30..3000 (seed 2018)",
        "stream_groups": groups,
        "parallelism": "single-gpu",
        "tiles": {"k_lbm": sim.variants(0)[sim.get_variant(0)], "k_thermal": sim.variants(1)[sim.get_variant(1)]},
        "variants": [sim.get_variant(0), sim.get_variant(1)]})
    line["sequential_mlups"] = round(sequential, 1)
    line["batched_over_sequential"] = round(batched / sequential, 3)
    line["sequential_variants"] = seq_var
    line["timing"] = {"repeats": len(reps), "ms_per_step_each": [round(r / args.steps, 6) for r in reps],
                      "statistic": "median", "window_aligned_to_launch_period": period,
                      "sequential": f"one window of {period} steps per run, aligned, after 20 steps and its tuning"}
    line["roofline"] = kernel_roofline(torch, sim, cfgs[0], prec, nodes, max(10, args.kernel_launches // 10),
                                       f"boiling-sweep-{len(cfgs)}-runs-{args.precision}", ms_step)
    line["wall_s"] = round(wall, 3)
    return line


if __name__ == "__main__":
    main()
