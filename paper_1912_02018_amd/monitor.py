"""Time series of the FP64 wall heat flux, Nusselt number and total mass of running simulations
(the quantities Sec. IV B of the paper follows in time), sampled every few steps and written as CSV or
JSON.  Sampling reads the library's FP64 reductions back to the host, so it synchronises the stream.
"""
from __future__ import annotations

import csv
import json

COLUMNS = ("step", "run", "q_mean", "nu", "nu_time_avg", "mass")


def record(sim, steps: int, every: int, runs=None, include_start: bool = True) -> list:
    """Advance ``sim`` by ``steps`` steps and sample every ``every`` steps (and at the start if
    include_start).  Returns one dict per sample and run with the keys of COLUMNS."""
    if every <= 0 or steps < 0:
        raise ValueError("need every > 0 and steps >= 0")
    runs = list(range(len(sim.cfgs))) if runs is None else list(runs)
    rows = []

    def sample():
        for r in runs:
            q, nu, nu_avg = sim.wall_heat_flux(r)
            rows.append({"step": sim.step_count, "run": r, "q_mean": q, "nu": nu, "nu_time_avg": nu_avg,
                         "mass": sim.total_mass(r)})

    if include_start:
        sample()
    done = 0
    while done < steps:
        n = min(every, steps - done)
        sim.step(n)
        done += n
        if n == every or done == steps:
            sample()
    return rows


def write_csv(path: str, rows: list):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=COLUMNS)
        w.writeheader()
        for row in rows:
            w.writerow({k: (repr(row[k]) if isinstance(row[k], float) else row[k]) for k in COLUMNS})


def write_json(path: str, rows: list):
    with open(path, "w") as fh:
        json.dump([{k: row[k] for k in COLUMNS} for row in rows], fh)


def read_csv(path: str) -> list:
    with open(path, newline="") as fh:
        return [{k: (int(v) if k in ("step", "run") else float(v)) for k, v in row.items()} for row in csv.DictReader(fh)]
