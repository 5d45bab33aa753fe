"""Time-series recorder (paper_1912_02018_amd.monitor): sampling schedule and exact CSV / JSON round
trips on the host; on the GPU the samples equal direct reads of a second, identical run."""
import json
import os

import numpy as np
import pytest

from paper_1912_02018_amd import monitor


class FakeSim:
    """Host stand-in with the attributes record() reads: a step counter and deterministic values."""

    def __init__(self, n_runs=2):
        self.cfgs = [None] * n_runs
        self.step_count = 0

    def step(self, n):
        self.step_count += n

    def wall_heat_flux(self, r):
        s = self.step_count
        return 1e-3 * (s + 1) / 3.0, 10.0 + s / 7.0 + r, 9.5 + r / 11.0

    def total_mass(self, r):
        return 1234.5 + self.step_count / 13.0 + r


def test_sampling_schedule_and_round_trips(tmp_path):
    sim = FakeSim()
    rows = monitor.record(sim, 25, 10)
    assert [(r["step"], r["run"]) for r in rows] == [(s, k) for s in (0, 10, 20, 25) for k in (0, 1)]
    only = monitor.record(FakeSim(), 20, 10, runs=[1], include_start=False)
    assert [(r["step"], r["run"]) for r in only] == [(10, 1), (20, 1)]
    p = os.path.join(tmp_path, "series.csv")
    monitor.write_csv(p, rows)
    back = monitor.read_csv(p)
    assert back == rows                       # floats written with repr: exact
    q = os.path.join(tmp_path, "series.json")
    monitor.write_json(q, rows)
    assert json.load(open(q)) == rows
    with pytest.raises(ValueError):
        monitor.record(FakeSim(), 10, 0)


@pytest.mark.gpu
def test_samples_equal_direct_reads():
    import torch
    assert torch.cuda.is_available()
    from paper_1912_02018_amd import lbm
    from paper_1912_02018_amd.config import FP64, cylinder_config
    cfg = cylinder_config(64, 32, 6, 20, re=100.0, u_in=0.02, dTr_wall=0.1, precision=FP64, warmup=0, diag_every=2)
    a, b = lbm.Simulation([cfg, cfg.replace(dTr_wall=0.2)]), lbm.Simulation([cfg, cfg.replace(dTr_wall=0.2)])
    rows = monitor.record(a, 30, 15)
    for s in (0, 15, 30):
        b.step(s - b.step_count)
        for r in (0, 1):
            row = next(x for x in rows if x["step"] == s and x["run"] == r)
            assert (row["q_mean"], row["nu"], row["nu_time_avg"]) == b.wall_heat_flux(r)
            assert row["mass"] == b.total_mass(r)
    assert np.isfinite([x["nu"] for x in rows]).all()
