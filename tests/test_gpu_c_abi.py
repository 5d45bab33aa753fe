"""The C ABI used from plain C (tests/c_abi_example.c, built with the library into
tests/c_abi_example.bin): a program with its own HIP workspace and stream, and no Python or PyTorch,
steps a heated-cylinder channel and reads back mass, heat flux and fields; they equal, bit for bit,
the same run through the Python binding (one library, one arithmetic)."""
import os
import subprocess

import numpy as np
import pytest

from paper_1912_02018_amd.config import FP32, FP64, cylinder_config

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "c_abi_example.bin")


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_c_program_matches_binding(precision):
    if not os.path.exists(EXE):
        pytest.skip("tests/c_abi_example.bin is built by __graft_entry__.build()")
    import torch
    assert torch.cuda.is_available()
    from paper_1912_02018_amd import lbm
    cfg = cylinder_config(64, 32, 6, 20, re=100.0, u_in=0.02, dTr_wall=0.1, precision=precision, warmup=0,
                          rk_stages=4, diag_every=5)
    steps = 60
    c = lbm.to_c_config(cfg)
    text = "".join(f"{name}={getattr(c, name)!r}\n" for name, _ in lbm._CONFIG_FIELDS) + f"steps={steps}\n"
    env = dict(os.environ)
    env["LD_LIBRARY_PATH"] = os.path.dirname(lbm.LIB_PATH) + os.pathsep + env.get("LD_LIBRARY_PATH", "")
    out = subprocess.run([EXE], input=text, capture_output=True, text=True, timeout=120, env=env)
    assert out.returncode == 0, out.stderr
    lines = out.stdout.split("\n")
    head = {l.split()[0]: float.fromhex(l.split()[1]) for l in lines[:4]}
    vals = np.array([float.fromhex(v) for v in lines[4:] if v])
    n = cfg.nx * cfg.ny
    assert vals.size == 4 * n

    sim = lbm.Simulation(cfg)
    sim.step(steps)
    f = sim.fields()
    q, nu, nu_avg = sim.wall_heat_flux()
    assert head["mass"] == sim.total_mass()
    assert (head["q"], head["nu"], head["nu_avg"]) == (q, nu, nu_avg)
    for k, name in enumerate(("rho", "ux", "uy", "T")):
        assert np.array_equal(vals[k * n:(k + 1) * n].reshape(cfg.ny, cfg.nx), f[name]), name
