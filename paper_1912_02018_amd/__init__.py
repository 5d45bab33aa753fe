"""MI355X-native central-moment pseudopotential lattice Boltzmann step for forced-convection
boiling on a heated cylinder (Saito et al., arXiv:1912.02018).

The compute path is ``liblbm.so``: hand-written HIP kernels for gfx950 behind a C ABI declared
in ``include/lbm.h``.  ``paper_1912_02018_amd.lbm`` is the thin ctypes binding; ``config`` holds
run configurations and ``inputs`` the seeded synthetic initial fields.
"""
from .config import LBMConfig, FP64, FP32, FP16S, BF16S  # noqa: F401

__all__ = ["LBMConfig", "FP64", "FP32", "FP16S", "BF16S"]
