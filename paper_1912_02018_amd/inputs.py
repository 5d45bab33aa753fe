"""Seeded synthetic initial fields shared by the oracle tests and the HIP path.

This module holds no arithmetic of the method: it only draws reproducible random numbers
(SplitMix64, Steele, Lea and Flood, OOPSLA 2014) and lays out macroscopic density / velocity
fields (a slab, a bubble, a shear wave, a uniform stream).  Every side turns these fields into
populations itself.
"""
from __future__ import annotations

import numpy as np

_M64 = (1 << 64) - 1


def splitmix64(seed: int, n: int) -> np.ndarray:
    """First n outputs of SplitMix64 started from ``seed`` (uint64)."""
    with np.errstate(over="ignore"):
        idx = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed & _M64) + idx * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int) -> np.ndarray:
    """n doubles in [0, 1) from the top 53 bits of SplitMix64."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_noise(seed: int, shape, amp: float) -> np.ndarray:
    """Additive noise uniform in (-amp, amp)."""
    n = int(np.prod(shape))
    return (amp * (2.0 * uniform01(seed, n) - 1.0)).reshape(shape)


def slab(nx: int, ny: int, x0: int, x1: int, rho_in: float, rho_out: float,
         noise_amp: float = 0.0, seed: int = 1912) -> np.ndarray:
    """Density of a slab x0 <= x < x1 (normal to x) of rho_in surrounded by rho_out."""
    rho = np.full((ny, nx), rho_out, dtype=np.float64)
    rho[:, x0:x1] = rho_in
    if noise_amp:
        rho += uniform_noise(seed, (ny, nx), noise_amp)
    return rho


def bubble(nx: int, ny: int, radius: float, rho_in: float, rho_out: float,
           width: float = 2.0, cx: float | None = None, cy: float | None = None) -> np.ndarray:
    """Circular region of rho_in (radius ``radius``) in rho_out, tanh profile of given width."""
    cx = (nx - 1) / 2.0 if cx is None else cx
    cy = (ny - 1) / 2.0 if cy is None else cy
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.hypot(x - cx, y - cy)
    return 0.5 * (rho_in + rho_out) - 0.5 * (rho_in - rho_out) * np.tanh(2.0 * (r - radius) / width)


def shear_wave(nx: int, ny: int, rho0: float, amp: float, mode: int = 1):
    """Uniform density with u_y = amp sin(2 pi mode x / nx), u_x = 0."""
    x = np.arange(nx, dtype=np.float64)
    uy = np.broadcast_to(amp * np.sin(2.0 * np.pi * mode * x / nx), (ny, nx)).copy()
    return np.full((ny, nx), rho0), np.zeros((ny, nx)), uy


def uniform(nx: int, ny: int, rho0: float, ux: float = 0.0, uy: float = 0.0):
    return np.full((ny, nx), rho0), np.full((ny, nx), ux), np.full((ny, nx), uy)


def random_fields(nx: int, ny: int, rho0: float, drho: float, du: float, seed: int):
    """Smooth-free random fields for parity tests: rho0 + U(-drho, drho), u ~ U(-du, du)."""
    rho = rho0 + uniform_noise(seed, (ny, nx), drho)
    ux = uniform_noise(seed + 1, (ny, nx), du)
    uy = uniform_noise(seed + 2, (ny, nx), du)
    return rho, ux, uy
