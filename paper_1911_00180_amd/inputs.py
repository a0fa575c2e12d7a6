"""Seeded synthetic inputs (initial temperatures, mean-free-path fields, probe
cells, random populations).

This module holds no arithmetic of the method itself: it only draws and shapes
input arrays.  The same arrays are fed to the GPU library and, in tests, to
the FP64 CPU oracle.  Every generator takes an explicit seed (numpy PCG64 via
``default_rng``).
"""
from __future__ import annotations

import numpy as np


def seeded_center(seed: int, nx: int, ny: int) -> tuple[int, int]:
    """Pulse centre (x0, y0) drawn uniformly on the lattice."""
    rng = np.random.default_rng(seed)
    x0, y0 = rng.integers(0, [nx, ny])
    return int(x0), int(y0)


def gaussian_pulse(nx: int, ny: int, sigma: float, x0: float, y0: float,
                   amplitude: float = 1.0, background: float = 0.0,
                   periodic: bool = True) -> np.ndarray:
    """T0[y, x] = background + amplitude * exp(-r^2 / (2 sigma^2)).

    With ``periodic`` the distance r is the minimum-image distance on the
    nx-by-ny torus, so the pulse is smooth across the wrap."""
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    dx = x - x0
    dy = y - y0
    if periodic:
        dx = (dx + nx / 2.0) % nx - nx / 2.0
        dy = (dy + ny / 2.0) % ny - ny / 2.0
    r2 = dy[:, None] ** 2 + dx[None, :] ** 2
    return background + amplitude * np.exp(-r2 / (2.0 * sigma * sigma))


def smooth_lognormal_field(nx: int, ny: int, seed: int, corr: float,
                           median: float, log_spread: float,
                           lo: float, hi: float) -> np.ndarray:
    """Smooth random positive field, e.g. a per-cell mean free path.

    White noise from ``default_rng(seed)`` is Gaussian-filtered on the periodic
    lattice (FFT, correlation length ``corr`` cells), standardised, and mapped
    to ``median * exp(log_spread * z)``, then clipped to [lo, hi]."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((ny, nx))
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.fftfreq(nx)[None, :]
    filt = np.exp(-2.0 * (np.pi * corr) ** 2 * (kx ** 2 + ky ** 2))
    z = np.real(np.fft.ifft2(np.fft.fft2(z) * filt))
    z = (z - z.mean()) / z.std()
    return np.clip(median * np.exp(log_spread * z), lo, hi)


def probe_cells(seed: int, nx: int, ny: int, count: int, margin: int = 0) -> np.ndarray:
    """``count`` distinct cells (x, y), at least ``margin`` cells from the edges."""
    rng = np.random.default_rng(seed)
    xs = np.arange(margin, nx - margin)
    ys = np.arange(margin, ny - margin)
    flat = rng.choice(xs.size * ys.size, size=count, replace=False)
    return np.stack([xs[flat % xs.size], ys[flat // xs.size]], axis=1)


def random_populations(seed: int, q: int, ny: int, nx: int,
                       dtype=np.float32) -> np.ndarray:
    """Nonnegative populations e[q, y, x] drawn uniformly from [0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.random((q, ny, nx)).astype(dtype)


def random_temperature(seed: int, ny: int, nx: int, dtype=np.float32) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.random((ny, nx)).astype(dtype)


def inverse_problem(n: int = 256, seed_field: int = 1, seed_target: int = 2):
    """Inputs of the n x n inverse problem (MFP field recovered from probe
    temperatures), with lengths scaled by s = n / 256: the MFP field
    ln MFP = ln 16 + (ln 4 / 2) z, z smooth (correlation 16 s cells) and
    standardised, clipped to [4, 64] cells, from default_rng(seed_field); the
    target field from default_rng(seed_target); a centred Gaussian pulse
    sigma0 = 16 s; 32 probe cells from default_rng(3), at least 8 s cells
    from the edges.  Returns (n, mfp, target_mfp, T0, probes) with float32
    fields and probes as int [32, 2] (x, y)."""
    s = n / 256.0
    spread = float(np.log(4.0) / 2.0)
    mfp = smooth_lognormal_field(n, n, seed_field, 16.0 * s, 16.0, spread, 4.0, 64.0)
    tgt = smooth_lognormal_field(n, n, seed_target, 16.0 * s, 16.0, spread, 4.0, 64.0)
    T0 = gaussian_pulse(n, n, 16.0 * s, n // 2, n // 2)
    probes = probe_cells(3, n, n, 32, margin=int(round(8 * s)))
    return n, mfp.astype(np.float32), tgt.astype(np.float32), T0.astype(np.float32), probes


def inverse_problem_256(seed_field: int = 1, seed_target: int = 2):
    """The 256 x 256 inverse problem (correlation 16 cells, sigma0 = 16,
    probes at least 8 cells from the edges)."""
    return inverse_problem(256, seed_field, seed_target)
