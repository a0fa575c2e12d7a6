"""FP64 reference of the in-plane film conductivity (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of oracle/.  A film of thickness ny
cells with adiabatic diffuse walls at y = -1/2 and ny - 1/2 is held between
blackbody columns x = 0 (T_h) and x = nx - 1 (T_c) (Sec. 3.5).  The
effective conductivity is read from the heat flux averaged over the last
`window` steps (Sec. 3.4 averages over ten steps), taken over the interior
columns 1 .. nx-2:

    kappa_eff = <q_x> (nx - 1) / (T_h - T_c),

and compared with the bulk value of the gray model with unit heat capacity
and group velocity, kappa = Lambda / d (Lambda the MFP in cells, d = 2, or 3
when the run emulates 3D with the factor 3/2 of Eq. W-correction).
Reading: the distance between the wall cells is nx - 1 cells.
"""
from __future__ import annotations

import numpy as np

from .worm_lbm import Config, Lattice


def kappa_ratio(cfg: Config, qx_avg: np.ndarray) -> float:
    """kappa_eff / kappa from a window-averaged q_x field [ny, nx]."""
    q_mean = float(np.mean(qx_avg[:, 1:cfg.nx - 1]))
    kappa_eff = q_mean * (cfg.nx - 1) / (cfg.t_x_lo - cfg.t_x_hi)
    d = 3.0 if cfg.emulate_3d else 2.0
    return kappa_eff / (float(cfg.mfp) / d)


def film_run(cfg: Config, nsteps: int, window: int = 10):
    """Film from T0 = 0 (walls imposed), nsteps steps; returns (lattice,
    window-averaged qx, qy)."""
    lat = Lattice(cfg)
    lat.set_temperature(np.zeros((cfg.ny, cfg.nx)))
    qx, qy = lat.run(nsteps, flux_window=window)
    return lat, qx, qy


def film_kappa(cfg: Config, nsteps: int, window: int = 10) -> float:
    _, qx, _ = film_run(cfg, nsteps, window)
    return kappa_ratio(cfg, qx)
