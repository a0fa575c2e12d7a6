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

The flux of Eq. q_corr, q = sum_i e_i s_i, is not exactly the energy that
the step carries across a face: the EED part W w_i E of every direction moves
along its pending worm move on every step, pauses included, and a diagonal
move is sqrt(2) long.  face_current() counts that energy exactly (from the
push form of Eq. algorithm); in a steady film it is the same on every face
(energy conservation, Eq. lbm-energy-density).  At large W the Eq. q_corr
flux exceeds it, by a share first order in W (measured in a wall-free slab
with Q = 16: 37 % at MFP 1.28 cells, 12 % at 4, 6 % at 8), which is why
kappa_eff / kappa read from q exceeds 1 for the thickest films at the
smallest Kn.
"""
from __future__ import annotations

import numpy as np

from .worm_lbm import D2Q8, Config, Lattice


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


def face_current(lat: Lattice) -> np.ndarray:
    """Energy that the next step carries across each face x + 1/2 between
    columns x and x + 1 (x = 0 .. nx - 2), per row: the packets of the push
    form of Eq. algorithm whose move has a +1 (-1) x component leave column x
    (x + 1) through that face; a hopping direction moves (1 - W) e_i + W w_i E,
    a pausing one only its EED part W w_i E.  Returns [nx - 1]."""
    c = lat.cfg
    n = lat.n + 1
    sch = lat.schedule(n)
    mv, hp = sch.move[n - 1], sch.hop[n - 1]
    E = lat.e.sum(axis=0)
    W = lat.Wc
    J = np.zeros(c.nx - 1)
    for i in range(c.q):
        sx, _ = D2Q8[int(mv[i])]
        moved = W * lat.w[i] * E
        if hp[i]:
            moved = moved + (1.0 - W) * lat.e[i]
        col = np.broadcast_to(moved, (c.ny, c.nx)).sum(axis=0)
        if sx == 1:
            J += col[:-1]
        elif sx == -1:
            J -= col[1:]
    return J / c.ny


def slab_steady(cfg: Config, settle: int, window: int):
    """A film started from the linear profile between its walls, run `settle`
    steps and then `window` more; returns (mean face current [nx - 1], mean
    q_x [ny, nx], temperature [ny, nx]) over the window."""
    lat = Lattice(cfg)
    T0 = np.linspace(cfg.t_x_lo, cfg.t_x_hi, cfg.nx)
    lat.set_temperature(np.tile(T0, (cfg.ny, 1)))
    lat.run(settle)
    J = np.zeros(cfg.nx - 1)
    qx = np.zeros((cfg.ny, cfg.nx))
    for _ in range(window):
        J += face_current(lat)
        lat.step()
        qx += lat.heat_flux()[0]
    return J / window, qx / window, lat.temperature()
