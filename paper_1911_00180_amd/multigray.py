"""Multigray transport: uncoupled gray bands on one grid (Sec. 2.2).

The paper notes that, instead of a full dispersion, several gray BTEs can be
solved in parallel without coupling and their results superposed.  Band b
carries a share c_b of the heat capacity, its own mean free path and its own
group velocity; on the worm lattice the velocity is the TAS grid speed v_b
(<= 1 cell per step: the fastest band sets the time step), which the
schedule imposes by pausing (Sec. 2.3).  With the linearised gray model each
band holds the energy c_b T, relaxes towards its own equilibrium, and the
temperature of the superposition is T = sum_b E_b / sum_b c_b.

With walls, the bands advance together in one batched launch per step
(bands with equal grid speeds share one schedule, the others have their
own); on a periodic lattice each band advances on its own, several steps
per launch.
"""
from __future__ import annotations

import numpy as np
import torch

from .lattice import Batch, Lattice


class Multigray:
    def __init__(self, nx: int, ny: int, q: int, bands, device="cuda",
                 t_x_lo: float = 0.0, t_x_hi: float = 0.0, t_y_lo: float = 0.0,
                 t_y_hi: float = 0.0, **kw):
        """bands: [(c_b, v_b, mfp_b)]: heat-capacity share, grid speed in
        (0, 1] and mean free path in cells of each band.  Other keyword
        arguments (edges, direction set, ...) go to every band's Lattice; the
        wall temperatures are shared and each band holds c_b of them."""
        self.bands = [(float(c), float(v), float(m)) for c, v, m in bands]
        if not self.bands or any(c <= 0 for c, _, _ in self.bands):
            raise ValueError("bands need positive heat-capacity shares")
        self.nx, self.ny, self.q = nx, ny, q
        self.device = torch.device(device)
        self.c_total = sum(c for c, _, _ in self.bands)
        self.lattices = []
        for c, v, mfp in self.bands:
            lat = Lattice(nx, ny, q, mfp=mfp, device=device, t_x_lo=c * t_x_lo,
                          t_x_hi=c * t_x_hi, t_y_lo=c * t_y_lo, t_y_hi=c * t_y_hi, **kw)
            if v != 1.0:
                lat.set_speeds(np.full(q, v))
            self.lattices.append(lat)
        p = self.lattices[0].params
        periodic = p.x_edge == 0 and p.y_edge == 0
        self.batch = Batch(self.lattices) if len(self.lattices) > 1 and not periodic else None

    def set_temperature(self, T0) -> None:
        T0 = torch.as_tensor(T0, dtype=torch.float32, device=self.device)
        for (c, _, _), lat in zip(self.bands, self.lattices):
            lat.set_temperature(c * T0)

    def step(self, n: int = 1) -> None:
        if self.batch is not None:
            self.batch.step(n)
        else:
            for lat in self.lattices:
                lat.step(n)

    def temperature(self) -> torch.Tensor:
        T = torch.zeros((self.ny, self.nx), dtype=torch.float32, device=self.device)
        for lat in self.lattices:
            lat.accumulate_temperature(1.0 / self.c_total, T)
        return T

    def close(self) -> None:
        if self.batch is not None:
            self.batch.close()
        for lat in self.lattices:
            lat.close()
