"""Probe temperatures of a worm-LBM run as a differentiable torch function.

``ProbeSeries(lattice, probes, nsteps, every, checkpoint_every)`` maps
(per-cell MFP field, initial temperature T0, blackbody wall temperatures) to
the temperatures T^m(p) at the probe cells p on the steps m = every,
2 every, ..., nsteps.  Its backward pass is the library's adjoint: for a fixed
relaxation field each step is affine in the populations (Sec. 2.3,
Eq. algorithm; Sec. 2.6), so dL/de follows the transposed steps backwards in
time, seeded with dL/dT at the probes.

Memory: the forward pass saves the state every ``checkpoint_every`` steps; the
backward pass restores each checkpoint, recomputes the states of its segment
into a tape (the forward kernel writes them there directly) and runs the
reverse steps over it.  Device memory: (nsteps / K + K) states plus the adjoint
workspace (two population sets).  Argument marshalling only: every step runs
in the library's HIP kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import wormlbm as W
from .lattice import Lattice


class ProbeSeries:
    def __init__(self, lattice: Lattice, probes, nsteps: int, every: int,
                 checkpoint_every: int = 50):
        if nsteps < 1 or every < 1 or checkpoint_every < 1:
            raise ValueError("nsteps, every and checkpoint_every must be >= 1")
        if lattice.params.y_edge == W.EDGE_DIFFUSE:
            raise ValueError("the adjoint covers periodic and blackbody edges")
        cells = np.asarray(probes, dtype=np.int64).reshape(-1, 2)
        if cells.size and (cells[:, 0].min() < 0 or cells[:, 0].max() >= lattice.nx
                           or cells[:, 1].min() < 0 or cells[:, 1].max() >= lattice.ny):
            raise ValueError("probe cells must lie inside the lattice")
        self.lat = lattice
        self.nsteps, self.every, self.K = nsteps, every, checkpoint_every
        self.cells = torch.as_tensor(cells.astype(np.int32), device=lattice.device).contiguous()
        self.nloss = nsteps // every
        self.nseg = (nsteps + self.K - 1) // self.K
        self.ck = lattice.new_states(self.nseg)
        self.tape = lattice.new_states(max(self.K - 1, 1))
        self._adj_ws = None
        self._generation = 0

    def __call__(self, mfp: torch.Tensor | None, T0: torch.Tensor,
                 walls: torch.Tensor | None = None) -> torch.Tensor:
        if walls is None:
            walls = torch.zeros(4, dtype=torch.float32, device=self.lat.device)
        return _ProbeRun.apply(mfp, T0, walls, self)

    # -- forward ---------------------------------------------------------------
    def run_forward(self, mfp, T0, walls) -> torch.Tensor:
        lat = self.lat
        self._generation += 1
        lat.set_mfp_field(None if mfp is None else mfp.detach())
        wl = [float(v) for v in walls.detach().cpu().tolist()]
        lat.set_wall_temperatures(*wl)
        lat.set_temperature(T0.detach())
        # restart the schedule at step 0 from this initial state
        lat.save_state(self.ck[0])
        lat.load_state(self.ck[0], 0)
        out = torch.empty((self.nloss, self.cells.shape[0]), dtype=torch.float32,
                          device=lat.device)
        m = 0
        for k in range(self.nseg):
            s1 = min((k + 1) * self.K, self.nsteps)
            if k > 0:
                lat.save_state(self.ck[k])
            while m < s1:
                nxt = min(s1, (m // self.every + 1) * self.every)
                lat.step(nxt - m)
                m = nxt
                if m % self.every == 0:
                    lat.read_probes(self.cells, out[m // self.every - 1])
        return out

    # -- backward --------------------------------------------------------------
    def run_backward(self, grad_out: torch.Tensor, generation: int):
        if generation != self._generation:
            raise RuntimeError("backward of a ProbeSeries call after a later forward call: "
                               "its checkpoints were overwritten")
        lat, h = self.lat, self.lat.handle
        grad_out = grad_out.to(torch.float32).contiguous()
        if self._adj_ws is None:
            self._adj_ws = torch.empty(W.wlbm_adjoint_bytes(h), dtype=torch.uint8,
                                       device=lat.device)
        lat._sync_stream()
        slot = self.tape.shape[1]
        W.wlbm_adjoint_begin(h, self._adj_ws.data_ptr(), self._adj_ws.numel(), self.nsteps)
        P = self.cells.shape[0]

        def seed(m):
            if m > 0 and m % self.every == 0 and P:
                W.wlbm_adjoint_seed(h, P, self.cells.data_ptr(),
                                    grad_out[m // self.every - 1].data_ptr())

        m = self.nsteps
        seed(m)
        for k in reversed(range(self.nseg)):
            s0 = k * self.K
            if m - s0 > 1:
                lat.load_state(self.ck[k], s0)
                lat.step_tape(m - s0 - 1, self.tape)   # tape[j] = state s0 + 1 + j
                lat._sync_stream()
            while m > s0:
                stop = max(s0, ((m - 1) // self.every) * self.every)
                if stop >= s0 + 1:
                    W.wlbm_adjoint_steps(h, m - stop, self.tape[stop - s0 - 1].data_ptr(), slot)
                else:
                    if m - 1 >= s0 + 1:
                        W.wlbm_adjoint_steps(h, m - s0 - 1, self.tape[0].data_ptr(), slot)
                    W.wlbm_adjoint_steps(h, 1, self.ck[k].data_ptr(), slot)
                m = stop
                seed(m)
        g_mfp = torch.empty((lat.ny, lat.nx), dtype=torch.float32, device=lat.device)
        g_T0 = torch.empty_like(g_mfp)
        g_walls = W.wlbm_adjoint_read(h, g_mfp.data_ptr(), g_T0.data_ptr())
        return g_mfp, g_T0, torch.tensor(g_walls, dtype=torch.float32, device=lat.device)


class _ProbeRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mfp, T0, walls, runner: ProbeSeries):
        out = runner.run_forward(mfp, T0, walls)
        ctx.runner = runner
        ctx.generation = runner._generation
        ctx.has_mfp = mfp is not None
        return out

    @staticmethod
    def backward(ctx, grad_out):
        g_mfp, g_T0, g_walls = ctx.runner.run_backward(grad_out, ctx.generation)
        return (g_mfp if ctx.has_mfp else None), g_T0, g_walls, None
