"""A worm-LBM lattice on one GPU, with PyTorch providing device memory and the
stream.  Thin convenience layer over the C-ABI binding: it allocates the
workspace and output tensors and passes their pointers; every step of the
method runs in the library's HIP kernels.
"""
from __future__ import annotations

import torch

from . import wormlbm as W


class Lattice:
    def __init__(self, nx: int, ny: int, q: int, mfp: float = float("inf"),
                 device: str | torch.device = "cuda", **kw):
        self.params = W.make_params(nx, ny, q, mfp=mfp, **kw)
        self.nx, self.ny, self.q = nx, ny, q
        self.device = torch.device(device)
        nbytes = W.wlbm_workspace_bytes(self.params)
        # the caching allocator returns at least 512-byte aligned blocks
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.handle = W.wlbm_create(self.params, self.workspace.data_ptr(), nbytes,
                                    self._stream())
        self._mfp_field = None

    def _stream(self) -> int:
        return torch.cuda.current_stream(self.device).cuda_stream

    def _sync_stream(self) -> None:
        W.wlbm_set_stream(self.handle, self._stream())

    def _field(self, t: torch.Tensor, shape) -> torch.Tensor:
        t = torch.as_tensor(t, dtype=torch.float32, device=self.device).contiguous()
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    # -- state ---------------------------------------------------------------
    def set_temperature(self, T0) -> None:
        self._sync_stream()
        t = self._field(T0, (self.ny, self.nx))
        W.wlbm_set_temperature(self.handle, t.data_ptr())
        self._keep = t

    def set_populations(self, e) -> None:
        self._sync_stream()
        t = self._field(e, (self.q, self.ny, self.nx))
        W.wlbm_set_populations(self.handle, t.data_ptr())
        self._keep = t

    def set_mfp_field(self, mfp) -> None:
        self._sync_stream()
        if mfp is None:
            W.wlbm_set_mfp_field(self.handle, None)
            self._mfp_field = None
            return
        t = self._field(mfp, (self.ny, self.nx))
        W.wlbm_set_mfp_field(self.handle, t.data_ptr())
        self._mfp_field = t

    def set_sources(self, cells, values) -> None:
        """Internal sources: cells [S, 2] (x, y), imposed DDEDs values [S, q];
        None (or S = 0) removes them.  The tensors are kept alive here."""
        self._sync_stream()
        if cells is None or len(cells) == 0:
            W.wlbm_set_sources(self.handle, 0, None, None)
            self._sources = None
            return
        c = torch.as_tensor(cells, dtype=torch.int32, device=self.device).contiguous()
        v = torch.as_tensor(values, dtype=torch.float32, device=self.device).contiguous()
        if c.dim() != 2 or c.shape[1] != 2 or tuple(v.shape) != (c.shape[0], self.q):
            raise ValueError("cells must be [S, 2] and values [S, q]")
        W.wlbm_set_sources(self.handle, c.shape[0], c.data_ptr(), v.data_ptr())
        self._sources = (c, v)

    def set_speeds(self, speeds) -> None:
        """Grid speed of each direction ([q] in (0, 1]; None = 1), at step 0."""
        W.wlbm_set_speeds(self.handle, self.q, speeds)

    def accumulate_temperature(self, scale: float, T: torch.Tensor) -> None:
        """T += scale * (this lattice's temperature), on the device."""
        self._sync_stream()
        W.wlbm_accumulate_temperature(self.handle, scale, T.data_ptr())

    def set_wall_temperatures(self, t_x_lo=0.0, t_x_hi=0.0, t_y_lo=0.0, t_y_hi=0.0) -> None:
        W.wlbm_set_wall_temperatures(self.handle, t_x_lo, t_x_hi, t_y_lo, t_y_hi)

    def set_flux_window(self, window: int) -> None:
        W.wlbm_set_flux_window(self.handle, window)

    def step(self, n: int = 1) -> None:
        self._sync_stream()
        W.wlbm_step(self.handle, n)

    @property
    def step_count(self) -> int:
        return W.wlbm_step_count(self.handle)

    # -- readout -------------------------------------------------------------
    def temperature(self) -> torch.Tensor:
        self._sync_stream()
        T = torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)
        W.wlbm_read_temperature(self.handle, T.data_ptr())
        return T

    def heat_flux(self, averaged: bool = False):
        self._sync_stream()
        qx = torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)
        qy = torch.empty_like(qx)
        W.wlbm_read_heat_flux(self.handle, qx.data_ptr(), qy.data_ptr(), int(averaged))
        return qx, qy

    def populations(self) -> torch.Tensor:
        self._sync_stream()
        e = torch.empty((self.q, self.ny, self.nx), dtype=torch.float32, device=self.device)
        W.wlbm_read_populations(self.handle, e.data_ptr())
        return e

    def totals(self):
        self._sync_stream()
        return W.wlbm_read_totals(self.handle)

    # -- saved states and tapes -----------------------------------------------
    @property
    def state_bytes(self) -> int:
        return W.wlbm_state_bytes(self.handle)

    def new_states(self, n: int) -> torch.Tensor:
        """n zero-filled state slots, [n, state_bytes] uint8 (a tape)."""
        return torch.zeros((n, self.state_bytes), dtype=torch.uint8, device=self.device)

    def save_state(self, buf: torch.Tensor) -> None:
        self._sync_stream()
        W.wlbm_save_state(self.handle, buf.data_ptr(), buf.numel())

    def load_state(self, buf: torch.Tensor, step: int) -> None:
        self._sync_stream()
        W.wlbm_load_state(self.handle, buf.data_ptr(), buf.numel(), step)

    def step_tape(self, n: int, tape: torch.Tensor) -> None:
        """n steps; the state after step k (1-based) goes to tape[k - 1]."""
        if tape.dim() != 2 or tape.shape[0] < n or not tape.is_contiguous():
            raise ValueError("tape must be a contiguous [slots >= n, slot_bytes] tensor")
        self._sync_stream()
        W.wlbm_step_tape(self.handle, n, tape.data_ptr(), tape.shape[1])

    def read_probes(self, cells: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """T at cells ([P, 2] int32 (x, y) on the device)."""
        self._sync_stream()
        if out is None:
            out = torch.empty(cells.shape[0], dtype=torch.float32, device=self.device)
        W.wlbm_read_probes(self.handle, cells.shape[0], cells.data_ptr(), out.data_ptr())
        return out

    # -- launch configuration -------------------------------------------------
    @property
    def dir_split(self) -> int:
        return W.wlbm_get_dir_split(self.handle)

    @property
    def steps_per_launch(self) -> int:
        """Time steps a kernel launch advances on this lattice (1: single-step
        kernel)."""
        return W.wlbm_get_steps_per_launch(self.handle)

    def block_rows(self, k: int) -> int:
        """Output rows per block of the kernel for k = 2, 3 or 4 steps per
        launch (fixed, tuned or the launch model's pick; 0 if this lattice runs
        one step per launch)."""
        return W.wlbm_get_block_rows(self.handle, k)

    def set_block_rows(self, k: int, rows: int) -> None:
        """Fix the output rows per block for k steps per launch (0: back to
        the launch model's pick)."""
        W.wlbm_set_block_rows(self.handle, k, rows)

    def tune_block_rows(self, k: int, launches: int = 6) -> int:
        """Time every candidate block height for k steps per launch on the
        current state (restored afterwards) and keep the fastest."""
        self._sync_stream()
        buf = torch.empty(self.state_bytes, dtype=torch.uint8, device=self.device)
        return W.wlbm_tune_block_rows(self.handle, buf.data_ptr(), buf.numel(), k, launches)

    def set_dir_split(self, split: int) -> None:
        W.wlbm_set_dir_split(self.handle, split)

    def autotune(self, steps: int = 20):
        """Keep the fastest direction split; returns (ms per step for splits
        1, 2, 4, chosen split).  The state is restored afterwards."""
        self._sync_stream()
        buf = torch.empty(self.state_bytes, dtype=torch.uint8, device=self.device)
        return W.wlbm_autotune(self.handle, buf.data_ptr(), buf.numel(), steps)

    def flux_mean(self, x0: int = 0, x1: int | None = None, averaged: bool = True):
        """Mean (q_x, q_y) over columns x0 <= x < x1, float64."""
        self._sync_stream()
        return W.wlbm_read_flux_mean(self.handle, x0, self.nx if x1 is None else x1,
                                     int(averaged))

    def close(self) -> None:
        if getattr(self, "handle", None):
            W.wlbm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Lattices advanced together in one kernel launch (same step count,
    split, per-cell field use and flux window; q, direction sets and grid
    speeds may differ): several steps per launch when every lattice takes the
    multi-step kernel with one q, else one step per launch, where
    ``set_graphs(True)`` replays whole schedule chunks as one HIP graph
    launch."""

    def __init__(self, lattices):
        self.lattices = list(lattices)
        self.device = self.lattices[0].device
        handles = [lat.handle for lat in self.lattices]
        nbytes = W.wlbm_batch_bytes(handles)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.handle = W.wlbm_batch_create(handles, self.workspace.data_ptr(), nbytes,
                                          torch.cuda.current_stream(self.device).cuda_stream)

    def step(self, n: int = 1) -> None:
        for lat in self.lattices:
            lat._sync_stream()
        W.wlbm_batch_step(self.handle, n)

    def set_graphs(self, on: bool) -> None:
        W.wlbm_batch_set_graphs(self.handle, 1 if on else 0)

    @property
    def steps_per_launch(self) -> int:
        """Time steps one launch advances every lattice (1: one per launch)."""
        return W.wlbm_batch_get_steps_per_launch(self.handle)

    def tune_block_rows(self, launches: int = 6) -> int:
        """Time every candidate block height of the batch's multi-step
        launches (one height for all lattices) on the current states
        (restored afterwards) and keep the fastest for every lattice."""
        for lat in self.lattices:
            lat._sync_stream()
        nbytes = sum((lat.state_bytes + 255) // 256 * 256 for lat in self.lattices)
        buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        rows = W.wlbm_batch_tune_block_rows(self.handle, buf.data_ptr(), buf.numel(), launches)
        del buf
        return rows

    def close(self) -> None:
        if getattr(self, "handle", None):
            W.wlbm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
