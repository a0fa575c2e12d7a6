"""Host logic of ProbeSeries (checkpoints, tapes, seeds), on the CPU.

The library calls are replaced by a recorder that tracks which forward state
each buffer holds, so the test checks that every reverse step m is given the
state of step m - 1, that each loss step is seeded exactly once (after the
reverse pass reaches it, before it moves below it), and that the forward pass
reads the probes on the loss steps.
"""
import types

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1911_00180_amd import autodiff  # noqa: E402


class FakeLattice:
    def __init__(self, nx=8, ny=8):
        self.nx, self.ny = nx, ny
        self.device = torch.device("cpu")
        self.params = types.SimpleNamespace(y_edge=0)
        self.handle = 1
        self.step_no = 0
        self.log = []
        self.bufs = {}          # data_ptr -> step of the state it holds

    # buffers: one row per state slot; record state steps by pointer
    def new_states(self, n):
        return torch.zeros((n, 256), dtype=torch.uint8)

    def _sync_stream(self):
        pass

    def set_mfp_field(self, m):
        pass

    def set_wall_temperatures(self, *w):
        pass

    def set_temperature(self, T0):
        self.step_no = 0

    def save_state(self, buf):
        self.bufs[buf.data_ptr()] = self.step_no

    def load_state(self, buf, step):
        assert self.bufs[buf.data_ptr()] == step
        self.step_no = step

    def step(self, n):
        self.step_no += n

    def step_tape(self, n, tape):
        for k in range(n):
            self.step_no += 1
            self.bufs[tape[k].data_ptr()] = self.step_no

    def read_probes(self, cells, out):
        self.log.append(("probe", self.step_no))
        out.fill_(float(self.step_no))


class FakeW:
    EDGE_DIFFUSE = 2

    def __init__(self, lat, slot):
        self.lat, self.slot, self.m = lat, slot, None
        self.seeds, self.used = [], []

    def wlbm_adjoint_bytes(self, h):
        return 64

    def wlbm_adjoint_begin(self, h, ptr, n, step):
        self.m = step

    def wlbm_adjoint_seed(self, h, n, cells, vals):
        self.seeds.append(self.m)

    def wlbm_adjoint_steps(self, h, n, states, slot):
        assert 0 < n <= self.m
        for k in range(n):
            m = self.m - k
            state_ptr = states + (n - 1 - k) * slot
            assert self.lat.bufs[state_ptr] == m - 1, (m, self.lat.bufs.get(state_ptr))
            self.used.append(m)
        self.m -= n

    def wlbm_adjoint_read(self, h, a, b):
        assert self.m == 0
        return (0.0, 0.0, 0.0, 0.0)


@pytest.mark.parametrize("nsteps,every,K", [(60, 5, 16), (70, 7, 7), (70, 7, 70), (23, 4, 5),
                                            (10, 10, 1), (1000, 10, 50), (31, 1, 3)])
def test_reverse_schedule(monkeypatch, nsteps, every, K):
    lat = FakeLattice()
    series = autodiff.ProbeSeries.__new__(autodiff.ProbeSeries)
    series.lat = lat
    series.nsteps, series.every, series.K = nsteps, every, K
    series.cells = torch.zeros((3, 2), dtype=torch.int32)
    series.nloss = nsteps // every
    series.nseg = (nsteps + K - 1) // K
    series.ck = lat.new_states(series.nseg)
    series.tape = lat.new_states(max(K - 1, 1))
    series._adj_ws = None
    series._generation = 0
    fake = FakeW(lat, series.tape.shape[1])
    monkeypatch.setattr(autodiff, "W", fake)
    out = series.run_forward(None, torch.zeros(8, 8), torch.zeros(4))
    assert [s for _, s in lat.log] == list(range(every, nsteps + 1, every))
    assert torch.equal(out[:, 0], torch.arange(every, nsteps + 1, every, dtype=torch.float32))
    series.run_backward(torch.zeros(series.nloss, 3), series._generation)
    assert fake.used == list(range(nsteps, 0, -1))
    assert fake.seeds == list(range((nsteps // every) * every, 0, -every))


def test_backward_after_newer_forward_is_refused(monkeypatch):
    lat = FakeLattice()
    series = autodiff.ProbeSeries.__new__(autodiff.ProbeSeries)
    series._generation = 2
    series.lat = lat
    with pytest.raises(RuntimeError):
        series.run_backward(torch.zeros(1, 1), 1)


def test_probe_cells_validated():
    lat = FakeLattice()
    with pytest.raises(ValueError):
        autodiff.ProbeSeries(lat, np.array([[8, 0]]), 10, 5)
