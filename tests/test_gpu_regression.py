"""The paper's benchmark set-ups on the GPU: the one-pixel source (Sec. 3.1),
cross-plane transport in the Fourier limit (Sec. 3.4, Eq. 1DT) and the one
hot - three cold walls (Sec. 3.6, Eq. 2DT).  Each runs against the FP64
oracle (1e-5 of the largest value, as for every forward field) on a short
run, and its physics is checked on the GPU's own longer run against the
same closed forms the oracle is pinned to."""
import math

import numpy as np
import pytest

import pins
from oracle import worm_lbm as o

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
RTOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_00180_amd import wormlbm
    wormlbm.lib()


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64) - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("q", [8, 16, 32, 512])
@pytest.mark.parametrize("mfp", [math.inf, 25.0])
def test_one_pixel_source(q, mfp):
    """51 x 51 periodic, the centre pixel held at T = 1 by an isotropic
    source, ring direction sets of the paper's figure, 20 steps."""
    from paper_1911_00180_amd.lattice import Lattice
    N, n = 51, 20
    c = N // 2
    lat = Lattice(N, N, q, mfp=mfp, dirs="ring")
    ora0 = o.Lattice(o.Config(nx=N, ny=N, q=q, dirs="ring", mfp=mfp))
    vals = ora0.w[None, :]
    cells = np.array([[c, c]], dtype=np.int32)
    lat.set_sources(cells, vals.astype(np.float32))
    ora = o.Lattice(o.Config(nx=N, ny=N, q=q, dirs="ring", mfp=mfp, source_cells=cells,
                             source_values=vals.astype(np.float32).astype(np.float64)))
    lat.set_temperature(torch.zeros((N, N)))
    ora.set_temperature(np.zeros((N, N)))
    lat.step(n)
    ora.run(n)
    T = lat.temperature().cpu().numpy()
    assert _rel(T, ora.temperature()) <= RTOL
    if math.isinf(mfp):
        x = np.arange(N) - c
        r = np.sqrt(x[None, :] ** 2 + x[:, None] ** 2)
        lit = T > 0
        assert r[lit].max() <= n + 1
        if q >= 2 * math.pi * n:
            assert lit[r <= n - 2].all()
    lat.close()


def test_cross_plane_fourier():
    """Ny = 1, blackbody walls T = 1 / 0, MFP 2 cells, Q = 16: parity with the
    oracle over 2000 steps, then the GPU run to 40000 steps against Eq. 1DT
    (the transient at 6000 steps, the linear steady state and a uniform
    flux at the end)."""
    from paper_1911_00180_amd.lattice import Lattice
    nx, mfp, q = 101, 2.0, 16
    L = nx - 1
    X = np.arange(nx) / L
    kw = dict(x_edge="blackbody", t_x_lo=1.0, t_x_hi=0.0)
    lat = Lattice(nx, 1, q, mfp=mfp, **kw)
    ora = o.Lattice(o.Config(nx=nx, ny=1, q=q, mfp=mfp, **kw))
    lat.set_temperature(torch.zeros((1, nx)))
    ora.set_temperature(np.zeros((1, nx)))
    lat.step(2000)
    ora.run(2000)
    assert _rel(lat.temperature().cpu().numpy(), ora.temperature()) <= RTOL
    lat.step(4000)
    T = lat.temperature().cpu().numpy()[0].astype(np.float64)
    ref = pins._cross_plane_series(X, (mfp / 2.0) * 6000 / L ** 2)
    assert np.abs(T - ref).max() < 0.012
    lat.step(34000 - 10)
    lat.set_flux_window(10)
    lat.step(10)
    T = lat.temperature().cpu().numpy()[0].astype(np.float64)
    assert np.abs(T - (1.0 - X))[1:-1].max() < 0.015
    qx, _ = lat.heat_flux(averaged=True)
    qx = qx.cpu().numpy()[0, 5:-5].astype(np.float64)
    assert (qx.max() - qx.min()) < 0.02 * qx.mean()
    # Fourier's law with kappa = MFP / 2 (C = v = 1) across the slab, up to
    # terms of order 1 / MFP (the oracle gives 1.12 x at MFP 2)
    assert abs(qx.mean() / ((mfp / 2.0) / L) - 1.0) < 0.15
    lat.close()


def test_one_hot_three_cold():
    """Blackbody walls, the upper one hot: parity with the oracle on 32 x 32
    over 500 steps, then 64 x 64 (MFP 1.5, Q = 16) run to steady state on the
    GPU against the Laplace series of Eq. 2DT in the middle half."""
    from paper_1911_00180_amd.lattice import Lattice
    kw = dict(x_edge="blackbody", y_edge="blackbody", t_y_hi=1.0)
    N = 32
    lat = Lattice(N, N, 16, mfp=1.5, **kw)
    ora = o.Lattice(o.Config(nx=N, ny=N, q=16, mfp=1.5, **kw))
    lat.set_temperature(torch.zeros((N, N)))
    ora.set_temperature(np.zeros((N, N)))
    lat.step(500)
    ora.run(500)
    assert _rel(lat.temperature().cpu().numpy(), ora.temperature()) <= RTOL
    lat.close()
    N = 64
    lat = Lattice(N, N, 16, mfp=1.5, **kw)
    lat.set_temperature(torch.zeros((N, N)))
    lat.step(30000)
    T = lat.temperature().cpu().numpy().astype(np.float64)
    X = np.arange(N)[None, :] / (N - 1)
    Y = np.arange(N)[:, None] / (N - 1)
    mid = slice(N // 4, 3 * N // 4 + 1)
    assert np.abs(T - pins.one_hot_three_cold_series(X, Y))[mid, mid].max() < 0.012
    lat.close()
