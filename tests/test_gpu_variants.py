"""Angle-dependent grid speeds and multigray bands on the GPU against the FP64
oracle (1e-5 of the largest value)."""
import numpy as np
import pytest

from oracle import worm_lbm as o
from paper_1911_00180_amd import inputs

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


@pytest.mark.parametrize("q,kind,edges", [
    (16, "uniform", dict(x_edge="blackbody", y_edge="diffuse", t_x_lo=1.0)),
    (24, "ring", dict()),
    (32, "uniform", dict(y_edge="diffuse", y_specularity=0.5))])
def test_angle_dependent_speeds(q, kind, edges):
    from paper_1911_00180_amd.lattice import Lattice
    nx, ny = 75, 33
    rng = np.random.default_rng(q)
    v = rng.uniform(0.25, 1.0, size=q)
    v[::4] = 1.0
    mfp = inputs.smooth_lognormal_field(nx, ny, 2, 6.0, 8.0, 0.5, 2.0, 40.0).astype(np.float32)
    lat = Lattice(nx, ny, q, mfp=10.0, dirs=kind, **edges)
    lat.set_mfp_field(torch.from_numpy(mfp))
    lat.set_speeds(v)
    ora = o.Lattice(o.Config(nx=nx, ny=ny, q=q, dirs=kind, mfp=mfp.astype(np.float64),
                             speeds=v, **edges))
    T0 = inputs.gaussian_pulse(nx, ny, 5.0, 30, 15).astype(np.float32)
    lat.set_temperature(torch.from_numpy(T0))
    ora.set_temperature(T0.astype(np.float64))
    lat.step(60)
    ora.run(60)
    assert _rel(lat.populations().cpu().numpy(), ora.e) <= RTOL
    lat.close()


def test_speeds_only_at_step_zero_and_batches_take_unequal_speeds():
    from paper_1911_00180_amd import wormlbm as W
    from paper_1911_00180_amd.lattice import Batch, Lattice
    a = Lattice(40, 30, 16, mfp=5.0)
    b = Lattice(40, 30, 16, mfp=5.0)
    b.set_speeds(np.full(16, 0.5))
    a2 = Lattice(40, 30, 16, mfp=5.0)
    b2 = Lattice(40, 30, 16, mfp=5.0)
    b2.set_speeds(np.full(16, 0.5))
    T0 = torch.from_numpy(inputs.random_temperature(3, 30, 40))
    for lat in (a, b, a2, b2):
        lat.set_temperature(T0)
    batch = Batch([a, b])          # two schedules in one launch per step
    batch.step(21)
    a2.step(21)
    b2.step(21)
    assert torch.equal(a.populations(), a2.populations())
    assert torch.equal(b.populations(), b2.populations())
    assert not torch.equal(a.populations(), b.populations())
    batch.close()
    for lat in (a, b, a2, b2):
        lat.close()
    c = Lattice(40, 30, 16, mfp=5.0)
    with pytest.raises(W.WormLBMError):
        c.set_speeds(np.full(16, 1.5))     # above one cell per step
    c.step(1)
    with pytest.raises(W.WormLBMError):
        c.set_speeds(np.full(16, 0.5))     # only at step 0
    c.close()


@pytest.mark.parametrize("speeds", [(1.0, 0.7, 0.4), (1.0, 1.0, 1.0)])
def test_multigray_superposition(speeds):
    """Three uncoupled bands (heat-capacity shares 0.5 / 0.3 / 0.2, MFPs 4 / 20
    / 200 cells) against the superposed oracle bands; with the blackbody wall
    both speed sets take the batched path (unequal speeds as separate
    schedules in one launch per step)."""
    from paper_1911_00180_amd.multigray import Multigray
    nx, ny, q = 66, 40, 16
    bands = [(0.5, speeds[0], 4.0), (0.3, speeds[1], 20.0), (0.2, speeds[2], 200.0)]
    mg = Multigray(nx, ny, q, bands, x_edge="blackbody", t_x_lo=1.0)
    assert mg.batch is not None
    T0 = inputs.gaussian_pulse(nx, ny, 6.0, 33, 20).astype(np.float32)
    mg.set_temperature(torch.from_numpy(T0))
    mg.step(45)
    got = mg.temperature().cpu().numpy()
    want = np.zeros((ny, nx))
    for c, v, mfp in bands:
        ora = o.Lattice(o.Config(nx=nx, ny=ny, q=q, mfp=mfp, x_edge="blackbody",
                                 t_x_lo=c * 1.0, speeds=np.full(q, v)))
        ora.set_temperature(c * T0.astype(np.float64))
        ora.run(45)
        want += ora.temperature()
    want /= sum(c for c, _, _ in bands)
    assert _rel(got, want) <= RTOL
    mg.close()
