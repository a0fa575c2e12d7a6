"""Specular / specular-diffuse walls and internal sources on the GPU against
the FP64 oracle (1e-5 of the largest value, as for every forward field), on
ragged multi-tile lattices, and through the batched step."""
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


def _pair(nx, ny, q, kind, mfp_field, **kw):
    from paper_1911_00180_amd.lattice import Lattice
    lat = Lattice(nx, ny, q, mfp=10.0, dirs=kind, **kw)
    lat.set_mfp_field(torch.from_numpy(mfp_field.astype(np.float32)))
    okw = {k: v for k, v in kw.items() if k != "dir_split"}
    ora = o.Lattice(o.Config(nx=nx, ny=ny, q=q, dirs=kind,
                             mfp=mfp_field.astype(np.float32).astype(np.float64), **okw))
    return lat, ora


@pytest.mark.parametrize("p", [0.35, 1.0])
@pytest.mark.parametrize("x_edge", ["periodic", "blackbody"])
@pytest.mark.parametrize("q,kind", [(16, "uniform"), (24, "ring")])
def test_specular_walls(p, x_edge, q, kind):
    nx, ny = 77, 23
    mfp = inputs.smooth_lognormal_field(nx, ny, 5, 6.0, 6.0, 0.5, 2.0, 30.0)
    lat, ora = _pair(nx, ny, q, kind, mfp, x_edge=x_edge, y_edge="diffuse", y_specularity=p,
                     t_x_lo=1.0, t_x_hi=0.25)
    e0 = inputs.random_populations(9, q, ny, nx)
    lat.set_populations(torch.from_numpy(e0))
    ora.set_populations(e0.astype(np.float64))
    ora._apply_blackbody(ora.e)
    lat.step(40)
    ora.run(40)
    assert _rel(lat.populations().cpu().numpy(), ora.e) <= RTOL
    assert _rel(lat.temperature().cpu().numpy(), ora.temperature()) <= RTOL
    if x_edge == "periodic":
        e, _, _ = lat.totals()
        assert abs(e - ora.energy()) <= 1e-6 * ora.energy()


@pytest.mark.parametrize("q,kind,x_edge,y_edge", [(16, "uniform", "periodic", "periodic"),
                                                  (24, "ring", "blackbody", "diffuse"),
                                                  (32, "uniform", "blackbody", "blackbody")])
def test_sources(q, kind, x_edge, y_edge):
    nx, ny = 70, 45
    rng = np.random.default_rng(12)
    cells = np.array([[3, 4], [35, 22], [0, 10], [69, 44], [12, 0]], dtype=np.int32)
    vals = rng.uniform(0.0, 2.0, size=(len(cells), q)).astype(np.float32)
    mfp = inputs.smooth_lognormal_field(nx, ny, 6, 6.0, 8.0, 0.5, 2.0, 40.0)
    lat, ora = _pair(nx, ny, q, kind, mfp, x_edge=x_edge, y_edge=y_edge, t_x_lo=0.5,
                     t_y_hi=0.3)
    ora.cfg.source_cells = cells
    ora.cfg.source_values = vals.astype(np.float64)
    lat.set_sources(cells, vals)
    T0 = inputs.random_temperature(3, ny, nx)
    lat.set_temperature(torch.from_numpy(T0))
    ora.set_temperature(T0.astype(np.float64))
    assert _rel(lat.populations().cpu().numpy(), ora.e) <= RTOL
    lat.step(30)
    ora.run(30)
    assert _rel(lat.populations().cpu().numpy(), ora.e) <= RTOL
    got = lat.populations().cpu().numpy()
    for (x, y), v in zip(cells, vals):
        assert np.array_equal(got[:, y, x], v)


def test_flux_source_and_removal():
    from paper_1911_00180_amd import wormlbm as W
    from paper_1911_00180_amd.lattice import Lattice
    q = 32
    lat = Lattice(40, 30, q, mfp=12.0)
    e = W.wlbm_flux_distribution(lat.params, 1.0, 0.2, 0.0)
    lat.set_sources(np.array([[20, 15]]), e[None, :])
    lat.set_temperature(torch.zeros((30, 40)))
    qx, qy = lat.heat_flux()
    assert qx[15, 20].item() == pytest.approx(0.2, abs=1e-6)
    assert qy[15, 20].item() == pytest.approx(0.0, abs=1e-6)
    lat.step(5)
    assert lat.temperature()[15, 20].item() == pytest.approx(1.0, rel=1e-6)
    lat.set_sources(None, None)
    lat.step(1)
    assert lat.temperature()[15, 20].item() != pytest.approx(1.0, rel=1e-3)
    with pytest.raises(W.WormLBMError):
        lat.set_sources(np.array([[1, 1], [1, 1]]), np.zeros((2, q)))
    with pytest.raises(W.WormLBMError):
        lat.set_sources(np.array([[40, 1]]), np.zeros((1, q)))
    lat.close()


def test_batch_with_sources_and_specular_walls():
    from paper_1911_00180_amd.lattice import Batch, Lattice
    q = 16
    cfgs = [dict(nx=70, ny=21, y_edge="diffuse", y_specularity=0.6, x_edge="blackbody",
                 t_x_lo=1.0),
            dict(nx=40, ny=40, y_edge="diffuse", y_specularity=1.0),
            dict(nx=33, ny=50)]
    rng = np.random.default_rng(2)

    def make():
        lats = []
        for k, c in enumerate(cfgs):
            lat = Lattice(c["nx"], c["ny"], q, mfp=7.0, sched_chunk=16,
                          **{a: b for a, b in c.items() if a not in ("nx", "ny")})
            lat.set_populations(torch.from_numpy(
                inputs.random_populations(k, q, c["ny"], c["nx"])))
            lats.append(lat)
        return lats

    srcs = [(np.array([[5, 5], [10, 3]]), rng.uniform(0, 1, (2, q))), None,
            (np.array([[0, 0]]), rng.uniform(0, 1, (1, q)))]
    a, b = make(), make()
    for lats in (a, b):
        for lat, sv in zip(lats, srcs):
            if sv is not None:
                lat.set_sources(*sv)
    batch = Batch(a)
    batch.step(37)
    for lat in b:
        lat.step(37)
    for x, y in zip(a, b):
        assert torch.equal(x.populations(), y.populations())
    batch.close()


def test_adjoint_rejects_sources():
    from paper_1911_00180_amd import wormlbm as W
    from paper_1911_00180_amd.lattice import Lattice
    lat = Lattice(32, 32, 16, mfp=5.0)
    lat.set_sources(np.array([[3, 3]]), np.ones((1, 16)))
    ws = torch.empty(W.wlbm_adjoint_bytes(lat.handle), dtype=torch.uint8, device="cuda")
    with pytest.raises(W.WormLBMError):
        W.wlbm_adjoint_begin(lat.handle, ws.data_ptr(), ws.numel(), 10)
    lat.close()


def test_specular_walls_uniform_weight():
    from paper_1911_00180_amd.lattice import Lattice
    nx, ny, q = 130, 9, 32
    lat = Lattice(nx, ny, q, mfp=4.0, y_edge="diffuse", y_specularity=0.5)
    ora = o.Lattice(o.Config(nx=nx, ny=ny, q=q, mfp=4.0, y_edge="diffuse", y_specularity=0.5))
    e0 = inputs.random_populations(19, q, ny, nx)
    lat.set_populations(torch.from_numpy(e0))
    ora.set_populations(e0.astype(np.float64))
    lat.step(50)
    ora.run(50)
    assert _rel(lat.populations().cpu().numpy(), ora.e) <= RTOL
