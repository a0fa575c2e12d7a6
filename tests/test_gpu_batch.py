"""Batched stepping, the split autotuner and the film readout on the GPU.

A batch step runs the same tile code as a single-lattice step, so batched
and one-by-one runs must agree bit for bit.  The film conductivity is
checked against the FP64 oracle (oracle/film.py): the window-averaged
column flux within 1e-5 of the wall temperature difference (the flux is a
sum of terms of either sign, so its error is measured against the
temperature scale, as for every flux check).
"""
import numpy as np
import pytest

from oracle import film as ofilm
from oracle import worm_lbm as o
from paper_1911_00180_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_00180_amd import wormlbm
    wormlbm.lib()


MIXED = [
    dict(nx=70, ny=45, mfp=6.0, x_edge="blackbody", y_edge="diffuse", t_x_lo=1.0),
    dict(nx=64, ny=64, mfp=20.0),
    dict(nx=131, ny=9, mfp=3.0, x_edge="periodic", y_edge="blackbody", t_y_lo=0.5),
    dict(nx=33, ny=100, mfp=1e4, x_edge="blackbody", y_edge="periodic", t_x_hi=2.0),
    dict(nx=200, ny=17, mfp=2.5, x_edge="blackbody", y_edge="blackbody", t_x_lo=1.0,
         t_y_hi=0.25),
]


def _make(q, cfg, seed, **kw):
    from paper_1911_00180_amd.lattice import Lattice
    lat = Lattice(cfg["nx"], cfg["ny"], q, **{k: v for k, v in cfg.items() if k not in
                                               ("nx", "ny")}, **kw)
    lat.set_populations(torch.from_numpy(inputs.random_populations(seed, q, cfg["ny"],
                                                                   cfg["nx"])))
    return lat


@pytest.mark.parametrize("q,split", [(16, 0), (32, 4), (24, 1)])
def test_batch_equals_one_by_one(q, split):
    from paper_1911_00180_amd.lattice import Batch
    kw = dict(dir_split=split, sched_chunk=16)
    a = [_make(q, c, 10 + k, **kw) for k, c in enumerate(MIXED)]
    b = [_make(q, c, 10 + k, **kw) for k, c in enumerate(MIXED)]
    for lat in a + b:
        lat.set_flux_window(5)
    batch = Batch(a)
    batch.step(37)          # crosses two schedule chunks, ends on odd parity
    batch.step(6)
    for lat in b:
        lat.step(37)
        lat.step(6)
    for x, y in zip(a, b):
        assert x.step_count == y.step_count == 43
        assert torch.equal(x.populations(), y.populations())
        assert torch.equal(x.temperature(), y.temperature())
        for u, v in zip(x.heat_flux(averaged=True), y.heat_flux(averaged=True)):
            assert torch.equal(u, v)
        assert x.flux_mean(averaged=True) == y.flux_mean(averaged=True)
    batch.close()
    for lat in a + b:
        lat.close()


def test_batch_rejects_mismatched_lattices():
    from paper_1911_00180_amd import wormlbm as W
    from paper_1911_00180_amd.lattice import Batch
    a = _make(16, MIXED[0], 1, dir_split=1)
    b = _make(32, MIXED[1], 2, dir_split=2)
    with pytest.raises(W.WormLBMError):
        Batch([a, b])          # splits differ
    b.close()
    b = _make(16, MIXED[1], 2, dir_split=1)
    b.set_mfp_field(torch.full((MIXED[1]["ny"], MIXED[1]["nx"]), 7.0))
    with pytest.raises(W.WormLBMError):
        Batch([a, b])          # per-cell field use differs
    c = _make(16, MIXED[1], 3, dir_split=1)
    c.step(1)
    with pytest.raises(W.WormLBMError):
        Batch([a, c])
    with pytest.raises(W.WormLBMError):
        Batch([a, a])
    for lat in (a, b, c):
        lat.close()


def test_autotune_restores_state_and_keeps_a_valid_split():
    lat = _make(64, dict(nx=300, ny=200, mfp=12.0, x_edge="blackbody", y_edge="diffuse",
                         t_x_lo=1.0), 4)
    lat.step(7)
    before = lat.populations()
    ms, chosen = lat.autotune(steps=5)
    assert chosen in (1, 2, 4) and lat.dir_split == chosen
    assert all(m > 0 for m in ms)
    assert lat.step_count == 7
    assert torch.equal(lat.populations(), before)
    lat.close()


@pytest.mark.parametrize("kn,ny", [(0.3, 8), (2.0, 12), (20.0, 16)])
def test_film_flux_matches_oracle(kn, ny):
    from paper_1911_00180_amd.films import FilmSweep
    nx, q, n = 48, 16, 1500
    sweep = FilmSweep([(kn, ny, kn * ny)], nx=nx, q=q)
    sweep.step_batched(n)
    qx, _ = sweep.lattices[0].flux_mean(1, nx - 1, averaged=True)
    cfg = o.Config(nx=nx, ny=ny, q=q, mfp=kn * ny, x_edge="blackbody", y_edge="diffuse",
                   t_x_lo=1.0, t_x_hi=0.0)
    _, oqx, _ = ofilm.film_run(cfg, n, window=10)
    assert abs(qx - float(np.mean(oqx[:, 1:nx - 1]))) <= 1e-5
    k = sweep.kappa_ratios()[0]
    assert k == pytest.approx(ofilm.kappa_ratio(cfg, oqx), abs=1e-5 * (nx - 1) / (kn * ny / 2))
    sweep.close()


def test_film_sweep_full_size_batched_equals_one_by_one():
    """The 24-film sweep at full size (Nx = 512, Q = 128) in the launch
    configuration the bench times: batched and one-by-one agree bit for bit."""
    from paper_1911_00180_amd.films import FilmSweep, film_set
    films = film_set()
    a = FilmSweep(films)
    b = FilmSweep(films)
    a.step_batched(60)
    b.step_each(60)
    for x, y in zip(a.lattices, b.lattices):
        assert torch.equal(x.temperature(), y.temperature())
    ka, kb = a.kappa_ratios(), b.kappa_ratios()
    assert ka == kb
    assert all(np.isfinite(ka))
    a.close()
    b.close()


def test_batch_graph_replays_equal_step_by_step():
    """Whole schedule chunks replayed as captured HIP graphs give the bits of
    step-by-step launches and of one-by-one lattices, over repeated replays
    of both ring slots with eager work between them (reads, new wall
    temperatures, a per-cell field that makes the batch capture again), and
    with chunk remainders that shift the buffer parity between calls."""
    from paper_1911_00180_amd import wormlbm as W
    from paper_1911_00180_amd.lattice import Batch
    q = 16
    kw = dict(sched_chunk=16)
    sets = [[_make(q, c, 30 + k, **kw) for k, c in enumerate(MIXED)] for _ in range(3)]
    graphed, eager, single = sets
    bg, be = Batch(graphed), Batch(eager)
    be.set_graphs(False)
    with pytest.raises(W.WormLBMError):
        W.wlbm_batch_set_graphs(bg.handle, 2)
    mfp = {id(c): torch.from_numpy(inputs.smooth_lognormal_field(c["nx"], c["ny"], 5, 4.0, 6.0,
                                                                 0.5, 2.0, 30.0)
                                   .astype(np.float32)) for c in MIXED}
    for call, n in enumerate((32, 16, 7, 48, 16, 33, 32, 48)):
        if call == 3:
            for lats in sets:
                for lat, c in zip(lats, MIXED):
                    lat.set_mfp_field(mfp[id(c)])
        if call == 5:
            for lats in sets:
                for lat in lats:
                    lat.set_wall_temperatures(0.75, 0.125, 0.5, 0.25)
        if call == 6:
            # every lattice stepped on its own by an odd count: the buffers
            # swap, and the next batch call's table (not the graph) follows
            for lats in sets:
                for lat in lats:
                    lat.step(3)
        bg.step(n)
        be.step(n)
        for lat in single:
            lat.step(n)
        for x, y, z in zip(graphed, eager, single):
            assert x.step_count == y.step_count == z.step_count
            assert torch.equal(x.populations(), y.populations()), (call, n)
            assert torch.equal(x.populations(), z.populations()), (call, n)
            assert torch.equal(x.temperature(), z.temperature()), (call, n)
    bg.close()
    be.close()
    for lats in sets:
        for lat in lats:
            lat.close()


def test_batch_of_different_direction_sets_equals_one_by_one():
    """Lattices with different Q, direction sets and grid speeds in one
    batch (each direction set has its own schedule ring; one launch per step
    covers all of them) give the bits of stepping each lattice alone; a
    member whose grid speeds change after the batch was made is refused."""
    from paper_1911_00180_amd import wormlbm as W
    from paper_1911_00180_amd.lattice import Batch
    specs = [(16, "uniform", False), (32, "ring", False), (24, "uniform", False),
             (16, "uniform", True), (48, "ring", False), (16, "uniform", False)]
    kw = dict(dir_split=1, sched_chunk=16)

    def build(seed0):
        lats = []
        for k, (q, kind, slow) in enumerate(specs):
            lat = _make(q, MIXED[k % len(MIXED)], seed0 + k, dirs=kind, **kw)
            if slow:
                lat.set_speeds(np.linspace(0.55, 1.0, q))
            lats.append(lat)
        return lats

    a, b = build(60), build(60)
    batch = Batch(a)
    for n in (37, 16, 5, 32):
        batch.step(n)
        for lat in b:
            lat.step(n)
        for x, y in zip(a, b):
            assert x.step_count == y.step_count
            assert torch.equal(x.populations(), y.populations()), (x.q, n)
            assert torch.equal(x.temperature(), y.temperature()), (x.q, n)
    batch.close()
    for lat in a + b:
        lat.close()
    c = build(70)
    batch = Batch(c)
    c[0].set_speeds(np.full(16, 0.8))
    with pytest.raises(W.WormLBMError):
        batch.step(1)
    batch.close()
    for lat in c:
        lat.close()


@pytest.mark.parametrize("q,per_cell,fusion", [(128, False, 1), (64, True, 1), (32, False, 3),
                                               (16, False, 4), (256, False, 1), (128, False, 3),
                                               (120, True, 4), (88, False, 2)])
def test_batched_multi_step_launches_keep_the_bits_of_single_steps(q, per_cell, fusion):
    """Films of several thicknesses (blackbody x, diffuse y) and a periodic and a
    blackbody-y lattice in one batch: the batch advances several steps per launch
    for all of them (each lattice's block height, one table of pull offsets per
    geometry), and matches lattices stepped one step per launch bit for bit,
    across schedule chunks, odd launch counts and a flux window."""
    from paper_1911_00180_amd.lattice import Batch
    cfgs = [dict(nx=150, ny=ny, mfp=mfp, x_edge="blackbody", y_edge="diffuse", t_x_lo=1.0,
                 t_x_hi=0.1) for ny, mfp in ((8, 2.0), (23, 9.0), (40, 30.0), (8, 5.0))]
    cfgs += [dict(nx=97, ny=30, mfp=12.0),
             dict(nx=64, ny=17, mfp=4.0, x_edge="periodic", y_edge="blackbody", t_y_lo=0.3)]
    kw = dict(sched_chunk=24)
    a = [_make(q, c, 40 + k, step_fusion=fusion, **kw) for k, c in enumerate(cfgs)]
    b = [_make(q, c, 40 + k, step_fusion=0, **kw) for k, c in enumerate(cfgs)]
    if per_cell:
        for x, y, c in zip(a, b, cfgs):
            f = torch.from_numpy(inputs.smooth_lognormal_field(c["nx"], c["ny"], 3, 4.0, 8.0,
                                                               0.5, 2.0, 30.0)
                                 .astype(np.float32))
            x.set_mfp_field(f)
            y.set_mfp_field(f)
    for lat in a + b:
        lat.set_flux_window(3)
    batch = Batch(a)
    for n in (50, 7, 24):
        batch.step(n)
        for lat in b:
            lat.step(n)
        for x, y in zip(a, b):
            assert x.step_count == y.step_count
            assert torch.equal(x.populations(), y.populations()), n
            for u, v in zip(x.heat_flux(averaged=True), y.heat_flux(averaged=True)):
                assert torch.equal(u, v)
            assert x.flux_mean(averaged=True) == y.flux_mean(averaged=True), n
    batch.close()
    for lat in a + b:
        lat.close()


def test_batch_block_height_tuner_restores_states_and_keeps_the_bits():
    """wlbm_batch_tune_block_rows: one height for every member, chosen among
    the candidates; the members end at their states and step counts, and the
    tuned batch keeps the bits of an untuned twin."""
    from paper_1911_00180_amd.lattice import Batch
    cfgs = [dict(nx=150, ny=ny, mfp=mfp, x_edge="blackbody", y_edge="diffuse", t_x_lo=1.0,
                 t_x_hi=0.1) for ny, mfp in ((8, 2.0), (23, 9.0), (40, 30.0))]
    a = [_make(64, c, 60 + k) for k, c in enumerate(cfgs)]
    b = [_make(64, c, 60 + k) for k, c in enumerate(cfgs)]
    for x in a + b:
        x.set_flux_window(5)
    ba, bb = Batch(a), Batch(b)
    k = ba.steps_per_launch
    assert k >= 2
    ba.step(24)
    bb.step(24)
    before = [x.populations().clone() for x in a]
    rows = ba.tune_block_rows(launches=2)
    assert rows >= 1 and (rows + 2 * (k - 1)) % 3 == 0
    for x, p0 in zip(a, before):
        assert x.step_count == 24
        assert x.block_rows(k) == rows
        assert torch.equal(x.populations(), p0)
    for n in (40, 7):
        ba.step(n)
        bb.step(n)
        for x, y in zip(a, b):
            assert torch.equal(x.populations(), y.populations()), n
            for u, v in zip(x.heat_flux(averaged=True), y.heat_flux(averaged=True)):
                assert torch.equal(u, v)
    ba.close()
    bb.close()
    for x in a + b:
        x.close()
