"""GPU path (HIP kernels through the C-ABI) against the FP64 oracle.

Tolerances: the worm/TAS schedule and W = 0 (pure advection) runs are
bit-exact; otherwise the FP32 fields must satisfy
max|x32 - x64| <= 1e-5 * max|x64| (temperature, populations).  The heat flux
is a sum of terms of either sign that can cancel to far below their own size
(|q| <= v_g T), so its error is measured against max|T64|.
"""
import math

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
    wormlbm.lib()  # the HIP library must be there; no fallback


def _lattice(**kw):
    from paper_1911_00180_amd.lattice import Lattice
    return Lattice(**kw)


def _oracle(nx, ny, q, mfp, **kw):
    okw = {k: v for k, v in kw.items() if k in ("dirs", "emulate_3d", "mfp_correction", "x_edge",
                                                "y_edge", "t_x_lo", "t_x_hi", "t_y_lo",
                                                "t_y_hi")}
    return o.Lattice(o.Config(nx=nx, ny=ny, q=q, mfp=mfp, **okw))


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64) - b)) / max(np.max(np.abs(b)), 1e-300))


def _run_pair(nx, ny, q, mfp, nsteps, T0=None, e0=None, mfp_field=None, **kw):
    """Same seeded input into the GPU lattice and the oracle; returns both."""
    lat = _lattice(nx=nx, ny=ny, q=q, mfp=mfp if mfp_field is None else 10.0, **kw)
    ora = _oracle(nx, ny, q, mfp if mfp_field is None else mfp_field.astype(np.float64), **kw)
    if mfp_field is not None:
        lat.set_mfp_field(torch.from_numpy(mfp_field.astype(np.float32)))
    if T0 is not None:
        lat.set_temperature(torch.from_numpy(T0.astype(np.float32)))
        ora.set_temperature(T0.astype(np.float32).astype(np.float64))
    else:
        lat.set_populations(torch.from_numpy(e0.astype(np.float32)))
        ora.set_populations(e0.astype(np.float32).astype(np.float64))
        ora._apply_blackbody(ora.e)
    lat.step(nsteps)
    ora.run(nsteps)
    return lat, ora


def test_c1_gaussian_64x64_q16():
    """64 x 64 periodic, Q = 16 evenly spaced, MFP 16, Gaussian pulse
    (sigma 4, amplitude 1) centred, 200 steps: T and q."""
    T0 = inputs.gaussian_pulse(64, 64, 4.0, 32, 32)
    lat, ora = _run_pair(64, 64, 16, 16.0, 200, T0=T0)
    assert _rel(lat.temperature().cpu().numpy(), ora.temperature()) <= RTOL
    qx, qy = lat.heat_flux()
    oqx, oqy = ora.heat_flux()
    scale = np.abs(ora.temperature()).max()
    assert np.abs(qx.cpu().numpy() - oqx).max() <= RTOL * scale
    assert np.abs(qy.cpu().numpy() - oqy).max() <= RTOL * scale
    e, sqx, sqy = lat.totals()
    assert abs(e - ora.energy()) <= 1e-6 * ora.energy()


@pytest.mark.parametrize("q,kind,nx,ny", [(16, "uniform", 70, 45), (24, "ring", 131, 67),
                                          (64, "uniform", 200, 9)])
def test_ballistic_bit_exact(q, kind, nx, ny):
    """W = 0: every population is a pure shift of its initial value, bit for
    bit (exact advection, no smearing)."""
    e0 = inputs.random_populations(5, q, ny, nx)
    lat, ora = _run_pair(nx, ny, q, math.inf, 37, e0=e0, dirs=kind)
    got = lat.populations().cpu().numpy()
    assert np.array_equal(got.astype(np.float64), ora.e)


EDGE_CASES = [
    dict(x_edge="blackbody", y_edge="diffuse", t_x_lo=1.0, t_x_hi=0.0),
    dict(x_edge="periodic", y_edge="diffuse"),
    dict(x_edge="blackbody", y_edge="periodic", t_x_lo=0.3, t_x_hi=0.8),
    dict(x_edge="blackbody", y_edge="blackbody", t_x_lo=1.0, t_x_hi=0.0, t_y_lo=0.25,
         t_y_hi=0.75),
    dict(x_edge="periodic", y_edge="blackbody", t_y_lo=0.5, t_y_hi=0.1),
    dict(x_edge="periodic", y_edge="periodic"),
]


@pytest.mark.parametrize("edges", EDGE_CASES, ids=lambda d: f"{d['x_edge']}-{d['y_edge']}")
@pytest.mark.parametrize("kind,q", [("uniform", 32), ("ring", 16)])
def test_walls_ragged(edges, kind, q):
    """Every edge combination on a ragged lattice (several tiles, partial
    last tiles), strong scattering, random initial populations."""
    nx, ny = 133, 37
    e0 = inputs.random_populations(11, q, ny, nx)
    lat, ora = _run_pair(nx, ny, q, 4.0, 60, e0=e0, dirs=kind, **edges)
    got = lat.populations().cpu().numpy()
    assert _rel(got, ora.e) <= RTOL
    assert _rel(lat.temperature().cpu().numpy(), ora.temperature()) <= RTOL


@pytest.mark.parametrize("split", [1, 2, 4])
@pytest.mark.parametrize("edges", [dict(x_edge="blackbody", y_edge="diffuse", t_x_lo=1.0),
                                   dict(x_edge="periodic", y_edge="periodic")],
                         ids=["walls", "periodic"])
def test_direction_splits_agree(split, edges):
    """Every split of the directions over waves gives the oracle's answer
    (and the flux window, which is summed across the split, too)."""
    nx, ny, q = 300, 70, 32
    e0 = inputs.random_populations(3, q, ny, nx)
    lat = _lattice(nx=nx, ny=ny, q=q, mfp=6.0, dir_split=split, **edges)
    ora = _oracle(nx, ny, q, 6.0, **edges)
    lat.set_populations(torch.from_numpy(e0))
    ora.set_populations(e0.astype(np.float64))
    ora._apply_blackbody(ora.e)
    lat.set_flux_window(5)
    lat.step(40)
    oqx, oqy = ora.run(40, flux_window=5)
    assert _rel(lat.populations().cpu().numpy(), ora.e) <= RTOL
    assert _rel(lat.temperature().cpu().numpy(), ora.temperature()) <= RTOL
    qx, qy = lat.heat_flux(averaged=True)
    scale = np.abs(ora.temperature()).max()
    assert np.abs(qx.cpu().numpy() - oqx).max() <= RTOL * scale
    assert np.abs(qy.cpu().numpy() - oqy).max() <= RTOL * scale


def test_per_cell_mfp_field():
    """Per-cell relaxation: a smooth lognormal MFP field (4 .. 64 cells)."""
    nx, ny, q = 96, 80, 16
    mfp = inputs.smooth_lognormal_field(nx, ny, seed=1, corr=8.0, median=16.0,
                                        log_spread=math.log(4.0) / 2, lo=4.0, hi=64.0)
    T0 = inputs.gaussian_pulse(nx, ny, 8.0, nx / 2, ny / 2)
    lat, ora = _run_pair(nx, ny, q, None, 150, T0=T0, mfp_field=mfp,
                         x_edge="blackbody", t_x_lo=0.5, y_edge="periodic")
    assert _rel(lat.temperature().cpu().numpy(), ora.temperature()) <= RTOL
    assert _rel(lat.populations().cpu().numpy(), ora.e) <= RTOL


def test_per_cell_field_with_diffuse_walls():
    nx, ny, q = 77, 29, 24
    mfp = inputs.smooth_lognormal_field(nx, ny, seed=4, corr=5.0, median=8.0,
                                        log_spread=0.5, lo=2.0, hi=40.0)
    e0 = inputs.random_populations(6, q, ny, nx)
    lat, ora = _run_pair(nx, ny, q, None, 50, e0=e0, mfp_field=mfp, dirs="ring",
                         x_edge="periodic", y_edge="diffuse")
    assert _rel(lat.populations().cpu().numpy(), ora.e) <= RTOL


def test_flux_window_average():
    """q averaged over the last 10 steps (Sec. 3.4) against the oracle."""
    nx, ny, q = 120, 40, 32
    lat = _lattice(nx=nx, ny=ny, q=q, mfp=20.0, x_edge="blackbody", y_edge="diffuse",
                   t_x_lo=1.0, t_x_hi=0.0)
    ora = _oracle(nx, ny, q, 20.0, x_edge="blackbody", y_edge="diffuse", t_x_lo=1.0, t_x_hi=0.0)
    T0 = np.zeros((ny, nx))
    lat.set_temperature(torch.zeros(ny, nx))
    ora.set_temperature(T0)
    lat.set_flux_window(10)
    lat.step(90)
    qx, qy = lat.heat_flux(averaged=True)
    oqx, oqy = ora.run(90, flux_window=10)
    scale = np.abs(ora.temperature()).max()
    assert np.abs(qx.cpu().numpy() - oqx).max() <= RTOL * scale
    assert np.abs(qy.cpu().numpy() - oqy).max() <= RTOL * scale
    from paper_1911_00180_amd import wormlbm as W
    lat.step(5)  # fewer steps than the window: no valid average
    with pytest.raises(W.WormLBMError) as ei:
        lat.heat_flux(averaged=True)
    assert ei.value.status == W.WLBM_ESTATE


def test_cross_plane_ballistic_wall():
    """Ny = 1 periodic, blackbody x walls, W = 0, Q = 64 (Sec. 3.4 set-up)."""
    nx, q, n = 130, 64, 100
    kw = dict(x_edge="blackbody", t_x_lo=1.0, t_x_hi=0.0)
    lat, ora = _run_pair(nx, 1, q, math.inf, n, T0=np.zeros((1, nx)), **kw)
    assert np.array_equal(lat.populations().cpu().numpy().astype(np.float64), ora.e)


def test_deterministic_and_chunk_independent():
    nx, ny, q = 150, 90, 32
    T0 = inputs.gaussian_pulse(nx, ny, 6.0, 40, 50)
    out = []
    for chunk in (16, 256, 16):
        lat = _lattice(nx=nx, ny=ny, q=q, mfp=7.0, y_edge="diffuse", sched_chunk=chunk)
        lat.set_temperature(torch.from_numpy(T0.astype(np.float32)))
        for k in (1, 30, 69):          # step in uneven pieces
            lat.step(k)
        out.append(lat.populations().cpu().numpy())
        assert lat.step_count == 100
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def test_unstable_mfp_field_rejected_and_previous_kept():
    from paper_1911_00180_amd import wormlbm as W
    nx, ny, q = 40, 30, 16
    lat = _lattice(nx=nx, ny=ny, q=q, mfp=10.0)
    good = torch.full((ny, nx), 5.0)
    lat.set_mfp_field(good)
    bad = good.clone()
    bad[3, 4] = 0.5                  # W_corr > 1
    with pytest.raises(W.WormLBMError) as ei:
        lat.set_mfp_field(bad)
    assert ei.value.status == W.WLBM_EUNSTABLE
    bad[3, 4] = -1.0
    with pytest.raises(W.WormLBMError):
        lat.set_mfp_field(bad)
    # the previous field is still active
    T0 = inputs.gaussian_pulse(nx, ny, 4.0, 20, 15)
    lat.set_temperature(torch.from_numpy(T0.astype(np.float32)))
    lat.step(20)
    ora = _oracle(nx, ny, q, np.full((ny, nx), 5.0))
    ora.set_temperature(T0.astype(np.float32).astype(np.float64))
    ora.run(20)
    assert _rel(lat.temperature().cpu().numpy(), ora.temperature()) <= RTOL


def test_full_size_1024_energy_and_sampled_cells():
    """1024 x 1024, Q = 64, MFP 102.4 (Kn = 0.1), the benchmarked launch
    configuration (four steps per launch, 48-column, 45-row blocks, the
    height the library's timing picked for this lattice in the benchmark run
    on MI355X): energy is conserved,
    the populations equal those of single steps bit for bit, and sampled
    cells after n steps equal the oracle run on the window that can influence
    them (signals move at most one cell per step, so a window of half-width
    n + 2 is exact at its centre)."""
    nx = ny = 1024
    q, n = 64, 48
    x0, y0 = inputs.seeded_center(1911, nx, ny)
    T0 = inputs.gaussian_pulse(nx, ny, 16.0, x0, y0).astype(np.float32)
    lat = _lattice(nx=nx, ny=ny, q=q, mfp=102.4)
    lat.set_block_rows(4, 45)
    lat.set_temperature(torch.from_numpy(T0))
    e0, _, _ = lat.totals()
    lat.step(n)
    e1, _, _ = lat.totals()
    assert abs(e1 - e0) <= 1e-6 * e0
    single = _lattice(nx=nx, ny=ny, q=q, mfp=102.4, step_fusion=0)
    single.set_temperature(torch.from_numpy(T0))
    single.step(n)
    assert torch.equal(lat.populations(), single.populations())
    single.close()
    T = lat.temperature().cpu().numpy()
    rng = np.random.default_rng(7)
    half = n + 2
    samples = [(x0, y0), ((x0 + 20) % nx, (y0 - 13) % ny), (0, 0), (nx - 1, 5)]
    samples += [tuple(int(v) for v in rng.integers(0, nx, 2)) for _ in range(2)]
    got, want, tmax = [], [], 0.0
    for (sx, sy) in samples:
        xs = (np.arange(sx - half, sx + half + 1)) % nx
        ys = (np.arange(sy - half, sy + half + 1)) % ny
        win = T0[np.ix_(ys, xs)].astype(np.float64)
        ora = _oracle(2 * half + 1, 2 * half + 1, q, 102.4)
        ora.set_temperature(win)
        ora.run(n)
        Tw = ora.temperature()
        want.append(Tw[half, half])
        got.append(T[sy, sx])
        tmax = max(tmax, float(np.abs(Tw).max()))
    # against the largest |T| of the oracle windows after the run (the
    # pulse's window holds the field's maximum), not of T0
    assert tmax > 0.0
    for (sx, sy), g, w in zip(samples, got, want):
        assert abs(g - w) <= RTOL * tmax, (sx, sy, g, w, tmax)


def _window(s, half, n, walled):
    """Cells of the oracle window around coordinate s on an axis of n cells,
    and that window's edge type: a periodic window when no wall is within
    reach, else one that starts or ends at the lattice's own wall (its other
    edge lies outside the region that can influence the sample)."""
    if walled and s <= half:
        return np.arange(0, s + half + 1), "lo"
    if walled and s >= n - 1 - half:
        return np.arange(s - half, n), "hi"
    return np.arange(s - half, s + half + 1) % n, None


def test_full_size_4096_q256_walls_sampled_cells():
    """4096 x 4096, Q = 256, Kn = 10 (MFP 40960 cells), blackbody x walls at
    T = 1 and 0, diffuse y walls, as the large benchmark runs it (two steps
    per launch, the library's default), from a random initial field:
    sampled cells after n steps, at the corners, along each wall and inside,
    equal the oracle run on the window that can influence them.  A window
    that reaches a wall ends at that wall; its far edge (a wall of the same
    kind, or a periodic wrap) is more than n cells from the sample."""
    nx = ny = 4096
    q, n, mfp = 256, 40, 40960.0
    walls = dict(x_edge="blackbody", y_edge="diffuse", t_x_lo=1.0, t_x_hi=0.0)
    T0 = inputs.random_temperature(11, ny, nx)
    lat = _lattice(nx=nx, ny=ny, q=q, mfp=mfp, **walls)
    lat.set_temperature(torch.from_numpy(T0))
    lat.step(n)
    T = lat.temperature().cpu().numpy()
    lat.close()
    assert np.isfinite(T).all()
    half = n + 2
    rng = np.random.default_rng(12)
    samples = [(0, 0), (1, 2), (nx - 1, ny - 1), (nx - 3, ny - 2), (2000, 0), (1500, ny - 1),
               (0, 2222), (nx - 1, 77), (5, 3000), (nx - 8, 1234), (30, 20)]
    samples += [tuple(int(v) for v in rng.integers(0, nx, 2)) for _ in range(2)]
    for (sx, sy) in samples:
        xs, wx = _window(sx, half, nx, True)
        ys, wy = _window(sy, half, ny, True)
        win = T0[np.ix_(ys, xs)].astype(np.float64)
        kw = dict(x_edge="blackbody" if wx else "periodic",
                  y_edge="diffuse" if wy else "periodic",
                  t_x_lo=1.0, t_x_hi=0.0)
        ora = _oracle(xs.size, ys.size, q, mfp, **kw)
        ora.set_temperature(win)
        ora.run(n)
        cx = int(np.nonzero(xs == sx)[0][0])
        cy = int(np.nonzero(ys == sy)[0][0])
        want = ora.temperature()[cy, cx]
        assert abs(T[sy, sx] - want) <= RTOL * 1.0, (sx, sy, T[sy, sx], want)


def test_full_size_4096_q256_walls_2000_steps_keep_the_bits_of_single_steps():
    """The same lattice for its full 2000 steps: two steps per launch (as
    benchmarked) against one step per launch, bit for bit in every cell's
    temperature and in the FP64 totals, after 500 and after 2000 steps (the
    oracle windows of the test above cover 40 steps; over 2000 steps they
    would span the lattice)."""
    nx = ny = 4096
    q, mfp = 256, 40960.0
    walls = dict(x_edge="blackbody", y_edge="diffuse", t_x_lo=1.0, t_x_hi=0.0)
    T0 = torch.from_numpy(inputs.random_temperature(11, ny, nx))
    a = _lattice(nx=nx, ny=ny, q=q, mfp=mfp, **walls)
    b = _lattice(nx=nx, ny=ny, q=q, mfp=mfp, step_fusion=0, **walls)
    assert a.steps_per_launch == 2 and b.steps_per_launch == 1
    for lat in (a, b):
        lat.set_temperature(T0)
    for n in (500, 1500):
        a.step(n)
        b.step(n)
        ta, tb = a.temperature(), b.temperature()
        assert torch.isfinite(ta).all()
        assert torch.equal(ta, tb), n
        assert a.totals() == b.totals(), n
    a.close()
    b.close()


@pytest.mark.parametrize("kn", [0.1, 10.0])
def test_crop_256_q64_4000_steps(kn):
    """The 256 x 256 periodic crop of the benchmarked workload (Q = 64 evenly
    spaced, MFP kn * 1024, Gaussian sigma0 = 16 at the seeded centre) run for
    4000 steps against stored FP64 oracle values (written by
    tests/golden/make_crop_reference.py): 2048 seeded cells, the row and the
    column through the centre, and the total energy."""
    import json
    import os
    golden = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    with open(os.path.join(golden, f"crop256_q64_kn{kn:g}.json")) as f:
        ref = json.load(f)
    n, q = 256, 64
    x0, y0 = inputs.seeded_center(1911, 1024, 1024)
    cx, cy = x0 % n, y0 % n
    assert [cx, cy] == ref["center"]
    T0 = inputs.gaussian_pulse(n, n, 16.0, cx, cy).astype(np.float32)
    lat = _lattice(nx=n, ny=n, q=q, mfp=ref["mfp"])
    lat.set_temperature(torch.from_numpy(T0))
    lat.step(ref["steps"])
    T = lat.temperature().cpu().numpy().astype(np.float64)
    tol = RTOL * ref["max_abs_T"]
    cells = np.asarray(ref["cells"])
    assert np.abs(T[cells[:, 1], cells[:, 0]] - np.asarray(ref["T_cells"])).max() <= tol
    assert np.abs(T[cy, :] - np.asarray(ref["T_row"])).max() <= tol
    assert np.abs(T[:, cx] - np.asarray(ref["T_col"])).max() <= tol
    assert abs(float(np.abs(T).max()) - ref["max_abs_T"]) <= tol
    e, _, _ = lat.totals()
    assert abs(e - ref["energy"]) <= 1e-6 * ref["energy"]


@pytest.mark.parametrize("q", [16, 32, 64])
def test_direction_splits_are_bit_identical(q):
    """E is summed in the same order (8-direction batch sums, added in batch
    order) whatever the split of the directions over waves, so every split,
    and the multi-step path, gives the same bits."""
    nx, ny = 141, 29
    e0 = torch.from_numpy(inputs.random_populations(5, q, ny, nx))
    runs = []
    for split in (1, 2, 4):
        if q // split < 8:
            continue
        for fusion in (False, True):
            for edges in (dict(x_edge="blackbody", y_edge="diffuse", t_x_lo=1.0), dict()):
                lat = _lattice(nx=nx, ny=ny, q=q, mfp=6.0, dir_split=split,
                               step_fusion=fusion, **edges)
                lat.set_populations(e0)
                lat.step(13)
                runs.append((bool(edges), split, fusion, lat.populations().cpu()))
                lat.close()
    for walls in (False, True):
        same = [r for r in runs if r[0] == walls]
        for r in same[1:]:
            assert torch.equal(r[3], same[0][3]), r[:3]
