"""Several steps per launch (k_stepk, K = 2 .. 4) against one step per launch
(k_step), on periodic lattices and on lattices with blackbody x and y edges
and adiabatic diffuse y walls.

The multi-step kernels use the same arithmetic and the same summation order
as the single-step kernel, so the populations must agree bit for bit,
whatever direction split the single steps use and whatever block height the
library picks, on ragged and tiny lattices, for step counts that leave single
steps at the end, across schedule chunks and inside flux windows (whose
float64 heat-flux sums the multi-step launches accumulate step by step).
Oracle parity of the multi-step path is covered by every periodic parity
test, which runs it by default.
"""
import numpy as np
import pytest

from paper_1911_00180_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_00180_amd import wormlbm
    wormlbm.lib()


def _pair(nx, ny, q, fusion=1, **kw):
    from paper_1911_00180_amd.lattice import Lattice
    a = Lattice(nx, ny, q, step_fusion=fusion, **kw)
    b = Lattice(nx, ny, q, step_fusion=0, **kw)
    return a, b


@pytest.mark.parametrize("fusion", [2, 3, 4])
@pytest.mark.parametrize("nx,ny,q,mfp", [(150, 41, 64, 9.0), (97, 23, 32, 4.0), (9, 8, 8, 1e9),
                                         (100, 30, 256, 6.0), (61, 19, 120, 5.0),
                                         (77, 26, 72, 3.0), (130, 50, 128, 8.0)])
def test_two_and_three_steps_per_launch(fusion, nx, ny, q, mfp):
    """At most two, three or four steps per launch against single steps, for
    counts that leave every remainder (and odd chunk ends)."""
    a, b = _pair(nx, ny, q, fusion=fusion, mfp=mfp, sched_chunk=17)
    e0 = torch.from_numpy(inputs.random_populations(8, q, ny, nx))
    for lat in (a, b):
        lat.set_populations(e0)
    for n in (3, 4, 5, 1, 2, 40):
        a.step(n)
        b.step(n)
        assert torch.equal(a.populations(), b.populations()), n
        assert torch.equal(a.temperature(), b.temperature()), n
    a.close()
    b.close()


@pytest.mark.parametrize("nx,ny,q,split,mfp,kind", [
    (1024, 64, 64, 0, 102.4, "uniform"),
    (131, 37, 64, 4, 6.0, "uniform"),
    (70, 45, 16, 2, 3.0, "uniform"),
    (20, 10, 32, 1, 9.0, "ring"),
    (5, 3, 8, 1, 2.0, "uniform"),
    (200, 17, 24, 1, 1e9, "ring"),
    (8, 2, 16, 2, 3.0, "uniform"),     # smallest lattice the multi-step kernels take
    (49, 5, 64, 0, 8.0, "uniform"),    # last strip holds one column
    (7, 9, 8, 1, 2.0, "uniform"),      # too narrow: single steps
    (128, 6, 128, 0, 20.0, "uniform"),
])
def test_fused_equals_single_steps(nx, ny, q, split, mfp, kind):
    a, b = _pair(nx, ny, q, mfp=mfp, dirs=kind, dir_split=split, sched_chunk=16)
    e0 = torch.from_numpy(inputs.random_populations(3, q, ny, nx))
    for lat in (a, b):
        lat.set_populations(e0)
    for n in (1, 2, 7, 16, 33):
        a.step(n)
        b.step(n)
        assert torch.equal(a.populations(), b.populations()), n
        assert torch.equal(a.temperature(), b.temperature()), n
    a.close()
    b.close()


def test_fused_with_mfp_field_and_flux_window():
    nx, ny, q = 150, 40, 32
    a, b = _pair(nx, ny, q, mfp=5.0, sched_chunk=16)
    mfp = torch.from_numpy(inputs.smooth_lognormal_field(nx, ny, 4, 5.0, 6.0, 0.6, 2.0, 30.0)
                           .astype(np.float32))
    T0 = torch.from_numpy(inputs.random_temperature(6, ny, nx))
    for lat in (a, b):
        lat.set_mfp_field(mfp)
        lat.set_temperature(T0)
        lat.set_flux_window(5)
    for n in (40, 13, 6):
        a.step(n)
        b.step(n)
        assert torch.equal(a.populations(), b.populations()), n
        for u, v in zip(a.heat_flux(averaged=True), b.heat_flux(averaged=True)):
            assert torch.equal(u, v)
    a.close()
    b.close()


@pytest.mark.parametrize("fusion", [2, 3, 4])
@pytest.mark.parametrize("nx,ny,q,kw", [
    (150, 41, 64, dict(mfp=9.0)),
    (70, 45, 32, dict(mfp=6.0, x_edge="blackbody", y_edge="diffuse", t_x_lo=1.0)),
    (61, 19, 128, dict(mfp=5.0, x_edge="blackbody", y_edge="diffuse", t_x_lo=1.0, t_x_hi=0.2)),
    (64, 17, 8, dict(mfp=4.0, x_edge="periodic", y_edge="blackbody", t_y_lo=0.3)),
    (100, 30, 256, dict(mfp=6.0)),
])
def test_flux_windows_inside_multi_step_launches(fusion, nx, ny, q, kw):
    """Flux-window steps run several per launch: windows that start at each
    step of a launch, or before the call, and span launches and schedule
    chunks keep the float64 window sums of single steps bit for bit (the
    per-cell averages and the fixed-order float64 means)."""
    a, b = _pair(nx, ny, q, fusion=fusion, sched_chunk=16, **kw)
    assert a.steps_per_launch >= 2
    e0 = torch.from_numpy(inputs.random_populations(21, q, ny, nx))
    for lat in (a, b):
        lat.set_populations(e0)
    for window, n in ((1, 9), (2, 9), (3, 10), (4, 12), (5, 11), (7, 7), (13, 50), (40, 45)):
        for lat in (a, b):
            lat.set_flux_window(window)
        a.step(n)
        b.step(n)
        assert torch.equal(a.populations(), b.populations()), (window, n)
        for u, v in zip(a.heat_flux(averaged=True), b.heat_flux(averaged=True)):
            assert torch.equal(u, v), (window, n)
        assert a.flux_mean(averaged=True) == b.flux_mean(averaged=True), (window, n)
        assert (a.flux_mean(1, nx - 1, averaged=True) ==
                b.flux_mean(1, nx - 1, averaged=True)), (window, n)
    a.close()
    b.close()


def test_fused_then_adjoint_tape_and_restart():
    """Tapes and restarts still run single steps; a fused run continued from a
    saved state matches an unfused one."""
    nx, ny, q = 90, 50, 16
    a, b = _pair(nx, ny, q, mfp=7.0)
    T0 = torch.from_numpy(inputs.random_temperature(8, ny, nx))
    for lat in (a, b):
        lat.set_temperature(T0)
        lat.step(11)
    tape = a.new_states(5)
    a.step_tape(5, tape)
    b.step(5)
    assert torch.equal(a.populations(), b.populations())
    a.load_state(tape[2], 14)
    a.step(9)
    b.load_state(tape[2], 14)
    b.step(9)
    assert torch.equal(a.populations(), b.populations())
    a.close()
    b.close()


def test_block_height_model_and_tuner_keep_bits():
    """Untuned, the k-step kernel runs the launch model's height (no timing
    inside the step call, never 0); wlbm_tune_block_rows times every
    candidate on a saved state, restores the state and the step count, and
    keeps a valid height; populations match single steps throughout."""
    nx, ny, q = 200, 130, 32
    a, b = _pair(nx, ny, q, fusion=3, mfp=12.0)
    r0 = a.block_rows(3)
    assert r0 in range(5, 63, 3) and r0 <= ny + 2
    assert a.block_rows(5) == -1 and a.block_rows(1) == -1
    assert b.block_rows(3) == 0          # one step per launch
    e0 = torch.from_numpy(inputs.random_populations(4, q, ny, nx))
    for lat in (a, b):
        lat.set_populations(e0)
    a.step(30)
    b.step(30)
    assert torch.equal(a.populations(), b.populations())
    assert a.block_rows(3) == r0
    rows = a.tune_block_rows(3, launches=3)
    assert rows in range(5, 63, 3) and rows <= ny + 2 and a.block_rows(3) == rows
    assert a.step_count == 30
    assert torch.equal(a.populations(), b.populations())
    a.step(33)
    b.step(33)
    assert torch.equal(a.populations(), b.populations())
    from paper_1911_00180_amd import wormlbm as W
    with pytest.raises(W.WormLBMError):
        b.tune_block_rows(3)             # b runs one step per launch
    a.set_block_rows(3, 0)
    assert a.block_rows(3) == r0
    a.close()
    b.close()


def test_fixed_block_heights():
    """Heights set by the caller skip the timing and keep the bits; invalid
    heights are rejected."""
    from paper_1911_00180_amd import wormlbm as W
    nx, ny, q = 120, 70, 16
    e0 = torch.from_numpy(inputs.random_populations(6, q, ny, nx))
    b = None
    for k, rows in ((2, 1), (3, 8), (4, 9), (4, 30)):
        a, b0 = _pair(nx, ny, q, fusion=k, mfp=5.0)
        if b is None:
            b = b0
            b.set_populations(e0)
            b.step(24)
        else:
            b0.close()
        a.set_block_rows(k, rows)
        assert a.block_rows(k) == rows
        a.set_populations(e0)
        a.step(24)
        assert torch.equal(a.populations(), b.populations()), (k, rows)
        for bad in (2, 63, -1):
            if bad and (bad + 2 * (k - 1)) % 3 == 0 and 0 < bad <= 62:
                continue
            with pytest.raises(W.WormLBMError):
                a.set_block_rows(k, bad)
        a.close()
    with pytest.raises(W.WormLBMError):
        b.set_block_rows(5, 3)
    b.close()


@pytest.mark.parametrize("seed", range(12))
def test_fused_random_shapes(seed):
    """Seeded random lattices (nx 8 .. 300, ny 2 .. 90, Q from 8 to 128,
    either direction set, uniform or per-cell MFP, random schedule chunk and
    step counts): any number of steps per launch gives the bits of single
    steps."""
    rng = np.random.default_rng(1000 + seed)
    nx = int(rng.integers(8, 301))
    ny = int(rng.integers(2, 91))
    q = int(rng.choice([8, 16, 24, 32, 48, 64, 72, 80, 88, 96, 104, 112, 120, 128]))
    kind = "ring" if rng.random() < 0.3 else "uniform"
    fusion = int(rng.integers(1, 5))
    chunk = int(rng.integers(16, 64))
    a, b = _pair(nx, ny, q, fusion=fusion, mfp=float(rng.uniform(2.0, 50.0)), dirs=kind,
                 sched_chunk=chunk)
    if rng.random() < 0.4:
        mfp = torch.from_numpy(inputs.smooth_lognormal_field(nx, ny, seed, 4.0, 8.0, 0.5, 2.0,
                                                             40.0).astype(np.float32))
        a.set_mfp_field(mfp)
        b.set_mfp_field(mfp)
    e0 = torch.from_numpy(inputs.random_populations(50 + seed, q, ny, nx))
    for lat in (a, b):
        lat.set_populations(e0)
    for n in rng.integers(1, 40, 3):
        a.step(int(n))
        b.step(int(n))
        assert torch.equal(a.populations(), b.populations()), (nx, ny, q, kind, fusion, chunk, n)
    a.close()
    b.close()


WALLED = {
    "bbx": dict(x_edge="blackbody", y_edge="periodic", t_x_lo=1.0, t_x_hi=0.25),
    "bby": dict(x_edge="periodic", y_edge="blackbody", t_y_lo=0.7, t_y_hi=0.1),
    "bbxy": dict(x_edge="blackbody", y_edge="blackbody", t_x_lo=1.0, t_x_hi=0.0, t_y_lo=0.5,
                 t_y_hi=0.2),
    "dify": dict(x_edge="periodic", y_edge="diffuse"),
    "bbx_dify": dict(x_edge="blackbody", y_edge="diffuse", t_x_lo=1.0, t_x_hi=0.0),
}


@pytest.mark.parametrize("fusion", [2, 3, 4])
@pytest.mark.parametrize("edges", sorted(WALLED))
@pytest.mark.parametrize("nx,ny,q,mfp,per_cell", [
    (150, 41, 64, 9.0, False), (97, 23, 32, 4.0, True), (9, 8, 8, 2.0, False),
    (70, 130, 128, 6.0, True), (200, 3, 16, 1.5, False), (90, 37, 256, 7.0, False),
    (60, 20, 192, 3.0, True), (45, 29, 88, 5.0, False), (103, 14, 104, 2.5, True)])
def test_walled_lattices_keep_the_bits_of_single_steps(fusion, edges, nx, ny, q, mfp, per_cell):
    """Blackbody x / y edges and diffuse y walls (Sec. 2.6) inside the
    multi-step kernel: every level overwrites blackbody cells, zeroes the rows
    beyond a non-periodic y edge and re-emits the diffuse nodes' inflow, so
    any number of steps per launch gives the bits of single steps."""
    a, b = _pair(nx, ny, q, fusion=fusion, mfp=mfp, sched_chunk=17, **WALLED[edges])
    assert a.block_rows(fusion) > 0 and b.block_rows(fusion) == 0
    if per_cell:
        f = torch.from_numpy(inputs.smooth_lognormal_field(nx, ny, 5, 4.0, 8.0, 0.5, 2.0,
                                                           40.0).astype(np.float32))
        a.set_mfp_field(f)
        b.set_mfp_field(f)
    e0 = torch.from_numpy(inputs.random_populations(9, q, ny, nx))
    for lat in (a, b):
        lat.set_populations(e0)
    for n in (3, 4, 5, 1, 2, 40):
        a.step(n)
        b.step(n)
        assert torch.equal(a.populations(), b.populations()), n
        assert torch.equal(a.temperature(), b.temperature()), n
    a.close()
    b.close()


@pytest.mark.parametrize("seed", range(10))
def test_walled_random_shapes(seed):
    """Seeded random walled lattices (edges, sizes, Q, direction set, per-cell
    field, chunk and step counts, wall temperatures): multi-step launches keep
    the bits of single steps."""
    rng = np.random.default_rng(2000 + seed)
    nx = int(rng.integers(8, 260))
    ny = int(rng.integers(2, 80))
    q = int(rng.choice([8, 16, 24, 32, 48, 64, 72, 80, 88, 96, 104, 112, 120, 128]))
    kind = "ring" if rng.random() < 0.3 else "uniform"
    edges = dict(WALLED[sorted(WALLED)[int(rng.integers(0, len(WALLED)))]])
    for key in ("t_x_lo", "t_x_hi", "t_y_lo", "t_y_hi"):
        if key in edges:
            edges[key] = float(rng.uniform(0.0, 1.0))
    fusion = int(rng.integers(1, 5))
    chunk = int(rng.integers(16, 64))
    a, b = _pair(nx, ny, q, fusion=fusion, mfp=float(rng.uniform(1.5, 50.0)), dirs=kind,
                 sched_chunk=chunk, **edges)
    if rng.random() < 0.4:
        mfp = torch.from_numpy(inputs.smooth_lognormal_field(nx, ny, seed, 4.0, 8.0, 0.5, 2.0,
                                                             40.0).astype(np.float32))
        a.set_mfp_field(mfp)
        b.set_mfp_field(mfp)
    e0 = torch.from_numpy(inputs.random_populations(70 + seed, q, ny, nx))
    for lat in (a, b):
        lat.set_populations(e0)
    for n in rng.integers(1, 40, 3):
        a.step(int(n))
        b.step(int(n))
        assert torch.equal(a.populations(), b.populations()), (nx, ny, q, kind, edges, fusion, n)
    a.close()
    b.close()
