"""The C-ABI library on the host (no GPU): it loads, exports every declared
symbol, validates its arguments, and its host tables match the oracle."""
import math
import re
import os

import numpy as np
import pytest

from oracle import worm_lbm as o
from paper_1911_00180_amd import wormlbm as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "wormlbm.h")


def test_exports_every_declared_symbol():
    src = open(HEADER).read()
    declared = set(re.findall(r"\b(wlbm_[a-z_0-9]+)\s*\(", src))
    assert declared == set(W.EXPORTS)
    L = W.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_exports_nothing_else():
    """The library is built with hidden visibility: its dynamic symbol table
    holds the declared entry points and nothing more of its own."""
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", W.LIB_PATH], capture_output=True,
                         text=True)
    if out.returncode != 0:
        pytest.skip("nm not available")
    text_syms = {ln.split()[-1] for ln in out.stdout.splitlines()
                 if len(ln.split()) == 3 and ln.split()[1] == "T"}
    assert text_syms == set(W.EXPORTS)


@pytest.mark.parametrize("q,kind", [(16, "uniform"), (64, "uniform"), (24, "ring")])
def test_schedule_with_speeds_bit_exact_against_oracle(q, kind):
    rng = np.random.default_rng(q)
    v = rng.uniform(0.2, 1.0, size=q)
    v[::5] = 1.0
    p = W.make_params(32, 32, q, mfp=10.0, dirs=kind)
    moves, pos = W.wlbm_get_schedule(p, 0, 1500, positions=True, speeds=v)
    sch = o.tas_schedule(o.make_directions(q, kind), 1500, speeds=v)
    want = np.where(sch.hop, sch.move, -sch.move).astype(np.int8)
    assert np.array_equal(moves, want)
    assert np.array_equal(pos, sch.pos)
    with pytest.raises(W.WormLBMError):
        W.wlbm_get_schedule(p, 0, 10, speeds=np.full(q, 1.5))


@pytest.mark.parametrize("q,kind", [(8, "uniform"), (16, "uniform"), (64, "uniform"),
                                    (128, "uniform"), (256, "uniform"), (16, "ring"),
                                    (64, "ring"), (128, "ring")])
def test_schedule_bit_exact_against_oracle(q, kind):
    """Closed-form worm paths + integer TAS (library) against the literal
    greedy search + TAS rule (oracle): identical move and hop tables."""
    nsteps = 3000 if q <= 64 else 1200
    p = W.make_params(32, 32, q, mfp=10.0, dirs=kind)
    moves, pos = W.wlbm_get_schedule(p, 0, nsteps, positions=True)
    sch = o.tas_schedule(o.make_directions(q, kind), nsteps)
    want = np.where(sch.hop, sch.move, -sch.move).astype(np.int8)
    assert np.array_equal(moves, want)
    assert np.array_equal(pos, sch.pos)


def test_schedule_window_matches_full_run():
    p = W.make_params(8, 8, 64, mfp=10.0)
    full, _ = W.wlbm_get_schedule(p, 0, 700)
    part, _ = W.wlbm_get_schedule(p, 500, 200)
    assert np.array_equal(full[500:], part)


@pytest.mark.parametrize("q,kind", [(8, "uniform"), (48, "uniform"), (16, "ring"), (96, "ring")])
def test_directions_and_constants_against_oracle(q, kind):
    p = W.make_params(8, 8, q, mfp=12.5, dirs=kind, emulate_3d=True)
    sx, sy, w = W.wlbm_get_directions(p)
    dirs = o.make_directions(q, kind)
    assert np.array_equal(sx, [d.sx for d in dirs])
    assert np.array_equal(sy, [d.sy for d in dirs])
    assert np.allclose(w, o.weights(dirs), rtol=0, atol=1e-15)
    lam, Wv, wc = W.wlbm_get_constants(p)
    assert abs(lam - o.lambda_corr(dirs)) < 1e-15
    assert Wv == 1 / 12.5
    assert abs(wc - o.w_corr(1 / 12.5, o.lambda_corr(dirs), True)) < 1e-16


@pytest.mark.parametrize("field,value,status", [
    ("q", 12, W.WLBM_EINVAL), ("q", 0, W.WLBM_EINVAL), ("q", 2048, W.WLBM_EINVAL),
    ("nx", 0, W.WLBM_EINVAL), ("ny", -3, W.WLBM_EINVAL), ("x_edge", 2, W.WLBM_EINVAL),
    ("y_edge", 7, W.WLBM_EINVAL), ("mfp_cells", 0.0, W.WLBM_EINVAL),
    ("mfp_cells", float("nan"), W.WLBM_EINVAL), ("mfp_cells", 0.5, W.WLBM_EUNSTABLE),
    ("dir_split", 3, W.WLBM_EINVAL), ("dir_split", 8, W.WLBM_EINVAL),
    ("sched_chunk", 5, W.WLBM_EINVAL), ("t_x_lo", float("inf"), W.WLBM_EINVAL),
    ("dirs", 5, W.WLBM_EINVAL), ("emulate_3d", 2, W.WLBM_EINVAL),
    ("step_fusion", 5, W.WLBM_EINVAL), ("step_fusion", -1, W.WLBM_EINVAL),
])
def test_validation_errors(field, value, status):
    p = W.make_params(16, 16, 16, mfp=8.0)
    setattr(p, field, value)
    with pytest.raises(W.WormLBMError) as ei:
        W.wlbm_workspace_bytes(p)
    assert ei.value.status == status
    assert W.wlbm_last_error()


def test_stability_limit_matches_app_a():
    """W_corr <= 1 accepted, W_corr > 1 rejected (App. A), also without the
    correction (plain W = 1/MFP)."""
    p = W.make_params(16, 16, 8, mfp=1.0, mfp_correction=False)
    W.wlbm_workspace_bytes(p)
    p.mfp_cells = 1.0 - 1e-9
    with pytest.raises(W.WormLBMError) as ei:
        W.wlbm_workspace_bytes(p)
    assert ei.value.status == W.WLBM_EUNSTABLE


def test_schedule_argument_checks():
    p = W.make_params(16, 16, 16, mfp=8.0)
    with pytest.raises(W.WormLBMError):
        W.wlbm_get_schedule(p, -1, 4)
    with pytest.raises(W.WormLBMError):
        W.wlbm_get_schedule(p, 2**31 - 2, 4)


def test_workspace_size_covers_double_buffered_populations():
    p = W.make_params(1024, 1024, 64, mfp=102.4)
    n = W.wlbm_workspace_bytes(p)
    assert n >= 2 * 64 * 1024 * 1024 * 4
    # plus E (two buffers), the weight field, the 1/MFP field and the two
    # flux fields (float64)
    assert n < (2 * 64 + 3) * 1026 * 1088 * 4 + 5 * 1024 * 1024 * 4 + (1 << 20)
    # the 4096 x 4096 x 256 lattice fits one MI355X (288 GB)
    p = W.make_params(4096, 4096, 256, mfp=40960.0, x_edge="blackbody", y_edge="diffuse")
    assert W.wlbm_workspace_bytes(p) < 40e9


def test_create_rejects_bad_workspace_without_touching_the_gpu():
    p = W.make_params(16, 16, 16, mfp=8.0)
    with pytest.raises(W.WormLBMError) as ei:
        W.wlbm_create(p, 0, 1 << 20, 0)
    assert ei.value.status == W.WLBM_EINVAL
    with pytest.raises(W.WormLBMError) as ei:
        W.wlbm_create(p, 256 * 1024, 16, 0)
    assert ei.value.status == W.WLBM_ENOMEM
    with pytest.raises(W.WormLBMError) as ei:
        W.wlbm_create(p, 256 * 1024 + 4, 1 << 30, 0)
    assert ei.value.status == W.WLBM_EINVAL


def test_size_limit_of_one_direction_group():
    """Eight padded direction planes are addressed through one 32-bit buffer
    window: 11000^2 fits, 12000^2 is rejected with a clear error."""
    W.wlbm_workspace_bytes(W.make_params(11000, 11000, 8, mfp=50.0))
    with pytest.raises(W.WormLBMError) as ei:
        W.wlbm_workspace_bytes(W.make_params(12000, 12000, 8, mfp=50.0))
    assert ei.value.status == W.WLBM_EINVAL
    assert "too large" in W.wlbm_last_error()


def test_direction_split_needs_divisible_q():
    W.wlbm_workspace_bytes(W.make_params(64, 64, 32, mfp=8.0, dir_split=4))
    with pytest.raises(W.WormLBMError) as ei:
        W.wlbm_workspace_bytes(W.make_params(64, 64, 24, mfp=8.0, dir_split=2))
    assert ei.value.status == W.WLBM_EINVAL


def test_flux_distribution_matches_oracle():
    import numpy as np

    from oracle import worm_lbm as o
    for q, kind in ((16, "uniform"), (64, "uniform"), (24, "ring"), (40, "ring")):
        p = W.make_params(16, 16, q, mfp=8.0, dirs=kind)
        e = W.wlbm_flux_distribution(p, 0.6, 0.03, -0.07)
        lat = o.Lattice(o.Config(nx=4, ny=4, q=q, dirs=kind))
        want = o.flux_distribution(lat.dirs, lat.w, 0.6, np.array([0.03, -0.07]))
        assert np.max(np.abs(e - want)) < 1e-15


def test_specularity_validated():
    p = W.make_params(16, 16, 16, mfp=8.0, y_edge="diffuse", y_specularity=1.5)
    with pytest.raises(W.WormLBMError) as ei:
        W.wlbm_workspace_bytes(p)
    assert ei.value.status == W.WLBM_EINVAL
    p = W.make_params(16, 16, 16, mfp=8.0, y_edge="diffuse", y_specularity=0.25)
    assert W.wlbm_workspace_bytes(p) > 0


def test_batch_entry_points_reject_null_handles_without_the_gpu():
    for call in (lambda: W.wlbm_batch_step(0, 1), lambda: W.wlbm_batch_set_graphs(0, 1)):
        with pytest.raises(W.WormLBMError) as ei:
            call()
        assert ei.value.status == W.WLBM_EINVAL
    W.wlbm_batch_destroy(0)     # NULL is accepted


def test_build_compiles_every_source_file():
    """Every HIP / C++ source under csrc is compiled into the library or the
    stream probe, once (a multi-step instantiation file left out of the list
    would leave its launch symbols undefined until load time)."""
    import os
    from paper_1911_00180_amd import build
    files = sorted(f for f in os.listdir(build.CSRC) if f.endswith((".hip", ".cpp")))
    listed = build.SOURCES + build.PROBE_SOURCES
    assert sorted(listed) == files
    assert len(set(listed)) == len(listed)
