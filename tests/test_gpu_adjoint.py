"""Adjoint (reverse-mode) path on the GPU against the FP64 oracle gradients.

The oracle (oracle/adjoint.py) is pinned on the CPU by the Jacobian transpose
of its forward step and by central differences.  Here the library's reverse
pass, driven through ProbeSeries (checkpoints + recomputed tapes), is compared
with it on ragged multi-tile lattices, and at the full 256 x 256, Q = 64,
1000-step size with directional central differences of the GPU forward.

Tolerances.  Probe temperatures: 1e-5 * max|T| as for every forward field.
Gradients: each reverse step is a convex combination of adjoint values plus
seeds, as well conditioned as a forward step, and the MFP gradient is summed
per step from terms whose equilibrium parts are taken out before rounding; so
the FP32 error grows at most like n * eps (n = 60 steps, eps = 6e-8, about
4e-6) and every gradient is held to 1e-5 of its largest value.  Central
differences of the FP32 forward (full size) carry their own truncation and
rounding error and are held to 2e-3.
"""
import os

import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import worm_lbm as o
from paper_1911_00180_amd import inputs

pytestmark = pytest.mark.gpu

# Gradient tolerance of the 1000-step full-size case (relative to the
# largest value of each gradient), as for the 60-step cases.
GRAD_RTOL_1000 = 1e-5

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_00180_amd import wormlbm
    wormlbm.lib()


def _series(nx, ny, q, dirs, x_edge, y_edge, probes, nsteps, every, K, **kw):
    from paper_1911_00180_amd.autodiff import ProbeSeries
    from paper_1911_00180_amd.lattice import Lattice
    lat = Lattice(nx, ny, q, mfp=8.0, dirs=dirs, x_edge=x_edge, y_edge=y_edge, **kw)
    return lat, ProbeSeries(lat, probes, nsteps, every, checkpoint_every=K)


def _gpu_grads(series, mfp, T0, walls, targets):
    dev = series.lat.device
    m = torch.tensor(mfp, dtype=torch.float32, device=dev, requires_grad=True)
    t = torch.tensor(T0, dtype=torch.float32, device=dev, requires_grad=True)
    w = torch.tensor(walls, dtype=torch.float32, device=dev, requires_grad=True)
    out = series(m, t, w)
    tg = torch.tensor(targets, dtype=torch.float32, device=dev)
    loss = ((out - tg) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    return (out.detach().cpu().numpy(), loss.item(), m.grad.cpu().numpy(),
            t.grad.cpu().numpy(), w.grad.cpu().numpy())


CASES = [
    # nx, ny, q, dirs, x_edge, y_edge, emulate_3d
    (70, 45, 16, "uniform", "blackbody", "periodic", False),
    (131, 37, 24, "ring", "blackbody", "blackbody", True),
    (64, 40, 32, "uniform", "periodic", "periodic", False),
    (50, 66, 16, "uniform", "periodic", "blackbody", False),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}-q{c[2]}-{c[4]}-{c[5]}")
def test_adjoint_matches_oracle(case):
    nx, ny, q, dirs, xe, ye, e3 = case
    nsteps, every, K = 60, 5, 16
    mfp = inputs.smooth_lognormal_field(nx, ny, 1, 6.0, 5.0, 0.5, 2.0, 16.0).astype(np.float32)
    T0 = inputs.gaussian_pulse(nx, ny, 6.0, nx // 2, ny // 2).astype(np.float32)
    probes = inputs.probe_cells(3, nx, ny, 12)
    targets = np.random.default_rng(2).uniform(0.0, 0.3, (nsteps // every, len(probes)))
    targets = targets.astype(np.float32)
    walls = np.array([0.5, 0.0, 0.25, 0.1], dtype=np.float32)
    lat, series = _series(nx, ny, q, dirs, xe, ye, probes, nsteps, every, K, emulate_3d=e3)
    out, loss, g_mfp, g_T0, g_w = _gpu_grads(series, mfp, T0, walls, targets)

    cfg = o.Config(nx=nx, ny=ny, q=q, mfp=mfp.astype(np.float64), dirs=dirs, x_edge=xe,
                   y_edge=ye, emulate_3d=e3, t_x_lo=float(walls[0]), t_x_hi=float(walls[1]),
                   t_y_lo=float(walls[2]), t_y_hi=float(walls[3]))
    oloss, og_mfp, og_T0, og_w = oadj.probe_loss_gradients(
        cfg, T0.astype(np.float64), nsteps, probes, every, targets.astype(np.float64))
    # forward probe temperatures
    _, olat, states = oadj.probe_loss(cfg, T0.astype(np.float64), nsteps, probes, every,
                                      targets.astype(np.float64), keep_states=True)
    oT = np.array([states[k * every].sum(axis=0)[probes[:, 1], probes[:, 0]]
                   for k in range(1, nsteps // every + 1)])
    Tmax = max(np.abs(T0).max(), max(walls))
    assert np.abs(out - oT).max() <= 1e-5 * Tmax
    assert abs(loss - oloss) <= 1e-4 * oloss
    err_mfp = np.abs(g_mfp - og_mfp).max() / np.abs(og_mfp).max()
    err_T0 = np.abs(g_T0 - og_T0).max() / np.abs(og_T0).max()
    print(f"relative gradient errors: mfp {err_mfp:.2e}, T0 {err_T0:.2e}")
    assert err_mfp <= 1e-5
    assert err_T0 <= 1e-5
    ow = np.array([og_w["x_lo"], og_w["x_hi"], og_w["y_lo"], og_w["y_hi"]])
    assert np.abs(g_w - ow).max() <= 1e-5 * max(np.abs(ow).max(), 1e-30)
    lat.close()


def test_checkpoint_interval_does_not_change_gradients():
    """Recomputed states are bit-identical to the forward ones, so the
    gradients do not depend on the checkpoint interval."""
    nx, ny, q = 70, 45, 16
    mfp = inputs.smooth_lognormal_field(nx, ny, 1, 6.0, 5.0, 0.5, 2.0, 16.0).astype(np.float32)
    T0 = inputs.gaussian_pulse(nx, ny, 6.0, 20, 30).astype(np.float32)
    probes = inputs.probe_cells(3, nx, ny, 9)
    targets = np.zeros((10, 9), dtype=np.float32)
    walls = np.array([1.0, 0.0, 0.0, 0.0], dtype=np.float32)
    res = []
    for K in (7, 50, 70):
        lat, series = _series(nx, ny, q, "uniform", "blackbody", "periodic", probes, 70, 7, K)
        res.append(_gpu_grads(series, mfp, T0, walls, targets))
        lat.close()
    for r in res[1:]:
        for a, b in zip(res[0][2:], r[2:]):
            assert np.array_equal(a, b)


def test_tape_and_restart_are_bit_exact():
    from paper_1911_00180_amd.lattice import Lattice
    nx, ny, q = 96, 40, 32
    T0 = torch.from_numpy(inputs.random_temperature(4, ny, nx))
    mk = lambda: Lattice(nx, ny, q, mfp=9.0, x_edge="blackbody", y_edge="periodic",  # noqa: E731
                         t_x_lo=1.0)
    a = mk()
    a.set_temperature(T0)
    a.step(150)
    want = a.populations()
    # tape: states after each step land in consecutive slots
    b = mk()
    b.set_temperature(T0)
    b.step(100)
    tape = b.new_states(50)
    b.step_tape(50, tape)
    assert b.step_count == 150
    assert torch.equal(b.populations(), want)
    # restart at a step that is not a snapshot boundary of the schedule
    c = mk()
    c.load_state(tape[36], 137)
    c.step(13)
    assert c.step_count == 150
    assert torch.equal(c.populations(), want)
    # save, run on, reload
    d = mk()
    buf = torch.zeros(d.state_bytes, dtype=torch.uint8, device="cuda")
    d.load_state(tape[36], 137)
    d.save_state(buf)
    d.step(5)
    d.load_state(buf, 137)
    d.step(13)
    assert torch.equal(d.populations(), want)
    for lat in (a, b, c, d):
        lat.close()


def test_probe_readout_and_bad_seed_cell():
    from paper_1911_00180_amd import wormlbm as W
    from paper_1911_00180_amd.lattice import Lattice
    lat = Lattice(40, 30, 16, mfp=5.0)
    T0 = inputs.random_temperature(5, 30, 40)
    lat.set_temperature(torch.from_numpy(T0))
    cells = torch.tensor([[3, 4], [39, 29], [40, 0]], dtype=torch.int32, device="cuda")
    T = lat.read_probes(cells).cpu().numpy()
    assert T[0] == pytest.approx(T0[4, 3], rel=1e-6)
    assert T[1] == pytest.approx(T0[29, 39], rel=1e-6)
    assert np.isnan(T[2])
    ws = torch.empty(W.wlbm_adjoint_bytes(lat.handle), dtype=torch.uint8, device="cuda")
    W.wlbm_adjoint_begin(lat.handle, ws.data_ptr(), ws.numel(), 10)
    vals = torch.ones(3, dtype=torch.float32, device="cuda")
    W.wlbm_adjoint_seed(lat.handle, 3, cells.data_ptr(), vals.data_ptr())
    with pytest.raises(W.WormLBMError):
        W.wlbm_adjoint_read(lat.handle, None, None)
    lat.close()


def test_adjoint_rejects_diffuse_walls():
    from paper_1911_00180_amd import wormlbm as W
    from paper_1911_00180_amd.lattice import Lattice
    lat = Lattice(32, 32, 16, mfp=5.0, y_edge="diffuse")
    ws = torch.empty(W.wlbm_adjoint_bytes(lat.handle), dtype=torch.uint8, device="cuda")
    with pytest.raises(W.WormLBMError):
        W.wlbm_adjoint_begin(lat.handle, ws.data_ptr(), ws.numel(), 10)
    lat.close()


GOLDEN_INVERSE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                              "inverse256_q64.npz")


def _golden_input_hash(mfp, tgt, T0, probes):
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_inverse_reference", os.path.join(os.path.dirname(GOLDEN_INVERSE),
                                               "make_inverse_reference.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.input_hash(mfp, tgt, T0, probes)


def test_c4_full_size_against_oracle_gradients():
    """The inverse problem at its stated size (256 x 256, Q = 64, per-cell MFP
    field, blackbody x walls 0.5 / 0, periodic y, 1000 steps, 32 probes, loss
    every 10 steps, checkpoints every 50) against the FP64 oracle's stored
    run (tests/golden/inverse256_q64.npz, written by make_inverse_reference.py
    from the oracle alone, targets included): probe temperatures within
    1e-5 of their largest value, the loss within 1e-4, and dL/dMFP, dL/dT0
    and the wall gradients element by element against their largest values
    (tolerance in the module docstring)."""
    from paper_1911_00180_amd.autodiff import ProbeSeries
    from paper_1911_00180_amd.lattice import Lattice
    ref = np.load(GOLDEN_INVERSE, allow_pickle=False)
    n, mfp, tgt, T0, probes = inputs.inverse_problem_256()
    assert str(ref["input_hash"]) == _golden_input_hash(mfp, tgt, T0, probes)
    lat = Lattice(n, n, 64, mfp=16.0, x_edge="blackbody", y_edge="periodic")
    series = ProbeSeries(lat, probes, 1000, 10, checkpoint_every=50)
    walls = np.array([0.5, 0.0, 0.0, 0.0], dtype=np.float32)
    out, loss, g_mfp, g_T0, g_w = _gpu_grads(series, mfp, T0, walls,
                                             ref["targets"].astype(np.float32))
    T_ref = ref["T_probes"]
    err_T = np.abs(out - T_ref).max() / np.abs(T_ref).max()
    err_mfp = np.abs(g_mfp - ref["g_mfp"]).max() / np.abs(ref["g_mfp"]).max()
    err_T0 = np.abs(g_T0 - ref["g_T0"]).max() / np.abs(ref["g_T0"]).max()
    err_w = np.abs(g_w - ref["g_walls"]).max() / np.abs(ref["g_walls"]).max()
    print(f"probe T {err_T:.2e}, loss {abs(loss - ref['loss']) / ref['loss']:.2e}, "
          f"dL/dMFP {err_mfp:.2e}, dL/dT0 {err_T0:.2e}, walls {err_w:.2e}")
    assert err_T <= 1e-5
    assert abs(loss - float(ref["loss"])) <= 1e-4 * float(ref["loss"])
    assert err_mfp <= GRAD_RTOL_1000
    assert err_T0 <= GRAD_RTOL_1000
    assert err_w <= GRAD_RTOL_1000
    lat.close()


def test_c4_full_size_directional_derivatives():
    """Full size: <grad, v> against central differences of the GPU forward
    along smooth directions of the MFP field and of T0, and for each wall."""
    n, mfp, tgt, T0, probes = inputs.inverse_problem_256()
    from paper_1911_00180_amd.autodiff import ProbeSeries
    from paper_1911_00180_amd.lattice import Lattice
    lat = Lattice(n, n, 64, mfp=16.0, x_edge="blackbody", y_edge="periodic")
    series = ProbeSeries(lat, probes, 1000, 10, checkpoint_every=50)
    dev = "cuda"
    walls = torch.tensor([0.5, 0.0, 0.0, 0.0], device=dev)
    with torch.no_grad():
        target = series(torch.from_numpy(tgt).to(dev), torch.from_numpy(T0).to(dev), walls)

    def loss_of(m, t, w):
        with torch.no_grad():
            out = series(m, t, w)
        return float(((out.double() - target.double()) ** 2).sum())

    m = torch.from_numpy(mfp).to(dev).requires_grad_(True)
    t = torch.from_numpy(T0).to(dev).requires_grad_(True)
    w = walls.clone().requires_grad_(True)
    out = series(m, t, w)
    ((out - target) ** 2).sum().backward()
    v = torch.from_numpy(inputs.smooth_lognormal_field(n, n, 7, 8.0, 1.0, 1.0, 0.1, 10.0)
                         .astype(np.float32)).to(dev)
    v = v / v.abs().max()
    for name, base, g, d, h in [("mfp", m, m.grad, v * torch.from_numpy(mfp).to(dev), 1e-3),
                                ("T0", t, t.grad, v, 1e-2)]:
        lp = loss_of(*(x.detach() + h * d if x is base else x.detach() for x in (m, t, w)))
        lm = loss_of(*(x.detach() - h * d if x is base else x.detach() for x in (m, t, w)))
        fd = (lp - lm) / (2 * h)
        an = float((g.double() * d.double()).sum())
        print(f"{name}: adjoint {an:.6e}  central difference {fd:.6e}")
        assert abs(an - fd) <= 2e-3 * abs(fd)
    for k in (0,):
        e = torch.zeros(4, device=dev)
        e[k] = 1.0
        h = 1e-2
        fd = (loss_of(m.detach(), t.detach(), w.detach() + h * e)
              - loss_of(m.detach(), t.detach(), w.detach() - h * e)) / (2 * h)
        an = float(w.grad[k])
        print(f"wall {k}: adjoint {an:.6e}  central difference {fd:.6e}")
        assert abs(an - fd) <= 2e-3 * abs(fd)
    lat.close()


def test_c5_adjoint_2048_q128_directional_derivatives():
    """The 2048 x 2048, Q = 128 inverse problem (MFP correlation 128 cells,
    pulse sigma0 = 128, blackbody x walls at 0.5 and 0, periodic y) over 200
    steps with a checkpoint every 20: <grad, v> against the chain rule through
    central differences of the GPU forward's probe temperatures,
    sum_k 2 (T_k - T^_k) (T_k(+h v) - T_k(-h v)) / 2h.  For a fixed MFP field
    the probe temperatures are affine in T0 and the wall temperatures, so these
    differences have no truncation error; the MFP direction uses a small
    relative step.  The sum can cancel (mismatches of both signs), so the
    error is held to 2e-3 of the sum of the magnitudes of its terms."""
    from paper_1911_00180_amd.autodiff import ProbeSeries
    from paper_1911_00180_amd.lattice import Lattice
    n, mfp, tgt, T0, probes = inputs.inverse_problem(2048)
    lat = Lattice(n, n, 128, mfp=16.0, x_edge="blackbody", y_edge="periodic")
    series = ProbeSeries(lat, probes, 200, 10, checkpoint_every=20)
    dev = "cuda"
    walls = torch.tensor([0.5, 0.0, 0.0, 0.0], device=dev)
    with torch.no_grad():
        target = series(torch.from_numpy(tgt).to(dev), torch.from_numpy(T0).to(dev), walls)

    def probes_of(m, t, w):
        with torch.no_grad():
            return series(m, t, w).double()

    m = torch.from_numpy(mfp).to(dev).requires_grad_(True)
    t = torch.from_numpy(T0).to(dev).requires_grad_(True)
    w = walls.clone().requires_grad_(True)
    out = series(m, t, w)
    loss = ((out - target) ** 2).sum()
    assert float(loss.detach()) > 0
    loss.backward()
    resid = 2.0 * (out.detach().double() - target.double())
    v = torch.from_numpy(inputs.smooth_lognormal_field(n, n, 7, 64.0, 1.0, 1.0, 0.1, 10.0)
                         .astype(np.float32)).to(dev)
    v = v / v.abs().max()
    e0 = torch.zeros(4, device=dev)
    e0[0] = 1.0
    checks = [("mfp", 0, m.grad, v * torch.from_numpy(mfp).to(dev), 1e-3),
              ("T0", 1, t.grad, v, 1e-2),
              ("wall 0", 2, w.grad, e0, 1e-2)]
    for name, k, g, d, h in checks:
        args_p = [x.detach() for x in (m, t, w)]
        args_m = [x.detach() for x in (m, t, w)]
        args_p[k] = args_p[k] + h * d
        args_m[k] = args_m[k] - h * d
        dout = (probes_of(*args_p) - probes_of(*args_m)) / (2 * h)
        fd = float((resid * dout).sum())
        scale = float((resid * dout).abs().sum())
        an = float((g.double() * d.double()).sum())
        print(f"{name}: adjoint {an:.6e}  central difference {fd:.6e}  scale {scale:.6e}")
        assert scale > 0
        assert abs(an - fd) <= 2e-3 * scale
    lat.close()
    del series, out, loss
    torch.cuda.empty_cache()
