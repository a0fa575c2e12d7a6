"""Pins of the FP64 oracle gradients (oracle/adjoint.py).

The transposed step is checked against the Jacobian of the oracle's forward
step built column by column (brute force on tiny lattices), and the loss
gradients against central differences of the forward loss.  The loss is
quadratic in the populations and the populations are affine in T0 and in the
wall temperatures, so central differences are exact there up to rounding; in
the mean free path they carry an O(h^2) error.
"""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import worm_lbm as o
from paper_1911_00180_amd import inputs

EDGES = [("periodic", "periodic"), ("blackbody", "periodic"),
         ("periodic", "blackbody"), ("blackbody", "blackbody")]


def _jacobian(lat, n):
    """d e^n / d e^{n-1} of oracle step n, one column per unit population."""
    c = lat.cfg
    N = c.q * c.ny * c.nx
    J = np.zeros((N, N))
    lat.set_populations(np.zeros((c.q, c.ny, c.nx)))
    lat.n = n - 1
    lat.step()
    base = lat.e.ravel().copy()
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        lat.set_populations(e.reshape(c.q, c.ny, c.nx))
        lat.n = n - 1
        lat.step()
        J[:, k] = lat.e.ravel() - base
    return J


@pytest.mark.parametrize("x_edge,y_edge", EDGES)
@pytest.mark.parametrize("q,kind", [(8, "uniform"), (16, "ring")])
def test_transposed_step_equals_jacobian_transpose(x_edge, y_edge, q, kind):
    rng = np.random.default_rng(5)
    nx, ny = 5, 4
    mfp = rng.uniform(1.5, 6.0, size=(ny, nx))
    cfg = o.Config(nx=nx, ny=ny, q=q, mfp=mfp, dirs=kind, x_edge=x_edge, y_edge=y_edge,
                   t_x_lo=0.3, t_x_hi=0.7, t_y_lo=0.2, t_y_hi=0.9)
    lat = o.Lattice(cfg)
    own = adj._wall_owner(cfg)
    for n in range(1, 13):
        J = _jacobian(lat, n)
        lam = rng.standard_normal((q, ny, nx))
        lam_p = lam.copy()
        lam_p[:, own != ""] = 0.0       # the overwritten outputs carry no state
        got, _ = adj.transposed_step(lat, n, lam_p)
        want = (J.T @ lam.ravel()).reshape(q, ny, nx)
        assert np.max(np.abs(got - want)) < 1e-13, n


def _problem(x_edge, y_edge, emulate_3d=False, q=16, kind="uniform"):
    nx, ny = 12, 10
    mfp = inputs.smooth_lognormal_field(nx, ny, 1, 3.0, 4.0, 0.6, 2.0, 12.0)
    cfg = o.Config(nx=nx, ny=ny, q=q, mfp=mfp, dirs=kind, x_edge=x_edge, y_edge=y_edge,
                   emulate_3d=emulate_3d, t_x_lo=0.5, t_x_hi=0.0, t_y_lo=0.25, t_y_hi=0.1)
    T0 = inputs.gaussian_pulse(nx, ny, 2.5, 6, 5, periodic=True)
    probes = inputs.probe_cells(3, nx, ny, 6)
    nsteps, every = 40, 5
    targets = np.random.default_rng(2).uniform(0.0, 0.3, size=(nsteps // every, len(probes)))
    return cfg, T0, nsteps, probes, every, targets


def _loss(cfg, T0, nsteps, probes, every, targets):
    return adj.probe_loss(cfg, T0, nsteps, probes, every, targets)[0]


def _with(cfg, **kw):
    d = dict(cfg.__dict__)
    d.update(kw)
    return o.Config(**d)


@pytest.mark.parametrize("x_edge,y_edge,emulate_3d,q,kind", [
    ("blackbody", "periodic", False, 16, "uniform"),
    ("blackbody", "blackbody", True, 16, "uniform"),
    ("periodic", "periodic", False, 24, "ring"),
])
def test_gradients_match_central_differences(x_edge, y_edge, emulate_3d, q, kind):
    cfg, T0, nsteps, probes, every, targets = _problem(x_edge, y_edge, emulate_3d, q, kind)
    loss, g_mfp, g_T0, g_Tb = adj.probe_loss_gradients(cfg, T0, nsteps, probes, every, targets)
    assert loss == pytest.approx(_loss(cfg, T0, nsteps, probes, every, targets), rel=1e-14)
    rng = np.random.default_rng(9)
    cells = [tuple(int(v) for v in rng.integers(0, [cfg.nx, cfg.ny])) for _ in range(6)]
    cells += [(0, 3), (cfg.nx - 1, 0), (5, 0)]          # wall and corner cells
    for (x, y) in cells:
        h = 1e-4 * cfg.mfp[y, x]
        mp, mm = cfg.mfp.copy(), cfg.mfp.copy()
        mp[y, x] += h
        mm[y, x] -= h
        fd = (_loss(_with(cfg, mfp=mp), T0, nsteps, probes, every, targets)
              - _loss(_with(cfg, mfp=mm), T0, nsteps, probes, every, targets)) / (2 * h)
        scale = max(np.abs(g_mfp).max(), 1e-300)
        assert abs(g_mfp[y, x] - fd) <= 1e-6 * scale, ("mfp", x, y)
        tp, tm = T0.copy(), T0.copy()
        tp[y, x] += 1e-3
        tm[y, x] -= 1e-3
        fd = (_loss(cfg, tp, nsteps, probes, every, targets)
              - _loss(cfg, tm, nsteps, probes, every, targets)) / 2e-3
        assert abs(g_T0[y, x] - fd) <= 1e-9 * max(np.abs(g_T0).max(), 1e-300), ("T0", x, y)
    walls = []
    if x_edge == "blackbody":
        walls += ["x_lo", "x_hi"]
    if y_edge == "blackbody":
        walls += ["y_lo", "y_hi"]
    for key in ("x_lo", "x_hi", "y_lo", "y_hi"):
        name = "t_" + key
        v = getattr(cfg, name)
        fd = (_loss(_with(cfg, **{name: v + 1e-3}), T0, nsteps, probes, every, targets)
              - _loss(_with(cfg, **{name: v - 1e-3}), T0, nsteps, probes, every, targets)) / 2e-3
        if key in walls:
            assert abs(g_Tb[key] - fd) <= 1e-9 * max(abs(fd), 1e-12), key
            assert fd != 0.0
        else:
            assert g_Tb[key] == 0.0 and fd == 0.0


def test_gradient_nonzero_where_signal_reaches():
    """Sanity of the setup used above: the probes see both the pulse and the
    walls within the horizon, so every gradient is exercised."""
    cfg, T0, nsteps, probes, every, targets = _problem("blackbody", "blackbody")
    _, g_mfp, g_T0, g_Tb = adj.probe_loss_gradients(cfg, T0, nsteps, probes, every, targets)
    assert np.count_nonzero(g_mfp) > 0.9 * g_mfp.size
    assert np.count_nonzero(g_T0) > 0.5 * g_T0.size
    assert all(v != 0.0 for v in g_Tb.values())


def test_diffuse_edges_rejected():
    cfg = o.Config(nx=8, ny=8, q=8, mfp=4.0, y_edge="diffuse")
    with pytest.raises(ValueError):
        adj.probe_loss(cfg, np.zeros((8, 8)), 4, np.array([[1, 1]]), 2, np.zeros((2, 1)))
