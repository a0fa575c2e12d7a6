"""Pins of the specular / specular-diffuse walls and the internal sources of
the oracle (Sec. 2.6, Eq. adiabatic-specular, Eq. isotropic, Eq. anisotropic,
Eq. lbm-heat-flux).

* Method of images: a film with specular y walls evolves exactly as the
  periodic film of twice the height whose upper half holds the mirror image
  (rows reversed, every direction replaced by its mirror direction) of the
  lower half, for any relaxation field that is mirrored too.
* Specular-diffuse walls conserve energy and, with a uniform relaxation
  weight, keep a uniform isotropic state fixed, for every specular fraction.
* A source cell in a ballistic (W = 0) periodic lattice lays its imposed
  values along each direction's worm path: after n steps direction i holds
  v_i at x0 + P_i(n) - P_i(m), m = 0 .. n, and zero elsewhere.
* Flux distributions: for the evenly spaced set sum_i w_i s_i s_i^T = I / 2,
  so the distribution with temperature T and flux q is w_i (T + 2 q . s_i).
"""
import numpy as np
import pytest

from oracle import worm_lbm as o


def _mirror_state(lat, e):
    """Doubled-height state: lower half e, upper half its mirror image."""
    q, ny, nx = e.shape
    e2 = np.zeros((q, 2 * ny, nx))
    e2[:, :ny] = e
    for i in range(q):
        e2[lat.mirror_y[i], ny:] = e[i, ::-1]
    return e2


@pytest.mark.parametrize("q,kind,x_edge", [(16, "uniform", "periodic"), (24, "ring", "periodic"),
                                           (16, "uniform", "blackbody")])
def test_specular_film_equals_mirrored_periodic_film(q, kind, x_edge):
    rng = np.random.default_rng(21)
    nx, ny = 11, 5
    mfp = rng.uniform(1.5, 8.0, size=(ny, nx))
    kw = dict(nx=nx, q=q, dirs=kind, x_edge=x_edge, t_x_lo=0.7, t_x_hi=0.2)
    film = o.Lattice(o.Config(ny=ny, mfp=mfp, y_edge="diffuse", y_specularity=1.0, **kw))
    twin = o.Lattice(o.Config(ny=2 * ny, mfp=np.vstack([mfp, mfp[::-1]]), y_edge="periodic",
                              **kw))
    e0 = rng.random((q, ny, nx))
    film.set_populations(e0)
    film._apply_blackbody(film.e)
    twin.set_populations(_mirror_state(film, film.e))
    for _ in range(40):
        film.step()
        twin.step()
        assert np.max(np.abs(twin.e[:, :ny] - film.e)) < 1e-12
        assert np.max(np.abs(twin.e - _mirror_state(film, film.e))) < 1e-12


@pytest.mark.parametrize("p", [0.0, 0.35, 1.0])
def test_specular_diffuse_conserves_energy_and_keeps_equilibrium(p):
    rng = np.random.default_rng(3)
    nx, ny, q = 9, 6, 16
    mfp = rng.uniform(1.5, 6.0, size=(ny, nx))
    lat = o.Lattice(o.Config(nx=nx, ny=ny, q=q, mfp=mfp, y_edge="diffuse", y_specularity=p))
    lat.set_populations(rng.random((q, ny, nx)))
    e0 = lat.energy()
    for _ in range(25):
        lat.step()
    assert abs(lat.energy() - e0) < 1e-12 * e0
    # (with a per-cell field a pause mixes the weights of two cells, so the
    # fixed point needs a uniform one)
    lat = o.Lattice(o.Config(nx=nx, ny=ny, q=q, mfp=3.5, y_edge="diffuse", y_specularity=p))
    lat.set_temperature(np.full((ny, nx), 0.8))
    for _ in range(25):
        lat.step()
    assert np.max(np.abs(lat.e - lat.w[:, None, None] * 0.8)) < 1e-14


@pytest.mark.parametrize("q,kind", [(16, "uniform"), (24, "ring")])
def test_source_lays_values_along_worm_paths(q, kind):
    rng = np.random.default_rng(8)
    nx = ny = 41
    x0, y0 = 20, 20
    vals = rng.uniform(0.5, 1.5, size=q)
    cfg = o.Config(nx=nx, ny=ny, q=q, dirs=kind, source_cells=np.array([[x0, y0]]),
                   source_values=vals[None, :])
    lat = o.Lattice(cfg)
    lat.set_temperature(np.zeros((ny, nx)))
    n = 15
    for _ in range(n):
        lat.step()
    pos = lat.schedule(n).pos   # worm positions after steps 1 .. n
    want = np.zeros((q, ny, nx))
    for i in range(q):
        P = np.vstack([[0, 0], pos[:n, i]])
        for m in range(n + 1):
            dx, dy = P[n] - P[m]
            want[i, (y0 + dy) % ny, (x0 + dx) % nx] = vals[i]
    assert np.array_equal(lat.e, want)


def test_source_wins_over_blackbody_wall_and_is_imposed_at_start():
    q = 8
    vals = np.arange(1, q + 1, dtype=float)
    cfg = o.Config(nx=6, ny=5, q=q, mfp=3.0, x_edge="blackbody", t_x_lo=2.0,
                   source_cells=np.array([[0, 2], [3, 3]]), source_values=np.vstack([vals, -vals]))
    lat = o.Lattice(cfg)
    lat.set_temperature(np.ones((5, 6)))
    assert np.array_equal(lat.e[:, 2, 0], vals) and np.array_equal(lat.e[:, 3, 3], -vals)
    lat.step()
    assert np.array_equal(lat.e[:, 2, 0], vals) and np.array_equal(lat.e[:, 3, 3], -vals)
    assert np.allclose(lat.e[:, 1, 0], lat.w * 2.0)


def test_flux_distribution_uniform_closed_form():
    rng = np.random.default_rng(4)
    for q in (8, 16, 64):
        lat = o.Lattice(o.Config(nx=4, ny=4, q=q))
        T, qv = 0.7, rng.normal(size=2) * 0.1
        e = o.flux_distribution(lat.dirs, lat.w, T, qv)
        assert np.allclose(e, lat.w * (T + 2.0 * (lat.s @ qv)), atol=1e-15)
    lat = o.Lattice(o.Config(nx=4, ny=4, q=24, dirs="ring"))
    e = o.flux_distribution(lat.dirs, lat.w, 0.3, np.array([0.02, -0.05]))
    assert abs(e.sum() - 0.3) < 1e-15
    assert np.allclose(lat.s.T @ e, [0.02, -0.05], atol=1e-15)


# ---------------------------------------------------------------------------
# Angle-dependent grid speed (Sec. 2.3)
# ---------------------------------------------------------------------------
def test_unit_speeds_give_the_isotropic_schedule():
    for q, kind in ((16, "uniform"), (24, "ring")):
        dirs = o.make_directions(q, kind)
        a = o.tas_schedule(dirs, 300)
        b = o.tas_schedule(dirs, 300, speeds=np.ones(q))
        assert np.array_equal(a.move, b.move) and np.array_equal(a.hop, b.hop)


@pytest.mark.parametrize("v", [0.5, 0.3, 0.75, 0.999])
def test_axial_hop_count_closed_form(v):
    """An axial direction at speed v has made min(n, floor(v n + 1)) hops
    after n steps (one hop per step at most; the worm may lead by one
    cell)."""
    dirs = o.make_directions(16, "uniform")
    sch = o.tas_schedule(dirs, 400, speeds=np.full(16, v))
    for n in range(1, 401):
        k = int(np.abs(sch.pos[n - 1, 0]).sum())       # direction 0 is +x
        assert k == min(n, int(np.floor(v * n + 1.0))), n


def test_worm_keeps_to_its_speed():
    """Every worm stays within radius v_i n + 1 and, once started, at most
    one diagonal hop (sqrt 2) plus the lead of one cell behind it."""
    rng = np.random.default_rng(5)
    for q, kind in ((16, "uniform"), (32, "ring")):
        dirs = o.make_directions(q, kind)
        v = rng.uniform(0.2, 1.0, size=q)
        sch = o.tas_schedule(dirs, 500, speeds=v)
        r = np.hypot(sch.pos[..., 0], sch.pos[..., 1])
        n = np.arange(1, 501)[:, None]
        assert np.all(r <= v[None, :] * n + 1.0 + 1e-12)
        assert np.all(r >= v[None, :] * n + 1.0 - np.sqrt(2.0) - 1.0)


def test_slowed_axis_travels_at_its_speed():
    """Directions nearer the x axis slowed to half speed: after n steps the
    +x worm is at v n + 1 and the +y worm at n."""
    q = 32
    lat0 = o.Lattice(o.Config(nx=4, ny=4, q=q))
    v = np.where(np.abs(lat0.s[:, 0]) > np.abs(lat0.s[:, 1]), 0.5, 1.0)
    n = 60
    sch = o.tas_schedule(lat0.dirs, n, speeds=v)
    assert tuple(sch.pos[n - 1, 0]) == (31, 0)        # direction 0: +x
    assert tuple(sch.pos[n - 1, q // 4]) == (0, 60)   # direction q/4: +y
