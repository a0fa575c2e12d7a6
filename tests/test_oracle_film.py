"""Pins of the film-conductivity oracle (oracle/film.py).

* Ballistic closed form: with W = 0 and no y walls, every direction that
  points away from the hot wall carries w_i T_h once it has crossed the film,
  the others carry T_c = 0 (or the initial 0), so the interior flux is
  exactly T_h * sum_{s_x > 0} w_i s_x,i.
* Ordering (Sec. 3.5: boundary scattering lowers the in-plane conductivity):
  kappa_eff/kappa falls as Kn grows, and diffuse walls conduct less than no
  walls at the same Kn.
* Scale of kappa_ratio, fixed independently of it: in a steady wall-free
  slab the exact energy current carried across each face by the step
  (face_current, counted from the push form) is the same on every face, it
  equals the lattice diffusivity measured from the spreading of a free pulse
  (second moment, d<r^2>/dt = 4 alpha) times the bulk gradient, and
  kappa_ratio fed with that current, times L*/(nx - 1) with L* = dT/|grad T|
  the effective length of the bulk profile, gives alpha / (Lambda / d).  A
  wrong length (nx for nx - 1), dimension or flux scale in kappa_ratio fails
  this (planted in copies of oracle/film.py below).
* The flux of Eq. q_corr exceeds that current at large W by a share first
  order in W: (q/J - 1) * MFP stays between 0.4 and 0.55 at MFP 1.28 and 4.
"""
import os

import numpy as np
import pytest

from oracle import film
from oracle import worm_lbm as o


def _cfg(nx, ny, q, mfp, y_edge, **kw):
    return o.Config(nx=nx, ny=ny, q=q, mfp=mfp, x_edge="blackbody", y_edge=y_edge,
                    t_x_lo=1.0, t_x_hi=0.0, **kw)


@pytest.mark.parametrize("q,kind", [(16, "uniform"), (24, "ring")])
def test_ballistic_flux_closed_form(q, kind):
    cfg = _cfg(20, 3, q, np.inf, "periodic", dirs=kind)
    _, qx, qy = film.film_run(cfg, 240, window=10)
    lat = o.Lattice(cfg)
    want = sum(lat.w[i] * lat.s[i, 0] for i in range(q) if lat.s[i, 0] > 1e-12)
    assert np.max(np.abs(qx[:, 1:-1] - want)) < 1e-13
    # no net flux across the film for a symmetric direction set
    assert np.max(np.abs(qy[:, 1:-1])) < 1e-13


def test_kappa_falls_with_knudsen_and_with_walls():
    ny, nx, n = 6, 24, 5000
    k_diffuse = [film.film_kappa(_cfg(nx, ny, 16, kn * ny, "diffuse"), n) for kn in (0.5, 2, 8)]
    k_free = [film.film_kappa(_cfg(nx, ny, 16, kn * ny, "periodic"), n) for kn in (0.5, 2, 8)]
    assert k_diffuse[0] > k_diffuse[1] > k_diffuse[2] > 0
    assert k_free[0] > k_free[1] > k_free[2] > 0
    for a, b in zip(k_diffuse, k_free):
        assert a < b


def _diffusivity(mfp, q, nx=160, sigma=6.0, n1=60, n2=200):
    """Lattice diffusivity from the growth of the second moment of a free
    Gaussian pulse on a periodic lattice (the pulse stays far from the
    edges): d<r^2>/dt = 4 alpha in 2D."""
    lat = o.Lattice(o.Config(nx=nx, ny=nx, q=q, mfp=mfp))
    x = np.arange(nx) - nx // 2
    r2 = x[None, :] ** 2 + x[:, None] ** 2
    lat.set_temperature(np.exp(-r2 / (2 * sigma ** 2)))
    lat.run(n1)
    T1 = lat.temperature()
    lat.run(n2)
    T2 = lat.temperature()
    return ((T2 * r2).sum() / T2.sum() - (T1 * r2).sum() / T1.sum()) / (4 * n2)


def _slab(fm, nx, mfp, settle):
    """Steady wall-free slab (periodic y, one row) between T_h = 1 and
    T_c = 0: (current per face, q_x, bulk gradient, L*)."""
    cfg = _cfg(nx, 1, 16, mfp, "periodic")
    J, qx, T = fm.slab_steady(cfg, settle=settle, window=1000)
    lo, hi = nx // 4, 3 * nx // 4
    g = abs(np.polyfit(np.arange(lo, hi), T[0, lo:hi], 1)[0])
    return cfg, J, qx, g, (cfg.t_x_lo - cfg.t_x_hi) / g


def check_kappa_scale(fm):
    mfp, nx = 1.28, 48
    cfg, J, qx, g, Lstar = _slab(fm, nx, mfp, settle=3200)
    Jm = J[1:-1].mean()
    assert np.abs(J[1:-1] - Jm).max() <= 1e-4 * abs(Jm)        # conservation
    alpha = _diffusivity(mfp, 16)
    assert abs(Jm / g - alpha) <= 5e-3 * alpha, (Jm / g, alpha)
    field = np.zeros((1, nx))
    field[:, 1:nx - 1] = Jm
    k = fm.kappa_ratio(cfg, field)
    want = alpha / (mfp / 2.0)
    assert abs(k * Lstar / (nx - 1) - want) <= 5e-3 * want, (k * Lstar / (nx - 1), want)
    return Jm, qx[0, 1:-1].mean()


def test_kappa_scale_pinned_by_energy_current_and_diffusivity():
    check_kappa_scale(film)


def test_q_corr_flux_exceeds_the_current_to_first_order():
    excess = []
    for mfp, nx, settle in ((1.28, 48, 3200), (4.0, 64, 2500)):
        _, J, qx, _, _ = _slab(film, nx, mfp, settle)
        ratio = qx[0, 1:-1].mean() / J[1:-1].mean()
        excess.append((ratio - 1.0) * mfp)
        assert ratio > 1.0
    for e in excess:
        assert 0.4 <= e <= 0.55, excess


FILM = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "oracle", "film.py")

FILM_MUTATIONS = {
    "kappa_length_nx": ("kappa_eff = q_mean * (cfg.nx - 1) / (cfg.t_x_lo - cfg.t_x_hi)",
                        "kappa_eff = q_mean * cfg.nx / (cfg.t_x_lo - cfg.t_x_hi)"),
    "kappa_dimension_three": ("d = 3.0 if cfg.emulate_3d else 2.0", "d = 3.0"),
    "kappa_interior_includes_walls": ("q_mean = float(np.mean(qx_avg[:, 1:cfg.nx - 1]))",
                                      "q_mean = float(np.mean(qx_avg))"),
    "current_without_eed_on_pause": ("        moved = W * lat.w[i] * E\n        if hp[i]:\n"
                                     "            moved = moved + (1.0 - W) * lat.e[i]",
                                     "        moved = 0.0 * E\n        if hp[i]:\n"
                                     "            moved = W * lat.w[i] * E + (1.0 - W) * lat.e[i]"),
}


@pytest.mark.parametrize("name", sorted(FILM_MUTATIONS))
def test_film_mutation_is_caught(name):
    import types
    old, new = FILM_MUTATIONS[name]
    with open(FILM) as f:
        src = f.read()
    assert src.count(old) == 1, f"snippet of {name} must occur exactly once"
    mod = types.ModuleType("oracle.film_mutant")
    mod.__file__ = FILM
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), FILM, "exec"), mod.__dict__)
    with pytest.raises(AssertionError):
        check_kappa_scale(mod)
