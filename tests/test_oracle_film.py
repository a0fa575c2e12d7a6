"""Pins of the film-conductivity oracle (oracle/film.py).

* Ballistic closed form: with W = 0 and no y walls, every direction that
  points away from the hot wall carries w_i T_h once it has crossed the film,
  the others carry T_c = 0 (or the initial 0), so the interior flux is
  exactly T_h * sum_{s_x > 0} w_i s_x,i.
* Ordering (Sec. 3.5: boundary scattering lowers the in-plane conductivity):
  kappa_eff/kappa falls as Kn grows, and diffuse walls conduct less than no
  walls at the same Kn.
"""
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
