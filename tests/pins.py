"""Pins of the FP64 oracle: facts that the paper or the mathematics fix.

Every pin is a function of the oracle module ``o`` that raises AssertionError
when the oracle disagrees.  The test suite runs them on the oracle as it is
(test_oracle_pins.py) and on copies of it with a planted mistake
(test_oracle_mutations.py), where at least one pin must fail.
"""
from __future__ import annotations

import math

import numpy as np

from conftest import read_golden


def _dir_index(o, dirs, vx, vy):
    for i, d in enumerate(dirs):
        if abs(d.sx - vx) < 1e-12 and abs(d.sy - vy) < 1e-12:
            return i
    raise AssertionError("direction not found")


# -- Sec. 2.3, Fig. 2: the TAS worked example --------------------------------
def pin_tas_d2q8_diagonal(o):
    g = read_golden("tas_d2q8_diagonal.txt")
    hops = [int(v) for v in g["hops"]]
    pauses = [int(v) for v in g["pauses"]]
    dirs = o.make_directions(8, "uniform")
    r2 = math.sqrt(0.5)
    for (vx, vy) in [(r2, r2), (-r2, r2), (-r2, -r2), (r2, -r2)]:
        i = _dir_index(o, dirs, vx, vy)
        sch = o.tas_schedule(dirs, 5)
        got_h = [n + 1 for n in range(5) if sch.hop[n, i]]
        got_p = [n + 1 for n in range(5) if not sch.hop[n, i]]
        assert got_h == hops and got_p == pauses, (got_h, got_p)


# -- Sec. 3.1 and Sec. 4: the propagation error is at most one cell -----------
def pin_propagation_error(o):
    for q, kind in [(16, "uniform"), (64, "uniform"), (16, "ring"), (48, "ring")]:
        dirs = o.make_directions(q, kind)
        nsteps = 300
        sch = o.tas_schedule(dirs, nsteps)
        n = np.arange(1, nsteps + 1)[:, None]
        r = np.hypot(sch.pos[..., 0], sch.pos[..., 1])
        assert np.all(r <= n + 1 + 1e-12), "outside the TAS circle"
        assert np.all(r >= n - 1 - 1e-12), "more than one cell behind"
        s = np.array([[d.sx, d.sy] for d in dirs])
        # perpendicular distance of the worm from the ray: at most one cell
        perp = np.abs(sch.pos[..., 0] * s[None, :, 1] - sch.pos[..., 1] * s[None, :, 0])
        assert perp.max() <= 1.0, perp.max()
        # axial directions are never paused (Sec. 3.1) and are exact
        for i, d in enumerate(dirs):
            if d.sx == 0.0 or d.sy == 0.0:
                assert sch.hop[:, i].all()
                assert np.array_equal(r[:, i], n[:, 0].astype(float))


# -- Sec. 2.5: a ring direction's worm path repeats every M hops --------------
def pin_worm_repeats_on_lattice_vector(o):
    for m in (1, 2, 3, 4, 5, 8):
        for d in o.ring_directions(m):
            path = o.worm_path(d, 3 * m)
            px = py = 0
            vx, vy = d.ring_vec
            for k, mv in enumerate(path, start=1):
                ux, uy = o.D2Q8[mv]
                # moves stay in the direction's octant: one step along the
                # major axis, and never against the minor component
                assert ux * vx >= 0 and uy * vy >= 0
                px += ux
                py += uy
                if k % m == 0:
                    assert (px, py) == (vx * k // m, vy * k // m), (d.ring_vec, k)
            # the sequence has period M
            assert path[:m] == path[m:2 * m] == path[2 * m:3 * m]


# -- Sec. 2.4, Fig. 4 and Sec. 2.2: angular weights --------------------------
def pin_weights(o):
    g = read_golden("d2q16_weight_gaps.txt")
    dirs = o.ring_directions(2)
    phi = [d.angle for d in dirs] + [2 * math.pi]
    gaps = [phi[j + 1] - phi[j] for j in range(16)]
    ga = [gaps[int(j) - 1] for j in g["group_a"]]
    gb = [gaps[int(j) - 1] for j in g["group_b"]]
    assert max(ga) - min(ga) < 1e-14 and max(gb) - min(gb) < 1e-14
    w = o.weights(dirs)
    # the weight of direction j spans half of each neighbouring gap
    for j in range(16):
        assert abs(w[j] - (gaps[j - 1] + gaps[j]) / (4 * math.pi)) < 1e-15
    assert abs(w[0] - math.atan(0.5) / (2 * math.pi)) < 1e-15
    assert abs(w[1] - 1.0 / 16.0) < 1e-15
    for q in (8, 16, 64, 256):
        for kind in ("uniform", "ring"):
            assert abs(math.fsum(o.weights(o.make_directions(q, kind))) - 1.0) < 1e-14
        assert np.allclose(o.weights(o.make_directions(q, "uniform")), 1.0 / q, rtol=0, atol=1e-15)
        # the gap rule itself gives 1/Q for evenly spaced directions
        phi = [2.0 * math.pi * i / q for i in range(q)] + [2.0 * math.pi]
        gap = [phi[j + 1] - phi[j] for j in range(q)]
        assert max(abs((gap[j - 1] + gap[j]) / (4 * math.pi) - 1.0 / q) for j in range(q)) < 1e-15


# -- Sec. 2.3 Eq. W-correction-factor and its generalisation in Sec. 2.4 ------
def pin_lambda_corr(o):
    g = read_golden("lambda_corr_d2q8.txt")
    ref = float(g["numerator"][0]) / (float(g["denominator_sqrt2_plus"][0]) + math.sqrt(2.0))
    for kind in ("uniform", "ring"):
        assert abs(o.lambda_corr(o.make_directions(8, kind)) - ref) < 1e-15
    # many directions: the mean of 1/max(|cos|,|sin|) over the circle is
    # (4/pi) ln(1 + sqrt 2), so Lambda_corr -> pi / (4 ln(1 + sqrt 2))
    lim = math.pi / (4.0 * math.log(1.0 + math.sqrt(2.0)))
    assert abs(o.lambda_corr(o.make_directions(4096, "uniform")) - lim) < 1e-6
    # ring set: the hop speed sqrt(1 + (j/M)^2) is sampled uniformly in
    # t = j/M, so Lambda_corr -> 1 / int_0^1 sqrt(1 + t^2) dt
    lim_ring = 2.0 / (math.sqrt(2.0) + math.asinh(1.0))
    assert abs(o.lambda_corr(o.make_directions(8 * 512, "ring")) - lim_ring) < 1e-5


def pin_w_corr_limits(o):
    g = read_golden("w_corr_limits.txt")
    for f3 in (False, True):
        f = float(g["ratio_at_zero"][0]) if f3 else 1.0
        for q in (8, 64):
            lam = o.lambda_corr(o.make_directions(q, "uniform"))
            assert abs(o.w_corr(1e-9, lam, f3) / 1e-9 - f) < 1e-8
            want = (float(g["value_at_one_over_lambda"][0]) if f3 else 1.0) * lam
            assert abs(o.w_corr(1.0, lam, f3) - want) < 1e-15


# -- App. A: the stability limit W_corr <= 1 is enforced ----------------------
def pin_stability_guard(o):
    try:
        o.Lattice(o.Config(nx=4, ny=4, q=8, mfp=0.5, mfp_correction=False))
    except ValueError:
        pass
    else:
        raise AssertionError("W = 2 accepted")
    o.Lattice(o.Config(nx=4, ny=4, q=8, mfp=1.0, mfp_correction=False))


# -- Sec. 1, Sec. 4: exact advection (no smearing) at W = 0 ------------------
def pin_ballistic_exact(o):
    for q, kind, nx, ny in [(16, "uniform", 24, 20), (24, "ring", 17, 23)]:
        rng = np.random.default_rng(q)
        T0 = rng.random((ny, nx)).astype(np.float32).astype(np.float64)
        lat = o.Lattice(o.Config(nx=nx, ny=ny, q=q, mfp=math.inf, dirs=kind))
        lat.set_temperature(T0)
        n = 31
        lat.run(n)
        sch = lat.schedule(n)
        want = o.ballistic_temperature(T0, lat.w, sch.pos[n - 1])
        assert np.max(np.abs(lat.temperature() - want)) < 1e-14
        # each direction individually: a pure shift of its initial field
        for i in range(q):
            p = sch.pos[n - 1, i]
            assert np.array_equal(lat.e[i], lat.w[i] * np.roll(T0, (int(p[1]), int(p[0])), (0, 1)))


# -- Sec. 2.2: the collision conserves energy ----------------------------------
def pin_energy_conservation(o):
    rng = np.random.default_rng(7)
    for y_edge in ("periodic", "diffuse"):
        for mfp in (3.0, rng.uniform(1.5, 9.0, size=(13, 11))):
            for kind, q in (("uniform", 16), ("ring", 24)):
                lat = o.Lattice(o.Config(nx=11, ny=13, q=q, mfp=mfp, dirs=kind, y_edge=y_edge))
                lat.set_populations(rng.random((q, 13, 11)))
                e0 = lat.energy()
                lat.run(25)
                assert abs(lat.energy() - e0) < 1e-13 * e0, (y_edge, kind)


# -- Sec. 2.2: the isotropic equilibrium is a fixed point ---------------------
def pin_equilibrium_fixed_point(o):
    for kw in ({}, {"y_edge": "diffuse"},
               {"x_edge": "blackbody", "y_edge": "blackbody", "t_x_lo": 0.7,
                "t_x_hi": 0.7, "t_y_lo": 0.7, "t_y_hi": 0.7},
               {"x_edge": "blackbody", "y_edge": "diffuse", "t_x_lo": 0.7, "t_x_hi": 0.7}):
        for kind in ("uniform", "ring"):
            lat = o.Lattice(o.Config(nx=9, ny=7, q=16, mfp=2.5, dirs=kind, **kw))
            lat.set_temperature(np.full((7, 9), 0.7))
            e0 = lat.e.copy()
            lat.run(20)
            assert np.max(np.abs(lat.e - e0)) < 1e-14, kw


# -- Sec. 2.3: W = 1 reduces to the standard D2Q8 scheme -----------------------
def pin_w1_is_standard_d2q8(o):
    rng = np.random.default_rng(3)
    nx, ny = 10, 8
    lat = o.Lattice(o.Config(nx=nx, ny=ny, q=8, mfp=1.0, mfp_correction=False))
    lat.set_populations(rng.random((8, ny, nx)))
    for _ in range(6):
        E = lat.e.sum(axis=0)
        lat.step()
        for i, d in enumerate(lat.dirs):
            big = max(abs(d.sx), abs(d.sy))
            cx, cy = int(round(d.sx / big)), int(round(d.sy / big))
            want = lat.w[i] * np.roll(E, (cy, cx), (0, 1))
            assert np.max(np.abs(lat.e[i] - want)) < 1e-15


# -- App. A, Eq. stabil-prop / Eq. stabil-pause: Fourier symbol of a step ------
def pin_von_neumann(o):
    nx, W = 16, 0.3
    lat = o.Lattice(o.Config(nx=nx, ny=1, q=8, mfp=1.0 / W, mfp_correction=False))
    lat.run(2)                      # step 3 is a pause step of the diagonals
    kx = 2.0 * math.pi * 3 / nx
    x = np.arange(nx)
    u = np.cos(kx * x) + 0.5 * np.sin(kx * x) + 2.0
    lat.set_populations(lat.w[:, None, None] * u[None, None, :])
    sch = lat.schedule(3)
    lat.step()
    for i in range(8):
        mvx = o.D2Q8[int(sch.move[2, i])][0]
        paused = not sch.hop[2, i]
        before = np.fft.fft(lat.w[i] * u)[3]
        after = np.fft.fft(lat.e[i, 0])[3]
        # the numpy transform uses e^{-ikx}: a shift by +s multiplies by e^{-iks}
        g = o.growth_factor(W, -kx * mvx, paused)
        assert abs(after / before - g) < 1e-12, (i, after / before, g)
        assert abs(g) <= 1.0 + 1e-15


# -- Sec. 3.3: Fourier limit at small Kn ---------------------------------------
def pin_fourier_limit(o):
    """A Gaussian pulse spreads as the 2D heat kernel, with the diffusivity
    v Lambda / d of the emulated dimension d (d = 3 with the 3/2 factor of
    Eq. W-correction, else 2), approached to first order in 1/MFP."""
    mfp, q, nx, n1, n2 = 4.0, 8, 256, 40, 400
    for f3 in (False, True):
        lat = o.Lattice(o.Config(nx=nx, ny=nx, q=q, mfp=mfp, emulate_3d=f3))
        c = nx // 2
        x = np.arange(nx) - c
        r2 = x[None, :] ** 2 + x[:, None] ** 2
        lat.set_temperature(np.exp(-r2 / (2 * (3 * mfp) ** 2)))
        lat.run(n1)
        T1 = lat.temperature()
        m1 = (T1 * r2).sum() / T1.sum()
        lat.run(n2)
        T2 = lat.temperature()
        m2 = (T2 * r2).sum() / T2.sum()
        alpha = (m2 - m1) / (4 * n2)
        d = 3.0 if f3 else 2.0
        ratio = alpha / (mfp / d)
        assert 0.93 < ratio < 1.0, ratio
        # the profile is the (periodic) 2D heat kernel of that diffusivity
        s2 = m1 / 2.0 + 2.0 * alpha * n2
        g = sum(np.exp(-(x + k * nx) ** 2 / (2 * s2)) for k in (-1, 0, 1))
        kern = g[None, :] * g[:, None]
        kern *= T2.sum() / kern.sum()
        assert np.max(np.abs(T2 - kern)) < 0.025 * T2.max()


# -- Sec. 3.4, Eq. 1D-ball-2D: ballistic emission of a blackbody wall ---------
def pin_ballistic_wall(o):
    q, nx, n = 64, 130, 100
    lat = o.Lattice(o.Config(nx=nx, ny=1, q=q, mfp=math.inf, x_edge="blackbody",
                             t_x_lo=1.0, t_x_hi=0.0))
    lat.set_temperature(np.zeros((1, nx)))
    lat.run(n)
    T = lat.temperature()[0]
    x = np.arange(nx, dtype=float)
    def theta(xx):
        return np.where(xx < n, np.arccos(np.clip(xx / n, 0.0, 1.0)), 0.0) / np.pi
    lo = np.minimum(theta(x - 1), theta(x + 1))
    hi = np.maximum(theta(x - 1), theta(x + 1))
    viol = np.maximum(lo - T, T - hi)[1:n - 1]
    assert viol.max() <= 1.0 / q, viol.max()
    # behind the front the wall's emission is a half-space of isotropic
    # radiation: T -> 1/2 and q_x -> (1/2pi) * int cos = 1/pi, q_y = 0
    qx, qy = lat.heat_flux()
    # (the two directions parallel to the wall never leave it: 1/Q short)
    assert abs(T[1] - 0.5) <= 1.0 / q + 1e-12
    assert abs(qx[0, 1] - 1.0 / math.pi) < 2.0 / q
    assert np.max(np.abs(qy)) < 1e-12


# -- Sec. 3.1: the one-pixel source and the angular-space-filling criterion --
def pin_one_pixel_source(o):
    """A pixel held at T = 1 by an isotropic source (Eq. isotropic) in a
    51 x 51 periodic domain at T = 0, ballistic, 20 steps, ring sets of the
    paper's figure (Q = 8, 16, 32, 512).  Q >= 2 pi n (ASF) fills every cell
    within the propagated radius; fewer directions leave rays with gaps that
    shrink as Q grows; nothing is lit farther than n + 1 cells (the
    propagation error is at most one pixel, the bound stated in the same
    section)."""
    N, n = 51, 20
    c = N // 2
    x = np.arange(N) - c
    r = np.sqrt(x[None, :] ** 2 + x[:, None] ** 2)
    ann = (r > 12) & (r <= n - 2)
    frac = {}
    for q in (8, 16, 32, 512):
        w = o.Lattice(o.Config(nx=N, ny=N, q=q, dirs="ring")).w
        lat = o.Lattice(o.Config(nx=N, ny=N, q=q, dirs="ring", source_cells=np.array([[c, c]]),
                                 source_values=w[None, :]))
        lat.set_temperature(np.zeros((N, N)))
        lat.run(n)
        lit = lat.temperature() > 0
        assert r[lit].max() <= n + 1, (q, r[lit].max())
        frac[q] = lit[ann].mean()
    assert 512 >= 2 * math.pi * n and frac[512] == 1.0
    assert frac[8] < frac[16] < frac[32] < 0.5, frac


# -- Sec. 3.4, Eq. 1DT: cross-plane transport in the Fourier limit -----------
def _cross_plane_series(X, a, terms=400):
    th = 1.0 - X
    for l in range(1, terms):
        th -= 2.0 / (math.pi * l) * np.sin(l * math.pi * X) * np.exp(-(l * math.pi) ** 2 * a)
    return th


def pin_cross_plane_fourier(o):
    """Ny = 1 periodic, blackbody walls T = 1 / 0 at x = 0 / Nx - 1, start at
    T = 0, MFP 2 cells (Kn 0.02), Q = 16: the profile follows the transient
    series of Eq. 1DT with the lattice diffusivity MFP / 2 (d = 2), to within
    the wall slip of order Kn, the closer the later."""
    nx, mfp = 101, 2.0
    L = nx - 1
    X = np.arange(nx) / L
    lat = o.Lattice(o.Config(nx=nx, ny=1, q=16, mfp=mfp, x_edge="blackbody", t_x_lo=1.0,
                             t_x_hi=0.0))
    lat.set_temperature(np.zeros((1, nx)))
    done = 0
    for n, tol in ((500, 0.04), (2000, 0.025), (6000, 0.012)):
        lat.run(n - done)
        done = n
        ref = _cross_plane_series(X, (mfp / 2.0) * n / L ** 2)
        err = np.abs(lat.temperature()[0] - ref).max()
        assert err < tol, (n, err)


# -- Sec. 3.6, Eq. 2DT: one hot - three cold walls, steady Fourier limit -----
def one_hot_three_cold_series(X, Y, terms=200):
    th = np.zeros(np.broadcast(X, Y).shape)
    for l in range(1, terms, 2):   # 1 - cos(l pi) = 2 for odd l, 0 for even
        # sinh(l pi Y) / sinh(l pi), written without overflow
        ratio = np.exp(l * math.pi * (Y - 1.0)) * (1.0 - np.exp(-2.0 * l * math.pi * Y)) / (
            1.0 - np.exp(-2.0 * l * math.pi))
        th += 4.0 / (l * math.pi) * np.sin(l * math.pi * X) * ratio
    return th


def pin_one_hot_three_cold(o):
    """Blackbody walls, the upper one at T = 1 and the others at 0, 32 x 32,
    MFP 1.5 cells, Q = 16: the steady state matches the Laplace series of
    Eq. 2DT in the middle half of the square (walls at cells 0 and N - 1)."""
    N = 32
    lat = o.Lattice(o.Config(nx=N, ny=N, q=16, mfp=1.5, x_edge="blackbody", y_edge="blackbody",
                             t_y_hi=1.0))
    lat.set_temperature(np.zeros((N, N)))
    lat.run(4000)
    X = np.arange(N)[None, :] / (N - 1)
    Y = np.arange(N)[:, None] / (N - 1)
    mid = slice(N // 4, 3 * N // 4 + 1)
    err = np.abs(lat.temperature() - one_hot_three_cold_series(X, Y))[mid, mid].max()
    assert err < 0.02, err
    # the series itself: 1/4 at the centre of the square (four rotated
    # copies of the problem add up to T = 1 everywhere)
    assert abs(one_hot_three_cold_series(np.array(0.5), np.array(0.5)) - 0.25) < 1e-12


ALL_PINS = [
    pin_tas_d2q8_diagonal,
    pin_propagation_error,
    pin_worm_repeats_on_lattice_vector,
    pin_weights,
    pin_lambda_corr,
    pin_w_corr_limits,
    pin_stability_guard,
    pin_ballistic_exact,
    pin_energy_conservation,
    pin_equilibrium_fixed_point,
    pin_w1_is_standard_d2q8,
    pin_von_neumann,
    pin_ballistic_wall,
    pin_fourier_limit,
    pin_one_pixel_source,
    pin_cross_plane_fourier,
    pin_one_hot_three_cold,
]
