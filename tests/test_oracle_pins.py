"""The FP64 oracle against what the paper and the mathematics fix."""
import math

import numpy as np
import pytest

import pins
from oracle import worm_lbm as o


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(o)


def test_worm_greedy_is_nearest_lattice_point():
    """The greedy of Eq. worm-paths puts the worm after k hops on the lattice
    point with major coordinate k nearest to the ray, ties resolved away from
    the major axis (the later, diagonal index wins)."""
    for q, kind in [(8, "uniform"), (16, "uniform"), (40, "uniform"), (64, "uniform"),
                    (16, "ring"), (24, "ring"), (64, "ring")]:
        for d in o.make_directions(q, kind):
            path = o.worm_path(d, 200)
            ax = d.major_axis()
            px = py = 0
            for k, mv in enumerate(path, start=1):
                px += o.D2Q8[mv][0]
                py += o.D2Q8[mv][1]
                pos = (px, py)
                tgt = d.target(k)
                assert abs(pos[ax]) == k
                minor = abs(tgt[1 - ax])
                want = math.floor(minor) + (1 if minor - math.floor(minor) >= 0.5 else 0)
                assert abs(pos[1 - ax]) == want


def test_d2q8_diagonal_hop_fraction():
    """Fig. 2 lower panel: the diagonal's travelled distance converges to the
    axial one, i.e. the hop fraction tends to 1/sqrt(2)."""
    dirs = o.make_directions(8, "uniform")
    sch = o.tas_schedule(dirs, 4000)
    frac = sch.hop[:, 1].mean()
    assert abs(frac - 1 / math.sqrt(2)) < 1e-3
    r = math.hypot(*sch.pos[-1, 1])
    assert abs(r - 4000) <= 1.0


def _pull_matrix(lat, n):
    """Affine step e^{n} = A_n e^{n-1} + b_n, built entry by entry from the
    pull form: the output population (i, y, x) gathers the DDED of direction i
    from the cell it came from and the EED of every direction j from the cell
    the pending move of i starts at."""
    c = lat.cfg
    q, ny, nx = c.q, c.ny, c.nx
    N = q * ny * nx
    A = np.zeros((N, N))
    b = np.zeros(N)
    sch = lat.schedule(n)
    mv, hp = sch.move[n - 1], sch.hop[n - 1]
    Wc = np.broadcast_to(np.asarray(lat.Wc, dtype=float), (ny, nx))
    idx = lambda i, y, x: (i * ny + y) * nx + x

    def src(x, y, dx, dy):
        sx_, sy_ = x - dx, y - dy
        if c.x_edge == "periodic":
            sx_ %= nx
        elif not 0 <= sx_ < nx:
            return None
        if c.y_edge == "periodic":
            sy_ %= ny
        elif not 0 <= sy_ < ny:
            return None
        return sx_, sy_

    for i in range(q):
        dx, dy = o.D2Q8[int(mv[i])]
        hx, hy = (dx, dy) if hp[i] else (0, 0)
        for y in range(ny):
            for x in range(nx):
                r = idx(i, y, x)
                s = src(x, y, hx, hy)
                if s is not None:
                    A[r, idx(i, s[1], s[0])] += 1.0 - Wc[s[1], s[0]]
                s = src(x, y, dx, dy)
                if s is not None:
                    for j in range(q):
                        A[r, idx(j, s[1], s[0])] += Wc[s[1], s[0]] * lat.w[i]
    if c.y_edge == "diffuse":
        # A boundary node behind each wall absorbs what streams into it and
        # emits it again isotropically: node column X holds w_k T_g(X) with
        # T_g(X) = R(X) / C(X), R the absorbed amount, C the share an
        # isotropic unit state delivers into the domain on this step.
        for wall, yrow in (("lo", 0), ("hi", ny - 1)):
            out_dy = -1 if wall == "lo" else 1
            in_dy = -out_dy
            for X in range(nx):
                Rcoef = np.zeros(N)          # R(X) as a linear form of e^{n-1}
                for j in range(q):
                    dx, dy = o.D2Q8[int(mv[j])]
                    if dy != out_dy:
                        continue
                    xs = X - dx
                    if c.x_edge == "periodic":
                        xs %= nx
                    elif not 0 <= xs < nx:
                        continue
                    if hp[j]:
                        Rcoef[idx(j, yrow, xs)] += 1.0 - Wc[yrow, xs]
                    for k in range(q):
                        Rcoef[idx(k, yrow, xs)] += Wc[yrow, xs] * lat.w[j]
                Wg = Wc[yrow, X]
                C = sum(lat.w[k] * ((1.0 - Wg) * hp[k] + Wg) for k in range(q)
                        if o.D2Q8[int(mv[k])][1] == in_dy)
                for k in range(q):
                    dx, dy = o.D2Q8[int(mv[k])]
                    if dy != in_dy:
                        continue
                    xd = X + dx
                    if c.x_edge == "periodic":
                        xd %= nx
                    elif not 0 <= xd < nx:
                        continue
                    a = lat.w[k] * ((1.0 - Wg) * hp[k] + Wg)
                    if c.x_edge == "blackbody" and X in (0, nx - 1):
                        # the corner node belongs to the blackbody wall
                        b[idx(k, yrow, xd)] += a * (c.t_x_lo if X == 0 else c.t_x_hi)
                    else:
                        A[idx(k, yrow, xd), :] += (a / C) * Rcoef
    bb = np.zeros((q, ny, nx), dtype=bool)
    if c.y_edge == "blackbody":
        bb[:, 0, :] = bb[:, ny - 1, :] = True
    if c.x_edge == "blackbody":
        bb[:, :, 0] = bb[:, :, nx - 1] = True
    A[bb.ravel(), :] = 0.0
    # blackbody cells hold w_i T_wall; the x walls win at the corners
    wall = np.zeros((q, ny, nx))
    if c.y_edge == "blackbody":
        wall[:, 0, :] = lat.w[:, None] * c.t_y_lo
        wall[:, ny - 1, :] = lat.w[:, None] * c.t_y_hi
    if c.x_edge == "blackbody":
        wall[:, :, 0] = lat.w[:, None] * c.t_x_lo
        wall[:, :, nx - 1] = lat.w[:, None] * c.t_x_hi
    b[bb.ravel()] = wall.ravel()[bb.ravel()]
    return A, b, bb


@pytest.mark.parametrize("x_edge,y_edge", [("periodic", "periodic"), ("periodic", "diffuse"),
                                           ("blackbody", "diffuse"), ("blackbody", "periodic"),
                                           ("blackbody", "blackbody"), ("periodic", "blackbody")])
@pytest.mark.parametrize("q,kind", [(8, "uniform"), (16, "uniform"), (16, "ring")])
def test_push_step_equals_pull_matrix(x_edge, y_edge, q, kind):
    """The oracle's push-form step equals the pull-form step matrix on tiny
    lattices, for every boundary combination and 12 consecutive steps
    (so that hops and pauses both occur)."""
    rng = np.random.default_rng(11)
    nx, ny = 5, 4
    mfp = rng.uniform(1.2, 6.0, size=(ny, nx))
    lat = o.Lattice(o.Config(nx=nx, ny=ny, q=q, mfp=mfp, dirs=kind, x_edge=x_edge,
                             y_edge=y_edge, t_x_lo=0.3, t_x_hi=0.9, t_y_lo=0.4, t_y_hi=0.6))
    lat.set_populations(rng.random((q, ny, nx)))
    for n in range(1, 13):
        A, b, bb = _pull_matrix(lat, n)
        e0 = lat.e.ravel().copy()
        lat.step()
        want = A @ e0 + b
        got = lat.e.ravel()
        assert np.max(np.abs(got - want)) < 1e-14
        # nonnegative coefficients: the step is a convex redistribution
        assert A.min() >= 0.0
