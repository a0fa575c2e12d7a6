"""FP64 reference implementation of the worm-LBM for the gray phonon BTE.

TEST INFRASTRUCTURE ONLY.  This module is the oracle that the GPU library is
checked against.  It is plain, slow and written to be compared with the paper
by eye: numpy in float64, a Python loop over time steps and over directions,
the literal greedy worm-path search and the integer TAS rule.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it; the
product path (the C-ABI library and its binding) never does, and the two share
no code.

Paper: Hammer, Fritz, Bedoya-Martinez, "The worm-LBM, an algorithm for a high
number of propagation directions on a lattice Boltzmann grid: the case of
phonon transport" (arXiv:1911.00180).  Citations below name the section and
equation label of that paper.

Lattice units throughout: one cell per axial hop, one time step per hop, group
velocity 1, so the mean free path in cells is 1/W (Sec. 2.2, Eq. W-Kn).

Readings of passages that the paper leaves open or prints garbled are listed
where they are used; each one is marked "Reading:".
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# D2Q8 basic moves (Sec. 2.2 Fig. 1 and Sec. 2.5 Fig. 5a).
# Reading: the figure is not available; the text fixes axial directions as
# 1-4 and diagonal directions as 5-8 (Sec. 2.4).  Within each group the order
# E, N, W, S / NE, NW, SW, SE is chosen.  Only "axial before diagonal" matters:
# it decides ties of the greedy search (the later index wins).
# ---------------------------------------------------------------------------
D2Q8 = {
    1: (1, 0), 2: (0, 1), 3: (-1, 0), 4: (0, -1),
    5: (1, 1), 6: (-1, 1), 7: (-1, -1), 8: (1, -1),
}
AXIAL = (1, 2, 3, 4)
DIAGONAL = (5, 6, 7, 8)


# ---------------------------------------------------------------------------
# Direction sets and angular weights (Sec. 2.4, Eq. weight, Fig. 4)
# ---------------------------------------------------------------------------
@dataclass
class Direction:
    """One propagation direction s_hat of the D2Q[M x 8] scheme."""
    sx: float            # unit vector, x component
    sy: float            # unit vector, y component
    angle: float         # polar angle in [0, 2 pi)
    ring_vec: tuple | None = None   # integer lattice vector V (ring set only)
    ring_m: int = 0                  # M of the ring set (ring set only)

    # -- geometry of the ray used by the worm-path search (Sec. 2.5) --------
    def major_axis(self) -> int:
        """0 if |s_x| >= |s_y| (ties, i.e. diagonals, pick x), else 1."""
        if self.ring_vec is not None:
            vx, vy = self.ring_vec
            return 0 if abs(vx) >= abs(vy) else 1
        return 0 if abs(self.sx) >= abs(self.sy) else 1

    def target(self, k: int) -> tuple:
        """Point of the ray whose major coordinate is k (in magnitude).

        Reading of Eq. worm-paths: the printed target "l * 8n/M" is read as the
        ray point reached after n worm hops, i.e. the point of the ray whose
        coordinate along its major axis equals n.  For the ring set this is
        (n/M)*V, evaluated as (n*V)/M so that half-integer coordinates are
        exact.  For angle-uniform directions the minor coordinate is
        n * t with t = |minor|/|major| of the FP64 unit vector.
        """
        if self.ring_vec is not None:
            vx, vy = self.ring_vec
            return (k * vx / self.ring_m, k * vy / self.ring_m)
        ax = self.major_axis()
        comp = (self.sx, self.sy)
        t = abs(comp[1 - ax]) / abs(comp[ax])
        out = [0.0, 0.0]
        out[ax] = math.copysign(float(k), comp[ax])
        out[1 - ax] = math.copysign(k * t, comp[1 - ax]) if comp[1 - ax] != 0.0 else 0.0
        return (out[0], out[1])

    def hop_speed(self) -> float:
        """Net displacement of one worm hop, c_i = 1/max(|s_x|,|s_y|).

        Reading of Eq. W-correction-factor-gereralized: c_i is the lattice speed
        of direction i, the length of the ray segment covered per hop; it gives
        1 (axial) and sqrt(2) (diagonal) for D2Q8, which reproduces
        Lambda_corr = 2/(1+sqrt(2)) of Eq. W-correction-factor.
        """
        if self.ring_vec is not None:
            vx, vy = self.ring_vec
            return math.hypot(vx, vy) / self.ring_m
        return 1.0 / max(abs(self.sx), abs(self.sy))


def uniform_directions(q: int) -> list[Direction]:
    """Q directions evenly spaced in angle, theta_i = 2 pi i / Q.

    Directions on the axes and diagonals (8i/Q an integer) are set to their
    exact unit vectors so that their worm paths are exact axial or diagonal
    moves.  The others use the host libm cos/sin in FP64.
    """
    if q % 8 != 0 or q <= 0:
        raise ValueError("Q must be a positive multiple of 8")
    dirs = []
    r2 = math.sqrt(0.5)
    exact = {0: (1.0, 0.0), 1: (r2, r2), 2: (0.0, 1.0), 3: (-r2, r2),
             4: (-1.0, 0.0), 5: (-r2, -r2), 6: (0.0, -1.0), 7: (r2, -r2)}
    for i in range(q):
        theta = 2.0 * math.pi * i / q
        if (8 * i) % q == 0:
            sx, sy = exact[(8 * i) // q]
        else:
            sx, sy = math.cos(theta), math.sin(theta)
        dirs.append(Direction(sx, sy, theta))
    return dirs


def ring_directions(m: int) -> list[Direction]:
    """The D2Q[M x 8] directions of Sec. 2.4: the 8M integer vectors V on the
    square ring max(|Vx|,|Vy|) = M, ordered counter-clockwise from (M, 0).

    Reading: the printed index range of theta_j = atan(j/M), j = 1..8M, is read
    as the first-octant angles atan(j/M), j = 0..M, continued by symmetry into
    all eight octants, which gives exactly these 8M vectors.
    """
    if m < 1:
        raise ValueError("M must be >= 1")
    vecs = set()
    for a in range(-m, m + 1):
        vecs.update({(m, a), (-m, a), (a, m), (a, -m)})
    def ang(v):
        return math.atan2(v[1], v[0]) % (2.0 * math.pi)
    vecs = sorted(vecs, key=ang)
    dirs = []
    for v in vecs:
        n = math.hypot(v[0], v[1])
        dirs.append(Direction(v[0] / n, v[1] / n, ang(v), ring_vec=v, ring_m=m))
    return dirs


def make_directions(q: int, kind: str) -> list[Direction]:
    if kind == "uniform":
        return uniform_directions(q)
    if kind == "ring":
        if q % 8 != 0:
            raise ValueError("Q must be a multiple of 8")
        return ring_directions(q // 8)
    raise ValueError(kind)


def weights(dirs: list[Direction]) -> np.ndarray:
    """Angular weights w_j (Sec. 2.4, Eq. weight; Sec. 2.2 uniform case).

    Reading: in Eq. weight the theta's are the angular gaps between
    neighbouring directions (the equalities listed under Fig. 4 only hold for
    gaps), so w_j is half the angle spanned from direction j-1 to j+1, divided
    by 2 pi:  w_j = (phi_{j+1} - phi_{j-1}) / (4 pi), cyclic.  Evenly spaced
    directions get w = 1/Q, the uniform case of Sec. 2.2.
    """
    q = len(dirs)
    if all(d.ring_vec is None for d in dirs):
        # evenly spaced: every gap is 2 pi / Q, so w_j = 1/Q exactly
        return np.full(q, 1.0 / q)
    phi = [d.angle for d in dirs]
    w = np.empty(q)
    for j in range(q):
        up = (phi[(j + 1) % q] - phi[j]) % (2.0 * math.pi)
        dn = (phi[j] - phi[(j - 1) % q]) % (2.0 * math.pi)
        w[j] = (up + dn) / (4.0 * math.pi)
    return w


def lambda_corr(dirs: list[Direction]) -> float:
    """Grid-MFP correction Lambda_corr = Q / sum_i c_i
    (Sec. 2.4, Eq. W-correction-factor-gereralized)."""
    return len(dirs) / math.fsum(d.hop_speed() for d in dirs)


def w_corr(w: float, lam: float, emulate_3d: bool = False) -> float:
    """Corrected relaxation weight (Sec. 2.3, Eq. W-correction):
    W_corr = f [ (1 - W) W + W (W Lambda_corr) ],  f = 3/2 only when a 2D run
    emulates 3D behaviour, else 1 (reading of the remark after the equation).
    """
    f = 1.5 if emulate_3d else 1.0
    return f * ((1.0 - w) * w + w * (w * lam))


# ---------------------------------------------------------------------------
# Worm paths (Sec. 2.5, Eq. worm-paths)
# ---------------------------------------------------------------------------
def worm_path(d: Direction, nhops: int) -> list[int]:
    """First `nhops` D2Q8 moves of the worm path of direction d.

    For hop k (1-based) the worm stands at p_{k-1} (its position after the
    previous hops) and takes the basic move whose landing point is nearest to
    the ray point reached after k hops.  The running minimum starts at
    delta = 1 and accepts "<=", so on a tie the later D2Q8 index wins
    (a diagonal beats an axial move).
    """
    px, py = 0, 0
    path = []
    for k in range(1, nhops + 1):
        tx, ty = d.target(k)
        delta = 1.0
        best = None
        for ihat in range(1, 9):
            ux, uy = D2Q8[ihat]
            dist = math.sqrt((px + ux - tx) ** 2 + (py + uy - ty) ** 2)
            if dist <= delta:
                delta = dist
                best = ihat
        if best is None:
            raise AssertionError("no D2Q8 move within one cell of the ray")
        path.append(best)
        px += D2Q8[best][0]
        py += D2Q8[best][1]
    return path


# ---------------------------------------------------------------------------
# Time-adaptive scheme (Sec. 2.3, Eq. algorithm; Sec. 2.5)
# ---------------------------------------------------------------------------
@dataclass
class Schedule:
    """Per step n (1-based, row n-1) and direction i: the pending worm move
    (D2Q8 index) and whether the DDED hops (True) or pauses (False)."""
    move: np.ndarray      # int8 [nsteps, Q], values 1..8
    hop: np.ndarray       # bool [nsteps, Q]
    pos: np.ndarray       # int64 [nsteps, Q, 2], worm position after step n


def tas_schedule(dirs: list[Direction], nsteps: int, step0: int = 0,
                 speeds=None) -> Schedule:
    """Worm-LBM schedule for steps step0+1 .. step0+nsteps.

    Reading of Eq. algorithm (x_cum, x_ax, Delta x): at step n the DDED of
    direction i may take its next worm move only if the worm stays inside the
    circle of radius x_ax + Delta x, where x_ax = n is the axial distance after
    this step and Delta x = 1 cell; x_cum is the length of the worm
    displacement after the candidate move.  In squared integers:
        hop  iff  |P + s|^2 <= (n + 1)^2 .
    Reading: the worm index advances only when the move is executed; a paused
    direction retries the same move at the next step.  This reproduces the
    D2Q8 diagonal example of Fig. 2 (hops at n = 1, 2, 4, 5, pause at n = 3).

    Angle-dependent grid speed (Sec. 2.3: the TAS can impose any
    direction-dependent velocity): with speeds v_i in (0, 1] cells per step
    (default 1) the axial distance after step n is v_i n, so
        hop  iff  |P + s|^2 <= (v_i n + 1)^2 ,
    evaluated in float64 when v_i != 1 (the integer rule when v_i = 1).
    """
    q = len(dirs)
    total = step0 + nsteps
    paths = [worm_path(d, total + 1) for d in dirs]
    P = [[0, 0] for _ in range(q)]
    k = [0] * q
    move = np.zeros((nsteps, q), dtype=np.int8)
    hop = np.zeros((nsteps, q), dtype=bool)
    pos = np.zeros((nsteps, q, 2), dtype=np.int64)
    for n in range(1, total + 1):
        for i in range(q):
            m = paths[i][k[i]]
            cx = P[i][0] + D2Q8[m][0]
            cy = P[i][1] + D2Q8[m][1]
            if speeds is None or speeds[i] == 1.0:
                h = cx * cx + cy * cy <= (n + 1) * (n + 1)
            else:
                r = speeds[i] * n + 1.0
                h = float(cx * cx + cy * cy) <= r * r
            if h:
                P[i] = [cx, cy]
                k[i] += 1
            if n > step0:
                move[n - step0 - 1, i] = m
                hop[n - step0 - 1, i] = h
                pos[n - step0 - 1, i] = P[i]
    return Schedule(move, hop, pos)


# ---------------------------------------------------------------------------
# Lattice, boundary conditions and one LBM step (Sec. 2.2, 2.3, 2.5, 2.6)
# ---------------------------------------------------------------------------
PERIODIC, BLACKBODY, DIFFUSE = "periodic", "blackbody", "diffuse"


@dataclass
class Config:
    nx: int
    ny: int
    q: int
    mfp: float | np.ndarray = math.inf   # cells; scalar or [ny, nx] field
    dirs: str = "uniform"                # "uniform" or "ring"
    emulate_3d: bool = False
    mfp_correction: bool = True          # False: plain W, no Eq. W-correction
    x_edge: str = PERIODIC               # PERIODIC or BLACKBODY
    y_edge: str = PERIODIC               # PERIODIC, BLACKBODY or DIFFUSE
    t_x_lo: float = 0.0
    t_x_hi: float = 0.0
    t_y_lo: float = 0.0
    t_y_hi: float = 0.0
    # fraction of what crosses a DIFFUSE y wall that is reflected specularly
    # (Eq. adiabatic-specular); the rest is scattered diffusely
    y_specularity: float = 0.0
    # internal sources (Eq. isotropic, Eq. anisotropic): cells [S, 2] (x, y)
    # whose DDEDs are overwritten every step by values [S, q]
    source_cells: np.ndarray | None = None
    source_values: np.ndarray | None = None
    # grid speed of each direction in cells per step (Sec. 2.3), None = 1
    speeds: np.ndarray | None = None


@dataclass
class Lattice:
    cfg: Config
    dirs: list = field(init=False)
    w: np.ndarray = field(init=False)
    s: np.ndarray = field(init=False)      # [Q, 2] unit vectors
    lam: float = field(init=False)
    Wc: np.ndarray | float = field(init=False)
    e: np.ndarray = field(init=False)      # [Q, ny, nx] DDEDs
    n: int = field(init=False, default=0)

    def __post_init__(self):
        c = self.cfg
        if c.x_edge not in (PERIODIC, BLACKBODY):
            raise ValueError("x edges: periodic or blackbody")
        if c.y_edge not in (PERIODIC, BLACKBODY, DIFFUSE):
            raise ValueError("y edges: periodic, blackbody or diffuse")
        self.dirs = make_directions(c.q, c.dirs)
        self.w = weights(self.dirs)
        self.s = np.array([[d.sx, d.sy] for d in self.dirs])
        self.lam = lambda_corr(self.dirs)
        mfp = np.asarray(c.mfp, dtype=np.float64)
        W = np.where(np.isinf(mfp), 0.0, 1.0 / np.where(np.isinf(mfp), 1.0, mfp))
        if c.mfp_correction:
            f = 1.5 if c.emulate_3d else 1.0
            Wc = f * ((1.0 - W) * W + W * (W * self.lam))      # Eq. W-correction
        else:
            Wc = W                   # the uncorrected scheme compared in Fig. 3
        if np.any(Wc > 1.0):                                    # App. A: W <= 1
            raise ValueError("unstable: corrected relaxation weight exceeds 1")
        if not 0.0 <= c.y_specularity <= 1.0:
            raise ValueError("y_specularity must lie in [0, 1]")
        if c.speeds is not None:
            v = np.asarray(c.speeds, dtype=np.float64)
            if v.shape != (c.q,) or np.any(~(v > 0.0)) or np.any(v > 1.0):
                raise ValueError("speeds must be q values in (0, 1]")
        # mirror image of each direction in a y wall: (sx, sy) -> (sx, -sy)
        self.mirror_y = np.array([self._find(d.sx, -d.sy) for d in self.dirs])
        self.Wc = float(Wc) if Wc.ndim == 0 else Wc
        self.e = np.zeros((c.q, c.ny, c.nx))
        self._sched = None

    def _find(self, sx: float, sy: float) -> int:
        for j, d in enumerate(self.dirs):
            if abs(d.sx - sx) < 1e-12 and abs(d.sy - sy) < 1e-12:
                return j
        raise ValueError("direction set is not symmetric under a y mirror")

    # -- state ------------------------------------------------------------
    def set_temperature(self, T0: np.ndarray) -> None:
        """e_i = w_i e_eq(T0): the weights set the initial condition (Sec. 2.4).
        Linear gray model e_eq = T (reading; see temperature())."""
        self.e = self.w[:, None, None] * np.asarray(T0, dtype=np.float64)[None]
        self._apply_blackbody(self.e)
        self._apply_sources(self.e)

    def set_populations(self, e: np.ndarray) -> None:
        self.e = np.array(e, dtype=np.float64)

    def schedule(self, nsteps: int) -> Schedule:
        """Schedule rows for steps 1..nsteps (cached, extended on demand)."""
        have = 0 if self._sched is None else self._sched.move.shape[0]
        if have < nsteps:
            self._sched = tas_schedule(self.dirs, max(nsteps, 2 * have, 16),
                                       speeds=self.cfg.speeds)
        return self._sched

    # -- one step ---------------------------------------------------------
    def _deposit(self, acc: np.ndarray, amount: np.ndarray, dx: int, dy: int) -> None:
        """Add `amount` (per source cell) into the ghost-padded accumulator at
        the destination x + (dx, dy)."""
        ny, nx = self.cfg.ny, self.cfg.nx
        acc[1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx] += amount

    def _fold(self, acc: np.ndarray):
        """Resolve packets that left the domain.  x first: wrap (periodic) or
        drop (blackbody).  Then y: wrap, drop, or return the packets that
        crossed a diffuse wall as per-column amounts absorbed by the boundary
        nodes of row -1 and row ny."""
        c = self.cfg
        nx, ny = c.nx, c.ny
        a = acc.copy()
        if c.x_edge == PERIODIC:
            a[:, nx] += a[:, 0]
            a[:, 1] += a[:, nx + 1]
        a = a[:, 1:nx + 1]
        r_lo = r_hi = None
        if c.y_edge == PERIODIC:
            a[ny] += a[0]
            a[1] += a[ny + 1]
        elif c.y_edge == DIFFUSE:
            r_lo = a[0].copy()
            r_hi = a[ny + 1].copy()
        return a[1:ny + 1], r_lo, r_hi

    def _apply_blackbody(self, e: np.ndarray) -> None:
        """Isotropic blackbody walls (Sec. 2.6, Eq. isotropic): all DDEDs of the
        wall cells are overwritten by w_i e_eq(T_wall) at every step.
        Reading: y walls first, then x walls (x wins at corners)."""
        c = self.cfg
        w = self.w[:, None]
        if c.y_edge == BLACKBODY:
            e[:, 0, :] = w * c.t_y_lo
            e[:, c.ny - 1, :] = w * c.t_y_hi
        if c.x_edge == BLACKBODY:
            e[:, :, 0] = w * c.t_x_lo
            e[:, :, c.nx - 1] = w * c.t_x_hi

    def _apply_sources(self, e: np.ndarray) -> None:
        """Internal sources (Sec. 2.6, Eq. isotropic and Eq. anisotropic): the
        DDEDs of each source cell are overwritten by the imposed distribution
        at every step.  Reading: after the blackbody walls, so a source on a
        wall cell wins."""
        c = self.cfg
        if c.source_cells is None:
            return
        for (x, y), vals in zip(np.asarray(c.source_cells), np.asarray(c.source_values)):
            e[:, int(y), int(x)] = vals

    def step(self) -> None:
        """Advance one time step n -> n+1 (push form).

        E(x) = sum_i e_i(x)                                (Eq. lbm-energy-density)
        e_i^eq(x) = w_i E(x)                               (Eq. lbm-energy-weighting)
        hop:   e_i(x + s_i) <- (1 - W) e_i(x) + W e_i^eq(x)          (Eq. algorithm)
        pause: e_i(x) keeps (1 - W) e_i(x), e_i(x + s_i) gets W e_i^eq(x)

        Reading (Eq. lbm-energy-weighting prints a sum over i): the equilibrium
        of direction i is w_i E, which matches the uniform case E/Q given in the
        same passage and Eq. isotropic.
        Reading (pause): the DDED part stays in its cell while the EED part
        moves along the pending worm move; App. A's pause growth factor
        (1 - W) + W e^{ik dx} states exactly this.
        The relaxation weight is W_corr (Sec. 2.3) evaluated per cell; the
        DDED that stays or hops uses W_corr of its own cell, the EED emitted by
        a cell uses W_corr of that cell.
        """
        c = self.cfg
        n = self.n + 1
        sch = self.schedule(n)
        mv = sch.move[n - 1]
        hp = sch.hop[n - 1]
        E = self.e.sum(axis=0)
        Wc = self.Wc
        new = np.zeros_like(self.e)
        r_lo = np.zeros(c.nx)
        r_hi = np.zeros(c.nx)
        p = c.y_specularity
        for i in range(c.q):
            sx, sy = D2Q8[int(mv[i])]
            acc = np.zeros((c.ny + 2, c.nx + 2))
            dded = (1.0 - Wc) * self.e[i]
            eed = Wc * self.w[i] * E
            if hp[i]:
                self._deposit(acc, dded, sx, sy)
            else:
                self._deposit(acc, dded, 0, 0)
            self._deposit(acc, eed, sx, sy)
            inside, lo, hi = self._fold(acc)
            new[i] += inside
            if lo is not None:
                r_lo += (1.0 - p) * lo
                r_hi += (1.0 - p) * hi
                if p > 0.0:
                    # Reading (Eq. adiabatic-specular): a packet that crosses
                    # the wall at y = -1/2 (ny - 1/2) is reflected there and
                    # ends the step in the wall-row cell it crossed under, in
                    # the mirrored direction.
                    j = self.mirror_y[i]
                    new[j, 0, :] += p * lo
                    new[j, c.ny - 1, :] += p * hi
        if c.y_edge == DIFFUSE:
            self._diffuse(new, r_lo, r_hi, mv, hp)
        self._apply_blackbody(new)
        self._apply_sources(new)
        self.e = new
        self.n = n

    def _diffuse(self, e: np.ndarray, r_lo: np.ndarray, r_hi: np.ndarray,
                 mv: np.ndarray, hp: np.ndarray) -> None:
        """Adiabatic diffuse walls (Sec. 2.6, Eq. adiabatic-diffuse).

        Reading: each wall is a row of boundary nodes just outside the domain
        (row -1 below, row ny above).  Everything that streams into a boundary
        node during the step (r_lo / r_hi, per column) is absorbed there and
        re-emitted isotropically: the node holds inward DDEDs w_i T_g, i.e.
        the sum of the DDEDs that travelled into the boundary distributed by
        the weights, as Eq. adiabatic-diffuse states.  These stream into the
        domain by the ordinary rule of the step: a direction whose pending move
        points inward delivers (hop (1 - W_g) + W_g) w_i T_g, and T_g is chosen
        so that the node emits exactly what it absorbed (adiabatic wall).
        W_g is the relaxation weight of the wall cell the node faces.
        With this normalisation a uniform isotropic state is an exact fixed
        point of the wall, also on steps where some directions pause.
        Reading (corners): the boundary node below or above a blackbody column
        belongs to the blackbody wall and emits at its temperature, as the
        blackbody overwrite wins at the corner cells themselves.
        Reading (specular-diffuse walls): r_lo / r_hi hold only the diffuse
        share (1 - p) of what crossed; the corner nodes emit that share of
        the wall temperature, so a fully specular wall (p = 1) emits nothing
        of its own and equals the mirror image of the domain.
        """
        c = self.cfg
        nx, ny = c.nx, c.ny
        Wc = np.broadcast_to(np.asarray(self.Wc, dtype=np.float64), (ny, nx))
        for r, yrow, dy_in in ((r_lo, 0, 1), (r_hi, ny - 1, -1)):
            Wg = Wc[yrow, :]
            crossing = []
            C = np.zeros(nx)
            for i in range(c.q):
                sx, sy = D2Q8[int(mv[i])]
                if sy == dy_in:
                    a = self.w[i] * ((1.0 - Wg) * (1.0 if hp[i] else 0.0) + Wg)
                    C += a
                    crossing.append((i, sx, a))
            Tg = r / C
            if c.x_edge == BLACKBODY:
                Tg[0] = (1.0 - c.y_specularity) * c.t_x_lo
                Tg[nx - 1] = (1.0 - c.y_specularity) * c.t_x_hi
            for i, sx, a in crossing:
                acc = np.zeros(nx + 2)
                acc[1 + sx:1 + sx + nx] += a * Tg
                if c.x_edge == PERIODIC:
                    acc[nx] += acc[0]
                    acc[1] += acc[nx + 1]
                e[i, yrow, :] += acc[1:nx + 1]

    def run(self, nsteps: int, flux_window: int = 0):
        """Advance nsteps; if flux_window > 0 also return the heat flux averaged
        over the last flux_window steps (Sec. 3.4: the flux is reported as an
        average over ten steps around the time of interest; reading: trailing
        window ending at the last step)."""
        qsum = None
        for k in range(nsteps):
            self.step()
            if flux_window and k >= nsteps - flux_window:
                qx, qy = self.heat_flux()
                if qsum is None:
                    qsum = [qx.copy(), qy.copy()]
                else:
                    qsum[0] += qx
                    qsum[1] += qy
        if qsum is not None:
            m = min(flux_window, nsteps)
            return qsum[0] / m, qsum[1] / m
        return None

    # -- readout ------------------------------------------------------------
    def temperature(self) -> np.ndarray:
        """Pseudo-temperature (Sec. 2.2, Eq. pseudo-T).

        Reading: linearised gray model with unit heat capacity, e_eq = T, so
        T = E = sum_i e_i.  The Bose-Einstein form of Eq. pseudo-T needs the
        atom density 3N/V, which the paper does not give in lattice units."""
        return self.e.sum(axis=0)

    def heat_flux(self):
        """q = v_g sum_i e_i s_hat_i (Sec. 2.2, Eq. q_corr), v_g = 1."""
        qx = np.tensordot(self.s[:, 0], self.e, axes=(0, 0))
        qy = np.tensordot(self.s[:, 1], self.e, axes=(0, 0))
        return qx, qy

    def energy(self) -> float:
        return math.fsum(self.e.ravel())


# ---------------------------------------------------------------------------
# Closed forms the method reaches exactly
# ---------------------------------------------------------------------------
def ballistic_temperature(T0: np.ndarray, w: np.ndarray, pos: np.ndarray) -> np.ndarray:
    """W = 0 on a periodic lattice: every DDED is carried without smearing
    (Sec. 1 and Sec. 4: no numerical smearing), so after n steps
    e_i(x) = w_i T0(x - P_i(n)) and T(x) = sum_i w_i T0(x - P_i(n)), with P_i(n)
    the worm position of direction i after step n."""
    out = np.zeros_like(np.asarray(T0, dtype=np.float64))
    for i in range(len(w)):
        out += w[i] * np.roll(T0, shift=(int(pos[i, 1]), int(pos[i, 0])), axis=(0, 1))
    return out


def flux_distribution(dirs: list[Direction], w: np.ndarray, T: float, q) -> np.ndarray:
    """DDEDs of a flux boundary or source (Sec. 2.6, Eq. lbm-heat-flux): the
    paper asks for the DDEDs to be prescribed uniquely; reading: the
    distribution linear in the direction, e_i = w_i (T + s_i . a), whose
    energy is T and whose flux sum_i e_i s_i is q, i.e. a = M^{-1} q with
    M = sum_i w_i s_i s_i^T (symmetric direction sets have sum_i w_i s_i = 0)."""
    S = np.array([[d.sx, d.sy] for d in dirs])
    M = (S * np.asarray(w)[:, None]).T @ S
    a = np.linalg.solve(M, np.asarray(q, dtype=np.float64))
    return np.asarray(w) * (T + S @ a)


def growth_factor(W: float, k: float, paused: bool) -> complex:
    """Von Neumann growth factor of one direction (App. A, Eq. stabil-prop and
    Eq. stabil-pause): propagate g = e^{ik}, pause g = 1 + W (e^{ik} - 1)."""
    z = complex(math.cos(k), math.sin(k))
    return z if not paused else 1.0 + W * (z - 1.0)
