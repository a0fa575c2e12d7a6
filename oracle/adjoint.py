"""FP64 reference gradients of a probe-temperature loss (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of oracle/.  Plain numpy, written
from the definition of the forward step in oracle/worm_lbm.py: the step is
affine in the populations for a fixed relaxation field,
    e^n = A_n e^{n-1} + b_n,
so the gradient of a loss of the states follows from the transposed
recursion lambda^{n-1} = A_n^T lambda^n + dL/de^{n-1}.

Loss (the adjoint workload of the build): with probe cells p and loss steps
k = every, 2*every, ..., nsteps,
    L = sum_k sum_p (T^k(p) - target_k(p))^2,   T = sum_i e_i.
Gradients: with respect to the per-cell mean free path (the relaxation time
tau in lattice units, W = 1/tau), the initial temperature T0 and the
blackbody wall temperatures.

Scope: periodic or blackbody edges (no diffuse walls).
"""
from __future__ import annotations

import numpy as np

from .worm_lbm import BLACKBODY, D2Q8, DIFFUSE, PERIODIC, Config, Lattice


def _wall_owner(cfg: Config):
    """Which blackbody wall sets each cell (None: a free cell).  The x walls
    win at corners, as in the forward overwrite."""
    own = np.full((cfg.ny, cfg.nx), "", dtype=object)
    if cfg.y_edge == BLACKBODY:
        own[0, :] = "y_lo"
        own[cfg.ny - 1, :] = "y_hi"
    if cfg.x_edge == BLACKBODY:
        own[:, 0] = "x_lo"
        own[:, cfg.nx - 1] = "x_hi"
    return own


def _pull(field: np.ndarray, dx: int, dy: int, cfg: Config) -> np.ndarray:
    """out(x) = field(x + (dx, dy)), wrapped on periodic edges and zero where
    x + (dx, dy) leaves the domain."""
    ny, nx = field.shape
    pad = np.zeros((ny + 2, nx + 2))
    pad[1:ny + 1, 1:nx + 1] = field
    if cfg.x_edge == PERIODIC:
        pad[1:ny + 1, 0] = field[:, nx - 1]
        pad[1:ny + 1, nx + 1] = field[:, 0]
    if cfg.y_edge == PERIODIC:
        pad[0, :] = pad[ny, :]
        pad[ny + 1, :] = pad[1, :]
    return pad[1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]


def transposed_step(lat: Lattice, n: int, lam: np.ndarray):
    """A_n^T lam: the adjoint of forward step n.

    Forward step n sends, from each source cell x and direction i, the DDED
    (1 - W(x)) e_i(x) to x + h_i (h_i = pending move on a hop, 0 on a pause)
    and the EED W(x) w_i E(x) to x + s_i.  Hence
        (A^T lam)_j(x) = (1 - W(x)) lam_j(x + h_j) + W(x) sum_i w_i lam_i(x + s_i)
    with lam read as zero outside the domain.  Returns (A^T lam, G) where
    G(x) = sum_i w_i lam_i(x + s_i)."""
    c = lat.cfg
    sch = lat.schedule(n)
    mv, hp = sch.move[n - 1], sch.hop[n - 1]
    W = np.broadcast_to(np.asarray(lat.Wc, dtype=np.float64), (c.ny, c.nx))
    G = np.zeros((c.ny, c.nx))
    for i in range(c.q):
        sx, sy = D2Q8[int(mv[i])]
        G += lat.w[i] * _pull(lam[i], sx, sy, c)
    out = np.empty_like(lam)
    for j in range(c.q):
        sx, sy = D2Q8[int(mv[j])]
        hx, hy = (sx, sy) if hp[j] else (0, 0)
        out[j] = (1.0 - W) * _pull(lam[j], hx, hy, c) + W * G
    return out, G


def probe_loss(cfg: Config, T0, nsteps, probes, every, targets, keep_states=False,
               checkpoint_every=None):
    """Forward run and loss.  probes: int [P, 2] (x, y); targets:
    [nsteps // every, P].  keep_states: also return every state e^0 ..
    e^nsteps; checkpoint_every = K: return the states e^0, e^K, e^2K, ... as a
    dict {step: state} instead."""
    if cfg.y_edge == DIFFUSE:
        raise ValueError("the adjoint covers periodic and blackbody edges")
    lat = Lattice(cfg)
    lat.set_temperature(np.asarray(T0, dtype=np.float64))
    lat.schedule(nsteps)
    states = [lat.e.copy()] if keep_states else None
    ck = {0: lat.e.copy()} if checkpoint_every else None
    loss = 0.0
    px, py = probes[:, 0], probes[:, 1]
    for n in range(1, nsteps + 1):
        lat.step()
        if keep_states:
            states.append(lat.e.copy())
        if ck is not None and n % checkpoint_every == 0:
            ck[n] = lat.e.copy()
        if n % every == 0:
            T = lat.temperature()
            d = T[py, px] - targets[n // every - 1]
            loss += float(np.sum(d * d))
    return loss, lat, (ck if ck is not None else states)


def probe_temperatures(cfg: Config, T0, nsteps, probes, every) -> np.ndarray:
    """T^k(p) of a forward run at steps k = every, 2 every, ..., nsteps:
    [nsteps // every, P]."""
    lat = Lattice(cfg)
    lat.set_temperature(np.asarray(T0, dtype=np.float64))
    lat.schedule(nsteps)
    px, py = probes[:, 0], probes[:, 1]
    out = []
    for n in range(1, nsteps + 1):
        lat.step()
        if n % every == 0:
            out.append(lat.temperature()[py, px].copy())
    return np.array(out)


class _Recomputed:
    """States e^n of a forward run from checkpoints every K steps: the states
    of the segment holding n are recomputed from its checkpoint by the
    forward step (the reverse pass asks for them in decreasing order, so one
    segment is held at a time)."""

    def __init__(self, lat: Lattice, ck: dict, K: int, nsteps: int):
        self.lat, self.ck, self.K, self.nsteps = lat, ck, K, nsteps
        self.base, self.seg = None, None

    def __getitem__(self, n: int) -> np.ndarray:
        base = (n // self.K) * self.K
        if base != self.base:
            self.lat.e = self.ck[base].copy()
            self.lat.n = base
            seg = [self.lat.e.copy()]
            for _ in range(min(self.K, self.nsteps + 1 - base) - 1):
                self.lat.step()
                seg.append(self.lat.e.copy())
            self.base, self.seg = base, seg
        return self.seg[n - base]


def probe_loss_gradients(cfg: Config, T0, nsteps, probes, every, targets,
                         checkpoint_every=None):
    """Loss and its gradients by the transposed recursion.

    checkpoint_every = K keeps only every K-th forward state and recomputes
    the others segment by segment during the reverse pass (same arithmetic,
    same results; for runs whose states do not all fit in memory).

    Returns (loss, dL/dmfp [ny, nx], dL/dT0 [ny, nx], dict of dL/dT_wall)."""
    if checkpoint_every:
        loss, lat, ck = probe_loss(cfg, T0, nsteps, probes, every, targets,
                                   checkpoint_every=checkpoint_every)
        states = _Recomputed(lat, ck, checkpoint_every, nsteps)
    else:
        loss, lat, states = probe_loss(cfg, T0, nsteps, probes, every, targets,
                                       keep_states=True)
    c = cfg
    own = _wall_owner(c)
    wall = own != ""
    px, py = probes[:, 0], probes[:, 1]
    W = np.broadcast_to(np.asarray(lat.Wc, dtype=np.float64), (c.ny, c.nx))
    gW = np.zeros((c.ny, c.nx))
    gTb = {"x_lo": 0.0, "x_hi": 0.0, "y_lo": 0.0, "y_hi": 0.0}

    def seed(n):
        s = np.zeros((c.ny, c.nx))
        if n % every == 0 and n > 0:
            T = states[n].sum(axis=0)
            d = T[py, px] - targets[n // every - 1]
            np.add.at(s, (py, px), 2.0 * d)
        return s

    def absorb_walls(lam):
        # overwritten cells feed the wall temperature, not earlier states
        contrib = np.tensordot(lat.w, lam, axes=(0, 0))
        for key in gTb:
            gTb[key] += float(contrib[own == key].sum())
        lam[:, wall] = 0.0

    lam = np.zeros((c.q, c.ny, c.nx))
    lam += seed(nsteps)[None]
    absorb_walls(lam)
    for n in range(nsteps, 0, -1):
        e_prev = states[n - 1]
        new, G = transposed_step(lat, n, lam)
        # dL/dW(x) at step n: from the DDED term -e_j(x) lam_j(x + h_j) and
        # the EED term w_i E(x) lam_i(x + s_i)
        sch = lat.schedule(n)
        mv, hp = sch.move[n - 1], sch.hop[n - 1]
        dd = np.zeros((c.ny, c.nx))
        for j in range(c.q):
            sx, sy = D2Q8[int(mv[j])]
            hx, hy = (sx, sy) if hp[j] else (0, 0)
            dd += e_prev[j] * _pull(lam[j], hx, hy, c)
        gW += -dd + e_prev.sum(axis=0) * G
        lam = new + seed(n - 1)[None]
        absorb_walls(lam)
    # e^0 = w_i T0 on free cells
    gT0 = np.tensordot(lat.w, lam, axes=(0, 0))
    gT0[wall] = 0.0
    # chain W_corr(W(mfp)): dW_corr/dW = f (1 - 2W + 2 W Lambda), dW/dmfp = -W^2
    mfp = np.broadcast_to(np.asarray(c.mfp, dtype=np.float64), (c.ny, c.nx))
    Wp = np.where(np.isinf(mfp), 0.0, 1.0 / np.where(np.isinf(mfp), 1.0, mfp))
    if c.mfp_correction:
        f = 1.5 if c.emulate_3d else 1.0
        dWc = f * (1.0 - 2.0 * Wp + 2.0 * Wp * lat.lam)
    else:
        dWc = np.ones_like(Wp)
    g_mfp = gW * dWc * (-Wp * Wp)
    del W
    return loss, g_mfp, gT0, gTb
