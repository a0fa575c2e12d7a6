"""In-plane conductivity of thin films versus Knudsen number (Sec. 3.5).

A film of thickness Ny cells with adiabatic diffuse walls (y) is held
between blackbody columns x = 0 (T = 1) and x = Nx - 1 (T = 0), starting
from T0 = 0.  The effective conductivity follows from the heat flux averaged
over the last ten steps (Sec. 3.4), over the interior columns:
kappa_eff = <q_x> (Nx - 1) / (T_h - T_c), against the bulk kappa = Lambda / 2
of the 2D gray model (unit heat capacity and group velocity).

For the steady state the run starts from the linear profile between the walls
(the steady state does not depend on T0) and averages the flux over whole
10000-step intervals; a film is steady when its kappa changes by less than
1e-6 between two consecutive intervals, twice in a row.

The sweep: 24 films, Nx = 512, Q = 128 evenly spaced directions,
Kn_j = 10^(-2 + 4j/23) per film thickness (MFP = Kn Ny cells), Ny_j drawn by
default_rng(180) from the thicknesses in {32, 64, 128, 256} for which the
MFP is at least one cell (W <= 1).  All films advance together through a
Batch (one kernel launch per two steps for all 24, with one block height for
the batch timed by `tune`); `step_each` advances them one after another for
comparison.

    python -m paper_1911_00180_amd.films [--steps N] [--steady] [--only J,...]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from .lattice import Batch, Lattice

THICKNESSES = (32, 64, 128, 256)


def film_set(n: int = 24, seed: int = 180):
    """[(Kn, Ny, MFP in cells)] of the sweep."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(n):
        kn = 10.0 ** (-2.0 + 4.0 * j / (n - 1))
        ok = [t for t in THICKNESSES if kn * t >= 1.0]
        ny = int(rng.choice(ok))
        out.append((kn, ny, kn * ny))
    return out


class FilmSweep:
    def __init__(self, films, nx: int = 512, q: int = 128, window: int = 10,
                 device="cuda", t_hot: float = 1.0, t_cold: float = 0.0, dir_split: int = 0,
                 start: str = "zero"):
        """start: "zero" (T0 = 0, the sweep's initial condition) or "linear"
        (T0 falling linearly from T_h to T_c between the walls; the steady
        state does not depend on T0, and this one is close to it)."""
        self.films = list(films)
        self.nx, self.q, self.window = nx, q, window
        self.t_hot, self.t_cold = t_hot, t_cold
        self.lattices = []
        for kn, ny, mfp in self.films:
            lat = Lattice(nx, ny, q, mfp=mfp, device=device, x_edge="blackbody",
                          y_edge="diffuse", t_x_lo=t_hot, t_x_hi=t_cold, dir_split=dir_split)
            if start == "linear":
                T0 = torch.linspace(t_hot, t_cold, nx).repeat(ny, 1)
            else:
                T0 = torch.zeros((ny, nx))
            lat.set_temperature(T0)
            lat.set_flux_window(window)
            self.lattices.append(lat)
        self.batch = Batch(self.lattices)

    @property
    def updates_per_step(self) -> int:
        return sum(self.nx * ny * self.q for _, ny, _ in self.films)

    def tune(self) -> int:
        """Time the candidate block heights of the batch's multi-step
        launches on the current states (restored) and keep the fastest for
        every film; 0 if the batch runs one step per launch."""
        if self.batch.steps_per_launch < 2:
            return 0
        return self.batch.tune_block_rows()

    def step_batched(self, n: int) -> None:
        self.batch.step(n)

    def step_each(self, n: int) -> None:
        for lat in self.lattices:
            lat.step(n)

    def kappa_ratios(self, only=None):
        """kappa_eff / kappa from the last flux window, of every film or of the
        films with the indices `only` (the others get None)."""
        out = []
        for j, ((kn, ny, mfp), lat) in enumerate(zip(self.films, self.lattices)):
            if only is not None and j not in only:
                out.append(None)
                continue
            qx, _ = lat.flux_mean(1, self.nx - 1, averaged=True)
            out.append(qx * (self.nx - 1) / (self.t_hot - self.t_cold) / (mfp / 2.0))
        return out

    def run_to_steady(self, check_every: int = 10000, rtol: float = 1e-6, repeats: int = 2,
                      max_steps: int = 1_000_000, log=None, only=None):
        """Step (batched) until, for every film, kappa averaged over whole
        check intervals changes by less than rtol (the sweep's criterion,
        1e-6) in `repeats` consecutive checks; films that have converged leave
        the batch.  (The flux of a single step carries the aperiodic TAS
        pattern: ten-step averages scatter by ~1e-2 from window to window,
        thousand-step averages by ~1e-5 - 1e-4, so the check interval is long.)
        Returns (kappa ratios, steps run, last relative change, converged
        flags) of the films run (`only`: their indices; default all).  `log`,
        if given, is called with a progress line after every check."""
        for lat in self.lattices:
            lat.set_flux_window(check_every)
        active = list(range(len(self.films))) if only is None else list(only)
        run = list(active)
        last = [None] * len(self.films)
        rel = [None] * len(self.films)
        calm = [0] * len(self.films)
        steps = [0] * len(self.films)
        done_k = [None] * len(self.films)
        batch = self.batch if only is None else Batch([self.lattices[j] for j in active])
        total = 0
        while active and total < max_steps:
            batch.step(check_every)
            total += check_every
            ks = self.kappa_ratios(only=active)
            still = []
            for j in active:
                steps[j] = total
                if last[j] is not None:
                    rel[j] = abs(ks[j] - last[j]) / abs(ks[j])
                if rel[j] is not None and rel[j] <= rtol:
                    calm[j] += 1
                else:
                    calm[j] = 0
                if calm[j] >= repeats:
                    done_k[j] = ks[j]
                else:
                    still.append(j)
                last[j] = ks[j]
            if still != active and still:
                if batch is not self.batch:
                    batch.close()
                batch = Batch([self.lattices[j] for j in still])
            active = still
            if log is not None:
                changes = [rel[j] for j in active if rel[j] is not None]
                worst = f", largest change {max(changes):.3g}" if changes else ""
                log(f"step {total}: {len(active)} films not yet steady{worst}")
        if batch is not self.batch:
            batch.close()
        for j in active:
            done_k[j] = last[j]
        return ([done_k[j] for j in run], [steps[j] for j in run], [rel[j] for j in run],
                [j not in active for j in run])

    def close(self) -> None:
        self.batch.close()
        for lat in self.lattices:
            lat.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--steps", type=int, default=10000, help="fixed steps for the timing")
    ap.add_argument("--window", type=int, default=10,
                    help="flux window of the timed steps (the last this many steps of each "
                         "call accumulate the heat flux; 0: none)")
    ap.add_argument("--steady", action="store_true", help="also run every film to steady state")
    ap.add_argument("--rtol", type=float, default=1e-6,
                    help="steady when kappa changes by less than this between checks")
    ap.add_argument("--check-every", type=int, default=10000,
                    help="steps per check (the flux is averaged over each interval)")
    ap.add_argument("--max-steps", type=int, default=1_000_000,
                    help="steps of the first steady-state pass at most")
    ap.add_argument("--second-steps", type=int, default=2_000_000,
                    help="steps of the second pass (ten times longer windows) for the films "
                         "not steady after the first; 0: none")
    ap.add_argument("--only", default="",
                    help="comma-separated indices of the films to run (default: all 24)")
    args = ap.parse_args()
    films = film_set()
    if args.only:
        films = [films[int(j)] for j in args.only.split(",")]
    sweep = FilmSweep(films, window=args.window)
    rows = sweep.tune()
    sweep.step_batched(10)
    torch.cuda.synchronize()
    t = time.perf_counter()
    sweep.step_batched(args.steps)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    other = FilmSweep(films, window=args.window)
    other.step_each(10)
    torch.cuda.synchronize()
    t = time.perf_counter()
    other.step_each(args.steps)
    torch.cuda.synchronize()
    te = time.perf_counter() - t
    res = {"films": [{"kn": kn, "ny": ny, "mfp": mfp} for kn, ny, mfp in films],
           "steps": args.steps, "window": args.window, "batch_block_rows": rows, "batched_s": tb, "one_by_one_s": te,
           "batched_gups": sweep.updates_per_step * args.steps / tb / 1e9,
           "one_by_one_gups": sweep.updates_per_step * args.steps / te / 1e9}
    other.close()
    sweep.close()
    if args.steady:
        steady = FilmSweep(films, start="linear")
        steady.tune()
        k, steps, rel, ok = steady.run_to_steady(
            check_every=args.check_every, rtol=args.rtol, max_steps=args.max_steps,
            log=lambda m: print(m, file=sys.stderr, flush=True))
        res["kappa_ratio"] = k
        res["steady_steps"] = steps
        res["last_relative_change"] = rel
        res["converged"] = ok
        res["criterion"] = {"rtol": args.rtol, "check_every": args.check_every, "repeats": 2,
                            "max_steps": args.max_steps}
        # films whose flux still scatters by more than rtol between windows
        # (the nearly ballistic ones) continue with ten times longer windows
        rest = [j for j, c in enumerate(ok) if not c]
        if rest and args.second_steps:
            k2, s2, r2, ok2 = steady.run_to_steady(
                check_every=10 * args.check_every, rtol=args.rtol, max_steps=args.second_steps,
                only=rest, log=lambda m: print(m, file=sys.stderr, flush=True))
            res["second_pass"] = {"films": rest, "check_every": 10 * args.check_every,
                                  "kappa_ratio": k2, "extra_steps": s2,
                                  "last_relative_change": r2, "converged": ok2}
        steady.close()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
