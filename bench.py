#!/usr/bin/env python3
"""Throughput of the worm-LBM collide-and-stream on one MI355X.

One bench step = one full time step of the method (every cell, every
direction: relaxation, worm/TAS streaming, boundary treatment) on the
workload below, run through the C-ABI library.  Prints one JSON line.

Workload (default): 1024 x 1024 periodic lattice, Q = 64 directions evenly
spaced in angle, TAS and grid-MFP correction, MFP 102.4 cells (Kn = 0.1 with
L = 1024), Gaussian pulse sigma0 = 16 at a seeded position.  Inputs are
synthetic (the paper's workloads are analytic initial conditions).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
CSRC = os.path.join(ROOT, "paper_1911_00180_amd", "csrc")
STEP_SOURCES = ("kernels.hip", "kernel_common.hpp", "device.hpp")
FUSED_SOURCES = ("fused.hip", "fused_kernel.hpp", "kernel_common.hpp", "device.hpp")
ADJOINT_SOURCES = ("adjoint.hip", "kernel_common.hpp", "device.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_1024x1024_q64_traffic.md")
FUSED_TRAFFIC_FILES = {k: os.path.join(ROOT, "profiles", f"k_stepk{k}_1024x1024_q64_traffic.md")
                       for k in (2, 3, 4)}
ADJOINT_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_adjoint_1024x1024_q64.md")
# the kernels that run the default workload (1024 x 1024 periodic, Q = 64),
# by time steps per launch
KERNELS = {1: "k_step<4, false, false>", 2: "k_stepk<8, 8, false, 2, false>",
           3: "k_stepk<8, 8, false, 3, false>", 4: "k_stepk<8, 8, false, 4, false>"}


def bytes_per_update(q: int, per_cell_w: bool = False) -> float:
    """Algorithmic HBM bytes per cell-direction update: the population is read
    once and written once (8 B); per cell, E is read and written (8/Q B);
    a per-cell weight field adds 4/Q B."""
    return 8.0 + 8.0 / q + (4.0 / q if per_cell_w else 0.0)


def kernel_hash(sources=STEP_SOURCES) -> str:
    """Hash of the sources a kernel is built from (first 16 hex digits)."""
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(path=TRAFFIC_FILE, sources=STEP_SOURCES):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or
    None if it is missing or was taken on different kernel sources."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.strip().startswith("- "):
                k, v = line.strip()[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_sha256_16") != kernel_hash(sources):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def run_gpu(nx, ny, q, mfp, steps, warmup, edges, split=0, seed=1911, fusion=1, block_rows=None,
            tune=True):
    """Time `steps` steps (after `warmup`) of the lattice; with several steps
    per launch the block height is fixed beforehand (given, timed by the
    library's tuner on a saved state that is then restored, or - tune False -
    the library's launch model), so that no tuning happens inside the timed
    region."""
    import numpy as np
    import torch

    from paper_1911_00180_amd import inputs
    from paper_1911_00180_amd.lattice import Lattice

    x0, y0 = inputs.seeded_center(seed, nx, ny)
    T0 = inputs.gaussian_pulse(nx, ny, 16.0, x0, y0).astype(np.float32)
    lat = Lattice(nx, ny, q, mfp=mfp, device="cuda:0", dir_split=split, step_fusion=fusion,
                  **edges)
    lat.set_temperature(torch.from_numpy(T0))
    for k, rows in (block_rows or {}).items():
        lat.set_block_rows(k, rows)
    spl = lat.steps_per_launch
    if tune and spl > 1 and lat.block_rows(spl) > 0 and spl not in (block_rows or {}):
        lat.tune_block_rows(spl)
    if spl > 1 and lat.block_rows(spl) <= 0:
        raise SystemExit(f"bench.py: no block height for {spl} steps per launch")
    lat.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    lat.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    energy, _, _ = lat.totals()
    # block height the library chose for the multi-step kernel, if any
    run_gpu.steps_per_launch = lat.steps_per_launch
    run_gpu.block_rows = (lat.block_rows(run_gpu.steps_per_launch)
                          if run_gpu.steps_per_launch > 1 else None)
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return ms, wall, energy


def run_stream_ceiling(sizes, repeats=10):
    """Read+write stream kernel (libwlbm_probe.so, 16-byte loads and stores)
    over buffers of the given byte sizes: the best GB/s (bytes read + bytes
    written per second) over its variants, per size."""
    import ctypes

    import torch

    path = os.path.join(ROOT, "paper_1911_00180_amd", "libwlbm_probe.so")
    probe = ctypes.CDLL(path)
    probe.wlbm_probe_copy.restype = ctypes.c_int
    probe.wlbm_probe_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    stream = torch.cuda.current_stream()
    out = {}
    for label, nbytes in sizes:
        nbytes = nbytes // 16 * 16
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        best = None
        for unroll in (1, 2, 4):
            for nt in (0, 1):
                def go():
                    rc = probe.wlbm_probe_copy(a.data_ptr(), b.data_ptr(), nbytes, unroll, nt,
                                               stream.cuda_stream)
                    if rc:
                        raise RuntimeError(f"stream probe failed: {rc}")
                go()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(repeats):
                    go()
                e1.record(stream)
                torch.cuda.synchronize()
                gbs = 2 * nbytes * repeats / (e0.elapsed_time(e1) * 1e-3) / 1e9
                if best is None or gbs > best[0]:
                    best = (gbs, unroll, nt)
        assert torch.equal(a[:1024], b[:1024])
        out[label] = {"bytes_per_buffer": nbytes, "GBs": round(best[0], 1),
                      "frac": round(best[0] / HBM_PEAK_GBS, 4),
                      "unroll": best[1], "nontemporal_stores": bool(best[2])}
        del a, b
        torch.cuda.empty_cache()
    return out


def adjoint_bytes_per_update(q: int, per_cell_w: bool = False) -> float:
    """Algorithmic HBM bytes per cell-direction update of one reverse step:
    adjoint populations read and written, forward state read (12 B); per cell
    the eight move-class partial sums read and written (64 B), the forward E
    read (4 B), the float64 gradient accumulator read and written (16 B), and
    a per-cell weight field (4 B)."""
    return 12.0 + (64.0 + 4.0 + 16.0 + (4.0 if per_cell_w else 0.0)) / q


def run_adjoint_ratio(n=256, q=64, steps=1000, K=50, repeats=3):
    """Forward (with checkpoints and probe reads) and backward (recompute +
    reverse steps) of the n x n, Q = q inverse problem; median times."""
    import numpy as np
    import torch

    from paper_1911_00180_amd import inputs
    from paper_1911_00180_amd.autodiff import ProbeSeries
    from paper_1911_00180_amd.lattice import Lattice

    n, mfp, tgt, T0, probes = inputs.inverse_problem(n)
    lat = Lattice(n, n, q, mfp=16.0, x_edge="blackbody", y_edge="periodic", device="cuda:0")
    series = ProbeSeries(lat, probes, steps, 10, checkpoint_every=K)
    dev = "cuda:0"
    walls = torch.tensor([0.5, 0.0, 0.0, 0.0], device=dev)
    T0d = torch.from_numpy(T0).to(dev)
    with torch.no_grad():
        target = series(torch.from_numpy(tgt).to(dev), T0d, walls)
    stream = torch.cuda.current_stream()
    fwd, bwd = [], []
    for r in range(repeats + 1):
        m = torch.from_numpy(mfp).to(dev).requires_grad_(True)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        torch.cuda.synchronize()
        e0.record(stream)
        out = series(m, T0d, walls)
        loss = ((out - target) ** 2).sum()
        e1.record(stream)
        loss.backward()
        e2.record(stream)
        torch.cuda.synchronize()
        if r:
            fwd.append(e0.elapsed_time(e1))
            bwd.append(e1.elapsed_time(e2))
    grad_ok = bool(torch.isfinite(m.grad).all())
    state_gb = (series.ck.numel() + series.tape.numel()) / 1e9
    lat.close()
    del out, loss, m, series, target
    torch.cuda.empty_cache()
    f, b = float(np.median(fwd)), float(np.median(bwd))
    return {"workload": f"{n}x{n}, Q={q}, lognormal MFP field (median 16, clipped 4..64, "
                        f"correlation {16 * n // 256}), blackbody x walls 0.5/0, periodic y, "
                        f"{steps} steps, 32 probes, loss every 10 steps, checkpoint every {K}",
            "forward_ms": round(f, 3), "backward_ms": round(b, 3),
            "ratio": round(b / f, 3), "grad_finite": grad_ok,
            "saved_states_GB": round(state_gb, 2),
            "forward_gups": round(n * n * q * steps / (f * 1e-3) / 1e9, 2)}


def run_adjoint_kernel(nx=1024, ny=1024, q=64, steps=20):
    """Reverse steps on the 1024 x 1024, Q = 64 periodic lattice (uniform
    MFP 102.4): average time per step over a tape of `steps` states."""
    import numpy as np
    import torch

    from paper_1911_00180_amd import inputs
    from paper_1911_00180_amd import wormlbm as W
    from paper_1911_00180_amd.lattice import Lattice

    x0, y0 = inputs.seeded_center(1911, nx, ny)
    T0 = inputs.gaussian_pulse(nx, ny, 16.0, x0, y0).astype(np.float32)
    lat = Lattice(nx, ny, q, mfp=102.4, device="cuda:0")
    lat.set_temperature(torch.from_numpy(T0))
    tape = lat.new_states(steps)
    lat.save_state(tape[0])
    lat.step_tape(steps - 1, tape[1:])
    ws = torch.empty(W.wlbm_adjoint_bytes(lat.handle), dtype=torch.uint8, device="cuda:0")
    cells = torch.tensor([[x0, y0]], dtype=torch.int32, device="cuda:0")
    seed = torch.ones(1, dtype=torch.float32, device="cuda:0")
    stream = torch.cuda.current_stream()
    times = []
    for r in range(4):
        lat._sync_stream()
        W.wlbm_adjoint_begin(lat.handle, ws.data_ptr(), ws.numel(), steps)
        W.wlbm_adjoint_seed(lat.handle, 1, cells.data_ptr(), seed.data_ptr())
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        W.wlbm_adjoint_steps(lat.handle, steps, tape[0].data_ptr(), tape.shape[1])
        e1.record(stream)
        torch.cuda.synchronize()
        if r:
            times.append(e0.elapsed_time(e1) / steps)
    lat.close()
    ms = float(np.median(times))
    bpu = adjoint_bytes_per_update(q)
    achieved = bpu * nx * ny * q / (ms * 1e-3) / 1e9
    return {"workload": f"{nx}x{ny} periodic, Q={q}, uniform MFP 102.4, {steps} reverse steps",
            "ms_per_step": round(ms, 5), "bytes_per_update": round(bpu, 4),
            "achieved_GBs": round(achieved, 1), "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": recorded_traffic(ADJOINT_TRAFFIC_FILE, ADJOINT_SOURCES)}


def run_films(steps=10000):
    """The 24-film sweep (Nx = 512, Q = 128, Ny 32..256, blackbody x, diffuse
    y): fixed steps batched (one launch for all films per two steps, block
    height tuned for the batch) against one-by-one."""
    import torch

    from paper_1911_00180_amd.films import FilmSweep, film_set

    films = film_set()
    out = {"workload": "24 films, Nx=512, Q=128, Ny from {32,64,128,256}, Kn 0.01..100, "
                       f"blackbody x 1/0, diffuse y, {steps} steps"}
    stream = torch.cuda.current_stream()
    for mode in ("batched", "batched_graphs", "one_by_one"):
        sw = FilmSweep(films)
        if mode == "batched_graphs":
            sw.batch.set_graphs(True)
        if mode != "one_by_one" and sw.batch.steps_per_launch > 1:
            # one block height for the whole batch, timed on a saved state
            # before the timed steps (one by one, each film keeps its own)
            out["batch_block_rows"] = sw.batch.tune_block_rows()
        go = sw.step_each if mode == "one_by_one" else sw.step_batched
        go(20)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        go(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        out[mode + "_ms_per_step"] = round(ms / steps, 5)
        out[mode + "_gups"] = round(sw.updates_per_step * steps / (ms * 1e-3) / 1e9, 2)
        sw.close()
    out["speedup"] = round(out["one_by_one_ms_per_step"] / out["batched_ms_per_step"], 3)
    out["graph_speedup"] = round(out["batched_ms_per_step"] / out["batched_graphs_ms_per_step"], 3)
    out.update(run_small_batch())
    return out


def run_small_batch(steps=4800):
    """A small batch, where per-step launch costs would show most: 24
    lattices of 64 x 64, Q = 16, blackbody x and diffuse y walls, MFP 4 .. 64
    cells; graph launches of whole schedule chunks against one launch per
    step."""
    import torch

    from paper_1911_00180_amd.lattice import Batch, Lattice

    out = {}
    stream = torch.cuda.current_stream()
    for graphs in (True, False):
        lats = [Lattice(64, 64, 16, mfp=4.0 * 16 ** (j / 23), x_edge="blackbody",
                        y_edge="diffuse", t_x_lo=1.0, device="cuda:0") for j in range(24)]
        batch = Batch(lats)
        batch.set_graphs(graphs)
        batch.step(480)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        batch.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        key = "small_batch_graphs_us_per_step" if graphs else "small_batch_no_graphs_us_per_step"
        out[key] = round(e0.elapsed_time(e1) * 1e3 / steps, 3)
        batch.close()
        for lat in lats:
            lat.close()
    out["small_batch_workload"] = ("24 lattices 64x64, Q=16, blackbody x, diffuse y, "
                                   f"MFP 4..64, {steps} steps")
    out["small_batch_graph_speedup"] = round(out["small_batch_no_graphs_us_per_step"] /
                                             out["small_batch_graphs_us_per_step"], 3)
    return out


def cpu_baseline(budget_s: float = 15.0):
    """The FP64 oracle on a bounded sample of the same workload: a 256 x 256
    periodic crop with the same Q and MFP, timed on the host."""
    import numpy as np

    from oracle import worm_lbm as o
    from paper_1911_00180_amd import inputs

    nx = ny = 256
    q = 64
    x0, y0 = inputs.seeded_center(1911, 1024, 1024)
    T0 = inputs.gaussian_pulse(nx, ny, 16.0, x0 % nx, y0 % ny)
    lat = o.Lattice(o.Config(nx=nx, ny=ny, q=q, mfp=102.4))
    lat.set_temperature(T0)
    lat.schedule(4000)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        lat.step()
        n += 1
    dt = time.perf_counter() - t0
    # the small parity lattice too: 64 x 64, Q = 16, MFP 16, 200 steps
    c1 = o.Lattice(o.Config(nx=64, ny=64, q=16, mfp=16.0))
    xx = np.arange(64) - 32
    c1.set_temperature(np.exp(-(xx[None, :] ** 2 + xx[:, None] ** 2) / (2 * 4.0 ** 2)))
    t1 = time.perf_counter()
    c1.run(200)
    d1 = time.perf_counter() - t1
    return {
        "value": nx * ny * q * n / dt / 1e9,
        "unit": "Gupdates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"256x256 periodic crop, Q=64, MFP 102.4, {n} steps of the FP64 numpy "
                  f"oracle in {dt:.1f} s (numpy elementwise ops, one thread; host has "
                  f"{os.cpu_count()} logical CPUs)",
        "small_lattice": {"workload": "64x64 periodic, Q=16, MFP 16, 200 steps",
                          "value": round(64 * 64 * 16 * 200 / d1 / 1e9, 4),
                          "unit": "Gupdates/s", "seconds": round(d1, 3)},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3840)
    ap.add_argument("--warmup", type=int, default=960)
    ap.add_argument("--kn", type=float, default=0.1, help="Knudsen number vs L = 1024")
    ap.add_argument("--split", type=int, default=0,
                    help="waves sharing one cell's directions (0 = library default)")
    ap.add_argument("--large", action="store_true",
                    help="also time the 2048 x 2048, Q = 128 inverse problem (about 160 GB "
                         "of checkpoints)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 4096 x 4096, Q = 256 wall-bounded lattice")
    ap.add_argument("--large-steps", type=int, default=200)
    ap.add_argument("--no-stream", action="store_true",
                    help="skip the read+write stream-kernel ceiling")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint measurements")
    ap.add_argument("--no-films", action="store_true", help="skip the batched film sweep")
    ap.add_argument("--steps-per-launch", type=int, default=4, choices=(1, 2, 3, 4),
                    help="time steps per kernel launch on the default lattice")
    ap.add_argument("--single-step", action="store_true",
                    help="same as --steps-per-launch 1")
    ap.add_argument("--film-steps", type=int, default=10000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--block-rows", default="",
                    help="fixed block heights of the multi-step kernels instead of the "
                         "library's timing, as K:R pairs, e.g. 4:9,3:8 (for profiling runs)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a device copy of this size (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)

    if args.copy_probe_mib:
        # five launches of the read+write stream kernel (16-byte loads and
        # stores, four per thread) over buffers of this size: the reference
        # for scaling the FETCH_SIZE and WRITE_SIZE counters
        import ctypes
        nbytes = args.copy_probe_mib * (1 << 20)
        probe = ctypes.CDLL(os.path.join(ROOT, "paper_1911_00180_amd", "libwlbm_probe.so"))
        probe.wlbm_probe_copy.restype = ctypes.c_int
        probe.wlbm_probe_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        a = torch.ones(nbytes // 4, device="cuda:0")
        b = torch.empty_like(a)
        stream = torch.cuda.current_stream().cuda_stream
        for _ in range(5):
            if probe.wlbm_probe_copy(a.data_ptr(), b.data_ptr(), nbytes, 4, 0, stream):
                sys.exit("bench.py: stream probe failed")
        torch.cuda.synchronize()
        assert torch.equal(a[:1024], b[:1024])
        print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes,
                          "launches": 5, "kernel": "k_copy (libwlbm_probe.so)"}))
        return

    nx = ny = 1024
    q = 64
    mfp = args.kn * nx
    spl = 1 if args.single_step else args.steps_per_launch
    # every launch must advance spl steps: whole schedule chunks (240 steps)
    # split evenly
    if args.steps % 240 % spl or args.steps % spl:
        sys.exit(f"bench.py: --steps must split into launches of {spl} steps "
                 "within 240-step schedule chunks")
    fixed_rows = {}
    for item in filter(None, args.block_rows.split(",")):
        k, rows = (int(v) for v in item.split(":"))
        fixed_rows[k] = rows
    ms, wall, energy = run_gpu(nx, ny, q, mfp, args.steps, args.warmup, {}, args.split,
                               fusion=spl if spl > 1 else 0, block_rows=fixed_rows)
    updates = nx * ny * q * args.steps
    gups = updates / (ms * 1e-3) / 1e9
    ms_step = ms / args.steps
    bpu = bytes_per_update(q)
    # Dominant kernel: the launch advancing spl steps.  Algorithmic bytes per
    # launch = the per-update figure (8 + 8/Q B: each population read and
    # written once per step, E read and written once per cell) times the
    # updates one launch processes, nx * ny * q * spl.  With several steps per
    # launch the kernel keeps the intermediate steps on chip, so this rate can
    # exceed the HBM peak; hbm_frac_one_pass is the share of the peak that
    # one pass over the arrays per launch (what it actually must move) takes.
    steps_per_launch = spl
    launches = args.steps // steps_per_launch
    ms_launch = ms / launches
    alg_bytes_launch = bpu * nx * ny * q * steps_per_launch
    one_pass_bytes = bpu * nx * ny * q
    achieved = alg_bytes_launch / (ms_launch * 1e-3) / 1e9
    traffic = (recorded_traffic(FUSED_TRAFFIC_FILES[spl], FUSED_SOURCES) if spl > 1
               else recorded_traffic())
    out = {
        "metric": "G cell-direction updates/s",
        "value": round(gups, 3),
        "unit": "Gupdates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {
            "workload": "worm-LBM collide-and-stream, 1024x1024 periodic, Q=64 evenly spaced "
                        "directions, TAS + grid-MFP correction, gray model",
            "nx": nx, "ny": ny, "q": q, "kn": args.kn, "mfp_cells": mfp,
            "initial": "Gaussian pulse sigma0=16 at default_rng(1911) position",
            "bytes_per_update": bpu,
            "steps_per_launch": steps_per_launch,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": KERNELS[spl],
            "block_rows": run_gpu.block_rows,
            "launches": launches,
            "ms_per_launch": round(ms_launch, 5),
            "algorithmic_bytes_per_launch": alg_bytes_launch,
            "one_pass_bytes_per_launch": one_pass_bytes,
            "hbm_frac_one_pass": round(one_pass_bytes / (ms_launch * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                       4),
            "hbm_frac_traffic": (round(traffic / (ms_launch * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                 if traffic else None),
        },
        "wall_s": round(wall, 4),
        "energy_after": energy,
    }
    # context: the same workload at fewer time steps per launch
    out["fewer_steps_per_launch"] = {}
    for k in range(1, spl):
        msk, _, _ = run_gpu(nx, ny, q, mfp, args.steps, args.warmup, {}, args.split,
                            fusion=k if k > 1 else 0, block_rows=fixed_rows)
        stk = msk / args.steps
        ak = bpu * nx * ny * q * k / (stk * k * 1e-3) / 1e9
        out["fewer_steps_per_launch"][str(k)] = {
            "kernel": KERNELS[k],
            "block_rows": run_gpu.block_rows,
            "value": round(updates / (msk * 1e-3) / 1e9, 3),
            "unit": "Gupdates/s",
            "ms_per_step": round(stk, 5),
            "ms_per_launch": round(stk * k, 5),
            "achieved_GBs": round(ak, 1),
            "frac": round(ak / HBM_PEAK_GBS, 4),
            "traffic": (recorded_traffic(FUSED_TRAFFIC_FILES[k], FUSED_SOURCES) if k > 1
                        else recorded_traffic()),
        }
    if not args.no_large:
        nl, ql = 4096, 256
        edges = dict(x_edge="blackbody", y_edge="diffuse", t_x_lo=1.0, t_x_hi=0.0)
        # block height timed on a saved state before the timed steps (about
        # 2 s: the 17 GB state is restored after each candidate)
        msl, walll, _ = run_gpu(nl, nl, ql, 10.0 * nl, args.large_steps, 10, edges, fusion=1)
        st = msl / args.large_steps
        kl = run_gpu.steps_per_launch
        bl = bytes_per_update(ql) * nl * nl * ql
        out["large"] = {
            "workload": "4096x4096, Q=256, blackbody x walls (T=1/0), diffuse y walls, Kn=10 "
                        "(MFP 40960 cells), Gaussian pulse sigma0=16 at the seeded position",
            "steps": args.large_steps,
            "value": round(nl * nl * ql / (st * 1e-3) / 1e9, 3),
            "unit": "Gupdates/s",
            "ms_per_step": round(st, 4),
            "steps_per_launch": kl,
            "block_rows": run_gpu.block_rows,
            "bytes_per_update": bytes_per_update(ql),
            # per-update bytes x updates per launch / launch time, and the
            # share of the peak one pass over the arrays per launch takes
            "roofline_frac": round(bl / (st * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "hbm_frac_one_pass": round(bl / kl / (st * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        }
    if args.large:
        # the 2048 x 2048, Q = 128 inverse problem, checkpoints sized to HBM
        out["large_adjoint"] = run_adjoint_ratio(n=2048, q=128, steps=1000, K=50, repeats=1)
    if not args.no_stream:
        pbytes = 4 * (nx + 64) * (ny + 2) * q
        out["stream_ceiling"] = run_stream_ceiling(
            [("1024x1024_q64", pbytes), ("4096x4096_q256", 4 * (4096 + 64) * 4098 * 256)])
    if not args.no_adjoint:
        adj = run_adjoint_ratio()
        adj["kernel"] = run_adjoint_kernel()
        out["adjoint"] = adj
    if not args.no_films:
        out["films"] = run_films(args.film_steps)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
