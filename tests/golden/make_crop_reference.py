"""Write tests/golden/crop256_q64_{kn}.json from the FP64 oracle.

The 256 x 256 periodic crop of the 1024 x 1024, Q = 64 workload: evenly
spaced directions, MFP 102.4 cells (Kn = 0.1 against L = 1024) or 10240
(Kn = 10), Gaussian sigma0 = 16 at (x0 mod 256, y0 mod 256) with (x0, y0)
drawn by default_rng(1911) on the 1024 lattice, 4000 steps.  Stored: T on
2048 seeded cells, on the row and the column through the pulse centre, the
maximum of |T| over the whole field and the total energy.  Calls only the
oracle and the seeded input module.

    python tests/golden/make_crop_reference.py [kn ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import worm_lbm as o  # noqa: E402
from paper_1911_00180_amd import inputs  # noqa: E402

N, Q, STEPS = 256, 64, 4000


def crop_input():
    x0, y0 = inputs.seeded_center(1911, 1024, 1024)
    cx, cy = x0 % N, y0 % N
    T0 = inputs.gaussian_pulse(N, N, 16.0, cx, cy).astype(np.float32)
    return T0, cx, cy


def sample_cells():
    return inputs.probe_cells(256, N, N, 2048)


def main(kns):
    T0, cx, cy = crop_input()
    cells = sample_cells()
    for kn in kns:
        mfp = kn * 1024
        lat = o.Lattice(o.Config(nx=N, ny=N, q=Q, mfp=mfp))
        lat.set_temperature(T0.astype(np.float64))
        t = time.time()
        lat.run(STEPS)
        T = lat.temperature()
        out = {
            "workload": f"256x256 periodic crop, Q={Q} uniform, MFP {mfp} cells, "
                        f"Gaussian sigma0=16 at ({cx},{cy}), {STEPS} steps",
            "kn": kn, "mfp": mfp, "steps": STEPS, "center": [cx, cy],
            "max_abs_T": float(np.abs(T).max()),
            "energy": lat.energy(),
            "cells": cells.tolist(),
            "T_cells": [float(T[y, x]) for x, y in cells],
            "T_row": [float(v) for v in T[cy, :]],
            "T_col": [float(v) for v in T[:, cx]],
        }
        path = os.path.join(HERE, f"crop256_q64_kn{kn:g}.json")
        with open(path, "w") as f:
            json.dump(out, f)
        print(f"{path}: {time.time() - t:.0f} s", flush=True)


if __name__ == "__main__":
    main([float(a) for a in sys.argv[1:]] or [0.1, 10.0])
