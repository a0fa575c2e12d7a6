"""Write tests/golden/inverse256_q64.npz from the FP64 oracle.

The 256 x 256, Q = 64 inverse problem at full size: evenly spaced directions,
per-cell MFP field (lognormal around 16 cells, clipped to 4 .. 64, correlation
16 cells, default_rng(1)), blackbody x walls at 0.5 and 0, periodic y, centred
Gaussian pulse sigma0 = 16, 1000 steps, 32 probe cells (default_rng(3)), loss
sum_k sum_p (T^k(p) - T^_k(p))^2 at k = 10, 20, ..., 1000.  The targets T^
are the oracle's own probe temperatures for the MFP field of default_rng(2).
The gradients come from the oracle's transposed recursion with a checkpoint
every 50 steps.  Stored: targets, the probe temperatures of the run, the loss,
dL/dMFP, dL/dT0 and the wall gradients, and a hash of the inputs.  Calls only
the oracle and the seeded input module.

    python tests/golden/make_inverse_reference.py
"""
import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import adjoint as oadj  # noqa: E402
from oracle import worm_lbm as o  # noqa: E402
from paper_1911_00180_amd import inputs  # noqa: E402

Q, STEPS, EVERY, K = 64, 1000, 10, 50
WALLS = (0.5, 0.0)
PATH = os.path.join(HERE, "inverse256_q64.npz")


def input_hash(mfp, tgt, T0, probes) -> str:
    h = hashlib.sha256()
    for a in (mfp, tgt, T0, probes):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


def config(n, mfp):
    return o.Config(nx=n, ny=n, q=Q, mfp=np.asarray(mfp, dtype=np.float64),
                    x_edge="blackbody", y_edge="periodic", t_x_lo=WALLS[0], t_x_hi=WALLS[1])


def main():
    n, mfp, tgt, T0, probes = inputs.inverse_problem_256()
    t = time.time()
    targets = oadj.probe_temperatures(config(n, tgt), T0.astype(np.float64), STEPS, probes,
                                      EVERY)
    print(f"targets: {time.time() - t:.0f} s", flush=True)
    t = time.time()
    T_run = oadj.probe_temperatures(config(n, mfp), T0.astype(np.float64), STEPS, probes, EVERY)
    print(f"probe temperatures: {time.time() - t:.0f} s", flush=True)
    t = time.time()
    loss, g_mfp, g_T0, g_w = oadj.probe_loss_gradients(
        config(n, mfp), T0.astype(np.float64), STEPS, probes, EVERY, targets,
        checkpoint_every=K)
    print(f"gradients: {time.time() - t:.0f} s", flush=True)
    np.savez_compressed(
        PATH, targets=targets, T_probes=T_run, loss=np.float64(loss), g_mfp=g_mfp, g_T0=g_T0,
        g_walls=np.array([g_w["x_lo"], g_w["x_hi"], g_w["y_lo"], g_w["y_hi"]]),
        input_hash=np.array(input_hash(mfp, tgt, T0, probes)))
    print(PATH, f"loss {loss:.6e}", flush=True)


if __name__ == "__main__":
    main()
