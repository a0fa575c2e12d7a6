"""FP64 CPU oracle of the worm-LBM (test infrastructure only).

Imported only by the test suite, the smoke check and the benchmark's
CPU-baseline leg.  The GPU library never imports or links anything here.
"""
from .worm_lbm import *  # noqa: F401,F403
