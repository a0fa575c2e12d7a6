"""MI355X-native worm-LBM (gray phonon BTE) hot path.

The compute path is the C-ABI library ``libwormlbm.so`` (hand-written HIP for
gfx950); :mod:`paper_1911_00180_amd.wormlbm` is its thin ctypes binding and
:mod:`paper_1911_00180_amd.lattice` a convenience wrapper that allocates the
device workspace with PyTorch.  Importing this package does not load the
library; the binding loads it on first use and raises if it is missing.
"""
__all__ = ["wormlbm", "lattice", "inputs"]
