"""Build libwormlbm.so in-tree with hipcc for gfx950.

Usage: python -m paper_1911_00180_amd.build   (or call build()).

Each source is compiled to an object file in parallel (no device code is
shared between sources), then the objects are linked into the library.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libwormlbm.so")
# Longest compiles first (the multi-step kernel instantiations), so that the
# parallel build ends soonest.
SOURCES = ["fused_batch_flux4.hip", "fused_batch_flux3.hip", "fused_batch_flux2.hip",
           "fused_flux4.hip", "fused_flux3.hip", "fused_flux2.hip", "fused_batch4.hip",
           "fused_batch3.hip", "fused_batch2.hip", "fused_walls4.hip", "fused_walls3.hip",
           "fused_walls2.hip", "fused.hip", "kernels.hip", "adjoint.hip", "reduce.hip",
           "api.hip", "api_states.hip", "api_batch.hip", "api_tune.hip", "api_noalloc.hip",
           "tables.cpp"]
# Stand-alone HBM stream kernel used by the benchmark to measure the
# practical read+write ceiling of the device (not part of the library).
PROBE_LIB = os.path.join(PKG, "libwlbm_probe.so")
PROBE_SOURCES = ["stream_probe.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-fvisibility=hidden",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wshadow",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    errs = [ln for ln in res.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if res.returncode != 0:
        sys.stderr.write(res.stderr)
        raise RuntimeError(f"hipcc failed with code {res.returncode}: {' '.join(cmd[-3:])}")
    if verbose and errs:
        sys.stderr.write("\n".join(errs) + "\n")


def _link(sources, out, tmpdir, verbose, jobs):
    objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in sources]
    cmds = [[hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-c",
             os.path.join(CSRC, s), "-o", o] for s, o in zip(sources, objs)]
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = out + ".tmp"
    _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, out)


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source into the shared library (and the stream probe);
    returns the library's path."""
    with tempfile.TemporaryDirectory(prefix="wlbm_build_") as tmpdir:
        _link(SOURCES, LIB, tmpdir, verbose, jobs)
        _link(PROBE_SOURCES, PROBE_LIB, tmpdir, verbose, jobs)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
