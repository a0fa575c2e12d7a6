"""ctypes binding of libwormlbm.so (C-ABI declared in include/wormlbm.h).

Argument marshalling only: every function forwards to the C function of the
same name; device pointers are passed as integers (e.g. ``tensor.data_ptr()``)
and streams as the raw HIP stream handle.  Failing calls raise WormLBMError
with the library's status and message.  The library is loaded on first use;
if it has not been built this raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_int8, c_int32, c_int64, \
    c_size_t, c_void_p

LIB_PATH = os.environ.get(
    "WORMLBM_LIB", os.path.join(os.path.dirname(os.path.abspath(__file__)), "libwormlbm.so"))

WLBM_OK = 0
WLBM_EINVAL = -1
WLBM_EUNSTABLE = -2
WLBM_ENOMEM = -3
WLBM_EHIP = -4
WLBM_ENONFINITE = -5
WLBM_ESTATE = -6

EDGE_PERIODIC, EDGE_BLACKBODY, EDGE_DIFFUSE = 0, 1, 2
DIRS_UNIFORM, DIRS_RING = 0, 1

STATUS_NAMES = {0: "WLBM_OK", -1: "WLBM_EINVAL", -2: "WLBM_EUNSTABLE", -3: "WLBM_ENOMEM",
                -4: "WLBM_EHIP", -5: "WLBM_ENONFINITE", -6: "WLBM_ESTATE"}

# every function the header declares, checked by the test suite
EXPORTS = (
    "wlbm_default_params", "wlbm_workspace_bytes", "wlbm_create", "wlbm_set_stream",
    "wlbm_set_temperature", "wlbm_set_populations", "wlbm_set_mfp_field",
    "wlbm_set_wall_temperatures", "wlbm_set_flux_window", "wlbm_step",
    "wlbm_read_temperature", "wlbm_read_heat_flux", "wlbm_read_populations",
    "wlbm_read_totals", "wlbm_get_directions", "wlbm_get_constants", "wlbm_get_schedule",
    "wlbm_step_count", "wlbm_last_error", "wlbm_destroy",
    "wlbm_state_bytes", "wlbm_save_state", "wlbm_load_state", "wlbm_step_tape",
    "wlbm_read_probes", "wlbm_adjoint_bytes", "wlbm_adjoint_begin", "wlbm_adjoint_seed",
    "wlbm_adjoint_steps", "wlbm_adjoint_read", "wlbm_adjoint_step_index",
    "wlbm_set_dir_split", "wlbm_get_dir_split", "wlbm_autotune", "wlbm_batch_bytes",
    "wlbm_batch_create", "wlbm_batch_step", "wlbm_batch_set_graphs", "wlbm_batch_destroy",
    "wlbm_read_flux_mean",
    "wlbm_set_sources", "wlbm_flux_distribution", "wlbm_set_speeds",
    "wlbm_accumulate_temperature", "wlbm_get_block_rows", "wlbm_set_block_rows",
    "wlbm_tune_block_rows", "wlbm_read_totals_noalloc", "wlbm_get_steps_per_launch",
    "wlbm_batch_get_steps_per_launch", "wlbm_batch_tune_block_rows",
)


class WlbmParams(ctypes.Structure):
    """Mirror of struct wlbm_params."""
    _fields_ = [
        ("nx", c_int32), ("ny", c_int32), ("q", c_int32), ("dirs", c_int32),
        ("mfp_cells", c_double),
        ("emulate_3d", c_int32), ("mfp_correction", c_int32),
        ("x_edge", c_int32), ("y_edge", c_int32),
        ("t_x_lo", c_double), ("t_x_hi", c_double), ("t_y_lo", c_double), ("t_y_hi", c_double),
        ("dir_split", c_int32), ("sched_chunk", c_int32),
        ("y_specularity", c_double),
        ("step_fusion", c_int32),
        ("reserved", c_int32 * 3),
    ]


class WormLBMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libwormlbm.so (once)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1911_00180_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = POINTER(WlbmParams)
    sig = {
        "wlbm_default_params": (None, [P]),
        "wlbm_workspace_bytes": (c_int, [P, POINTER(c_size_t)]),
        "wlbm_create": (c_int, [P, c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]),
        "wlbm_set_stream": (c_int, [c_void_p, c_void_p]),
        "wlbm_set_temperature": (c_int, [c_void_p, c_void_p]),
        "wlbm_set_populations": (c_int, [c_void_p, c_void_p]),
        "wlbm_set_mfp_field": (c_int, [c_void_p, c_void_p]),
        "wlbm_set_wall_temperatures": (c_int, [c_void_p, c_double, c_double, c_double, c_double]),
        "wlbm_set_flux_window": (c_int, [c_void_p, c_int32]),
        "wlbm_step": (c_int, [c_void_p, c_int64]),
        "wlbm_read_temperature": (c_int, [c_void_p, c_void_p]),
        "wlbm_read_heat_flux": (c_int, [c_void_p, c_void_p, c_void_p, c_int32]),
        "wlbm_read_populations": (c_int, [c_void_p, c_void_p]),
        "wlbm_read_totals": (c_int, [c_void_p, POINTER(c_double), POINTER(c_double),
                                     POINTER(c_double)]),
        "wlbm_get_directions": (c_int, [P, POINTER(c_double), POINTER(c_double),
                                        POINTER(c_double)]),
        "wlbm_get_constants": (c_int, [P, POINTER(c_double), POINTER(c_double),
                                       POINTER(c_double)]),
        "wlbm_get_schedule": (c_int, [P, POINTER(c_double), c_int64, c_int64, POINTER(c_int8),
                                      POINTER(c_int64)]),
        "wlbm_step_count": (c_int64, [c_void_p]),
        "wlbm_last_error": (c_char_p, []),
        "wlbm_destroy": (c_int, [c_void_p]),
        "wlbm_state_bytes": (c_int, [c_void_p, POINTER(c_size_t)]),
        "wlbm_save_state": (c_int, [c_void_p, c_void_p, c_size_t]),
        "wlbm_load_state": (c_int, [c_void_p, c_void_p, c_size_t, c_int64]),
        "wlbm_step_tape": (c_int, [c_void_p, c_int64, c_void_p, c_size_t]),
        "wlbm_read_probes": (c_int, [c_void_p, c_int32, c_void_p, c_void_p]),
        "wlbm_adjoint_bytes": (c_int, [c_void_p, POINTER(c_size_t)]),
        "wlbm_adjoint_begin": (c_int, [c_void_p, c_void_p, c_size_t, c_int64]),
        "wlbm_adjoint_seed": (c_int, [c_void_p, c_int32, c_void_p, c_void_p]),
        "wlbm_adjoint_steps": (c_int, [c_void_p, c_int64, c_void_p, c_size_t]),
        "wlbm_adjoint_read": (c_int, [c_void_p, c_void_p, c_void_p, POINTER(c_double)]),
        "wlbm_adjoint_step_index": (c_int64, [c_void_p]),
        "wlbm_set_dir_split": (c_int, [c_void_p, c_int32]),
        "wlbm_get_dir_split": (c_int32, [c_void_p]),
        "wlbm_get_block_rows": (c_int32, [c_void_p, c_int32]),
        "wlbm_set_block_rows": (c_int, [c_void_p, c_int32, c_int32]),
        "wlbm_tune_block_rows": (c_int, [c_void_p, c_void_p, c_size_t, c_int32, c_int32,
                                         POINTER(c_int32)]),
        "wlbm_read_totals_noalloc": (c_int, [c_void_p, c_void_p]),
        "wlbm_get_steps_per_launch": (c_int32, [c_void_p]),
        "wlbm_autotune": (c_int, [c_void_p, c_void_p, c_size_t, c_int32, POINTER(ctypes.c_float),
                                  POINTER(c_int32)]),
        "wlbm_batch_bytes": (c_int, [POINTER(c_void_p), c_int32, POINTER(c_size_t)]),
        "wlbm_batch_create": (c_int, [POINTER(c_void_p), c_int32, c_void_p, c_size_t, c_void_p,
                                      POINTER(c_void_p)]),
        "wlbm_batch_step": (c_int, [c_void_p, c_int64]),
        "wlbm_batch_set_graphs": (c_int, [c_void_p, c_int32]),
        "wlbm_batch_get_steps_per_launch": (c_int32, [c_void_p]),
        "wlbm_batch_tune_block_rows": (c_int, [c_void_p, c_void_p, c_size_t, c_int32,
                                               ctypes.POINTER(c_int32)]),
        "wlbm_batch_destroy": (c_int, [c_void_p]),
        "wlbm_read_flux_mean": (c_int, [c_void_p, c_int32, c_int32, c_int32, POINTER(c_double),
                                        POINTER(c_double)]),
        "wlbm_set_sources": (c_int, [c_void_p, c_int32, c_void_p, c_void_p]),
        "wlbm_flux_distribution": (c_int, [P, c_double, c_double, c_double, POINTER(c_double)]),
        "wlbm_set_speeds": (c_int, [c_void_p, POINTER(c_double)]),
        "wlbm_accumulate_temperature": (c_int, [c_void_p, c_double, c_void_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status: int) -> None:
    if status != WLBM_OK:
        msg = lib().wlbm_last_error().decode(errors="replace")
        raise WormLBMError(status, msg)


def _ptr(x):
    """Device or host pointer from an int, a torch tensor or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return c_void_p(x)
    return c_void_p(x.data_ptr())


# -- one wrapper per C function ---------------------------------------------
def wlbm_default_params() -> WlbmParams:
    p = WlbmParams()
    lib().wlbm_default_params(byref(p))
    return p


def wlbm_workspace_bytes(p: WlbmParams) -> int:
    n = c_size_t(0)
    _check(lib().wlbm_workspace_bytes(byref(p), byref(n)))
    return n.value


def wlbm_create(p: WlbmParams, d_workspace, ws_bytes: int, stream) -> int:
    h = c_void_p()
    _check(lib().wlbm_create(byref(p), _ptr(d_workspace), ws_bytes, c_void_p(stream or 0),
                             byref(h)))
    return h.value


def wlbm_set_stream(h: int, stream) -> None:
    _check(lib().wlbm_set_stream(c_void_p(h), c_void_p(stream or 0)))


def wlbm_set_temperature(h: int, d_T0) -> None:
    _check(lib().wlbm_set_temperature(c_void_p(h), _ptr(d_T0)))


def wlbm_set_populations(h: int, d_e) -> None:
    _check(lib().wlbm_set_populations(c_void_p(h), _ptr(d_e)))


def wlbm_set_mfp_field(h: int, d_mfp) -> None:
    _check(lib().wlbm_set_mfp_field(c_void_p(h), _ptr(d_mfp)))


def wlbm_set_wall_temperatures(h: int, t_x_lo: float, t_x_hi: float, t_y_lo: float,
                               t_y_hi: float) -> None:
    _check(lib().wlbm_set_wall_temperatures(c_void_p(h), t_x_lo, t_x_hi, t_y_lo, t_y_hi))


def wlbm_set_flux_window(h: int, window: int) -> None:
    _check(lib().wlbm_set_flux_window(c_void_p(h), window))


def wlbm_step(h: int, nsteps: int) -> None:
    _check(lib().wlbm_step(c_void_p(h), nsteps))


def wlbm_read_temperature(h: int, d_T) -> None:
    _check(lib().wlbm_read_temperature(c_void_p(h), _ptr(d_T)))


def wlbm_read_heat_flux(h: int, d_qx, d_qy, averaged: int = 0) -> None:
    _check(lib().wlbm_read_heat_flux(c_void_p(h), _ptr(d_qx), _ptr(d_qy), averaged))


def wlbm_read_populations(h: int, d_e) -> None:
    _check(lib().wlbm_read_populations(c_void_p(h), _ptr(d_e)))


def wlbm_read_totals(h: int):
    e, qx, qy = c_double(), c_double(), c_double()
    _check(lib().wlbm_read_totals(c_void_p(h), byref(e), byref(qx), byref(qy)))
    return e.value, qx.value, qy.value


def wlbm_get_directions(p: WlbmParams):
    import numpy as np
    sx, sy, w = (np.zeros(p.q) for _ in range(3))
    D = POINTER(c_double)
    _check(lib().wlbm_get_directions(byref(p), sx.ctypes.data_as(D), sy.ctypes.data_as(D),
                                     w.ctypes.data_as(D)))
    return sx, sy, w


def wlbm_get_constants(p: WlbmParams):
    lam, w, wc = c_double(), c_double(), c_double()
    _check(lib().wlbm_get_constants(byref(p), byref(lam), byref(w), byref(wc)))
    return lam.value, w.value, wc.value


def _host_doubles(v, n):
    import numpy as np
    if v is None:
        return None, None
    a = np.ascontiguousarray(v, dtype=np.float64)
    if a.shape != (n,):
        raise ValueError(f"expected {n} values")
    return a, a.ctypes.data_as(POINTER(c_double))


def wlbm_get_schedule(p: WlbmParams, step0: int, n: int, positions: bool = False,
                      speeds=None):
    """(moves [n, q] int8, positions [n, q, 2] int64 or None)."""
    import numpy as np
    moves = np.zeros((n, p.q), dtype=np.int8)
    pos = np.zeros((n, p.q, 2), dtype=np.int64) if positions else None
    keep, sp = _host_doubles(speeds, p.q)
    _check(lib().wlbm_get_schedule(
        byref(p), sp, step0, n, moves.ctypes.data_as(POINTER(c_int8)),
        pos.ctypes.data_as(POINTER(c_int64)) if positions else None))
    return moves, pos


def wlbm_set_speeds(h: int, q: int, speeds) -> None:
    keep, sp = _host_doubles(speeds, q)
    _check(lib().wlbm_set_speeds(c_void_p(h), sp))


def wlbm_accumulate_temperature(h: int, scale: float, d_T) -> None:
    _check(lib().wlbm_accumulate_temperature(c_void_p(h), scale, _ptr(d_T)))


def wlbm_step_count(h: int) -> int:
    return lib().wlbm_step_count(c_void_p(h))


def wlbm_last_error() -> str:
    return lib().wlbm_last_error().decode(errors="replace")


def wlbm_destroy(h: int) -> None:
    _check(lib().wlbm_destroy(c_void_p(h)))


def wlbm_state_bytes(h: int) -> int:
    n = c_size_t(0)
    _check(lib().wlbm_state_bytes(c_void_p(h), byref(n)))
    return n.value


def wlbm_save_state(h: int, d_buf, nbytes: int) -> None:
    _check(lib().wlbm_save_state(c_void_p(h), _ptr(d_buf), nbytes))


def wlbm_load_state(h: int, d_buf, nbytes: int, step: int) -> None:
    _check(lib().wlbm_load_state(c_void_p(h), _ptr(d_buf), nbytes, step))


def wlbm_step_tape(h: int, nsteps: int, d_tape, slot_bytes: int) -> None:
    _check(lib().wlbm_step_tape(c_void_p(h), nsteps, _ptr(d_tape), slot_bytes))


def wlbm_read_probes(h: int, n: int, d_cells, d_T) -> None:
    _check(lib().wlbm_read_probes(c_void_p(h), n, _ptr(d_cells), _ptr(d_T)))


def wlbm_adjoint_bytes(h: int) -> int:
    n = c_size_t(0)
    _check(lib().wlbm_adjoint_bytes(c_void_p(h), byref(n)))
    return n.value


def wlbm_adjoint_begin(h: int, d_ws, nbytes: int, step: int) -> None:
    _check(lib().wlbm_adjoint_begin(c_void_p(h), _ptr(d_ws), nbytes, step))


def wlbm_adjoint_seed(h: int, n: int, d_cells, d_dT) -> None:
    _check(lib().wlbm_adjoint_seed(c_void_p(h), n, _ptr(d_cells), _ptr(d_dT)))


def wlbm_adjoint_steps(h: int, n: int, d_states, slot_bytes: int) -> None:
    _check(lib().wlbm_adjoint_steps(c_void_p(h), n, _ptr(d_states), slot_bytes))


def wlbm_adjoint_read(h: int, d_g_mfp, d_g_T0):
    """Returns the four wall gradients (x_lo, x_hi, y_lo, y_hi)."""
    walls = (c_double * 4)()
    _check(lib().wlbm_adjoint_read(c_void_p(h), _ptr(d_g_mfp), _ptr(d_g_T0), walls))
    return tuple(walls)


def wlbm_adjoint_step_index(h: int) -> int:
    return lib().wlbm_adjoint_step_index(c_void_p(h))


def wlbm_set_dir_split(h: int, split: int) -> None:
    _check(lib().wlbm_set_dir_split(c_void_p(h), split))


def wlbm_get_dir_split(h: int) -> int:
    return lib().wlbm_get_dir_split(c_void_p(h))


def wlbm_get_block_rows(h: int, k: int) -> int:
    return lib().wlbm_get_block_rows(c_void_p(h), k)


def wlbm_set_block_rows(h: int, k: int, rows: int) -> None:
    _check(lib().wlbm_set_block_rows(c_void_p(h), k, rows))


def wlbm_get_steps_per_launch(h: int) -> int:
    return lib().wlbm_get_steps_per_launch(c_void_p(h))


def wlbm_read_totals_noalloc(h: int, d_totals) -> None:
    _check(lib().wlbm_read_totals_noalloc(c_void_p(h), _ptr(d_totals)))


def wlbm_tune_block_rows(h: int, d_state, nbytes: int, k: int, launches: int) -> int:
    rows = c_int32(0)
    _check(lib().wlbm_tune_block_rows(c_void_p(h), _ptr(d_state), nbytes, k, launches,
                                      byref(rows)))
    return rows.value


def wlbm_autotune(h: int, d_state, nbytes: int, steps: int):
    """(ms per step for splits 1, 2, 4 (-1 if invalid), chosen split)."""
    ms = (ctypes.c_float * 3)()
    chosen = c_int32(0)
    _check(lib().wlbm_autotune(c_void_p(h), _ptr(d_state), nbytes, steps, ms, byref(chosen)))
    return tuple(ms), chosen.value


def _handles(hs):
    arr = (c_void_p * len(hs))(*[c_void_p(h) for h in hs])
    return arr


def wlbm_batch_bytes(handles) -> int:
    n = c_size_t(0)
    _check(lib().wlbm_batch_bytes(_handles(handles), len(handles), byref(n)))
    return n.value


def wlbm_batch_create(handles, d_ws, nbytes: int, stream) -> int:
    b = c_void_p()
    _check(lib().wlbm_batch_create(_handles(handles), len(handles), _ptr(d_ws), nbytes,
                                   c_void_p(stream or 0), byref(b)))
    return b.value


def wlbm_batch_step(b: int, nsteps: int) -> None:
    _check(lib().wlbm_batch_step(c_void_p(b), nsteps))


def wlbm_batch_get_steps_per_launch(b: int) -> int:
    return lib().wlbm_batch_get_steps_per_launch(c_void_p(b))


def wlbm_batch_tune_block_rows(b: int, d_states, nbytes: int, launches: int) -> int:
    rows = c_int32(0)
    _check(lib().wlbm_batch_tune_block_rows(c_void_p(b), _ptr(d_states), nbytes, launches,
                                            byref(rows)))
    return rows.value


def wlbm_batch_set_graphs(b: int, on: int) -> None:
    _check(lib().wlbm_batch_set_graphs(c_void_p(b), on))


def wlbm_batch_destroy(b: int) -> None:
    _check(lib().wlbm_batch_destroy(c_void_p(b)))


def wlbm_read_flux_mean(h: int, x0: int, x1: int, averaged: int = 1):
    qx, qy = c_double(), c_double()
    _check(lib().wlbm_read_flux_mean(c_void_p(h), x0, x1, averaged, byref(qx), byref(qy)))
    return qx.value, qy.value


def wlbm_set_sources(h: int, n: int, d_cells, d_values) -> None:
    _check(lib().wlbm_set_sources(c_void_p(h), n, _ptr(d_cells), _ptr(d_values)))


def wlbm_flux_distribution(p: WlbmParams, T: float, qx: float, qy: float):
    import numpy as np
    e = np.zeros(p.q)
    _check(lib().wlbm_flux_distribution(byref(p), T, qx, qy, e.ctypes.data_as(POINTER(c_double))))
    return e


def make_params(nx: int, ny: int, q: int, mfp: float = float("inf"), dirs: str = "uniform",
                emulate_3d: bool = False, mfp_correction: bool = True,
                x_edge: str = "periodic", y_edge: str = "periodic",
                t_x_lo: float = 0.0, t_x_hi: float = 0.0, t_y_lo: float = 0.0,
                t_y_hi: float = 0.0, dir_split: int = 0,
                sched_chunk: int = 0, y_specularity: float = 0.0,
                step_fusion: int = 1) -> WlbmParams:
    """Parameters from keyword arguments (edge and direction names as strings).
    step_fusion: 1 / True = library default (up to four time steps per launch
    where the lattice allows it), 2 .. 4 = at most that many, 0 / False = one
    step per launch."""
    edges = {"periodic": EDGE_PERIODIC, "blackbody": EDGE_BLACKBODY, "diffuse": EDGE_DIFFUSE}
    p = wlbm_default_params()
    p.nx, p.ny, p.q = nx, ny, q
    p.dirs = {"uniform": DIRS_UNIFORM, "ring": DIRS_RING}[dirs]
    p.mfp_cells = mfp
    p.emulate_3d = int(emulate_3d)
    p.mfp_correction = int(mfp_correction)
    p.x_edge = edges[x_edge]
    p.y_edge = edges[y_edge]
    p.t_x_lo, p.t_x_hi, p.t_y_lo, p.t_y_hi = t_x_lo, t_x_hi, t_y_lo, t_y_hi
    p.dir_split, p.sched_chunk = dir_split, sched_chunk
    p.y_specularity = y_specularity
    p.step_fusion = int(step_fusion)
    return p
