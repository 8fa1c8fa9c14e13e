"""Python binding of the C ABI in ``include/rwpt.h`` (ctypes; marshalling only).

Every step of the method runs in the HIP kernels of ``librwpt.so``.  There is
no CPU fallback: if the library is missing, importing this module's functions
raises.  Functions keep the C names; ``Ensemble`` is a thin convenience
wrapper that owns one context.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librwpt.so")

RWPT_OK, RWPT_EINVAL, RWPT_ENOMEM, RWPT_EDEVICE, RWPT_ESTATE, RWPT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
RWPT_FP32, RWPT_FP64 = 0, 1
RWPT_NORM_SYM, RWPT_NORM_ROW = 0, 1
RWPT_PATH_AUTO, RWPT_PATH_SPARSE, RWPT_PATH_DENSE = 0, 1, 2
RWPT_PROBE_FMA, RWPT_PROBE_EXP, RWPT_PROBE_ROWSUM, RWPT_PROBE_EXCHANGE = 0, 1, 2, 3

STATUS_NAMES = {0: "RWPT_OK", -1: "RWPT_EINVAL", -2: "RWPT_ENOMEM", -3: "RWPT_EDEVICE",
                -4: "RWPT_ESTATE", -5: "RWPT_EUNSUPPORTED"}

# Every symbol include/rwpt.h declares.
EXPORTED = [
    "rwpt_config_default", "rwpt_create", "rwpt_init_ensemble", "rwpt_init_ensemble_device",
    "rwpt_step", "rwpt_sync", "rwpt_stats",
    "rwpt_query_masses", "rwpt_query_positions", "rwpt_audit", "rwpt_steps_taken",
    "rwpt_count_pairs", "rwpt_neighbors", "rwpt_debug_rowsums", "rwpt_profile_enable", "rwpt_profile_reset",
    "rwpt_profile_read", "rwpt_profile_phase_name", "rwpt_probe_rate", "rwpt_get_tiling",
    "rwpt_autotune", "rwpt_transfer_noalloc", "rwpt_last_error", "rwpt_version", "rwpt_destroy",
]


class rwpt_config(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("n_species", ctypes.c_int32),
        ("react_a", ctypes.c_int32),
        ("react_b", ctypes.c_int32),
        ("box_lo", ctypes.c_double * 3),
        ("box_hi", ctypes.c_double * 3),
        ("kappa", ctypes.c_double),
        ("rw_ratio", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("norm", ctypes.c_int32),
        ("path", ctypes.c_int32),
        ("tile_lanes", ctypes.c_int32),
        ("cell_refine", ctypes.c_double * 3),
        ("device", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("stream", ctypes.c_void_p),
        ("velocity", ctypes.c_double * 3),
        ("alpha_l", ctypes.c_double),
        ("alpha_t", ctypes.c_double),
    ]


class rwpt_stats_t(ctypes.Structure):
    _fields_ = [
        ("n_particles", ctypes.c_int64),
        ("n_real", ctypes.c_int32),
        ("tile_lanes", ctypes.c_int32),
        ("cell_refine", ctypes.c_double * 3),
        ("n_cells", ctypes.c_int64),
        ("steps_taken", ctypes.c_int64),
        ("ordered_pairs", ctypes.c_int64),
        ("candidate_evals", ctypes.c_int64),
        ("n_phases", ctypes.c_int32),
        ("graph_captures", ctypes.c_int32),
        ("phase_ms", ctypes.c_double * 16),
        ("phase_launches", ctypes.c_int64 * 16),
    ]


class RwptError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


_lib = None


def load_library(path: str | None = None):
    """Load librwpt.so (raises if it has not been built); ``path`` defaults to
    the module's LIB_PATH at call time."""
    global _lib
    if _lib is not None:
        return _lib
    path = LIB_PATH if path is None else path
    if not os.path.exists(path):
        raise ImportError("librwpt.so is not built (%s); build it with python -m paper_1811_05474_amd._build" % path)
    lib = ctypes.CDLL(path)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pcfg = ctypes.POINTER(rwpt_config)
    sig = {
        "rwpt_config_default": (None, [pcfg]),
        "rwpt_create": (i32, [pcfg, ctypes.POINTER(vp)]),
        "rwpt_init_ensemble": (i32, [vp, i32, vp, vp, vp, vp]),
        "rwpt_init_ensemble_device": (i32, [vp, i32, vp, vp, vp, vp]),
        "rwpt_stats": (i32, [vp, ctypes.POINTER(rwpt_stats_t)]),
        "rwpt_step": (i32, [vp, f64, f64, i32]),
        "rwpt_sync": (i32, [vp]),
        "rwpt_query_masses": (i32, [vp, vp]),
        "rwpt_query_positions": (i32, [vp, vp]),
        "rwpt_audit": (i32, [vp, vp]),
        "rwpt_steps_taken": (i32, [vp, ctypes.POINTER(i64)]),
        "rwpt_count_pairs": (i32, [vp, f64, f64, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "rwpt_neighbors": (i32, [vp, f64, f64, vp, vp, ctypes.POINTER(i64)]),
        "rwpt_debug_rowsums": (i32, [vp, f64, f64, i32, vp]),
        "rwpt_profile_enable": (i32, [vp, i32]),
        "rwpt_profile_reset": (i32, [vp]),
        "rwpt_profile_read": (i32, [vp, vp, vp, ctypes.POINTER(i32)]),
        "rwpt_profile_phase_name": (ctypes.c_char_p, [i32]),
        "rwpt_probe_rate": (i32, [vp, i32, ctypes.POINTER(f64)]),
        "rwpt_get_tiling": (i32, [vp, ctypes.POINTER(i32), vp]),
        "rwpt_autotune": (i32, [vp, f64, f64, i32]),
        "rwpt_transfer_noalloc": (i32, [pcfg, i32, vp, vp, vp, f64, f64]),
        "rwpt_last_error": (ctypes.c_char_p, [vp]),
        "rwpt_version": (ctypes.c_char_p, []),
        "rwpt_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(st: int, ctx=None):
    if st != RWPT_OK:
        msg = load_library().rwpt_last_error(ctx)
        raise RwptError(st, (msg or b"").decode())


# ------------------------------------------------------------ C-named calls --

def rwpt_config_default() -> rwpt_config:
    cfg = rwpt_config()
    load_library().rwpt_config_default(ctypes.byref(cfg))
    return cfg


def rwpt_create(cfg: rwpt_config):
    out = ctypes.c_void_p()
    st = load_library().rwpt_create(ctypes.byref(cfg), ctypes.byref(out))
    _check(st, None)
    return out


def rwpt_init_ensemble(ctx, n_per_real, pos: np.ndarray, mass: np.ndarray, d_scale=None):
    sizes = np.ascontiguousarray(np.asarray(n_per_real, dtype=np.int64).reshape(-1))
    pos = np.ascontiguousarray(np.asarray(pos, dtype=np.float64))
    mass = np.ascontiguousarray(np.asarray(mass, dtype=np.float64))
    ds = None
    if d_scale is not None:
        ds = np.ascontiguousarray(np.asarray(d_scale, dtype=np.float64).reshape(-1))
        assert ds.size == sizes.size
    st = load_library().rwpt_init_ensemble(ctx, int(sizes.size), _p(sizes), _p(pos), _p(mass),
                                           None if ds is None else _p(ds))
    _check(st, ctx)


def rwpt_init_ensemble_device(ctx, n_per_real, pos_dev_ptr: int, mass_dev_ptr: int, d_scale=None):
    """pos_dev_ptr / mass_dev_ptr: device addresses of contiguous binary64
    arrays in the layouts of rwpt_init_ensemble (e.g. ``tensor.data_ptr()``)."""
    sizes = np.ascontiguousarray(np.asarray(n_per_real, dtype=np.int64).reshape(-1))
    ds = None
    if d_scale is not None:
        ds = np.ascontiguousarray(np.asarray(d_scale, dtype=np.float64).reshape(-1))
        assert ds.size == sizes.size
    st = load_library().rwpt_init_ensemble_device(ctx, int(sizes.size), _p(sizes),
                                                  ctypes.c_void_p(pos_dev_ptr), ctypes.c_void_p(mass_dev_ptr),
                                                  None if ds is None else _p(ds))
    _check(st, ctx)


def rwpt_stats(ctx) -> dict:
    st = rwpt_stats_t()
    lib = load_library()
    _check(lib.rwpt_stats(ctx, ctypes.byref(st)), ctx)
    out = {name: getattr(st, name) for name, _ in rwpt_stats_t._fields_ if name not in ("phase_ms", "phase_launches")}
    out["cell_refine"] = tuple(st.cell_refine)
    out["phases"] = {lib.rwpt_profile_phase_name(i).decode(): (float(st.phase_ms[i]), int(st.phase_launches[i]))
                     for i in range(st.n_phases)}
    return out


def rwpt_step(ctx, dt: float, D: float, n_steps: int = 1):
    _check(load_library().rwpt_step(ctx, float(dt), float(D), int(n_steps)), ctx)


def rwpt_sync(ctx):
    _check(load_library().rwpt_sync(ctx), ctx)


def rwpt_query_masses(ctx, n: int, S: int) -> np.ndarray:
    out = np.zeros((S, n), dtype=np.float64)
    _check(load_library().rwpt_query_masses(ctx, _p(out)), ctx)
    return out


def rwpt_query_positions(ctx, n: int, dim: int) -> np.ndarray:
    out = np.zeros((n, dim), dtype=np.float64)
    _check(load_library().rwpt_query_positions(ctx, _p(out)), ctx)
    return out


def rwpt_audit(ctx, n_real: int, S: int) -> np.ndarray:
    out = np.zeros((n_real, S + 1), dtype=np.float64)
    _check(load_library().rwpt_audit(ctx, _p(out)), ctx)
    return out


def rwpt_steps_taken(ctx) -> int:
    v = ctypes.c_int64()
    _check(load_library().rwpt_steps_taken(ctx, ctypes.byref(v)), ctx)
    return int(v.value)


def rwpt_count_pairs(ctx, dt: float, D: float):
    p, e = ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().rwpt_count_pairs(ctx, float(dt), float(D), ctypes.byref(p), ctypes.byref(e)), ctx)
    return int(p.value), int(e.value)


def rwpt_neighbors(ctx, dt: float, D: float, n: int):
    nnz = ctypes.c_int64()
    lib = load_library()
    _check(lib.rwpt_neighbors(ctx, float(dt), float(D), None, None, ctypes.byref(nnz)), ctx)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    cols = np.zeros(max(1, nnz.value), dtype=np.int32)
    _check(lib.rwpt_neighbors(ctx, float(dt), float(D), _p(rowptr), _p(cols), ctypes.byref(nnz)), ctx)
    return rowptr, cols[: nnz.value]


def rwpt_debug_rowsums(ctx, dt: float, D: float, n: int, unit_weights: bool = False) -> np.ndarray:
    out = np.zeros(n, dtype=np.float64)
    _check(load_library().rwpt_debug_rowsums(ctx, float(dt), float(D), 1 if unit_weights else 0, _p(out)), ctx)
    return out


def rwpt_profile_enable(ctx, on: bool):
    _check(load_library().rwpt_profile_enable(ctx, 1 if on else 0), ctx)


def rwpt_profile_reset(ctx):
    _check(load_library().rwpt_profile_reset(ctx), ctx)


def rwpt_profile_read(ctx) -> dict:
    ms = np.zeros(16, dtype=np.float64)
    cnt = np.zeros(16, dtype=np.int64)
    n = ctypes.c_int32()
    lib = load_library()
    _check(lib.rwpt_profile_read(ctx, _p(ms), _p(cnt), ctypes.byref(n)), ctx)
    return {lib.rwpt_profile_phase_name(i).decode(): (float(ms[i]), int(cnt[i])) for i in range(n.value)}


def rwpt_probe_rate(ctx, kind: int) -> float:
    """Attainable rate of one probe kind (lane ops/s or candidate evaluations/s)."""
    v = ctypes.c_double()
    _check(load_library().rwpt_probe_rate(ctx, int(kind), ctypes.byref(v)), ctx)
    return float(v.value)


def rwpt_get_tiling(ctx):
    lanes = ctypes.c_int32()
    ref = np.zeros(3, dtype=np.float64)
    _check(load_library().rwpt_get_tiling(ctx, ctypes.byref(lanes), _p(ref)), ctx)
    return int(lanes.value), tuple(float(v) for v in ref)


def rwpt_autotune(ctx, dt: float, D: float, trial_steps: int = 3):
    _check(load_library().rwpt_autotune(ctx, float(dt), float(D), int(trial_steps)), ctx)


def rwpt_transfer_noalloc(cfg: rwpt_config, n: int, pos_dev_ptr: int, mass_in_dev_ptr: int,
                          mass_out_dev_ptr: int, dt: float, D: float):
    """pos / mass_in / mass_out: device addresses (e.g. ``tensor.data_ptr()``)
    of contiguous arrays in the path's precision: positions n x dim, masses
    S x n.  Queued on cfg.stream; returns without waiting."""
    st = load_library().rwpt_transfer_noalloc(ctypes.byref(cfg), int(n), ctypes.c_void_p(pos_dev_ptr),
                                              ctypes.c_void_p(mass_in_dev_ptr), ctypes.c_void_p(mass_out_dev_ptr),
                                              float(dt), float(D))
    _check(st, None)


def rwpt_last_error(ctx=None) -> str:
    return (load_library().rwpt_last_error(ctx) or b"").decode()


def rwpt_version() -> str:
    return load_library().rwpt_version().decode()


def rwpt_destroy(ctx):
    load_library().rwpt_destroy(ctx)


# ------------------------------------------------------------- convenience --

class Ensemble:
    """One context: ``Ensemble(dim=2, ...)`` then ``init(sizes, pos, mass)``, ``step(dt, D, n)``."""

    def __init__(self, dim=2, n_species=2, react=(0, 1), box_lo=(0.0, 0.0, 0.0), box_hi=(1.0, 1.0, 1.0),
                 kappa=3.0, rw_ratio=1.0, precision=RWPT_FP32, norm=RWPT_NORM_SYM, path=RWPT_PATH_AUTO,
                 tile_lanes=0, cell_refine=(0.0, 0.0, 0.0), device=0, use_graph=1, seed=0, stream=None,
                 velocity=(0.0, 0.0, 0.0), alpha_l=0.0, alpha_t=0.0):
        cfg = rwpt_config_default()
        cfg.dim = dim
        cfg.n_species = n_species
        cfg.react_a, cfg.react_b = (-1, -1) if react is None else react
        for k in range(3):
            cfg.box_lo[k] = box_lo[k] if k < len(box_lo) else 0.0
            cfg.box_hi[k] = box_hi[k] if k < len(box_hi) else 1.0
            cfg.cell_refine[k] = cell_refine[k]
        cfg.kappa = math.inf if kappa is None else float(kappa)
        cfg.rw_ratio = float(rw_ratio)
        cfg.precision = precision
        cfg.norm = norm
        cfg.path = path
        cfg.tile_lanes = tile_lanes
        cfg.device = device
        cfg.use_graph = use_graph
        cfg.seed = seed
        cfg.stream = stream
        for k in range(3):
            cfg.velocity[k] = velocity[k] if k < len(velocity) else 0.0
        cfg.alpha_l = float(alpha_l)
        cfg.alpha_t = float(alpha_t)
        self.cfg = cfg
        self.dim, self.S = dim, n_species
        self.n, self.n_real = 0, 0
        self.ctx = rwpt_create(cfg)

    def init(self, n_per_real, pos, mass, d_scale=None):
        rwpt_init_ensemble(self.ctx, n_per_real, pos, mass, d_scale)
        sizes = np.asarray(n_per_real).reshape(-1)
        self.n, self.n_real = int(sizes.sum()), int(sizes.size)
        return self

    def step(self, dt, D, n=1):
        rwpt_step(self.ctx, dt, D, n)
        return self

    def sync(self):
        rwpt_sync(self.ctx)

    def masses(self):
        return rwpt_query_masses(self.ctx, self.n, self.S)

    def positions(self):
        return rwpt_query_positions(self.ctx, self.n, self.dim)

    def audit(self):
        return rwpt_audit(self.ctx, self.n_real, self.S)

    def steps_taken(self):
        return rwpt_steps_taken(self.ctx)

    def count_pairs(self, dt, D):
        return rwpt_count_pairs(self.ctx, dt, D)

    def stats(self):
        return rwpt_stats(self.ctx)

    def probe_rate(self, kind):
        return rwpt_probe_rate(self.ctx, kind)

    def neighbors(self, dt, D):
        return rwpt_neighbors(self.ctx, dt, D, self.n)

    def rowsums(self, dt, D, unit_weights=False):
        return rwpt_debug_rowsums(self.ctx, dt, D, self.n, unit_weights)

    def close(self):
        if self.ctx:
            rwpt_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
