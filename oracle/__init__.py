"""CPU oracle for the particle mass-transfer step (arXiv:1811.05474).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark import this package.  The product library never
imports, links or executes anything here, and this package never imports the
product package.

Two independent implementations live here:

* ``rwpt_oracle.c`` (loaded through ctypes): FP64 random walk, neighbour lists
  and the explicit mass transfer + reaction of Eqs. (3)-(6) of the paper, with
  a full-matrix mode (Sec. 1.1 "brute force") and a cutoff mode (Sec. 2,
  s_max = kappa*sigma).
* ``numpy_ref.py``: a dense NumPy brute force for small N, written separately
  from the C file, used to cross-check it.

Every function cites the passage of the paper it follows; the readings taken
where the paper is ambiguous are listed in the header of ``rwpt_oracle.c``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rwpt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

NORM_SYM = 0
NORM_ROW = 1

GCC_FLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-std=c99", "-Wall", "-Wno-unused-function"]


def build(force: bool = False) -> str:
    """Compile ``rwpt_oracle.c`` into ``liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build()
        lib = ctypes.CDLL(_LIB)
        i64, i32, u64, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_double
        vp = ctypes.c_void_p
        lib.orc_philox4x32_10.argtypes = [vp, vp, vp]
        lib.orc_philox4x32_10.restype = None
        lib.orc_normals.argtypes = [ctypes.c_uint32, u64, u64, vp]
        lib.orc_normals.restype = None
        lib.orc_walk.argtypes = [i64, i32, vp, vp, u64, u64, f64, f64, vp, vp]
        lib.orc_walk.restype = i32
        lib.orc_walk_adv.argtypes = [i64, i32, vp, vp, u64, u64, f64, f64, vp, vp, vp, f64, f64]
        lib.orc_walk_adv.restype = i32
        lib.orc_neighbors.argtypes = [i64, i32, vp, f64, f64, f64, i32, vp, vp, i64]
        lib.orc_neighbors.restype = i64
        lib.orc_neighbors_rows.argtypes = [i64, i32, vp, f64, f64, f64, i32, vp, i64, vp, vp, i64]
        lib.orc_neighbors_rows.restype = i64
        lib.orc_transfer_rows.argtypes = [i64, i32, i32, vp, vp, vp, f64, f64, f64, i32, i32, i32,
                                          i32, vp, i64, vp]
        lib.orc_transfer_rows.restype = i32
        lib.orc_num_threads.argtypes = []
        lib.orc_num_threads.restype = i32
        lib.orc_set_num_threads.argtypes = [i32]
        lib.orc_set_num_threads.restype = None
        _lib = lib
        return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(t: int) -> None:
    _load().orc_set_num_threads(int(t))


def philox4x32_10(counter, key) -> np.ndarray:
    """Philox4x32-10 of Salmon et al. (SC'11) on one 128-bit counter."""
    c = np.ascontiguousarray(np.asarray(counter, dtype=np.uint32).reshape(4))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def normals(pid: int, seed: int, step: int) -> np.ndarray:
    """The three standard normals the walk of particle ``pid`` draws at ``step``."""
    z = np.zeros(3, dtype=np.float64)
    _load().orc_normals(ctypes.c_uint32(pid), ctypes.c_uint64(seed), ctypes.c_uint64(step), _ptr(z))
    return z


def walk(x: np.ndarray, ids: np.ndarray, seed: int, step: int, D_rw: float, dt: float,
         lo, hi, velocity=None, alpha_l: float = 0.0, alpha_t: float = 0.0) -> np.ndarray:
    """Random-walk move of Eq. (1)/(2) with reflecting walls (Sec. 3).

    Without ``velocity`` the move is pure diffusion with D_rw; with a constant
    velocity v it adds the drift v dt and the hydrodynamic dispersion of
    Eq. (1) with dispersivities alpha_l >= alpha_t >= 0.  ``x`` is (n, d)
    float64; returns a new array."""
    x = np.ascontiguousarray(np.array(x, dtype=np.float64, copy=True))
    n, d = x.shape
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32))
    lo = np.ascontiguousarray(np.asarray(lo, dtype=np.float64).reshape(-1)[:d])
    hi = np.ascontiguousarray(np.asarray(hi, dtype=np.float64).reshape(-1)[:d])
    if velocity is not None:
        vel = np.zeros(3, dtype=np.float64)
        v = np.asarray(velocity, dtype=np.float64).reshape(-1)[:d]
        vel[:v.size] = v
        rc = _load().orc_walk_adv(n, d, _ptr(x), _ptr(ids), ctypes.c_uint64(seed), ctypes.c_uint64(step),
                                  float(D_rw), float(dt), _ptr(lo), _ptr(hi), _ptr(vel), float(alpha_l),
                                  float(alpha_t))
        if rc != 0:
            raise ValueError("orc_walk_adv failed (%d)" % rc)
        return x
    rc = _load().orc_walk(n, d, _ptr(x), _ptr(ids), ctypes.c_uint64(seed), ctypes.c_uint64(step),
                          float(D_rw), float(dt), _ptr(lo), _ptr(hi))
    if rc != 0:
        raise ValueError("orc_walk failed (%d)" % rc)
    return x


def neighbors(x: np.ndarray, kappa: float, D: float, dt: float, prec: int = 32, rows=None):
    """Neighbour lists within s_max = kappa*sqrt(8 D dt) (Sec. 2.1/2.2), j = i included.

    Returns (rowptr int64[m+1], cols int32[nnz]) with ascending columns, for
    every particle (m = n) or, with ``rows``, for those particles in that
    order (m = len(rows))."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    n, d = x.shape
    lib = _load()
    if rows is not None:
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64).reshape(-1))
        rows_p, m = _ptr(rows), rows.size
    else:
        rows_p, m = None, n
    args = (n, d, _ptr(x), float(kappa), float(D), float(dt), int(prec), rows_p, m if rows is not None else 0)
    total = lib.orc_neighbors_rows(*args, None, None, -1)
    if total < 0:
        raise ValueError("orc_neighbors failed (%d)" % total)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    cols = np.zeros(max(int(total), 1), dtype=np.int32)
    got = lib.orc_neighbors_rows(*args, _ptr(rowptr), _ptr(cols), int(total))
    assert got == total
    return rowptr, cols[:total]


def transfer(x: np.ndarray, M: np.ndarray, D: float, dt: float, kappa: float = 3.0,
             norm: int = NORM_SYM, prec: int = 64, react=(0, 1), rows=None, return_r=False):
    """One explicit mass-transfer step (Eqs. 3-6) followed by the A+B reaction.

    x: (n, d) positions exactly as the path stores them; M: (S, n) masses.
    kappa = inf gives the full-matrix brute force of Sec. 1.1.  ``prec`` is the
    precision of the cutoff predicate only (the weights are always FP64).
    ``rows`` restricts the output to a subset of particles (all row sums are
    still computed, which the symmetric normalisation needs)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    M = np.ascontiguousarray(np.asarray(M, dtype=np.float64))
    n, d = x.shape
    S = M.shape[0]
    assert M.shape == (S, n)
    ra, rb = (-1, -1) if react is None else react
    if rows is not None:
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64).reshape(-1))
        out = np.zeros((S, rows.size), dtype=np.float64)
        rows_p, nrows = _ptr(rows), rows.size
    else:
        out = np.zeros((S, n), dtype=np.float64)
        rows_p, nrows = None, 0
    r = np.zeros(max(n, 1), dtype=np.float64)
    rc = _load().orc_transfer_rows(n, d, S, _ptr(x), _ptr(M), _ptr(out), float(D), float(dt),
                                   float(kappa), int(norm), int(prec), int(ra), int(rb), rows_p,
                                   nrows, _ptr(r))
    if rc != 0:
        raise ValueError("orc_transfer failed (%d)" % rc)
    if return_r:
        return out, r[:n]
    return out


def audit(M: np.ndarray, react=(0, 1)):
    """Exactly rounded sums: [sum M_0, ..., sum M_{S-1}, sum(M_a - M_b)] (conservation, Sec. 6)."""
    M = np.asarray(M, dtype=np.float64)
    sums = [math.fsum(M[s].tolist()) for s in range(M.shape[0])]
    if react is not None and react[0] >= 0:
        a, b = react
        sums.append(math.fsum(M[a].tolist() + (-M[b]).tolist()))
    else:
        sums.append(0.0)
    return np.array(sums)
