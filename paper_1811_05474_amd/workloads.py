"""Seeded synthetic workloads shaped like the paper's test problems.

This module only draws random inputs (positions, masses, ensemble sizes) and
names the workload shapes; it holds none of the mass-transfer arithmetic, so
both the GPU path and the CPU oracle may be fed from it.

Shapes follow the paper's own synthetic setups: particles placed uniformly at
random in a box with reflecting walls (Sec. 3), two reacting species A and B
(Sec. 3), fixed time step dt = 0.1 (Sec. 3), 1-D and 2-D domains (Sec. 3,
Sec. 5.1) and a 10^6-particle ensemble (Sec. 6.2).  Masses are
(1/N)(1 + 0.1 xi) with xi ~ N(0, 1) independent per particle and species.
Random numbers come from NumPy's PCG64 (``numpy.random.default_rng``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    dim: int
    n: int                 # particles per realisation (single-realisation workloads)
    n_species: int
    D: float               # mass-transfer diffusion coefficient (D_m of Eq. 3)
    dt: float
    steps: int
    kappa: float           # cutoff in units of sigma = sqrt(8 D dt); inf = full matrix
    rw_ratio: float        # random-walk diffusion D_rw = rw_ratio * D (0 = fixed positions)
    seed: int
    react: tuple = (0, 1)
    box_lo: tuple = (0.0, 0.0, 0.0)
    box_hi: tuple = (1.0, 1.0, 1.0)
    n_real: int = 1
    D_choices: tuple = field(default_factory=tuple)
    init: str = "uniform"  # "uniform" masses, or the segregated "interface" of Sec. 3
    x0: float | None = None  # interface position (default: the middle of the box)
    velocity: tuple = (0.0, 0.0, 0.0)  # constant velocity of the walk (Eq. 1)
    alpha_l: float = 0.0   # longitudinal dispersivity
    alpha_t: float = 0.0   # transverse dispersivity


WORKLOADS = {
    # 1-D, full matrix, fixed positions, FP64 -- small enough for the oracle
    "plain1d_n2000": Workload("plain1d_n2000", 1, 2000, 2, 1e-4, 0.1, 100, math.inf, 0.0, 1000),
    # 1-D, N = 32768: dense full-matrix and sparse kappa = 3 paths
    "plain1d_n32768": Workload("plain1d_n32768", 1, 32768, 2, 1e-4, 0.1, 500, 3.0, 0.0, 2000),
    # the same particles with every pair interacting (full matrix, no cutoff)
    "full1d_n32768": Workload("full1d_n32768", 1, 32768, 2, 1e-4, 0.1, 500, math.inf, 0.0, 2000),
    # 2-D, N = 10^6 in the unit square, kappa = 3, random walk between transfers
    "walk2d_n1e6": Workload("walk2d_n1e6", 2, 1_000_000, 2, 1e-5, 0.1, 200, 3.0, 1.0, 3000),
    # 64 independent 2-D realisations, N log-uniform in [1e4, 2e5], D in {1e-5, 1e-4}
    "batch2d_64": Workload("batch2d_64", 2, 0, 2, 1e-5, 0.1, 100, 3.0, 1.0, 4000, n_real=64,
                           D_choices=(1e-5, 1e-4)),
    # 3-D, N = 8e6, eight species, reaction on the first pair
    "walk3d_n8e6_s8": Workload("walk3d_n8e6_s8", 3, 8_000_000, 8, 1e-6, 0.1, 50, 3.0, 1.0, 5000),
    # the paper's verification problem (Sec. 3): segregated interface on
    # [0, 50], total D = 1 split equally between transfer and walk, t = 10;
    # species are the conservative components C1, C2 (no reaction term)
    "interface1d_l50": Workload("interface1d_l50", 1, 2000, 2, 0.5, 0.1, 100, 3.0, 1.0, 6000,
                                react=None, box_hi=(50.0, 1.0, 1.0), n_real=75, init="interface"),
    # the 2-D verification problem: 80 x 80 box, interface at x = 40
    "interface2d_l80": Workload("interface2d_l80", 2, 20000, 2, 0.5, 0.1, 100, 3.0, 1.0, 9000,
                                react=None, box_hi=(80.0, 80.0, 1.0), n_real=8, init="interface"),
    # the same interface at x0 = 10 advected with v = 1 and longitudinal
    # dispersivity 1 (Eq. 2 plus the transfer): the front reaches x = 20 at t = 10
    "advect1d_l50": Workload("advect1d_l50", 1, 2000, 2, 0.5, 0.1, 100, 3.0, 1.0, 8000,
                             react=None, box_hi=(50.0, 1.0, 1.0), n_real=75, init="interface", x0=10.0,
                             velocity=(1.0, 0.0, 0.0), alpha_l=1.0),
}


def interface(n: int, dim: int, L, seed: int, x0: float | None = None):
    """Segregated initial condition of the paper's test problem (Sec. 3, 5.1):
    uniform positions in [0, L]^dim; C1 = 1 for x > x0 (0 below; x0 = L/2 by
    default), C2 the complement; masses are concentration times the particle
    volume ds = |box| / n.  Returns positions (n, dim) and masses (2, n)."""
    L = np.broadcast_to(np.asarray(L, dtype=np.float64), (dim,))
    x = positions(n, dim, seed, (0.0,) * dim, tuple(L))
    ds = float(np.prod(L)) / n
    right = x[:, 0] > (0.5 * L[0] if x0 is None else float(x0))
    M = np.stack([right * ds, (~right) * ds]).astype(np.float64)
    return x, M


def positions(n: int, dim: int, seed: int, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)) -> np.ndarray:
    """(n, dim) float64 positions, i.i.d. uniform in the box."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo[:dim], dtype=np.float64)
    hi = np.asarray(hi[:dim], dtype=np.float64)
    u = rng.random((n, dim))
    return lo + (hi - lo) * u


def masses(n: int, n_species: int, seed: int) -> np.ndarray:
    """(S, n) float64 masses (1/N)(1 + 0.1 xi), xi ~ N(0,1)."""
    rng = np.random.default_rng(seed + 7919)
    xi = rng.standard_normal((n_species, n))
    return (1.0 + 0.1 * xi) / float(max(n, 1))


def batch_sizes(n_real: int, seed: int, lo: float = 1e4, hi: float = 2e5) -> np.ndarray:
    """Realisation sizes drawn log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed + 104729)
    u = rng.random(n_real)
    return np.rint(np.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * u)).astype(np.int64)


def make_inputs(w: Workload, n: int | None = None):
    """Positions (N, dim), masses (S, N), per-realisation sizes and D values.

    ``n`` overrides the particle count of a single-realisation workload (for
    scaled-down parity cases).  Realisation r of an "interface" workload is
    drawn with seed w.seed + r."""
    if w.init == "interface":
        n = w.n if n is None else int(n)
        parts = [interface(n, w.dim, w.box_hi[:w.dim], w.seed + r, x0=w.x0) for r in range(w.n_real)]
        return (np.concatenate([p[0] for p in parts], 0), np.concatenate([p[1] for p in parts], 1),
                np.full(w.n_real, n, dtype=np.int64), np.full(w.n_real, w.D))
    if w.n_real == 1:
        n = w.n if n is None else int(n)
        x = positions(n, w.dim, w.seed, w.box_lo, w.box_hi)
        M = masses(n, w.n_species, w.seed)
        return x, M, np.array([n], dtype=np.int64), np.array([w.D])
    sizes = batch_sizes(w.n_real, w.seed)
    if n is not None:  # scale the whole batch down, keeping the size mix
        sizes = np.maximum(1, np.rint(sizes * (float(n) / sizes.sum()))).astype(np.int64)
    xs, Ms = [], []
    for r, nr in enumerate(sizes):
        xs.append(positions(int(nr), w.dim, w.seed + r, w.box_lo, w.box_hi))
        Ms.append(masses(int(nr), w.n_species, w.seed + r))
    D = np.array([w.D_choices[r % len(w.D_choices)] for r in range(w.n_real)], dtype=np.float64)
    return np.concatenate(xs, 0), np.concatenate(Ms, 1), sizes, D
