"""Neighbour sets of the kernels a step actually launches, against the oracle.

The cutoff predicate decides an integer (whether j is a neighbour of i), so the
sets must match the oracle's bit for bit ("within" s_max, Sec. 2.1).  Two
views of the step's own pair kernels are checked:

* rwpt_neighbors enumerates the candidates through the same templates the
  step's pair kernels use for the tiling in use (the chunked candidate rows of
  the binary32 four-lane tiles, whole tiles or one block per tile; the own
  cutoff-box walk of the one-lane-per-particle row sum), with the same
  predicate arithmetic: the exported CSR must equal the oracle's;
* rwpt_debug_rowsums runs the step's real row-sum kernel in its launch shape
  with every weight replaced by exp(0) = 1: r_i must equal |N(i)| exactly.

Positions are the seeded inputs (never taken from the GPU).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1811_05474_amd import rwpt, workloads as W

pytestmark = pytest.mark.gpu

F32 = rwpt.RWPT_FP32
F64 = rwpt.RWPT_FP64


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def ensemble(dim, prec, lanes, S=2, seed=1):
    return rwpt.Ensemble(dim=dim, n_species=S, react=(0, 1), kappa=3.0, rw_ratio=0.0, precision=prec,
                         tile_lanes=lanes, seed=seed)


def D_for_neighbours(dim, n, mean_nb, dt=0.1):
    """D whose cutoff 3 sqrt(8 D dt) holds about mean_nb neighbours in the unit box."""
    unit = {1: 2.0, 2: math.pi, 3: 4.0 * math.pi / 3.0}[dim]
    rc = (mean_nb / ((n - 1) * unit)) ** (1.0 / dim)
    return rc * rc / (72.0 * dt)


# (dim, n, lanes, mean neighbours): the four-lane row-broadcast tiles with one
# block per tile (<= 4096 tiles of 16) and with whole tiles per wave; one lane
# per particle with every lane cached (few neighbours) and most lanes beyond
# the per-lane cache (many); the vector-load tiles.  Sparse four-lane whole
# tiles: most segments end in a short chunk of at most 16 or 32 candidates,
# evaluated in 4 or 8 broadcast steps
CASES = [
    (1, 32768, 4, 60.0), (1, 80000, 4, 60.0),
    (1, 80000, 4, 4.0), (2, 80000, 4, 3.0), (2, 80000, 4, 12.0),
    (2, 40000, 4, 200.0), (2, 120000, 4, 200.0),
    (3, 40000, 4, 30.0), (3, 80000, 4, 30.0),
    (1, 30000, -1, 3.0), (2, 30000, -1, 2.5), (2, 30000, -1, 12.0),
    (3, 50000, -1, 0.7), (3, 50000, -1, 12.0),
    (2, 30000, 8, 100.0), (3, 30000, 16, 20.0),
]


@pytest.mark.parametrize("prec", [F32, F64])
@pytest.mark.parametrize("dim,n,lanes,mean_nb", CASES)
def test_hot_kernel_neighbour_sets_bit_exact(dim, n, lanes, mean_nb, prec):
    dt = 0.1
    D = D_for_neighbours(dim, n, mean_nb, dt)
    x = f32(W.positions(n, dim, 600 + n % 97 + dim))
    M = W.masses(n, 2, 600 + dim)
    p = 32 if prec == F32 else 64
    ens = ensemble(dim, prec, lanes)
    ens.init([n], x, M)
    rp0, cols0 = oracle.neighbors(x, 3.0, D, dt, p)
    rp, cols = ens.neighbors(dt, D)
    same = np.array_equal(rp, rp0) and np.array_equal(cols, cols0)
    counts = ens.rowsums(dt, D, unit_weights=True)
    bad = np.flatnonzero(counts != np.diff(rp0))
    pairs, evals = ens.count_pairs(dt, D)
    ntiles = -(-n // (64 if lanes in (-1, 1) else 64 // abs(lanes)))
    print("dim %d n %d lanes %d (%d tiles) prec %d: %.1f neighbours/particle, %d candidate evaluations "
          "for %d entries; CSR equal %s; unit-weight row sums off in %d rows"
          % (dim, n, lanes, ntiles, p, rp0[-1] / n, evals, rp0[-1], same, bad.size))
    assert same
    assert bad.size == 0, bad[:10]
    assert pairs == rp0[-1] - n and evals >= rp0[-1]
    # the real row sums against the oracle's r_i = sum_j w_ij (FP64 weights)
    _, r0 = oracle.transfer(x, M, D, dt, kappa=3.0, prec=p, return_r=True)
    r = ens.rowsums(dt, D)
    rel = np.abs(r - r0).max() / np.abs(r0).max()
    print("row sums: max relative difference %.2e" % rel)
    assert rel < (1e-5 if prec == F32 else 1e-13)
    ens.close()


def test_split_and_whole_tile_forms_are_both_exercised():
    # one block per tile up to 4096 tiles of 16 particles, one wave per tile beyond
    assert -(-40000 // 16) <= 4096 < -(-120000 // 16)
    assert -(-32768 // 16) <= 4096 < -(-80000 // 16)


@pytest.mark.parametrize("name,rows_n", [("walk2d_n1e6", 3000), ("walk3d_n8e6_s8", 3000)])
def test_full_size_launch_shape_neighbour_sets(name, rows_n):
    """The 10^6-particle 2-D case (four-lane tiles, one wave per tile, 62 500
    tiles) and the 8e6-particle 3-D case (one lane per particle) in the launch
    shape the benchmark times: unit-weight row sums of the real row-sum kernel
    and exported rows of sampled particles against the oracle's rows, plus the
    total pair count from both views."""
    w = W.WORKLOADS[name]
    x, M, sizes, _ = W.make_inputs(w)
    x = f32(x)
    ens = rwpt.Ensemble(dim=w.dim, n_species=w.n_species, react=w.react, kappa=w.kappa, rw_ratio=w.rw_ratio,
                        precision=F32, seed=w.seed)
    ens.init(sizes, x, M)
    counts = ens.rowsums(w.dt, w.D, unit_weights=True)
    assert ens.stats()["tile_lanes"] == (4 if w.dim == 2 else -1)
    rows = np.random.default_rng(11).choice(w.n, rows_n, replace=False)
    rp0, cols0 = oracle.neighbors(x, w.kappa, w.D, w.dt, 32, rows=rows)
    assert np.array_equal(counts[rows], np.diff(rp0).astype(np.float64))
    pairs, evals = ens.count_pairs(w.dt, w.D)
    assert counts.sum() == pairs + w.n
    rp, cols = ens.neighbors(w.dt, w.D)
    assert rp[-1] == pairs + w.n
    for t, i in enumerate(rows):
        assert np.array_equal(cols[rp[i]:rp[i + 1]], cols0[rp0[t]:rp0[t + 1]]), i
    print("%s: %d ordered pairs, %.1f candidate evaluations per neighbour entry"
          % (name, pairs, evals / (pairs + w.n)))
    ens.close()
