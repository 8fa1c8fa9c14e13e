"""The half-stencil tiling (tile_lanes = -2): every unordered pair evaluated
once and its share delivered to both ends (the paper's Sec. 6.1 remark that
the looping scheme does about half as many operations), against the oracle.

* unit-weight row sums through the tiling's own passes equal |N(i)| exactly,
  so no pair is dropped or counted twice ("within" s_max, Sec. 2.1);
* masses after one and several steps against the oracle at the binary32 bar
  (symmetric and row normalisation, with and without the reaction);
* bitwise reproducible: the same bits from replayed graphs and eager launches.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1811_05474_amd import rwpt, workloads as W

import _oracle_steps as OS

pytestmark = pytest.mark.gpu

F32 = rwpt.RWPT_FP32
HALF = -2


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def D_for(dim, n, mean_nb, dt=0.1, box=1.0):
    unit = {1: 2.0, 2: math.pi, 3: 4.0 * math.pi / 3.0}[dim]
    rc = box * (mean_nb / ((n - 1) * unit)) ** (1.0 / dim)
    return rc * rc / (72.0 * dt)


def check_err(got, ref, bar, label=""):
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("normwise error %.3e (bar %.0e) %s" % (err, bar, label))
    assert err < bar, (err, label)


def make(dim, S=2, react=(0, 1), rw=0.0, norm=rwpt.RWPT_NORM_SYM, seed=1, graph=1, refine=(0, 0, 0), lanes=HALF):
    return rwpt.Ensemble(dim=dim, n_species=S, react=react, kappa=3.0, rw_ratio=rw, precision=F32, norm=norm,
                         tile_lanes=lanes, seed=seed, use_graph=graph, cell_refine=refine)


@pytest.mark.parametrize("dim,n,mean_nb", [(1, 20000, 40.0), (2, 30000, 3.0), (2, 30000, 60.0), (2, 60000, 225.0),
                                          (3, 40000, 1.5), (3, 40000, 30.0)])
def test_half_stencil_row_sums_count_every_neighbour_once(dim, n, mean_nb):
    dt = 0.1
    D = D_for(dim, n, mean_nb, dt)
    x = f32(W.positions(n, dim, 900 + dim))
    M = W.masses(n, 2, 900 + dim)
    ens = make(dim)
    ens.init([n], x, M)
    counts = ens.rowsums(dt, D, unit_weights=True)
    rp0, _ = oracle.neighbors(x, 3.0, D, dt, 32)
    bad = np.flatnonzero(counts != np.diff(rp0))
    print("dim %d n %d: %.1f neighbours per particle, row sums off in %d rows" % (dim, n, rp0[-1] / n, bad.size))
    assert ens.stats()["tile_lanes"] == HALF
    assert bad.size == 0, (bad[:8], counts[bad[:8]], np.diff(rp0)[bad[:8]])
    _, r0 = oracle.transfer(x, M, D, dt, kappa=3.0, prec=32, return_r=True)
    rel = np.abs(ens.rowsums(dt, D) - r0).max() / r0.max()
    print("row sums: max relative difference %.2e" % rel)
    assert rel < 1e-5
    ens.close()


@pytest.mark.parametrize("norm", [rwpt.RWPT_NORM_SYM, rwpt.RWPT_NORM_ROW])
@pytest.mark.parametrize("dim,n,mean_nb,S", [(1, 20000, 40.0, 2), (2, 40000, 100.0, 2), (2, 30000, 8.0, 3),
                                             (3, 40000, 20.0, 8)])
def test_half_stencil_transfer_matches_oracle(dim, n, mean_nb, S, norm):
    dt = 0.1
    D = D_for(dim, n, mean_nb, dt)
    x = f32(W.positions(n, dim, 910 + dim))
    M = f32(W.masses(n, S, 910 + dim))
    ens = make(dim, S=S, norm=norm)
    ens.init([n], x, M)
    onorm = oracle.NORM_SYM if norm == rwpt.RWPT_NORM_SYM else oracle.NORM_ROW
    ref = M
    for step in range(3):
        ens.step(dt, D, 1)
        ref = oracle.transfer(x, ref, D, dt, kappa=3.0, prec=32, norm=onorm)
        check_err(ens.masses(), ref, 1e-5, "step %d" % step)
    if norm == rwpt.RWPT_NORM_SYM:
        a0, a1 = oracle.audit(M), ens.audit()[0]
        drift = abs(a1[S] - a0[S]) / (a0[0] + a0[1])
        print("sum(A - B) drift %.2e" % drift)
        assert drift < 1e-6
    ens.close()


def test_half_stencil_with_the_walk_against_the_oracle_trajectory():
    n, D, dt, seed = 30000, 2e-4, 0.1, 99
    x = f32(W.positions(n, 2, seed))
    M = f32(W.masses(n, 2, seed))
    ens = make(2, rw=1.0, seed=seed)
    ens.init([n], x, M)
    u = float(np.spacing(np.float32(1.0)))
    bar = 1e-5 + 0.3 * 2.0 * 3.0 * 2.0 * u / math.sqrt(8.0 * D * dt)
    for step, (xr, mr) in enumerate(OS.steps(x, M, 3, D, dt, seed, (0, 0), (1, 1), True)):
        ens.step(dt, D, 1)
        assert np.abs(ens.positions() - xr).max() <= 2 * u
        check_err(ens.masses(), mr, bar, "walked step %d" % step)
    ens.close()


def test_half_stencil_batch_with_empty_single_and_uneven_realisations():
    sizes = [0, 1, 37, 0, 5000, 1, 20000, 300]
    scale = [1.0, 1.0, 1.0, 1.0, 0.25, 1.0, 1.0, 4.0]
    n = sum(sizes)
    x = f32(W.positions(n, 2, 8))
    M = f32(W.masses(n, 2, 8))
    D, dt = 2e-4, 0.1
    ens = make(2)
    ens.init(sizes, x, M, d_scale=scale)
    ens.step(dt, D, 2)
    got = ens.masses()
    off = np.concatenate([[0], np.cumsum(sizes)])
    for r, sz in enumerate(sizes):
        if sz == 0:
            continue
        b, e = off[r], off[r + 1]
        ref = M[:, b:e]
        for _ in range(2):
            ref = oracle.transfer(x[b:e], ref, D * scale[r], dt, kappa=3.0, prec=32)
        check_err(got[:, b:e], ref, 1e-5, "realisation %d (%d particles)" % (r, sz))
    ens.close()


def test_half_stencil_bitwise_reproducible_graph_and_eager():
    n, D, dt = 30000, 2e-4, 0.1
    x = W.positions(n, 2, 17)
    M = W.masses(n, 2, 17)
    outs = []
    for graph in (1, 0, 1):
        e = make(2, rw=1.0, seed=3, graph=graph)
        e.init([n], x, M)
        e.step(dt, D, 6)
        outs.append((e.masses(), e.positions(), e.audit()))
        e.close()
    for o in outs[1:]:
        assert np.array_equal(outs[0][0], o[0]) and np.array_equal(outs[0][1], o[1])
        assert np.array_equal(outs[0][2], o[2])


@pytest.mark.parametrize("refine", [(16.0, 2.0, 0.0), (8.0, 1.0, 0.0), (32.0, 4.0, 0.0)])
def test_half_stencil_full_size_on_identical_positions(refine):
    """The 10^6-particle 2-D workload with the walk off, two steps, sampled
    particles against the oracle, for cell grids of several refinements."""
    w = W.WORKLOADS["walk2d_n1e6"]
    x, M, sizes, _ = W.make_inputs(w)
    x, M = f32(x), f32(M)
    ens = make(2, rw=0.0, seed=w.seed, refine=refine)
    ens.init(sizes, x, M)
    rows = np.random.default_rng(23).choice(w.n, 3000, replace=False)
    ens.step(w.dt, w.D, 1)
    m1 = oracle.transfer(x, M, w.D, w.dt, kappa=3.0, prec=32)
    check_err(ens.masses()[:, rows], m1[:, rows], 1e-5, "step 1, refine %s" % (refine,))
    ens.step(w.dt, w.D, 1)
    m2 = oracle.transfer(x, m1, w.D, w.dt, kappa=3.0, prec=32, rows=rows)
    check_err(ens.masses()[:, rows], m2, 1e-5, "step 2")
    counts = ens.rowsums(w.dt, w.D, unit_weights=True)
    rp0, _ = oracle.neighbors(x, 3.0, w.D, w.dt, 32, rows=rows)
    assert np.array_equal(counts[rows], np.diff(rp0).astype(np.float64))
    ens.close()
