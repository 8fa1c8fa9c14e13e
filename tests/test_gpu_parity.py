"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (normwise, max |dM| / max |M|):
  * FP64 path vs oracle: 1e-12 per compared state;
  * FP32 path vs oracle: 1e-5 (weights computed from binary32 positions with
    the hardware exp2, binary32 exchanges flushed into binary64 row partials);
  * neighbour lists: bit-exact (same binary32 / binary64 predicate);
  * conservation: FP64 path |d sum(A-B)| / sum(A+B) <= 1e-12, FP32 path <= 1e-6.
Steps with the walk are compared with the oracle's own trajectory (its walk,
then its transfer, from its own previous state; tests/_oracle_steps.py): no
oracle input comes from the GPU.  Positions agree within 2e-6 in the unit box
(binary32 Box-Muller vs binary64, one binary32 ulp per move), and the masses
within the bars above plus the effect of that ulp on the weights (walk_tol).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1811_05474_amd import rwpt, workloads as W

import _oracle_steps as OS

pytestmark = pytest.mark.gpu

F32 = rwpt.RWPT_FP32
F64 = rwpt.RWPT_FP64


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def walk_tol(prec, D, dt, xmax=1.0, kappa=3.0):
    """Normwise bar for a step that includes the walk, against the oracle's own
    walk: the GPU and the oracle may place a particle one or two ulps apart
    (u = ulp(xmax) in the path's precision), which changes a weight by up to
    2 kappa u / sigma relative (sigma^2 = 8 D dt); an exchanged mass difference
    is at most ~0.3 of the largest mass.  Added to the bar of the same step on
    identical positions (1e-5 binary32, 1e-12 binary64)."""
    u = float(np.spacing(np.float32(xmax))) if prec == F32 else float(np.spacing(np.float64(xmax)))
    sigma = math.sqrt(8.0 * D * dt)
    return (1e-5 if prec == F32 else 1e-12) + 0.3 * 2.0 * kappa * 2.0 * u / sigma


def exact_sums(m, react=(0, 1)):
    """Exactly rounded totals of a mass array: what the binary64 audit of those
    masses must give (a property of the audit, not an oracle result)."""
    sums = [math.fsum(m[s].tolist()) for s in range(m.shape[0])]
    a, b = react
    sums.append(math.fsum(m[a].tolist() + (-m[b]).tolist()))
    return sums


def normerr(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def check_pos(pos, ref, prec, xmax=1.0, ulps=2.0):
    """Walked positions against the oracle's walk: within `ulps` units in the
    last place of the largest coordinate (the premise of walk_tol)."""
    u = float(np.spacing(np.float32(xmax))) if prec == F32 else float(np.spacing(np.float64(xmax)))
    d = float(np.abs(pos - ref).max())
    print("max position difference %.3e = %.2f ulp of %g" % (d, d / u, xmax))
    assert d <= ulps * u, (d, d / u)


def check_err(got, ref, bar, label=None):
    """Normwise error max |got - ref| / max |ref| against its bar, printed so
    that the margin under the bar is visible in the test log."""
    err = normerr(got, ref)
    print("normwise error %.3e (bar %.3e, margin %.1fx)%s"
          % (err, bar, bar / max(err, 1e-300), "" if label is None else " [%s]" % (label,)))
    assert err < bar, (err, bar, label)
    return err


def make(dim=2, S=2, react=(0, 1), kappa=3.0, rw=0.0, prec=F32, norm=rwpt.RWPT_NORM_SYM, lanes=0,
         refine=(0, 0, 0), graph=1, seed=1, box_lo=(0, 0, 0), box_hi=(1, 1, 1)):
    return rwpt.Ensemble(dim=dim, n_species=S, react=react, kappa=kappa, rw_ratio=rw, precision=prec,
                         norm=norm, tile_lanes=lanes, cell_refine=refine, use_graph=graph, seed=seed,
                         box_lo=box_lo, box_hi=box_hi)


def oracle_run(x, M, D, dt, steps, kappa, prec, norm=oracle.NORM_SYM, react=(0, 1)):
    for _ in range(steps):
        M = oracle.transfer(x, M, D, dt, kappa=kappa, prec=prec, norm=norm, react=react)
    return M


# ------------------------------------------------------------------ c1 ----

@pytest.mark.parametrize("prec,kappa,tol", [(F64, math.inf, 1e-12), (F32, math.inf, 1e-5),
                                            (F64, 3.0, 1e-12), (F32, 3.0, 1e-5)])
def test_plain1d_n2000_full_run(prec, kappa, tol):
    w = W.WORKLOADS["plain1d_n2000"]
    x, M, sizes, _ = W.make_inputs(w)
    if prec == F32:
        x, M = f32(x), f32(M)
    ens = make(dim=1, kappa=kappa, prec=prec, seed=w.seed)
    ens.init(sizes, x, M)
    ens.step(w.dt, w.D, w.steps)
    got = ens.masses()
    pos = ens.positions()
    assert np.array_equal(pos, x)  # no walk: positions never move
    ref = oracle_run(x, M, w.D, w.dt, w.steps, kappa, 64 if prec == F64 else 32)
    check_err(got, ref, tol)
    a = ens.audit()[0]
    a0 = oracle.audit(M)
    cons_tol = 1e-12 if prec == F64 else 1e-6
    assert abs(a[2] - a0[2]) / (a0[0] + a0[1]) < cons_tol
    ens.close()


@pytest.mark.parametrize("prec,tol,lanes", [(F64, 1e-12, 0), (F32, 1e-5, 4), (F32, 1e-5, 1)])
def test_plain1d_n2000_row_normalisation(prec, tol, lanes):
    w = W.WORKLOADS["plain1d_n2000"]
    x, M, sizes, _ = W.make_inputs(w)
    if prec == F32:
        x, M = f32(x), f32(M)
    ens = make(dim=1, kappa=3.0, prec=prec, norm=rwpt.RWPT_NORM_ROW, lanes=lanes)
    ens.init(sizes, x, M)
    ens.step(w.dt, w.D, 20)
    ref = oracle_run(x, M, w.D, w.dt, 20, 3.0, 64 if prec == F64 else 32, norm=oracle.NORM_ROW)
    check_err(ens.masses(), ref, tol)
    ens.close()


# ------------------------------------------------------------------ c2 ----

@pytest.mark.parametrize("lanes", [1, 4, 8, 16])
def test_plain1d_n32768_sparse(lanes):
    w = W.WORKLOADS["plain1d_n32768"]
    x, M, sizes, _ = W.make_inputs(w)
    x, M = f32(x), f32(M)
    ens = make(dim=1, kappa=3.0, prec=F32, lanes=lanes)
    ens.init(sizes, x, M)
    ens.step(w.dt, w.D, 3)
    ref = oracle_run(x, M, w.D, w.dt, 3, 3.0, 32)
    check_err(ens.masses(), ref, 1e-5)
    ens.close()


def test_neighbor_lists_bit_exact_1d():
    w = W.WORKLOADS["plain1d_n32768"]
    x, M, sizes, _ = W.make_inputs(w, n=8000)
    x = f32(x)
    for prec, p in ((F32, 32), (F64, 64)):
        ens = make(dim=1, kappa=3.0, prec=prec)
        ens.init(sizes, x, M)
        rp, cols = ens.neighbors(w.dt, w.D)
        rp0, cols0 = oracle.neighbors(x, 3.0, w.D, w.dt, p)
        assert np.array_equal(rp, rp0) and np.array_equal(cols, cols0)
        ens.close()


# ------------------------------------------------------------------ 2-D ----

@pytest.mark.parametrize("prec", [F32, F64])
@pytest.mark.parametrize("lanes", [-1, 1, 4, 8, 16])
def test_neighbor_lists_bit_exact_2d(prec, lanes):
    n, D, dt = 40000, 2e-4, 0.1  # about the neighbour count of the 10^6-particle case
    x = f32(W.positions(n, 2, 321))
    M = W.masses(n, 2, 321)
    ens = make(dim=2, prec=prec, lanes=lanes)
    ens.init([n], x, M)
    rp, cols = ens.neighbors(dt, D)
    rp0, cols0 = oracle.neighbors(x, 3.0, D, dt, 32 if prec == F32 else 64)
    assert np.array_equal(rp, rp0)
    assert np.array_equal(cols, cols0)
    pairs, evals = ens.count_pairs(dt, D)
    assert pairs == rp0[-1] - n
    assert evals >= rp0[-1]
    ens.close()


@pytest.mark.parametrize("prec", [F32, F64])
@pytest.mark.parametrize("dim,lanes", [(1, 0), (1, 16), (2, 0), (2, -1), (2, 8), (3, 0), (3, 4)])
def test_lattice_pairs_exactly_at_the_cutoff(dim, lanes, prec):
    # spacing h = 3/32 and kappa^2 8 D dt = 9 * 2^-10 = h^2, exact in binary32:
    # axis neighbours sit exactly on the cutoff and are included, diagonal
    # ones are not; the lists match the oracle's bit for bit
    m = {1: 10, 2: 10, 3: 6}[dim]
    idx = np.stack(np.meshgrid(*([np.arange(m)] * dim), indexing="ij"), -1).reshape(-1, dim)
    x = (2.0 + 3.0 * idx) / 32.0
    n = x.shape[0]
    D, dt = 2.0 ** -10, 0.125
    M = W.masses(n, 2, 7)
    ens = make(dim=dim, prec=prec, lanes=lanes)
    ens.init([n], x, M)
    rp, cols = ens.neighbors(dt, D)
    rp0, cols0 = oracle.neighbors(x, 3.0, D, dt, 32 if prec == F32 else 64)
    assert np.array_equal(rp, rp0) and np.array_equal(cols, cols0)
    expect = 1 + sum((idx[:, k] > 0).astype(int) + (idx[:, k] < m - 1).astype(int) for k in range(dim))
    assert np.array_equal(np.diff(rp), expect)
    ens.step(dt, D, 1)
    ref = oracle_run(x, M, D, dt, 1, 3.0, 32 if prec == F32 else 64)
    check_err(ens.masses(), ref, (1e-5 if prec == F32 else 1e-12))
    ens.close()


@pytest.mark.parametrize("prec", [F32, F64])
@pytest.mark.parametrize("lanes", [0, -1, 1, 4, 8, 16])
def test_walk2d_step_with_walk_replayed(prec, lanes):
    n, D, dt, seed = 30000, 2e-4, 0.1, 99
    x = W.positions(n, 2, seed)
    M = W.masses(n, 2, seed)
    if prec == F32:
        x, M = f32(x), f32(M)
    ens = make(dim=2, rw=1.0, prec=prec, seed=seed, lanes=lanes)
    ens.init([n], x, M)
    for step, (xr, mr) in enumerate(OS.steps(x, M, 3, D, dt, seed, (0, 0), (1, 1), prec == F32)):
        ens.step(dt, D, 1)
        check_pos(ens.positions(), xr, prec)
        got = ens.masses()
        check_err(got, mr, walk_tol(prec, D, dt), step)
    ens.close()


@pytest.mark.parametrize("prec", [F32, F64])
def test_walk2d_n1e6_one_step_sampled(prec):
    w = W.WORKLOADS["walk2d_n1e6"]
    x, M, sizes, _ = W.make_inputs(w)
    if prec == F32:
        x, M = f32(x), f32(M)
    ens = make(dim=2, rw=1.0, prec=prec, seed=w.seed)
    ens.init(sizes, x, M)
    ens.step(w.dt, w.D, 1)
    pos = ens.positions()
    got = ens.masses()
    rows = np.random.default_rng(5).choice(w.n, 4000, replace=False)
    (xr, ref), = OS.steps(x, M, 1, w.D, w.dt, w.seed, (0, 0), (1, 1), prec == F32, rows=rows)
    check_pos(pos, xr, prec)
    check_err(got[:, rows], ref, walk_tol(prec, w.D, w.dt))
    # mean in-cutoff neighbours near the closed-form value for the unit square
    pairs, _ = ens.count_pairs(w.dt, w.D)
    r = 3 * math.sqrt(8 * w.D * w.dt)
    F = math.pi * r * r - 8 * r ** 3 / 3 + r ** 4 / 2
    expect = w.n * (w.n - 1) * F
    # ordered pairs: variance ~ 2 E (1 + 4 n F) (pairs sharing a particle correlate)
    assert abs(pairs - expect) < 6 * math.sqrt(2 * expect * (1 + 4 * w.n * F))
    ens.close()


@pytest.mark.parametrize("prec", [F32, F64])
def test_walk3d_n8e6_one_step_sampled(prec):
    """The 3-D, eight-species workload at full size (8e6 particles) in the
    tiling the benchmark times (one lane per particle): one step, sampled
    particles against the oracle, and the pair count against the closed form."""
    w = W.WORKLOADS["walk3d_n8e6_s8"]
    x, M, sizes, _ = W.make_inputs(w)
    if prec == F32:
        x, M = f32(x), f32(M)
    ens = make(dim=3, S=8, rw=1.0, prec=prec, seed=w.seed)
    ens.init(sizes, x, M)
    ens.step(w.dt, w.D, 1)
    assert ens.stats()["tile_lanes"] == -1
    pos = ens.positions()
    got = ens.masses()
    rows = np.random.default_rng(6).choice(w.n, 4000, replace=False)
    (xr, ref), = OS.steps(x, M, 1, w.D, w.dt, w.seed, (0, 0, 0), (1, 1, 1), prec == F32, rows=rows)
    check_pos(pos, xr, prec)
    check_err(got[:, rows], ref, walk_tol(prec, w.D, w.dt))
    # the binary64 audit of all eight species and of A - B over 8e6 particles
    # (many reduction chunks in one realisation) against exactly rounded sums
    ex = np.asarray(exact_sums(got))
    assert np.all(np.abs(ens.audit()[0] - ex) <= 1e-12 * np.abs(ex[:8]).sum())
    # ordered pairs: n (n - 1) F(r) with the unit-cube pair-distance CDF
    # F(r) = 4 pi r^3 / 3 - 3 pi r^4 / 2 + 8 r^5 / 5 - r^6 / 6 (r <= 1)
    pairs, _ = ens.count_pairs(w.dt, w.D)
    r = 3 * math.sqrt(8 * w.D * w.dt)
    F = 4 * math.pi * r ** 3 / 3 - 1.5 * math.pi * r ** 4 + 1.6 * r ** 5 - r ** 6 / 6
    expect = w.n * (w.n - 1) * F
    assert abs(pairs - expect) < 6 * math.sqrt(2 * expect * (1 + 4 * w.n * F))
    ens.close()


def test_walk2d_n1e6_conservation_over_steps():
    w = W.WORKLOADS["walk2d_n1e6"]
    x, M, sizes, _ = W.make_inputs(w)
    for prec, tol in ((F32, 1e-6), (F64, 1e-12)):
        ens = make(dim=2, rw=1.0, prec=prec, seed=w.seed)
        ens.init(sizes, x, M)
        a0 = ens.audit()[0]
        ens.step(w.dt, w.D, 20)
        a1 = ens.audit()[0]
        assert abs(a1[2] - a0[2]) / (a0[0] + a0[1]) < tol
        m = ens.masses()
        assert np.all(np.minimum(m[0], m[1]) == 0.0)
        exact = exact_sums(m)
        assert abs(exact[2] - a1[2]) <= 1e-12 * (a0[0] + a0[1])
        ens.close()


# --------------------------------------------------------------- batched ----

def test_batched_realisations_match_independent_oracles():
    w = W.WORKLOADS["batch2d_64"]
    x, M, sizes, Ds = W.make_inputs(w, n=60000)
    x, M = f32(x), f32(M)
    sizes = sizes.copy()
    ens = make(dim=2, rw=0.0, prec=F32, seed=w.seed)
    ens.init(sizes, x, M, d_scale=Ds)
    ens.step(w.dt, 1.0, 2)
    got = ens.masses()
    a = ens.audit()
    off = np.concatenate([[0], np.cumsum(sizes)])
    for r in range(len(sizes)):
        b, e = off[r], off[r + 1]
        ref = oracle_run(x[b:e], M[:, b:e], Ds[r], w.dt, 2, 3.0, 32)
        check_err(got[:, b:e], ref, 1e-5, r)
        assert abs(a[r, 0] - exact_sums(got[:, b:e])[0]) < 1e-12
    ens.close()


def test_batch2d_64_full_size_sampled():
    """All 64 realisations (4.24e6 particles, D alternating 1e-5 / 1e-4) with
    the walk, in the launch configuration the benchmark times: sampled
    particles of six realisations against the oracle's walk and transfer."""
    w = W.WORKLOADS["batch2d_64"]
    x, M, sizes, Ds = W.make_inputs(w)
    x, M = f32(x), f32(M)
    ens = make(dim=2, rw=1.0, prec=F32, seed=w.seed)
    ens.init(sizes, x, M, d_scale=Ds / w.D)
    ens.step(w.dt, w.D, 1)
    pos = ens.positions()
    got = ens.masses()
    off = np.concatenate([[0], np.cumsum(sizes)])
    order = np.argsort(sizes)
    rng = np.random.default_rng(8)
    for r in [int(order[0]), int(order[1]), int(order[-1]), int(order[-2]), 10, 11]:
        b, e = int(off[r]), int(off[r + 1])
        rows = rng.choice(e - b, min(400, e - b), replace=False)
        # realisation r alone: its particles keep their global Philox ids
        walked = oracle.walk(x[b:e], np.arange(b, e, dtype=np.uint32), w.seed, 0, Ds[r], w.dt, (0, 0), (1, 1))
        xr = f32(walked)
        check_pos(pos[b:e], xr, F32)
        ref = oracle.transfer(xr, M[:, b:e], Ds[r], w.dt, kappa=3.0, prec=32, rows=rows)
        check_err(got[:, b + rows], ref, walk_tol(F32, Ds[r], w.dt), r)
    ens.close()


def test_batch_with_empty_and_single_realisations():
    sizes = [0, 1, 37, 0, 130, 1]
    n = sum(sizes)
    x = f32(W.positions(n, 2, 8))
    M = W.masses(n, 2, 8)
    ens = make(dim=2, prec=F64)
    ens.init(sizes, x, M, d_scale=[1, 1, 1, 1, 0.5, 1])
    D, dt = 5e-3, 0.1
    ens.step(dt, D, 2)
    got = ens.masses()
    off = np.concatenate([[0], np.cumsum(sizes)])
    for r, s in enumerate(sizes):
        if s == 0:
            continue
        b, e = off[r], off[r + 1]
        ref = oracle_run(x[b:e], M[:, b:e], D * [1, 1, 1, 1, 0.5, 1][r], dt, 2, 3.0, 64)
        check_err(got[:, b:e], ref, 1e-12)
    ens.close()


# --------------------------------------------------------------------- 3-D ----

@pytest.mark.parametrize("prec", [F32, F64])
@pytest.mark.parametrize("lanes", [0, -1, 4])
def test_walk3d_eight_species(prec, lanes):
    n, D, dt = 50000, 4e-5, 0.1
    x = W.positions(n, 3, 55)
    M = W.masses(n, 8, 55)
    if prec == F32:
        x, M = f32(x), f32(M)
    ens = make(dim=3, S=8, rw=1.0, prec=prec, seed=55, lanes=lanes)
    ens.init([n], x, M)
    # neighbour sets and counts on the initial positions (the same input on both sides)
    rp, cols = ens.neighbors(dt, D)
    rp0, cols0 = oracle.neighbors(x, 3.0, D, dt, 32 if prec == F32 else 64)
    assert np.array_equal(rp, rp0) and np.array_equal(cols, cols0)
    pairs, evals = ens.count_pairs(dt, D)
    assert pairs == rp0[-1] - n and evals >= rp0[-1]
    # one step with the walk against the oracle's own step
    ens.step(dt, D, 1)
    (xr, mr), = OS.steps(x, M, 1, D, dt, 55, (0, 0, 0), (1, 1, 1), prec == F32)
    assert np.abs(ens.positions() - xr).max() < (2e-6 if prec == F32 else 1e-12)
    check_err(ens.masses(), mr, walk_tol(prec, D, dt))
    if ens.stats()["tile_lanes"] == -1:
        # one lane per particle: only the cells of its own cutoff box (about
        # 2 x 2 x 2 cells of two cutoffs, ~16 candidates here for ~2 neighbours
        # including itself), not the candidate union of a 64-particle tile
        assert evals < 16 * rp0[-1]
    ens.close()


def test_walk3d_row_broadcast_tiles_whole_and_split():
    """The binary32 row-broadcast kernels in 3-D, eight species: 80000
    particles (5000 tiles, one wave per tile) and 40000 (2500 tiles, one block
    per tile with the candidate chunks split over its four waves)."""
    D, dt = 4e-5, 0.1
    for n in (80000, 40000):
        x = f32(W.positions(n, 3, 56))
        M = f32(W.masses(n, 8, 56))
        ens = make(dim=3, S=8, rw=1.0, prec=F32, seed=56, lanes=4)
        ens.init([n], x, M)
        ens.step(dt, D, 1)
        assert ens.stats()["tile_lanes"] == 4
        (xr, mr), = OS.steps(x, M, 1, D, dt, 56, (0, 0, 0), (1, 1, 1), True)
        assert np.abs(ens.positions() - xr).max() < 2e-6, n
        check_err(ens.masses(), mr, walk_tol(F32, D, dt), n)
        ens.close()


@pytest.mark.parametrize("S", [1, 3, 5])
def test_species_counts_and_no_reaction(S):
    n, D, dt = 5000, 1e-3, 0.1
    x = f32(W.positions(n, 2, 12))
    M = W.masses(n, S, 12)
    ens = make(dim=2, S=S, react=None, prec=F64)
    ens.init([n], x, M)
    ens.step(dt, D, 2)
    ref = oracle_run(x, M, D, dt, 2, 3.0, 64, react=None)
    check_err(ens.masses(), ref, 1e-12)
    a = ens.audit()[0]
    assert np.allclose(a[:S], M.sum(axis=1), rtol=1e-12, atol=0)
    ens.close()


# ------------------------------------------------------------- edge cases ----

def test_single_particle_and_ragged_sizes():
    for n in (1, 2, 63, 64, 65, 127, 129):
        x = f32(W.positions(n, 2, n))
        M = W.masses(n, 2, n)
        ens = make(dim=2, prec=F64, lanes=8)
        ens.init([n], x, M)
        ens.step(0.1, 0.05, 1)
        ref = oracle_run(x, M, 0.05, 0.1, 1, 3.0, 64)
        check_err(ens.masses(), ref, 1e-12, n)
        ens.close()


def test_all_particles_coincident():
    n = 300
    x = np.full((n, 2), 0.25)
    M = W.masses(n, 2, 4)
    ens = make(dim=2, prec=F64, react=None)
    ens.init([n], x, M)
    ens.step(0.1, 1e-4, 1)
    mean = M.mean(axis=1, keepdims=True)
    check_err(ens.masses(), 0.5 * (M + mean), 1e-13)
    ens.close()


def test_zero_diffusion_and_zero_steps():
    n = 500
    x = f32(W.positions(n, 2, 2))
    M = f32(W.masses(n, 2, 2))
    ens = make(dim=2, prec=F32, rw=1.0)
    ens.init([n], x, M)
    ens.step(0.1, 0.0, 0)
    assert ens.steps_taken() == 0
    ens.step(0.1, 0.0, 3)
    got = ens.masses()
    ref = M.copy()
    m = np.maximum(0, np.minimum(ref[0], ref[1]))
    ref[0] -= m
    ref[1] -= m
    check_err(got, ref, 1e-7)
    assert np.array_equal(ens.positions(), x)
    ens.close()


def test_particles_on_the_walls_and_corners():
    pts = np.array([[0, 0], [1, 1], [0, 1], [1, 0], [0.5, 0], [0.5, 1], [0, 0.5], [1, 0.5],
                    [1e-7, 1e-7], [1 - 1e-7, 0.5]], dtype=np.float64)
    x = f32(np.concatenate([pts, W.positions(500, 2, 3)]))
    n = len(x)
    M = W.masses(n, 2, 3)
    ens = make(dim=2, prec=F64)
    ens.init([n], x, M)
    ens.step(0.1, 2e-3, 1)
    ref = oracle_run(x, M, 2e-3, 0.1, 1, 3.0, 64)
    check_err(ens.masses(), ref, 1e-12)
    ens.close()


def test_non_unit_box():
    n = 3000
    lo, hi = (-2.0, 5.0), (3.0, 6.5)
    x = f32(W.positions(n, 2, 31, lo, hi))
    M = W.masses(n, 2, 31)
    ens = make(dim=2, prec=F32, box_lo=lo + (0,), box_hi=hi + (1,))
    ens.init([n], x, M)
    ens.step(0.1, 1e-3, 2)
    ref = oracle_run(x, M, 1e-3, 0.1, 2, 3.0, 32)
    check_err(ens.masses(), ref, 1e-5)
    ens.close()


def test_non_unit_box_3d():
    n = 4000
    lo, hi = (-1.0, 0.0, 2.0), (1.0, 0.5, 3.0)
    x = f32(W.positions(n, 3, 33, lo, hi))
    M = W.masses(n, 2, 33)
    for lanes in (0, 4):
        ens = make(dim=3, prec=F32, lanes=lanes, box_lo=lo, box_hi=hi)
        ens.init([n], x, M)
        ens.step(0.1, 1e-3, 2)
        ref = oracle_run(x, M, 1e-3, 0.1, 2, 3.0, 32)
        check_err(ens.masses(), ref, 1e-5, lanes)
        ens.close()


@pytest.mark.parametrize("prec", [F32, F64])
@pytest.mark.parametrize("dim,kappa,lanes", [(1, 4.5, 0), (2, 2.0, 0), (2, 5.0, 4), (2, 5.0, 8),
                                             (3, 2.5, 0), (3, 2.5, 4)])
def test_other_cutoff_multiples(dim, kappa, lanes, prec):
    # kappa sets the cutoff kappa * sigma (Sec. 2.2), hence the cell size and
    # the stencils; masses after two steps follow the oracle at that kappa
    n, dt = {1: 3000, 2: 4000, 3: 5000}[dim], 0.1
    D = {1: 2e-4, 2: 3e-4, 3: 2e-3}[dim]
    x = W.positions(n, dim, 40 + dim)
    if prec == F32:
        x = f32(x)
    M = W.masses(n, 2, 40 + dim)
    ens = make(dim=dim, prec=prec, kappa=kappa, lanes=lanes)
    ens.init([n], x, M)
    ens.step(dt, D, 2)
    ref = oracle_run(x, M, D, dt, 2, kappa, 32 if prec == F32 else 64)
    check_err(ens.masses(), ref, (1e-5 if prec == F32 else 1e-12))
    ens.close()


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_cutoff_wider_than_the_box(dim):
    # kappa * sigma (3.8) exceeds the box diagonal: every pair interacts, so
    # the sparse path gives the full matrix's result
    n, D, dt = 1500, 2.0, 0.1
    x = f32(W.positions(n, dim, 50 + dim))
    M = W.masses(n, 2, 50 + dim)
    ens = make(dim=dim, prec=F32)
    ens.init([n], x, M)
    ens.step(dt, D, 1)
    assert ens.count_pairs(dt, D)[0] == n * (n - 1)
    ref = oracle_run(x, M, D, dt, 1, math.inf, 32)
    check_err(ens.masses(), ref, 1e-5)
    ens.close()


# --------------------------------------------------- determinism / resume ----

def test_bitwise_deterministic_and_resumable():
    n, D, dt = 20000, 1e-4, 0.1
    x = W.positions(n, 2, 17)
    M = W.masses(n, 2, 17)
    outs = []
    for graph in (1, 0):
        e1 = make(dim=2, rw=1.0, prec=F32, seed=3, graph=graph)
        e1.init([n], x, M)
        e1.step(dt, D, 10)
        outs.append((e1.masses(), e1.positions()))
        e1.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    e2 = make(dim=2, rw=1.0, prec=F32, seed=3)
    e2.init([n], x, M)
    e2.step(dt, D, 4)
    e2.step(dt, D, 6)
    assert e2.steps_taken() == 10
    assert np.array_equal(e2.masses(), outs[0][0]) and np.array_equal(e2.positions(), outs[0][1])
    # re-initialising from the queried state continues the same trajectory
    # when the step counter is carried (the walk draws depend on id, step, seed)
    e2.close()


# -------------------------------------------------------------- autotuner ----

def test_autotune_restores_state_and_keeps_parity(tmp_path, monkeypatch):
    n, D, dt = 30000, 2e-4, 0.1
    x = W.positions(n, 2, 41)
    M = W.masses(n, 2, 41)
    monkeypatch.setenv("RWPT_TUNE_CACHE", str(tmp_path / "tune.txt"))
    ens = make(dim=2, rw=1.0, prec=F32, seed=41)
    ens.init([n], x, M)
    ens.step(dt, D, 2)
    m0, p0, a0, s0 = ens.masses(), ens.positions(), ens.audit(), ens.steps_taken()
    rwpt.rwpt_autotune(ens.ctx, dt, D, 2)
    assert np.array_equal(ens.masses(), m0) and np.array_equal(ens.positions(), p0)
    assert np.array_equal(ens.audit(), a0) and ens.steps_taken() == s0
    lanes, ref = rwpt.rwpt_get_tiling(ens.ctx)
    assert lanes in (1, 4, 8, 16)
    ens.step(dt, D, 1)
    # the tuned context continues the oracle's own three-step trajectory
    xr, mr = list(OS.steps(f32(x), f32(M), 3, D, dt, 41, (0, 0), (1, 1), True))[-1]
    assert np.abs(ens.positions() - xr).max() < 2e-6
    check_err(ens.masses(), mr, walk_tol(F32, D, dt))
    ens.close()
    # a second context with the same shape takes the cached choice
    text = (tmp_path / "tune.txt").read_text()
    assert text.count("|") == 1
    e2 = make(dim=2, rw=1.0, prec=F32, seed=41)
    e2.init([n], x, M)
    rwpt.rwpt_autotune(e2.ctx, dt, D, 2)
    assert rwpt.rwpt_get_tiling(e2.ctx) == (lanes, ref)
    assert (tmp_path / "tune.txt").read_text() == text
    e2.close()


@pytest.mark.parametrize("lanes", [-1, 1, 4, 8, 16])
@pytest.mark.parametrize("rw", [1.0, 0.0])
def test_three_warm_up_steps_capture_every_graph_the_timed_steps_replay(lanes, rw):
    # the autotuner times each candidate tiling after three untimed steps; a
    # step's graph depends on the mass buffer it starts from, so every graph
    # that later steps replay must already exist after those three
    n, D, dt = 20000, 2e-4, 0.1
    ens = make(dim=2, rw=rw, prec=F32, seed=4, lanes=lanes)
    ens.init([n], f32(W.positions(n, 2, 4)), f32(W.masses(n, 2, 4)))
    ens.step(dt, D, 3)
    before = ens.stats()["graph_captures"]
    ens.step(dt, D, 5)
    after = ens.stats()["graph_captures"]
    print("lanes %d, walk %g: %d graphs captured in the warm-up, %d more in five steps" % (lanes, rw, before,
                                                                                      after - before))
    assert 1 <= before <= 4 and after == before
    ens.close()


# ------------------------------------------------- full matrix on MFMA ----

@pytest.mark.parametrize("dim,n,S,norm", [(1, 2000, 2, rwpt.RWPT_NORM_SYM), (1, 8192, 2, rwpt.RWPT_NORM_SYM),
                                         (2, 3000, 2, rwpt.RWPT_NORM_SYM), (3, 2000, 8, rwpt.RWPT_NORM_SYM),
                                         (2, 3000, 3, rwpt.RWPT_NORM_ROW), (1, 1000, 8, rwpt.RWPT_NORM_ROW),
                                         (1, 77, 1, rwpt.RWPT_NORM_SYM)])
def test_dense_full_matrix_matches_oracle(dim, n, S, norm):
    D = {1: 1e-4, 2: 2e-3, 3: 1e-2}[dim]
    dt, steps = 0.1, 5
    x = f32(W.positions(n, dim, 500 + n))
    M = f32(W.masses(n, S, 500 + n))
    react = (0, 1) if S >= 2 else None
    ens = rwpt.Ensemble(dim=dim, n_species=S, react=react, kappa=None, rw_ratio=0.0, precision=F32,
                        norm=norm, path=rwpt.RWPT_PATH_DENSE, seed=3)
    ens.init([n], x, M)
    ens.step(dt, D, steps)
    ref = oracle_run(x, M, D, dt, steps, math.inf, 32,
                     norm=oracle.NORM_SYM if norm == rwpt.RWPT_NORM_SYM else oracle.NORM_ROW, react=react)
    check_err(ens.masses(), ref, 1e-5)
    if norm == rwpt.RWPT_NORM_SYM:
        # conserved by transfer and reaction: sum(A - B), or sum(M) without a reaction
        a0 = oracle.audit(M, react)
        a = ens.audit()[0]
        k = S if react is not None else 0
        assert abs(a[k] - a0[k]) <= 1e-6 * M[:2].sum()
    ens.close()


def test_dense_plain1d_n32768_two_steps_and_walk():
    w = W.WORKLOADS["plain1d_n32768"]
    x, M, sizes, _ = W.make_inputs(w)
    x, M = f32(x), f32(M)
    ens = rwpt.Ensemble(dim=1, n_species=2, kappa=None, rw_ratio=0.0, precision=F32,
                        path=rwpt.RWPT_PATH_DENSE, seed=3)
    ens.init(sizes, x, M)
    ens.step(w.dt, w.D, 2)
    ref = oracle_run(x, M, w.D, w.dt, 2, math.inf, 32)
    check_err(ens.masses(), ref, 1e-5)
    ens.close()
    # with the walk: one step against the oracle's own walk + full-matrix transfer
    n = 6000
    x = f32(W.positions(n, 2, 9))
    M = f32(W.masses(n, 2, 9))
    ens = rwpt.Ensemble(dim=2, n_species=2, kappa=None, rw_ratio=1.0, precision=F32,
                        path=rwpt.RWPT_PATH_DENSE, seed=9)
    ens.init([n], x, M)
    ens.step(0.1, 1e-3, 1)
    (xr, mr), = OS.steps(x, M, 1, 1e-3, 0.1, 9, (0, 0), (1, 1), True, kappa=math.inf)
    assert np.abs(ens.positions() - xr).max() < 2e-6
    check_err(ens.masses(), mr, walk_tol(F32, 1e-3, 0.1))
    ens.close()


def test_dense_path_requires_full_matrix_binary32_single_realisation():
    with pytest.raises(rwpt.RwptError) as ei:
        rwpt.Ensemble(dim=1, kappa=3.0, path=rwpt.RWPT_PATH_DENSE)
    assert ei.value.status == rwpt.RWPT_EINVAL
    with pytest.raises(rwpt.RwptError) as ei:
        rwpt.Ensemble(dim=1, kappa=None, precision=F64, path=rwpt.RWPT_PATH_DENSE)
    assert ei.value.status == rwpt.RWPT_EUNSUPPORTED
    ens = rwpt.Ensemble(dim=1, kappa=None, path=rwpt.RWPT_PATH_DENSE)
    with pytest.raises(rwpt.RwptError) as ei:
        ens.init([10, 10], W.positions(20, 1, 1), W.masses(20, 2, 1))
    assert ei.value.status == rwpt.RWPT_EUNSUPPORTED
    ens.close()


# ------------------------------------------ interface verification (Sec. 3) ----

def interface_ensemble(n, n_real, seed0):
    parts = [W.interface(n, 1, 50.0, seed0 + r) for r in range(n_real)]
    return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts], 1)


@pytest.mark.parametrize("prec", [F32, F64])
def test_interface_steps_replayed(prec):
    # three realisations with the walk, four steps against the oracle's own
    # trajectory (global particle ids).  Binary32 positions up to 50 resolve
    # 3.8e-6, so the two trajectories drift apart by a few such units
    n, R, seed = 2000, 3, 6000
    x, M = interface_ensemble(n, R, seed)
    if prec == F32:
        x, M = f32(x), f32(M)
    ens = make(dim=1, react=None, rw=1.0, prec=prec, seed=seed, box_hi=(50.0, 1, 1))
    ens.init([n] * R, x, M)
    traj = OS.steps(x, M, 4, 0.5, 0.1, seed, (0.0,), (50.0,), prec == F32, sizes=[n] * R, react=None)
    for step, (xr, mr) in enumerate(traj):
        ens.step(0.1, 0.5, 1)
        pos, got = ens.positions(), ens.masses()
        assert np.abs(pos - xr).max() < (1e-4 if prec == F32 else 1e-12)
        errs = [normerr(got[:, r * n:(r + 1) * n], mr[:, r * n:(r + 1) * n]) for r in range(R)]
        print("step", step, "max position difference %.2e" % np.abs(pos - xr).max(), "mass errors", errs)
        assert max(errs) < walk_tol(prec, 0.5, 0.1, xmax=50.0), (step, errs)
    ens.close()


@pytest.mark.parametrize("prec", [F32, F64])
def test_interface1d_l50_matches_erfc(prec):
    # the full verification workload: 75 realisations of N = 2000 on [0, 50],
    # D = 1 split equally between transfer and walk, 100 steps to t = 10.
    # The oracle's ensemble gives a per-realisation RMSE of 0.012 and a binned
    # ensemble profile within 0.0017 (RMS) of erfc.
    from scipy.special import erfc
    w = W.WORKLOADS["interface1d_l50"]
    L, n, R = w.box_hi[0], w.n, w.n_real
    x, M, sizes, _ = W.make_inputs(w)
    assert np.array_equal(x, interface_ensemble(n, R, w.seed)[0])
    ds = L / n
    ens = make(dim=1, react=None, rw=w.rw_ratio, prec=prec, seed=w.seed, box_hi=w.box_hi)
    ens.init(sizes, x, M)
    a0 = ens.audit()
    ens.step(w.dt, w.D, w.steps)
    pos, got = ens.positions()[:, 0], ens.masses()
    a1 = ens.audit()
    # the two components stay complementary and each is conserved per realisation
    assert np.abs((got[0] + got[1]) / ds - 1.0).max() < (1e-5 if prec == F32 else 1e-12)
    assert np.abs(a1[:, :2] - a0[:, :2]).max() < (1e-5 if prec == F32 else 1e-12) * L
    c = got[0] / ds
    exact = 0.5 * erfc((0.5 * L - pos) / math.sqrt(4 * (2 * w.D) * w.steps * w.dt))
    per_real = np.sqrt(np.mean(((c - exact) ** 2).reshape(R, n), axis=1))
    assert per_real.mean() < 0.02 and per_real.max() < 0.04
    bins = np.linspace(0.0, L, 51)
    b = np.clip(np.digitize(pos, bins) - 1, 0, 49)
    prof = np.bincount(b, c, 50) / np.bincount(b, None, 50)
    mid = 0.5 * (bins[1:] + bins[:-1])
    ex_mid = 0.5 * erfc((0.5 * L - mid) / math.sqrt(4 * (2 * w.D) * w.steps * w.dt))
    assert math.sqrt(np.mean((prof - ex_mid) ** 2)) < 0.004
    assert np.abs(prof - ex_mid).max() < 0.012
    ens.close()


# ----------------------------- four-lane whole tiles, short last chunks ----

@pytest.mark.parametrize("dim,mean_nb", [(1, 4.0), (2, 3.0), (2, 12.0), (2, 40.0)])
@pytest.mark.parametrize("S,norm", [(2, rwpt.RWPT_NORM_SYM), (2, rwpt.RWPT_NORM_ROW), (8, rwpt.RWPT_NORM_SYM)])
def test_four_lane_whole_tiles_with_short_last_chunks(dim, mean_nb, S, norm):
    # more than 4096 tiles of 16 (one wave per tile) at few neighbours: most
    # segments end in a chunk of at most 16 or 32 candidates, evaluated in 4
    # or 8 broadcast steps; the exchange on identical positions (no walk) must
    # match the oracle to the binary32 bar after each of two steps
    n, dt, seed = 80000, 0.1, 7300 + dim
    unit = {1: 2.0, 2: math.pi}[dim]
    rc = (mean_nb / ((n - 1) * unit)) ** (1.0 / dim)
    D = rc * rc / (72.0 * dt)
    x = f32(W.positions(n, dim, seed))
    M = f32(W.masses(n, S, seed))
    ens = make(dim=dim, S=S, prec=F32, norm=norm, seed=seed, lanes=4)
    ens.init([n], x, M)
    onorm = oracle.NORM_SYM if norm == rwpt.RWPT_NORM_SYM else oracle.NORM_ROW
    ref = M
    for step in range(2):
        ens.step(dt, D, 1)
        ref = oracle.transfer(x, ref, D, dt, kappa=3.0, prec=32, norm=onorm, react=(0, 1))
        check_err(ens.masses(), ref, 1e-5, step)
    assert ens.stats()["tile_lanes"] == 4 and -(-n // 16) > 4096
    pairs, evals = ens.count_pairs(dt, D)
    assert 0.5 * mean_nb * n < pairs < 1.5 * mean_nb * n
    ens.close()


# ------------------------------------- one lane per particle, neighbour cache ----

@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("mean_nb", [0.7, 2.5, 6.0, 12.0])
@pytest.mark.parametrize("prec,norm", [(F32, rwpt.RWPT_NORM_SYM), (F64, rwpt.RWPT_NORM_ROW)])
def test_private_lists_cached_and_missed_neighbours(dim, mean_nb, prec, norm):
    # mean in-cutoff neighbours per particle from 0.7 (every lane cached) to 12
    # (most lanes above the per-lane limit of 8, waves beyond their region):
    # cached lanes, missed lanes and mixed waves must all match the oracle
    n, dt, seed = 20000, 0.1, 7000 + dim
    unit = {1: 2.0, 2: math.pi, 3: 4.0 * math.pi / 3.0}[dim]
    rc = (mean_nb / ((n - 1) * unit)) ** (1.0 / dim)
    D = rc * rc / (72.0 * dt)
    x = W.positions(n, dim, seed)
    M = W.masses(n, 2, seed)
    if prec == F32:
        x, M = f32(x), f32(M)
    lo, hi = (0.0,) * dim, (1.0,) * dim
    ens = make(dim=dim, rw=1.0, prec=prec, norm=norm, seed=seed, lanes=-1)
    ens.init([n], x, M)
    onorm = oracle.NORM_SYM if norm == rwpt.RWPT_NORM_SYM else oracle.NORM_ROW
    for step, (xr, mr) in enumerate(OS.steps(x, M, 2, D, dt, seed, lo, hi, prec == F32, norm=onorm)):
        ens.step(dt, D, 1)
        pos, got = ens.positions(), ens.masses()
        assert np.abs(pos - xr).max() < (2e-6 if prec == F32 else 1e-12)
        check_err(got, mr, walk_tol(prec, D, dt), step)
    pairs, _ = ens.count_pairs(dt, D)
    assert 0.5 * mean_nb * n < pairs < 1.5 * mean_nb * n
    ens.close()


@pytest.mark.parametrize("mean_nb", [2.5, 6.0])
@pytest.mark.parametrize("prec,norm", [(F32, rwpt.RWPT_NORM_SYM), (F64, rwpt.RWPT_NORM_ROW)])
def test_private_lists_eight_species_in_several_rounds(mean_nb, prec, norm):
    # 3-D, eight species: a wave keeps 2.5 or 6 neighbours per lane on average,
    # so its cached entries take three or four rounds of 64 lanes (6.0: many
    # waves also fill their 256-entry region and send lanes to the stencil
    # walk); every species of every staged entry must reach its own lane
    n, dt, seed = 20000, 0.1, 7100
    rc = (mean_nb / ((n - 1) * 4.0 * math.pi / 3.0)) ** (1.0 / 3.0)
    D = rc * rc / (72.0 * dt)
    x = W.positions(n, 3, seed)
    M = W.masses(n, 8, seed)
    if prec == F32:
        x, M = f32(x), f32(M)
    ens = make(dim=3, S=8, rw=1.0, prec=prec, norm=norm, seed=seed, lanes=-1)
    ens.init([n], x, M)
    onorm = oracle.NORM_SYM if norm == rwpt.RWPT_NORM_SYM else oracle.NORM_ROW
    lo, hi = (0.0,) * 3, (1.0,) * 3
    for step, (xr, mr) in enumerate(OS.steps(x, M, 2, D, dt, seed, lo, hi, prec == F32, norm=onorm)):
        ens.step(dt, D, 1)
        pos, got = ens.positions(), ens.masses()
        assert np.abs(pos - xr).max() < (2e-6 if prec == F32 else 1e-12)
        check_err(got, mr, walk_tol(prec, D, dt), step)
    pairs, _ = ens.count_pairs(dt, D)
    assert 0.5 * mean_nb * n < pairs < 1.5 * mean_nb * n
    ens.close()


# ---------------------------------------------- device input and state summary ----

def test_init_from_device_buffers_matches_host_init():
    import torch
    n, seed = 5000, 31
    x = W.positions(n, 2, seed)
    M = W.masses(n, 2, seed)
    xd = torch.from_numpy(x).to("cuda").contiguous()
    Md = torch.from_numpy(M).to("cuda").contiguous()
    torch.cuda.synchronize()
    a = make(dim=2, rw=1.0, prec=F64, seed=seed)
    a.init([n], x, M)
    b = make(dim=2, rw=1.0, prec=F64, seed=seed)
    rwpt.rwpt_init_ensemble_device(b.ctx, [n], xd.data_ptr(), Md.data_ptr())
    b.n, b.n_real = n, 1
    assert np.array_equal(a.audit(), b.audit())
    a.step(0.1, 2e-4, 3)
    b.step(0.1, 2e-4, 3)
    assert np.array_equal(a.masses(), b.masses())
    assert np.array_equal(a.positions(), b.positions())
    # device input is validated like host input
    bad = xd.clone()
    bad[7, 1] = 2.0
    torch.cuda.synchronize()
    with pytest.raises(rwpt.RwptError) as ei:
        rwpt.rwpt_init_ensemble_device(b.ctx, [n], bad.data_ptr(), Md.data_ptr())
    assert ei.value.status == rwpt.RWPT_EINVAL and "outside" in str(ei.value)
    a.close()
    b.close()


def test_stats_summarise_the_state():
    n, D, dt = 20000, 2e-4, 0.1
    ens = make(dim=2, rw=1.0, prec=F32, seed=3)
    ens.init([n], f32(W.positions(n, 2, 3)), f32(W.masses(n, 2, 3)))
    st = ens.stats()
    assert st["n_particles"] == n and st["ordered_pairs"] == -1 and st["steps_taken"] == 0
    rwpt.rwpt_profile_enable(ens.ctx, True)
    ens.step(dt, D, 2)
    st = ens.stats()
    pairs, evals = ens.count_pairs(dt, D)
    assert st["steps_taken"] == 2 and st["ordered_pairs"] == pairs and st["candidate_evals"] == evals
    assert st["n_cells"] > 0 and st["tile_lanes"] == rwpt.rwpt_get_tiling(ens.ctx)[0]
    assert st["phases"]["exchange"][1] == 2 and st["phases"]["rowsum"][1] == 2
    ens.close()


def test_walk2d_n1e6_mixing_limited_decay_slope():
    # Continuum asymptote of the A + B -> 0 decay from Gaussian fluctuations:
    # sum A ~ t^(-d/4) while the particle spacing << sqrt(2 D_eff t) << box
    # (D_eff = D + D_rw); in 2-D at 10^6 particles that is steps ~10 - 200.
    w = W.WORKLOADS["walk2d_n1e6"]
    x, M, sizes, _ = W.make_inputs(w)
    ens = make(dim=2, rw=1.0, prec=F32, seed=w.seed)
    ens.init(sizes, x, M)
    marks, sums, done = [20, 40, 80, 160], [], 0
    for m in marks:
        ens.step(w.dt, w.D, m - done)
        done = m
        sums.append(ens.audit()[0, 0])
    slope = np.polyfit(np.log(marks), np.log(sums), 1)[0]
    assert -0.6 < slope < -0.4, slope
    ens.close()


def test_dense_full_matrix_at_its_maximum_size():
    # one realisation of 2^17 particles, the largest the matrix-core path
    # takes; sampled rows against the oracle's full matrix (every pair)
    n, D, dt = 1 << 17, 1e-4, 0.1
    x = f32(W.positions(n, 1, 17))
    M = f32(W.masses(n, 2, 17))
    ens = rwpt.Ensemble(dim=1, n_species=2, kappa=None, rw_ratio=0.0, precision=F32,
                        path=rwpt.RWPT_PATH_DENSE, seed=17)
    ens.init([n], x, M)
    ens.step(dt, D, 1)
    got = ens.masses()
    rows = np.random.default_rng(17).choice(n, 64, replace=False)
    # the oracle at kappa = 7 equals its full matrix to e^-49 of the kernel
    # (far below any tolerance here) and runs on its cell grid
    ref = oracle.transfer(x, M, D, dt, kappa=7.0, prec=32, rows=rows)
    check_err(got[:, rows], ref, 1e-5)
    a = ens.audit()[0]
    assert abs(a[2] - oracle.audit(M)[2]) < 1e-6 * (a[0] + a[1])
    ens.close()


# ------------------------------------------- advection and dispersion (Eq. 1) ----

@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("prec", [F32, F64])
def test_advective_walk_replayed(dim, prec):
    n, D, dt, seed = 20000, 1e-4, 0.1, 123
    vel = (0.02, -0.015, 0.01)[:dim]
    aL, aT = 0.01, 0.002
    x = W.positions(n, dim, seed)
    M = W.masses(n, 2, seed)
    if prec == F32:
        x, M = f32(x), f32(M)
    lo, hi = (0.0,) * dim, (1.0,) * dim
    ens = rwpt.Ensemble(dim=dim, n_species=2, rw_ratio=1.0, precision=prec, seed=seed, velocity=vel,
                        alpha_l=aL, alpha_t=aT)
    ens.init([n], x, M)
    traj = OS.steps(x, M, 3, D, dt, seed, lo, hi, prec == F32, velocity=vel, alpha_l=aL, alpha_t=aT)
    for step, (xr, mr) in enumerate(traj):
        ens.step(dt, D, 1)
        pos, got = ens.positions(), ens.masses()
        assert np.abs(pos - xr).max() < (2e-6 if prec == F32 else 1e-12)
        check_err(got, mr, walk_tol(prec, D, dt), step)
    ens.close()


@pytest.mark.parametrize("prec", [F32, F64])
def test_advected_interface_follows_the_shifted_erfc(prec):
    # 1-D interface at x0 = 10 on [0, 50] advected with v = 1 for t = 10, transfer
    # D_m = 0.5, walk share 0.5, longitudinal dispersivity 1: C1 follows
    # erfc((x0 + v t - x) / sqrt(4 (D_m + D_rw + alpha_L v) t)) / 2 near the front
    from scipy.special import erfc
    L, n, R, x0, v, aL = 50.0, 4000, 3, 10.0, 1.0, 1.0
    parts = [W.interface(n, 1, L, 8000 + r, x0=x0) for r in range(R)]
    x = np.concatenate([p[0] for p in parts])
    M = np.concatenate([p[1] for p in parts], 1)
    ens = rwpt.Ensemble(dim=1, n_species=2, react=None, rw_ratio=1.0, precision=prec, seed=8000,
                        box_hi=(L, 1, 1), velocity=(v, 0, 0), alpha_l=aL)
    ens.init([n] * R, x, M)
    ens.step(0.1, 0.5, 100)
    pos, got = ens.positions()[:, 0], ens.masses()
    front = x0 + v * 10.0
    sel = np.abs(pos - front) < 8.0
    exact = 0.5 * erfc((front - pos[sel]) / math.sqrt(4 * (0.5 + 0.5 + aL * v) * 10.0))
    rmse = math.sqrt(np.mean((got[0][sel] / (L / n) - exact) ** 2))
    assert rmse < 0.045, rmse
    # the components stay complementary
    assert np.abs((got[0] + got[1]) / (L / n) - 1.0).max() < (1e-5 if prec == F32 else 1e-12)
    ens.close()


@pytest.mark.parametrize("prec", [F32, F64])
def test_interface2d_l80_matches_erfc(prec):
    from scipy.special import erfc
    w = W.WORKLOADS["interface2d_l80"]
    L, n, R = w.box_hi[0], w.n, w.n_real
    x, M, sizes, _ = W.make_inputs(w)
    ens = make(dim=2, react=None, rw=w.rw_ratio, prec=prec, seed=w.seed, box_hi=w.box_hi)
    ens.init(sizes, x, M)
    # the first steps against the oracle's own trajectory (realisation 0)
    x0, m0 = (f32(x[:n]), f32(M[:, :n])) if prec == F32 else (x[:n], M[:, :n])
    traj = OS.steps(x0, m0, 2, w.D, w.dt, w.seed, (0, 0), (L, L), prec == F32, react=None)
    for step, (xr, mr) in enumerate(traj):
        ens.step(w.dt, w.D, 1)
        pos, got = ens.positions()[:n], ens.masses()[:, :n]
        assert np.abs(pos - xr).max() < (2e-4 if prec == F32 else 1e-11)
        err = normerr(got, mr)
        print("step", step, "max position difference %.2e" % np.abs(pos - xr).max(), "mass error %.2e" % err)
        assert err < walk_tol(prec, w.D, w.dt, xmax=L)
    ens.step(w.dt, w.D, w.steps - 2)
    pos, got = ens.positions(), ens.masses()
    ds = L * L / n
    exact = 0.5 * erfc((0.5 * L - pos[:, 0]) / math.sqrt(4 * (2 * w.D) * w.steps * w.dt))
    per_real = np.sqrt(np.mean(((got[0] / ds - exact) ** 2).reshape(R, n), axis=1))
    assert per_real.max() < 0.025 and per_real.mean() < 0.02, per_real
    ens.close()


@pytest.mark.parametrize("lanes,rw,prec", [(-1, 1.0, F32), (-1, 0.0, F32), (-1, 1.0, F64), (4, 1.0, F32),
                                           (4, 0.0, F32)])
def test_graph_eager_split_and_interleaved_queries_agree_bitwise(lanes, rw, prec):
    # the one-lane-per-particle path leaves the masses in place during a sort
    # and alternates the two mass buffers: replayed graphs (one per parity),
    # eager launches, steps split at odd counts, and queries that sort in
    # between (neighbour export before the first step) must all give the
    # same bits
    n, dt = 20000, 0.1
    rc = math.sqrt(3.0 / (math.pi * n))     # about 3 neighbours per particle
    D = rc * rc / (72.0 * dt)
    x = W.positions(n, 2, 23)
    M = W.masses(n, 2, 23)
    runs = []
    for mode in ("graph", "eager", "split", "queries"):
        e = make(dim=2, rw=rw, prec=prec, seed=5, lanes=lanes, graph=0 if mode == "eager" else 1)
        e.init([n], x, M)
        if mode == "split":
            for k in (1, 2, 3, 1):
                e.step(dt, D, k)
        elif mode == "queries":
            e.neighbors(dt, D)
            e.step(dt, D, 1)
            e.count_pairs(dt, D)
            e.step(dt, D, 2)
            e.stats()
            e.audit()
            e.masses()
            e.step(dt, D, 4)
        else:
            e.step(dt, D, 7)
        assert e.steps_taken() == 7
        runs.append((e.masses(), e.positions(), e.audit()))
        e.close()
    for other in runs[1:]:
        assert np.array_equal(runs[0][0], other[0]) and np.array_equal(runs[0][1], other[1])
        assert np.array_equal(runs[0][2], other[2])
    # and the result is the oracle's (replayed on the final positions is not
    # possible after a walk; without the walk it is 7 transfers)
    if rw == 0.0:
        ref = oracle_run(f32(x) if prec == F32 else x, f32(M) if prec == F32 else M, D, dt, 7, 3.0,
                         32 if prec == F32 else 64)
        check_err(runs[0][0], ref, (1e-5 if prec == F32 else 1e-12))


def test_cell_grids_of_different_refinement_agree_over_steps():
    """Ten FP64 steps with the walk on a grid of 11 k cells and on one of 44 k
    cells give the same masses and positions (same neighbour sets, summation
    order aside): the cell counts restart from zero every step."""
    n, D, dt = 30000, 1e-4, 0.1
    x = W.positions(n, 2, 78)
    M = W.masses(n, 2, 78)
    out = []
    for refine in ((4.0, 2.0, 0.0), (16.0, 2.0, 0.0)):
        ens = make(dim=2, prec=F64, rw=1.0, refine=refine, seed=78)
        ens.init([n], x, M)
        ens.step(dt, D, 10)
        st = ens.stats()
        out.append((st["n_cells"], ens.masses(), ens.positions(), ens.count_pairs(dt, D)[0]))
        ens.close()
    (cells_a, m_a, x_a, p_a), (cells_b, m_b, x_b, p_b) = out
    assert 2 * cells_a < cells_b
    assert np.array_equal(x_a, x_b) and p_a == p_b
    check_err(m_a, m_b, 1e-12)


def test_cell_scan_both_forms_agree():
    """Grids of more than 256 scan blocks (1.05e6 cells) take the three-launch
    cell scan, smaller ones the two-launch form: the same FP64 step on both
    grids gives the same masses (same neighbour sets, summation order aside)."""
    n, D, dt = 5_000_000, 1e-6, 0.1
    x = W.positions(n, 2, 77)
    M = W.masses(n, 2, 77)
    out = []
    for refine in ((32.0, 32.0, 0.0), (2.0, 2.0, 0.0)):
        ens = make(dim=2, prec=F64, refine=refine, seed=77)
        ens.init([n], x, M)
        ens.step(dt, D, 1)
        st = ens.stats()
        out.append((st["n_cells"], ens.masses(), ens.count_pairs(dt, D)[0]))
        ens.close()
    (cells_big, m_big, p_big), (cells_small, m_small, p_small) = out
    assert cells_big > 256 * 4096 >= cells_small
    assert p_big == p_small
    check_err(m_big, m_small, 1e-12)


# ----------------------- full sizes on identical positions (no walk) ----

def default_lanes(dim, prec):
    return {1: 4 if prec == F32 else 16, 2: 4 if prec == F32 else 8, 3: -1}[dim]


@pytest.mark.parametrize("prec", [F32, F64])
@pytest.mark.parametrize("name", ["walk2d_n1e6", "walk3d_n8e6_s8"])
def test_full_size_transfer_on_identical_positions(name, prec):
    """The 10^6-particle 2-D and 8e6-particle 3-D workloads in the launch
    configuration the benchmark times, with the walk switched off so that both
    sides see the same positions: two steps (the first sorts the seeded input,
    and the one-lane-per-particle path then reads the masses through the
    previous order; the second does not sort), sampled particles against the
    oracle at the stated bars with no walk allowance."""
    w = W.WORKLOADS[name]
    x, M, sizes, _ = W.make_inputs(w)
    if prec == F32:
        x, M = f32(x), f32(M)
    p = 32 if prec == F32 else 64
    ens = make(dim=w.dim, S=w.n_species, rw=0.0, prec=prec, seed=w.seed)
    ens.init(sizes, x, M)
    rows = np.random.default_rng(21).choice(w.n, 4000, replace=False)
    ens.step(w.dt, w.D, 1)
    assert ens.stats()["tile_lanes"] == default_lanes(w.dim, prec)
    m1 = oracle.transfer(x, M, w.D, w.dt, kappa=w.kappa, prec=p, react=w.react)
    check_err(ens.masses()[:, rows], m1[:, rows], 1e-5 if prec == F32 else 1e-12, "step 1")
    ens.step(w.dt, w.D, 1)
    m2 = oracle.transfer(x, m1, w.D, w.dt, kappa=w.kappa, prec=p, react=w.react, rows=rows)
    check_err(ens.masses()[:, rows], m2, 1e-5 if prec == F32 else 1e-12, "step 2")
    ens.close()


def test_batch2d_64_full_size_on_identical_positions():
    """All 64 realisations (4.24e6 particles) in the benchmark's launch
    configuration, walk off: sampled particles of the smallest, the largest
    and two mid-size realisations after two steps at the binary32 bar."""
    w = W.WORKLOADS["batch2d_64"]
    x, M, sizes, Ds = W.make_inputs(w)
    x, M = f32(x), f32(M)
    ens = make(dim=2, rw=0.0, prec=F32, seed=w.seed)
    ens.init(sizes, x, M, d_scale=Ds / w.D)
    ens.step(w.dt, w.D, 2)
    got = ens.masses()
    off = np.concatenate([[0], np.cumsum(sizes)])
    order = np.argsort(sizes)
    rng = np.random.default_rng(22)
    for r in [int(order[0]), int(order[-1]), int(order[31]), int(order[32])]:
        b, e = int(off[r]), int(off[r + 1])
        rows = rng.choice(e - b, min(500, e - b), replace=False)
        m1 = oracle.transfer(x[b:e], M[:, b:e], Ds[r], w.dt, kappa=3.0, prec=32)
        ref = oracle.transfer(x[b:e], m1, Ds[r], w.dt, kappa=3.0, prec=32, rows=rows)
        check_err(got[:, b + rows], ref, 1e-5, "realisation %d, %d particles, D %g" % (r, e - b, Ds[r]))
    ens.close()


# ---------------------------------------------- the stated run lengths ----

def _long_runs():
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "make_long_runs.py")
    spec = importlib.util.spec_from_file_location("make_long_runs", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("run,prec,path", [("plain1d_n32768_k3_fp32", F32, rwpt.RWPT_PATH_SPARSE),
                                           ("plain1d_n32768_k3_fp64", F64, rwpt.RWPT_PATH_SPARSE),
                                           ("plain1d_n32768_k7_fp32", F32, rwpt.RWPT_PATH_DENSE),
                                           ("walk2d_n1e6_rw0_fp32", F32, rwpt.RWPT_PATH_SPARSE),
                                           ("walk2d_n1e6_rw0_fp64", F64, rwpt.RWPT_PATH_SPARSE)])
def test_full_run_length_against_stored_oracle_runs(run, prec, path):
    """The plain 1-D workload for its 500 steps (cutoff 3 sigma in both
    precisions, and the full matrix on matrix cores against the oracle at
    7 sigma, which equals the full matrix to e^-49 of the kernel) and the
    10^6-particle 2-D workload for its 200 steps with positions fixed: the
    error accumulated over the whole run against the oracle's run, written by
    tests/golden/make_long_runs.py from the oracle alone."""
    LR = _long_runs()
    w, x, M, steps, kappa, p, rows_expected = LR.inputs(run)
    rows, ref = LR.load(run)
    assert np.array_equal(rows, rows_expected)
    dense = path == rwpt.RWPT_PATH_DENSE
    ens = rwpt.Ensemble(dim=w.dim, n_species=w.n_species, react=w.react, kappa=None if dense else kappa,
                        rw_ratio=0.0, precision=prec, path=path, seed=w.seed)
    ens.init([w.n], x, M)
    ens.step(w.dt, w.D, steps)
    got = ens.masses()
    check_err(got[:, rows], ref, 1e-5 if prec == F32 else 1e-12, "%s after %d steps" % (run, steps))
    a0, a1 = oracle.audit(M, w.react), ens.audit()[0]
    drift = abs(a1[-1] - a0[-1]) / (a0[0] + a0[1])
    print("sum(A - B) drift over the run %.2e of sum(A + B)" % drift)
    assert drift < (1e-6 if prec == F32 else 1e-12)
    ens.close()
