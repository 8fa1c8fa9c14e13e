"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests re-types the oracle's formula: each checks a published
value (Philox known answers, the paper's printed pad ratios), a closed form
of a special case, an invariant, or agreement with the separately written
dense NumPy brute force.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import numpy_ref
from paper_1811_05474_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


# ---------------------------------------------------------------- Philox ----

def test_philox_known_answer_vectors():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        out = oracle.philox4x32_10(v[0:4], v[4:6])
        assert [int(o) for o in out] == v[6:10]


# ------------------------------------------------------- closed forms -------

@pytest.mark.parametrize("norm", [oracle.NORM_SYM, oracle.NORM_ROW])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_two_particles_at_one_sigma(norm, d):
    # Two isolated particles at separation s = sigma = sqrt(8 D dt):
    # nu_12/nu_11 = e^-1, P_12 = e^-1/(1+e^-1) = 1/(e+1) in both readings,
    # so M_1' = M_1 + (M_2 - M_1) / (2 (e + 1))  (Eq. 4, Eq. 6).
    D, dt = 0.02, 0.5
    sigma = math.sqrt(8 * D * dt)
    x = np.zeros((2, d))
    x[1] = sigma / math.sqrt(d)
    M = np.array([[3.0, 1.0], [0.25, 2.0]])
    out = oracle.transfer(x, M, D, dt, kappa=3.0, norm=norm, prec=64, react=None)
    exp = M[:, 0] + (M[:, 1] - M[:, 0]) / (2 * (math.e + 1))
    assert np.allclose(out[:, 0], exp, rtol=1e-14, atol=0)
    exp1 = M[:, 1] + (M[:, 0] - M[:, 1]) / (2 * (math.e + 1))
    assert np.allclose(out[:, 1], exp1, rtol=1e-14, atol=0)


@pytest.mark.parametrize("dim,m", [(1, 10), (2, 10), (3, 6)])
@pytest.mark.parametrize("prec", [32, 64])
def test_lattice_neighbours_exactly_at_the_cutoff(dim, m, prec):
    # Lattice spacing h = 3/32 with 8 D dt = 2^-10, so kappa^2 8 D dt = h^2
    # exactly in binary32 and binary64: axis neighbours sit exactly on the
    # cutoff and count ("within" s_max, Sec. 2.1), diagonal ones (2 h^2) do not.
    idx = np.stack(np.meshgrid(*([np.arange(m)] * dim), indexing="ij"), -1).reshape(-1, dim)
    x = (2.0 + 3.0 * idx) / 32.0
    rp, cols = oracle.neighbors(x, 3.0, 2.0 ** -10, 0.125, prec)
    expect = 1 + sum((idx[:, k] > 0).astype(int) + (idx[:, k] < m - 1).astype(int) for k in range(dim))
    assert np.array_equal(np.diff(rp), expect)
    for i in (0, len(x) // 2):
        nb = cols[rp[i]:rp[i + 1]]
        assert np.all(np.abs(idx[nb] - idx[i]).sum(axis=1) <= 1)


def test_two_particles_at_cutoff_edge():
    # At s = 3 sigma the weight is e^-9 (Sec. 2.2: the pad captures the
    # density out to 3 sigma); just beyond, the pair does not interact.
    D, dt = 1e-4, 0.1
    sigma = math.sqrt(8 * D * dt)
    M = np.array([[1.0, 0.0]])
    x_in = np.array([[0.0], [3 * sigma * (1 - 1e-9)]])
    x_out = np.array([[0.0], [3 * sigma * (1 + 1e-6)]])
    w = math.exp(-9.0 * (1 - 1e-9) ** 2)
    out = oracle.transfer(x_in, M, D, dt, kappa=3.0, prec=64, react=None)
    assert out[0, 0] == pytest.approx(1.0 - 0.5 * w / (1 + w), rel=1e-12)
    out = oracle.transfer(x_out, M, D, dt, kappa=3.0, prec=64, react=None)
    assert out[0, 0] == 1.0 and out[0, 1] == 0.0


def test_coincident_cluster_relaxes_halfway_to_its_mean():
    # k coincident particles far from everything else: all weights 1, r = k,
    # P_ij = 1/k, so dM_i = (mean - M_i)/2 and M_i' = (M_i + mean)/2.
    k = 7
    rng = np.random.default_rng(5)
    x = np.concatenate([np.full((k, 2), 0.3), np.array([[0.9, 0.9], [0.95, 0.1]])])
    M = rng.random((2, k + 2))
    for norm in (oracle.NORM_SYM, oracle.NORM_ROW):
        out = oracle.transfer(x, M, 1e-5, 0.1, kappa=3.0, norm=norm, prec=32, react=None)
        mean = M[:, :k].mean(axis=1, keepdims=True)
        assert np.allclose(out[:, :k], 0.5 * (M[:, :k] + mean), rtol=1e-14, atol=0)
        # the two far particles are isolated: no change
        assert np.array_equal(out[:, k:], M[:, k:])


def test_uniform_masses_do_not_move():
    x = W.positions(500, 2, 3)
    M = np.full((2, 500), 0.125)
    out = oracle.transfer(x, M, 1e-3, 0.1, kappa=3.0, react=None)
    assert np.array_equal(out, M)


def test_zero_diffusion_is_a_no_op():
    x = W.positions(100, 1, 3)
    M = W.masses(100, 2, 3)
    out = oracle.transfer(x, M, 0.0, 0.1, kappa=3.0, react=None)
    assert np.array_equal(out, M)


def test_well_mixed_limit_halves_deviation_each_step():
    # When every pair has weight 1 (kernel much wider than the box), P_ij = 1/N
    # and M(n) - mean = 2^-n (M(0) - mean).
    n = 300
    x = W.positions(n, 2, 9)
    M0 = W.masses(n, 2, 9)
    M = M0.copy()
    D, dt = 1e12, 0.1
    for step in range(1, 9):
        M = oracle.transfer(x, M, D, dt, kappa=math.inf, react=None)
        mean = M0.mean(axis=1, keepdims=True)
        assert np.allclose(M - mean, 2.0 ** -step * (M0 - mean), rtol=0, atol=1e-12 * abs(M0).max())


# ------------------------------------------------------------ invariants ----

def _case(n=800, d=2, seed=21):
    x = f32(W.positions(n, d, seed))
    M = W.masses(n, 2, seed)
    return x, M


def test_sym_conserves_mass_and_row_does_not():
    x, M = _case()
    D, dt = 2e-4, 0.1
    Ms, Mr = M.copy(), M.copy()
    for _ in range(20):
        Ms = oracle.transfer(x, Ms, D, dt, kappa=3.0, norm=oracle.NORM_SYM, prec=32, react=None)
        Mr = oracle.transfer(x, Mr, D, dt, kappa=3.0, norm=oracle.NORM_ROW, prec=32, react=None)
    tot0 = oracle.audit(M, None)[:2]
    assert np.allclose(oracle.audit(Ms, None)[:2], tot0, rtol=1e-13, atol=0)
    # the literal row normalisation is not symmetric, so mass drifts
    assert np.max(np.abs(oracle.audit(Mr, None)[:2] - tot0) / tot0) > 1e-6


def test_sym_conserves_mass_over_a_walked_run():
    # Sec. 2.1: the symmetric exchange moves mass between pairs only, so the
    # totals of a walk + transfer run stay put to rounding (no reaction).
    n = 600
    x = W.positions(n, 2, 31)
    M = W.masses(n, 2, 31)
    ids = np.arange(n, dtype=np.uint32)
    tot0 = oracle.audit(M, None)[:2]
    for k in range(40):
        x = oracle.walk(x, ids, 77, k, 5e-4, 0.1, lo=(0, 0), hi=(1, 1))
        M = oracle.transfer(x, M, 5e-4, 0.1, kappa=3.0, norm=oracle.NORM_SYM, prec=64, react=None)
    assert np.all(np.abs(oracle.audit(M, None)[:2] - tot0) <= 1e-12 * tot0)
    assert np.max(np.abs(M - W.masses(n, 2, 31))) > 1e-2 * np.max(M)


def test_transfer_is_linear_in_mass():
    x, M = _case()
    M2 = W.masses(800, 2, 99)
    a, b = 0.75, -2.5
    T = lambda m: oracle.transfer(x, m, 3e-4, 0.1, kappa=3.0, prec=32, react=None)
    assert np.allclose(T(a * M + b * M2), a * T(M) + b * T(M2), rtol=0, atol=1e-15)


def test_permutation_equivariance():
    x, M = _case(n=600, d=3)
    perm = np.random.default_rng(1).permutation(600)
    out = oracle.transfer(x, M, 3e-3, 0.1, kappa=3.0, prec=32)
    outp = oracle.transfer(x[perm], M[:, perm], 3e-3, 0.1, kappa=3.0, prec=32)
    assert np.allclose(outp, out[:, perm], rtol=1e-13, atol=1e-19)


@pytest.mark.parametrize("norm", [oracle.NORM_SYM, oracle.NORM_ROW])
def test_translation_invariance(norm):
    # Eqs. (3)-(6) see positions only through separations.  On a 2^-20 grid
    # both the shift and every separation are exact in binary64, so no pair
    # can cross the cutoff; only the order of the sums may change.
    n, d = 700, 3
    x = np.floor(W.positions(n, d, 8) * 2.0 ** 20) / 2.0 ** 20
    M = W.masses(n, 2, 8)
    shift = np.array([0.375, -0.25, 3.5])
    out = oracle.transfer(x, M, 2e-3, 0.1, kappa=3.0, norm=norm, prec=64)
    outs = oracle.transfer(x + shift, M, 2e-3, 0.1, kappa=3.0, norm=norm, prec=64)
    assert np.max(np.abs(out - M)) > 1e-3 * np.max(M)
    assert np.allclose(outs, out, rtol=1e-13, atol=1e-19)


def test_cutoff_converges_to_full_matrix():
    # The cutoff drops only the kernel mass beyond kappa*sigma, so the gap to
    # the full-matrix brute force shrinks with kappa (Sec. 2.2).
    x, M = _case(n=1000, d=1)
    D, dt = 1e-4, 0.1
    dense = oracle.transfer(x, M, D, dt, kappa=math.inf, react=None)
    gaps = []
    for kappa in (1.5, 2.0, 3.0, 4.0, 7.0):
        sp = oracle.transfer(x, M, D, dt, kappa=kappa, prec=64, react=None)
        gaps.append(np.abs(sp - dense).max() / np.abs(M).max())
    assert all(g1 > g2 for g1, g2 in zip(gaps[:3], gaps[1:4]))
    assert gaps[2] < 1e-4       # kappa = 3
    assert gaps[-1] < 1e-15     # kappa = 7: exp(-49) is below rounding


def test_reaction_leaves_no_coexisting_reactants_and_keeps_a_minus_b():
    x, M = _case()
    D, dt = 2e-4, 0.1
    Mr = M.copy()
    Mlin = M.copy()
    for _ in range(15):
        Mr = oracle.transfer(x, Mr, D, dt, kappa=3.0, prec=32, react=(0, 1))
        Mlin = oracle.transfer(x, Mlin, D, dt, kappa=3.0, prec=32, react=None)
        assert np.all(np.minimum(Mr[0], Mr[1]) == 0.0)
    # A - B evolves by the same linear operator with or without the reaction
    # (the conservative-component argument of Sec. 3), so A = max(delta, 0).
    delta = Mlin[0] - Mlin[1]
    scale = np.abs(M).max()
    assert np.allclose(Mr[0] - Mr[1], delta, rtol=0, atol=1e-14 * scale)
    assert np.allclose(Mr[0], np.maximum(delta, 0), rtol=0, atol=1e-14 * scale)


# ------------------------------------------ independent implementation -----

@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("prec", [32, 64])
def test_neighbor_lists_match_dense_predicate(d, prec):
    n = 700
    x = f32(W.positions(n, d, 40 + d))
    D = {1: 1e-4, 2: 1e-3, 3: 5e-3}[d]
    rowptr, cols = oracle.neighbors(x, 3.0, D, 0.1, prec)
    mask = numpy_ref.neighbor_mask(x, 3.0, D, 0.1, prec)
    assert rowptr[-1] == mask.sum()
    for i in range(n):
        assert np.array_equal(cols[rowptr[i]:rowptr[i + 1]], np.nonzero(mask[i])[0])


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("kappa", [3.0, math.inf])
@pytest.mark.parametrize("norm", ["sym", "row"])
def test_c_oracle_matches_numpy_brute_force(d, kappa, norm):
    n = 500
    x = f32(W.positions(n, d, 60 + d))
    M = W.masses(n, 3, 60 + d)
    D = {1: 1e-4, 2: 1e-3, 3: 5e-3}[d]
    a = oracle.transfer(x, M, D, 0.1, kappa=kappa, prec=32, react=(0, 2),
                        norm=oracle.NORM_SYM if norm == "sym" else oracle.NORM_ROW)
    b = numpy_ref.transfer(x, M, D, 0.1, kappa=kappa, prec=32, react=(0, 2), norm=norm)
    assert np.allclose(a, b, rtol=0, atol=1e-14 * np.abs(M).max())


def test_expected_pair_count_in_unit_square():
    # Unordered pairs within r of i.i.d. uniform points in the unit square:
    # N(N-1)/2 * F2(r), F2(r) = pi r^2 - 8 r^3 / 3 + r^4 / 2 (exact pair-distance CDF).
    n, D, dt = 20000, 1e-5, 0.1
    x = f32(W.positions(n, 2, 77))
    rowptr, _ = oracle.neighbors(x, 3.0, D, dt, 32)
    pairs = (rowptr[-1] - n) / 2
    r = 3 * math.sqrt(8 * D * dt)
    F = math.pi * r * r - 8 * r ** 3 / 3 + r ** 4 / 2
    mean = n * (n - 1) / 2 * F
    assert abs(pairs - mean) < 6 * math.sqrt(mean * (1 + 4 * n * math.pi * r * r))


@pytest.mark.parametrize("n,r", [(20000, 0.05), (3000, 0.3)])
def test_expected_pair_count_in_unit_cube(n, r):
    # The same in the unit cube: F3(r) = 4 pi r^3 / 3 - 3 pi r^4 / 2 + 8 r^5 / 5
    # - r^6 / 6 (r <= 1, from integrating (1 - |u1|)(1 - |u2|)(1 - |u3|) over
    # the ball of radius r).  At r = 0.3 the r^4 wall term shifts the count by
    # about 1.5 bounds, so a formula without it fails.
    dt = 0.1
    D = r * r / (72.0 * dt)  # cutoff 3 sqrt(8 D dt) = r
    x = W.positions(n, 3, 78)
    rowptr, _ = oracle.neighbors(x, 3.0, D, dt, 64)
    pairs = (rowptr[-1] - n) / 2
    F = 4 * math.pi * r ** 3 / 3 - 1.5 * math.pi * r ** 4 + 1.6 * r ** 5 - r ** 6 / 6
    mean = n * (n - 1) / 2 * F
    assert abs(pairs - mean) < 6 * math.sqrt(mean * (1 + 4 * n * F))


# ------------------------------------------------------ paper arithmetic ----

def test_pad_ratios_printed_in_the_paper():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "paper_pad_ratios.txt"))
            if l.strip() and not l.startswith("#")]
    for sec, Dm, dt, kappa, L, P, ratio, tol in rows:
        Dm, dt, kappa, L, P, ratio, tol = map(float, (Dm, dt, kappa, L, P, ratio, tol))
        if sec == "sec6.2":
            # the cutoff this library uses: kappa * sqrt(8 D_m dt); verify that the
            # oracle's neighbour predicate switches exactly there
            pad = kappa * math.sqrt(8 * Dm * dt)
            x = np.array([[0.0], [pad * (1 - 1e-12)], [100.0], [100.0 + pad * (1 + 1e-9)]])
            rowptr, cols = oracle.neighbors(x, kappa, Dm, dt, 64)
            assert list(cols[rowptr[0]:rowptr[1]]) == [0, 1]
            assert list(cols[rowptr[2]:rowptr[3]]) == [2]
        else:
            pad = kappa * math.sqrt(4 * Dm * dt)
        assert abs(pad / (L / P) - ratio) <= tol
    # the combined pads at P = 8 of Sec. 4: "42 %"
    assert abs(2 * 3 * math.sqrt(4 * 0.5 * 0.1) / (50 / 8) - 0.42) < 0.02


# ------------------------------------------------------------------ walk ----

def test_walk_statistics_and_reflection():
    n = 200000
    rng = np.random.default_rng(3)
    x0 = 0.25 + 0.5 * rng.random((n, 2))
    ids = np.arange(n, dtype=np.uint32)
    D_rw, dt = 1e-4, 0.1
    x1 = oracle.walk(x0, ids, seed=12345, step=7, D_rw=D_rw, dt=dt, lo=(0, 0), hi=(1, 1))
    dx = (x1 - x0) / math.sqrt(2 * D_rw * dt)
    assert abs(dx.mean()) < 5 / math.sqrt(dx.size)
    assert abs(dx.var() - 1) < 5 * math.sqrt(2 / dx.size)
    from scipy import stats
    assert stats.kstest(dx[:, 0], "norm").pvalue > 1e-4
    assert stats.kstest(dx[:, 1], "norm").pvalue > 1e-4
    assert abs(np.corrcoef(dx[:, 0], dx[:, 1])[0, 1]) < 5 / math.sqrt(n)
    # reflection at zero-flux walls keeps every particle in the closed box
    xw = oracle.walk(rng.random((n, 2)), ids, seed=1, step=0, D_rw=0.05, dt=0.1, lo=(0, 0), hi=(1, 1))
    assert xw.min() >= 0.0 and xw.max() <= 1.0
    # a particle near the wall reflects: x = 0.001, step -0.004 -> 0.003
    z = oracle.normals(0, 99, 5)
    amp = 0.01 / abs(z[0])
    xr = oracle.walk(np.array([[0.001]]), np.array([0], np.uint32), 99, 5, amp * amp / 0.2, 0.1,
                     lo=(0,), hi=(1,))
    expect = 0.001 + 0.01 * np.sign(z[0])
    assert xr[0, 0] == pytest.approx(expect if expect >= 0 else -expect, abs=1e-15)


def test_walk_normals_independent_across_dimensions():
    # Box-Muller (Box & Muller, 1958) on two independent uniform pairs gives
    # three independent standard normals per particle and step.
    z = np.array([oracle.normals(i, 2024, 11) for i in range(60000)])
    assert np.all(np.abs(z.mean(axis=0)) < 5 / math.sqrt(len(z)))
    assert np.all(np.abs(z.var(axis=0) - 1) < 5 * math.sqrt(2 / len(z)))
    c = np.corrcoef(z.T)
    assert np.all(np.abs(c[np.triu_indices(3, 1)]) < 5 / math.sqrt(len(z)))
    # squares are uncorrelated too (a shared uniform would correlate them)
    c2 = np.corrcoef((z * z).T)
    assert np.all(np.abs(c2[np.triu_indices(3, 1)]) < 6 / math.sqrt(len(z)))
    from scipy import stats
    for k in range(3):
        assert stats.kstest(z[:, k], "norm").pvalue > 1e-4


def test_walk_draws_depend_only_on_id_step_seed():
    a = oracle.normals(17, 5, 3)
    b = oracle.normals(17, 5, 3)
    c = oracle.normals(17, 5, 4)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


# ----------------------------------------------- the transfer operator T ----
# One step with fixed positions is M' = M T^T for a matrix T that does not
# depend on M (linearity); transferring the unit masses e_j (as N species)
# gives T column by column.

def _operator(x, D, dt, norm, kappa=3.0):
    # rows of the result are unit-mass species: entry (j, i) = T_ij
    n = x.shape[0]
    eye = np.eye(n)
    blocks = [oracle.transfer(x, eye[b:b + 64], D, dt, kappa=kappa, norm=norm, prec=64, react=None)
              for b in range(0, n, 64)]
    return np.concatenate(blocks, axis=0)


@pytest.mark.parametrize("d", [1, 2])
def test_transfer_operator_symmetry_and_unit_sums(d):
    n = 60
    x = W.positions(n, d, 70 + d)
    D, dt = 4e-3, 0.1
    Ts = _operator(x, D, dt, oracle.NORM_SYM)
    Tr = _operator(x, D, dt, oracle.NORM_ROW)
    # SYM: P_ij = P_ji is computed identically from both ends, so T is
    # symmetric bit for bit; its rows and columns sum to 1 (uniform masses
    # stay put, total mass is conserved)
    assert np.array_equal(Ts, Ts.T)
    assert np.allclose(Ts.sum(axis=0), 1.0, rtol=0, atol=1e-15)
    assert np.allclose(Ts.sum(axis=1), 1.0, rtol=0, atol=1e-15)
    # ROW: rows still sum to 1, columns do not (mass is not conserved)
    assert np.allclose(Tr.sum(axis=0), 1.0, rtol=0, atol=1e-15)
    assert np.abs(Tr.sum(axis=1) - 1.0).max() > 1e-4
    # the row sums r_i include the self weight
    _, r = oracle.transfer(x, W.masses(n, 2, 1), D, dt, kappa=3.0, prec=64, react=None, return_r=True)
    assert np.all(r >= 1.0)


def test_mixing_limited_decay_matches_its_exact_expectation():
    # A - B = delta evolves by T with or without the reaction, and after the
    # reaction A = max(delta, 0).  With Gaussian mass fluctuations delta(0) has
    # independent entries of variance v0 = 2 (0.1 / N)^2 and mean 0, so
    # E[sum_i A_i(n)] = sqrt(v0 / 2 pi) sum_i || row i of T^n ||_2  exactly,
    # for fixed positions.  The oracle with the reaction is checked against
    # this over independent mass draws (statistically, within 4 standard
    # errors), which pins transfer and reaction together.
    n, D, dt, steps, draws = 120, 3.5e-4, 0.1, 8, 400
    x = W.positions(n, 1, 77)
    T = _operator(x, D, dt, oracle.NORM_SYM).T   # M' = T M for one species row
    v0 = 2.0 * (0.1 / n) ** 2
    expect, Tn = [], np.eye(n)
    for _ in range(steps):
        Tn = T @ Tn
        expect.append(math.sqrt(v0 / (2.0 * math.pi)) * np.linalg.norm(Tn, axis=1).sum())
    sums = np.zeros((draws, steps))
    for k in range(draws):
        M = W.masses(n, 2, 1000 + k)
        for s in range(steps):
            M = oracle.transfer(x, M, D, dt, kappa=3.0, prec=64, react=(0, 1))
            sums[k, s] = M[0].sum()
    mean = sums.mean(axis=0)
    se = sums.std(axis=0, ddof=1) / math.sqrt(draws)
    assert np.all(np.abs(mean - np.array(expect)) < 4.0 * se)
    # and the decay is monotone
    assert np.all(np.diff(expect) < 0)


def test_well_mixed_decay_reaches_the_global_excess():
    # every weight 1: delta relaxes to its mean by 2^-n, so sum A -> max(sum delta, 0)
    n = 200
    x = W.positions(n, 2, 5)
    for seed in (3, 4):
        M = W.masses(n, 2, seed)
        excess = max((M[0] - M[1]).sum(), 0.0)
        for _ in range(45):
            M = oracle.transfer(x, M, 1e12, 0.1, kappa=math.inf, react=(0, 1))
        assert abs(M[0].sum() - excess) < 1e-13 * np.abs(M).sum()
        assert abs(M[1].sum() - max(-(M[0] - M[1]).sum(), 0.0)) < 1e-13 * np.abs(M).sum()


@pytest.mark.parametrize("d", [1, 2, 3])
def test_cutoff_gap_is_bounded_by_the_neglected_kernel_mass(d):
    # w = exp(-s^2 / sigma^2) is a Gaussian of variance sigma^2 / 2 per axis;
    # the fraction of its mass beyond s = 3 sigma is erfc(3) in 1-D, e^-9 in
    # 2-D and erfc(3) + (6 / sqrt(pi)) e^-9 in 3-D.  Dropping it changes each
    # transfer by at most that fraction of the mass differences.
    from scipy.special import erfc
    n = {1: 1000, 2: 1500, 3: 1500}[d]
    x = f32(W.positions(n, d, 50 + d))
    M = W.masses(n, 2, 50 + d)
    rc = {1: 0.03, 2: 0.08, 3: 0.2}[d]
    D = (rc / 3.0) ** 2 / (8 * 0.1)
    dense = oracle.transfer(x, M, D, 0.1, kappa=math.inf, react=None)
    sparse = oracle.transfer(x, M, D, 0.1, kappa=3.0, prec=64, react=None)
    gap = np.abs(sparse - dense).max() / np.abs(M).max()
    tail = {1: erfc(3.0), 2: math.exp(-9.0), 3: erfc(3.0) + 6.0 / math.sqrt(math.pi) * math.exp(-9.0)}[d]
    assert tail / 1000 < gap < tail


# ------------------------------------------------- row-subset modes ----------

@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("kappa", [3.0, math.inf])
@pytest.mark.parametrize("norm", [oracle.NORM_SYM, oracle.NORM_ROW])
@pytest.mark.parametrize("react", [(0, 1), None])
def test_transfer_row_subset_equals_the_full_output(d, kappa, norm, react):
    # The explicit transfer of Eqs. (3)-(6) computes every particle's new
    # masses from the same beginning-of-step state, so asking for a subset of
    # rows (in any order, with repeats) must give exactly those columns of the
    # full output, bit for bit; the row sums stay those of all particles.
    n, S = {1: 700, 2: 900, 3: 800}[d], 3
    D, dt = {1: 2e-4, 2: 1e-3, 3: 4e-3}[d], 0.1
    x = f32(W.positions(n, d, 90 + d))
    M = W.masses(n, S, 90 + d)
    full, r_full = oracle.transfer(x, M, D, dt, kappa=kappa, norm=norm, prec=32, react=react, return_r=True)
    rng = np.random.default_rng(91 + d)
    rows = np.concatenate([rng.choice(n, 60, replace=False)[::-1], [n - 1, 0, 5, 5, n - 1]])
    sub, r_sub = oracle.transfer(x, M, D, dt, kappa=kappa, norm=norm, prec=32, react=react, rows=rows,
                                 return_r=True)
    assert sub.shape == (S, rows.size)
    assert np.array_equal(sub, full[:, rows])
    assert np.array_equal(r_sub, r_full)
    # an index slip would move a value to another column: every column differs
    assert len({tuple(full[:, i]) for i in range(n)}) == n


def test_transfer_row_subset_rejects_rows_outside_the_ensemble():
    x = W.positions(50, 2, 1)
    M = W.masses(50, 2, 1)
    for bad in ([0, 50], [-1], [3, 7, 1 << 40]):
        with pytest.raises(ValueError):
            oracle.transfer(x, M, 1e-3, 0.1, rows=np.array(bad))
    with pytest.raises(ValueError):
        oracle.neighbors(x, 3.0, 1e-3, 0.1, rows=np.array([0, 50]))
    assert oracle.transfer(x, M, 1e-3, 0.1, rows=np.array([], dtype=np.int64)).shape == (2, 0)


@pytest.mark.parametrize("d,prec", [(1, 32), (2, 32), (2, 64), (3, 32)])
def test_neighbor_row_subset_equals_the_full_lists(d, prec):
    # the row-subset export lists exactly the full lists' rows, in the order asked
    n = {1: 3000, 2: 4000, 3: 4000}[d]
    D, dt = {1: 1e-4, 2: 5e-4, 3: 3e-3}[d], 0.1
    x = f32(W.positions(n, d, 70 + d))
    rp, cols = oracle.neighbors(x, 3.0, D, dt, prec)
    rows = np.random.default_rng(d).choice(n, 300, replace=False)
    rows = np.concatenate([rows, rows[:7]])
    rp_s, cols_s = oracle.neighbors(x, 3.0, D, dt, prec, rows=rows)
    assert rp_s.size == rows.size + 1
    for t, i in enumerate(rows):
        assert np.array_equal(cols_s[rp_s[t]:rp_s[t + 1]], cols[rp[i]:rp[i + 1]])
