"""The paper's own verification problem (Sec. 3): a segregated interface of
two conservative components diffusing with total D, simulated as mass
transfer with D/2 plus a random walk with D/2.  C1 must approach the
analytical profile C1(x, t) = erfc((x0 - x) / sqrt(4 D t)) / 2 (the printed
formula is garbled; this is its dimensionally consistent reading, with
C1(x, 0) = H(x - x0) as in Sec. 5.1).

This pins the oracle's transfer + walk against a closed form: at N = 2000 the
equal split gives an RMSE near 0.013, while a kernel of the wrong width, a
missing walk or a wrong diffusion split leave errors two to three times
larger (0.027 - 0.038), and the walk alone about 0.22."""
import math

import numpy as np
from scipy.special import erfc

import oracle
from paper_1811_05474_amd import workloads as W

L, DT, STEPS = 50.0, 0.1, 100


def rmse_after(n, D_transfer, D_walk, seed):
    x, M = W.interface(n, 1, L, seed)
    ds = L / n
    ids = np.arange(n, dtype=np.uint32)
    for s in range(STEPS):
        if D_walk > 0:
            x = oracle.walk(x, ids, seed, s, D_walk, DT, (0.0,), (L,))
        M = oracle.transfer(x, M, D_transfer, DT, kappa=3.0, prec=64, react=None)
    exact = 0.5 * erfc((0.5 * L - x[:, 0]) / math.sqrt(4 * 1.0 * STEPS * DT))
    # the conservative components stay complementary: C1 + C2 = 1 everywhere
    assert np.allclose((M[0] + M[1]) / ds, 1.0, atol=1e-9)
    return math.sqrt(np.mean((M[0] / ds - exact) ** 2))


def test_interface_profile_matches_erfc_with_the_equal_split():
    errs = [rmse_after(2000, 0.5, 0.5, 6000 + r) for r in range(4)]
    assert np.mean(errs) < 0.02


def test_transfer_alone_diffuses_with_its_own_coefficient():
    # without the walk, transfer with D_m = 1 alone must give the D = 1 profile:
    # pins the kernel width sigma^2 = 8 D dt of Eq. (3)
    errs = [rmse_after(2000, 1.0, 0.0, 6100 + r) for r in range(4)]
    assert np.mean(errs) < 0.02
    # half the diffusivity in the transfer and no walk is clearly wrong
    bad = [rmse_after(2000, 0.5, 0.0, 6100 + r) for r in range(4)]
    assert np.mean(bad) > 0.03


def test_interface_error_falls_with_particle_number():
    small = np.mean([rmse_after(500, 0.5, 0.5, 6200 + r) for r in range(6)])
    large = np.mean([rmse_after(4000, 0.5, 0.5, 6200 + r) for r in range(6)])
    assert large < small


def rmse_2d(D_transfer, D_walk, seed, n=20000):
    L = 80.0
    x, M = W.interface(n, 2, L, seed)
    ds = L * L / n
    ids = np.arange(n, dtype=np.uint32)
    for s in range(STEPS):
        if D_walk > 0:
            x = oracle.walk(x, ids, seed, s, D_walk, DT, (0.0, 0.0), (L, L))
        M = oracle.transfer(x, M, D_transfer, DT, kappa=3.0, prec=64, react=None)
    exact = 0.5 * erfc((0.5 * L - x[:, 0]) / math.sqrt(4 * 1.0 * STEPS * DT))
    return math.sqrt(np.mean((M[0] / ds - exact) ** 2))


def test_interface_2d_80x80():
    # the 2-D form of the verification problem (80 x 80 box, interface at
    # x = 40): the profile across the interface is the same erfc
    assert rmse_2d(0.5, 0.5, 9000) < 0.02
    assert rmse_2d(1.0, 0.0, 9000) < 0.02       # kernel width in 2-D
    assert rmse_2d(0.5, 0.0, 9000) > 0.03       # missing walk
