"""Pins of the oracle's advective walk (Eq. 1, Eq. 2): a constant velocity v
and hydrodynamic dispersion alpha_T |v| I + (alpha_L - alpha_T) v v^T / |v| on
top of the isotropic walk share D_rw.

The displacement of one step is Gaussian with mean v dt and covariance
2 dt [(D_rw + alpha_T |v|) I + (alpha_L - alpha_T) v v^T / |v|]; an advected
segregated interface follows C1 = erfc((x0 + v t - x) / sqrt(4 D t)) / 2 with
D = D_m + D_rw + alpha_L |v| (1-D, the paper's Eq. (2) plus the transfer)."""
import math

import numpy as np
from scipy.special import erfc

import oracle
from paper_1811_05474_amd import workloads as W


def test_zero_velocity_is_the_plain_walk_bit_for_bit():
    x = W.positions(2000, 3, 1)
    ids = np.arange(2000)
    a = oracle.walk(x, ids, 5, 3, 2e-4, 0.1, (0, 0, 0), (1, 1, 1))
    b = oracle.walk(x, ids, 5, 3, 2e-4, 0.1, (0, 0, 0), (1, 1, 1), velocity=(0, 0, 0), alpha_l=0.3, alpha_t=0.1)
    assert np.array_equal(a, b)


def test_step_moments_along_and_across_the_flow():
    n, dt, Drw = 200000, 0.1, 0.05
    v = np.array([0.6, 0.8])
    aL, aT = 0.5, 0.1
    x0 = np.full((n, 2), 500.0)        # far from the walls of a large box
    x1 = oracle.walk(x0, np.arange(n), 11, 0, Drw, dt, (0, 0), (1000, 1000), velocity=v, alpha_l=aL, alpha_t=aT)
    dx = x1 - x0
    speed = np.linalg.norm(v)
    u = v / speed
    perp = np.array([-u[1], u[0]])
    along, across = dx @ u, dx @ perp
    var_l = 2 * dt * (Drw + aL * speed)
    var_t = 2 * dt * (Drw + aT * speed)
    se = lambda var: math.sqrt(var / n)
    assert abs(along.mean() - speed * dt) < 5 * se(var_l)
    assert abs(across.mean()) < 5 * se(var_t)
    # sample variances within 5 standard errors (sqrt(2 / n) relative)
    assert abs(along.var() / var_l - 1) < 5 * math.sqrt(2.0 / n)
    assert abs(across.var() / var_t - 1) < 5 * math.sqrt(2.0 / n)
    assert abs(np.mean(along * across)) < 5 * math.sqrt(var_l * var_t / n)


def advected_interface_rmse(alpha_walk, v_walk, seed):
    L, dt, steps, n, x0 = 50.0, 0.1, 100, 4000, 10.0
    Dm, Drw, v, aL = 0.5, 0.5, 1.0, 1.0
    x, M = W.interface(n, 1, L, seed, x0=x0)
    ds = L / n
    ids = np.arange(n, dtype=np.uint32)
    for s in range(steps):
        x = oracle.walk(x, ids, seed, s, Drw, dt, (0.0,), (L,), velocity=(v_walk,), alpha_l=alpha_walk)
        M = oracle.transfer(x, M, Dm, dt, kappa=3.0, prec=64, react=None)
    t = steps * dt
    front = x0 + v * t
    sel = np.abs(x[:, 0] - front) < 8.0   # the front, away from both walls
    exact = 0.5 * erfc((front - x[sel, 0]) / math.sqrt(4 * (Dm + Drw + aL * v) * t))
    return math.sqrt(np.mean((M[0][sel] / ds - exact) ** 2))


def test_advected_interface_follows_the_shifted_erfc():
    good = np.mean([advected_interface_rmse(1.0, 1.0, 8000 + r) for r in range(3)])
    assert good < 0.045
    # without the longitudinal dispersion the front is too steep; without the
    # drift it is in the wrong place
    assert np.mean([advected_interface_rmse(0.0, 1.0, 8000 + r) for r in range(3)]) > 0.05
    assert advected_interface_rmse(1.0, 0.0, 8000) > 0.3
