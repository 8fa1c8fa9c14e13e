"""Dense NumPy brute force of the explicit mass-transfer step (small N only).

TEST INFRASTRUCTURE ONLY -- a second, separately written implementation of
Eqs. (3)-(6) of arXiv:1811.05474 used to cross-check the C oracle.  It builds
the full N x N matrices the paper's "brute force" description names (Sec. 1.1):
the separation matrix s, the weights nu (Eq. 3, prefactor dropped because the
normalisation cancels it), the normalised P, and dM via Eq. (4).  Memory is
O(N^2); keep N <= ~3000.
"""
from __future__ import annotations

import numpy as np


def squared_separation_f32(x: np.ndarray) -> np.ndarray:
    """s_ij^2 evaluated in binary32 in dimension order, each op rounded."""
    xf = np.asarray(x, dtype=np.float32)
    acc = None
    for k in range(xf.shape[1]):
        dk = xf[None, :, k] - xf[:, None, k]  # dk[i, j] = x_j - x_i
        sq = dk * dk
        acc = sq if acc is None else acc + sq
    return acc


def squared_separation_f64(x: np.ndarray) -> np.ndarray:
    xd = np.asarray(x, dtype=np.float64)
    acc = None
    for k in range(xd.shape[1]):
        dk = xd[None, :, k] - xd[:, None, k]
        sq = dk * dk
        acc = sq if acc is None else acc + sq
    return acc


def neighbor_mask(x: np.ndarray, kappa: float, D: float, dt: float, prec: int = 32) -> np.ndarray:
    """Boolean N x N mask of pairs within s_max = kappa*sqrt(8 D dt) (Sec. 2.2)."""
    n = x.shape[0]
    if np.isinf(kappa):
        return np.ones((n, n), dtype=bool)
    rc2 = kappa * kappa * (8.0 * D * dt)
    if prec == 32:
        return squared_separation_f32(x) <= np.float32(rc2)
    return squared_separation_f64(x) <= rc2


def transfer(x: np.ndarray, M: np.ndarray, D: float, dt: float, kappa: float = np.inf,
             norm: str = "sym", prec: int = 64, react=(0, 1)) -> np.ndarray:
    """One explicit transfer + reaction step, dense matrices, FP64 weights.

    x: (n, d); M: (S, n).  norm 'row' is P_ij = nu_ij / sum_j nu_ij as printed;
    'sym' is (P + P^T)/2."""
    x = np.asarray(x, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    if D == 0.0:
        out = M.copy()
    else:
        s2 = squared_separation_f64(x)
        nu = np.exp(-s2 / (8.0 * D * dt))
        nu = np.where(neighbor_mask(x, kappa, D, dt, prec), nu, 0.0)
        rsum = nu.sum(axis=1)
        P = nu / rsum[:, None]
        if norm == "sym":
            P = 0.5 * (P + P.T)
        # Eq. (4): dM_i = 1/2 sum_j P_ij (M_j - M_i), for each species
        dM = np.empty_like(M)
        for s in range(M.shape[0]):
            diff = M[s][None, :] - M[s][:, None]
            dM[s] = 0.5 * (P * diff).sum(axis=1)
        out = M + dM
    if react is not None and react[0] >= 0:
        a, b = react
        m = np.maximum(0.0, np.minimum(out[a], out[b]))
        out[a] = out[a] - m
        out[b] = out[b] - m
    return out
