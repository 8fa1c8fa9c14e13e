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


def fma32(a: np.ndarray, b: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Correctly rounded binary32 fma(a, b, c), elementwise.

    a*b of two binary32 values is exact in binary64; the binary64 sum s and its
    exact error e (TwoSum) give a + b*c exactly as s + e.  Rounding s to
    binary32 is correct unless s lies exactly on a binary32 midpoint, where the
    sign of e decides."""
    a = np.asarray(a, dtype=np.float32).astype(np.float64)
    b = np.asarray(b, dtype=np.float32).astype(np.float64)
    c = np.asarray(c, dtype=np.float32).astype(np.float64)
    p = a * b
    s = p + c
    bp = s - p
    e = (p - (s - bp)) + (c - bp)
    f = s.astype(np.float32)
    # neighbours of f in binary32 and the midpoint on the side of s
    up = np.nextafter(f, np.float32(np.inf))
    dn = np.nextafter(f, np.float32(-np.inf))
    other = np.where(s > f.astype(np.float64), up, dn)
    mid = 0.5 * (f.astype(np.float64) + other.astype(np.float64))
    tie = (s == mid) & (e != 0)
    # at an exact tie the true value lies on the side of e
    fix = np.where(e > 0, np.maximum(f, other), np.minimum(f, other))
    return np.where(tie, fix, f).astype(np.float32)


def squared_separation_f32(x: np.ndarray) -> np.ndarray:
    """s_ij^2 in binary32: dx*dx, then fma(dy, dy, .), fma(dz, dz, .)."""
    xf = np.asarray(x, dtype=np.float32)
    acc = None
    for k in range(xf.shape[1]):
        dk = xf[None, :, k] - xf[:, None, k]  # dk[i, j] = x_j - x_i
        acc = dk * dk if acc is None else fma32(dk, dk, acc)
    return acc


def squared_separation_f64(x: np.ndarray) -> np.ndarray:
    """s_ij^2 in binary64 in the same operation order but unfused (each step
    rounded); neighbor_mask re-decides the pairs near the cutoff exactly."""
    xd = np.asarray(x, dtype=np.float64)
    acc = None
    for k in range(xd.shape[1]):
        dk = xd[None, :, k] - xd[:, None, k]
        acc = dk * dk if acc is None else dk * dk + acc
    return acc


def neighbor_mask(x: np.ndarray, kappa: float, D: float, dt: float, prec: int = 32) -> np.ndarray:
    """Boolean N x N mask of pairs within s_max = kappa*sqrt(8 D dt) (Sec. 2.2)."""
    n = x.shape[0]
    if np.isinf(kappa):
        return np.ones((n, n), dtype=bool)
    rc2 = kappa * kappa * (8.0 * D * dt)
    if prec == 32:
        return squared_separation_f32(x) <= np.float32(rc2)
    s2 = squared_separation_f64(x)
    mask = s2 <= rc2
    # pairs within a few ulps of the cutoff: decide with the exactly rounded
    # fma sequence (Fractions), since the unfused binary64 sum above may differ
    near = np.argwhere(np.abs(s2 - rc2) <= 1e-12 * rc2)
    if near.size:
        from fractions import Fraction
        xd = np.asarray(x, dtype=np.float64)
        for i, j in near:
            acc = None
            for k in range(xd.shape[1]):
                d = float(xd[j, k] - xd[i, k])
                acc = d * d if acc is None else float(Fraction(d) * Fraction(d) + Fraction(acc))
            mask[i, j] = acc <= rc2
    return mask


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
