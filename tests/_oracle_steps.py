"""The oracle's own trajectory of walk + transfer steps, for the replay tests.

Every input of every step comes from the oracle itself (the previous step's
positions and masses), never from the GPU path.  In the binary32 form the
walked positions are rounded to binary32 after every move, as that path stores
them; the remaining differences from the GPU (an ulp of position per move,
the hardware transcendentals of its Box-Muller) are covered by the tolerances
the tests state."""
import numpy as np

import oracle


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def steps(x, M, n_steps, D, dt, seed, lo, hi, prec32, sizes=None, d_scale=None, rw=1.0, kappa=3.0,
          norm=None, react=(0, 1), step0=0, velocity=None, alpha_l=0.0, alpha_t=0.0, rows=None):
    """Yields (positions, masses) after each of n_steps steps.

    x: (N, d) positions and M: (S, N) masses in the caller's order, with
    realisations of `sizes` (default one) laid out one after the other; particle
    i has Philox id i (its global index).  D is the transfer coefficient of
    realisation r times d_scale[r]; the walk uses rw times that.  rows (one
    realisation only): the masses of these particles only (the row sums still
    cover every particle)."""
    n = x.shape[0]
    sizes = [n] if sizes is None else [int(s) for s in sizes]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    scale = np.ones(len(sizes)) if d_scale is None else np.asarray(d_scale, dtype=np.float64)
    kw = {} if norm is None else {"norm": norm}
    xc, mc = np.array(x, dtype=np.float64), np.array(M, dtype=np.float64)
    for k in range(n_steps):
        xn = np.empty_like(xc)
        mn = np.empty_like(mc)
        for r in range(len(sizes)):
            b, e = int(off[r]), int(off[r + 1])
            if e == b:
                continue
            Dr = D * scale[r]
            if rw > 0.0:
                w = oracle.walk(xc[b:e], np.arange(b, e, dtype=np.uint32), seed, step0 + k, rw * Dr, dt, lo, hi,
                                velocity=velocity, alpha_l=alpha_l, alpha_t=alpha_t)
                xn[b:e] = f32(w) if prec32 else w
            else:
                xn[b:e] = xc[b:e]
            if rows is not None and k == n_steps - 1:
                assert len(sizes) == 1
                yield xn, oracle.transfer(xn, mc, Dr, dt, kappa=kappa, prec=32 if prec32 else 64,
                                          react=react, rows=rows, **kw)
                return
            mn[:, b:e] = oracle.transfer(xn[b:e], mc[:, b:e], Dr, dt, kappa=kappa, prec=32 if prec32 else 64,
                                         react=react, **kw)
        xc, mc = xn, mn
        yield xc, mc
