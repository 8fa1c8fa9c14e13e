"""The allocation-free transfer (rwpt_transfer_noalloc) against rwpt_step.

For callers that cannot allocate: one explicit transfer step of a single
realisation in caller device arrays, all intermediates in the library's fixed
scratch area.  It runs the kernels of rwpt_step, so on the same inputs (walk
off) its masses must match rwpt_step's to the path's bar (1e-5 binary32,
1e-12 binary64; they are expected bitwise equal).  Two calls in a row, the
second smaller, check that the scratch area's leftovers from the first call
do not leak into the second.
"""
import math

import numpy as np
import pytest

from paper_1811_05474_amd import rwpt, workloads as W

pytestmark = pytest.mark.gpu

F32 = rwpt.RWPT_FP32
F64 = rwpt.RWPT_FP64


def config(dim, S, prec, lanes, react=(0, 1), norm=rwpt.RWPT_NORM_SYM):
    cfg = rwpt.rwpt_config_default()
    cfg.dim = dim
    cfg.n_species = S
    cfg.react_a, cfg.react_b = (-1, -1) if react is None else react
    cfg.kappa = 3.0
    cfg.rw_ratio = 0.0
    cfg.precision = prec
    cfg.norm = norm
    cfg.tile_lanes = lanes
    cfg.seed = 5
    return cfg


def with_context(cfg, x, M, dt, D):
    """Masses after one rwpt_step of a context on the same inputs."""
    ens = rwpt.Ensemble(dim=cfg.dim, n_species=cfg.n_species,
                        react=None if cfg.react_a < 0 else (cfg.react_a, cfg.react_b), kappa=cfg.kappa,
                        rw_ratio=0.0, precision=cfg.precision, norm=cfg.norm, tile_lanes=cfg.tile_lanes,
                        seed=cfg.seed)
    ens.init([x.shape[0]], x, M)
    ens.step(dt, D, 1)
    out = ens.masses()
    ens.close()
    return out


def without_allocation(cfg, x, M, dt, D):
    import torch

    dt_t = torch.float32 if cfg.precision == F32 else torch.float64
    pos = torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dt_t).contiguous()
    m_in = torch.from_numpy(np.ascontiguousarray(M)).to(device="cuda", dtype=dt_t).contiguous()
    m_out = torch.full_like(m_in, float("nan"))
    torch.cuda.synchronize()
    rwpt.rwpt_transfer_noalloc(cfg, x.shape[0], pos.data_ptr(), m_in.data_ptr(), m_out.data_ptr(), dt, D)
    torch.cuda.synchronize()
    return m_out.double().cpu().numpy()


# (dim, species, precision, lanes): the default tilings of each dimension and
# precision (row-broadcast four-lane tiles, one lane per particle, vector-load
# tiles) and a forced one-lane-per-particle 2-D case with the row normalisation
CASES = [(2, 2, F32, 0, rwpt.RWPT_NORM_SYM), (3, 8, F32, 0, rwpt.RWPT_NORM_SYM), (1, 2, F32, 0, rwpt.RWPT_NORM_SYM),
         (2, 2, F64, 0, rwpt.RWPT_NORM_SYM), (3, 3, F64, 0, rwpt.RWPT_NORM_SYM), (1, 1, F64, 0, rwpt.RWPT_NORM_SYM),
         (2, 2, F32, -1, rwpt.RWPT_NORM_ROW)]


@pytest.mark.parametrize("dim,S,prec,lanes,norm", CASES)
def test_noalloc_matches_step_on_two_calls_the_second_smaller(dim, S, prec, lanes, norm):
    import torch

    assert torch.cuda.is_available()
    dt = 0.1
    bar = 1e-5 if prec == F32 else 1e-12
    react = (0, 1) if S >= 2 else None
    cfg = config(dim, S, prec, lanes, react=react, norm=norm)
    for call, (n, mean_nb, seed) in enumerate(((60000, 40.0, 31), (7001, 12.0, 32))):
        unit = {1: 2.0, 2: math.pi, 3: 4.0 * math.pi / 3.0}[dim]
        rc = (mean_nb / ((n - 1) * unit)) ** (1.0 / dim)
        D = rc * rc / (72.0 * dt)
        x = W.positions(n, dim, seed + dim)
        M = W.masses(n, S, seed + dim)
        if prec == F32:
            x = x.astype(np.float32).astype(np.float64)
            M = M.astype(np.float32).astype(np.float64)
        ref = with_context(cfg, x, M, dt, D)
        got = without_allocation(cfg, x, M, dt, D)
        assert np.all(np.isfinite(got))
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print("call %d: n %d, dim %d, S %d, binary%d, lanes %d: normwise difference %.3e (bar %.0e), bitwise equal %s"
              % (call, n, dim, S, 32 if prec == F32 else 64, lanes, err, bar, np.array_equal(got, ref)))
        assert err < bar


def test_noalloc_refuses_what_exceeds_its_scratch_area():
    # 3-D binary64 with eight species needs a few hundred bytes per particle:
    # 10^6 particles exceed the fixed area and are refused before any launch
    cfg = config(3, 8, F64, 0)
    with pytest.raises(rwpt.RwptError) as ei:
        rwpt.rwpt_transfer_noalloc(cfg, 1_000_000, 1, 2, 3, 0.1, 1e-6)
    assert ei.value.status == rwpt.RWPT_EUNSUPPORTED and "scratch" in str(ei.value)
