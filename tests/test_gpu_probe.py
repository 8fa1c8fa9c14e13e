"""GPU: the instruction-rate probes (rwpt_probe_rate) return rates consistent
with the device and with each other, and the row-broadcast pair kernels do
not run faster than the attainable rate of their own inner loop."""
import numpy as np
import pytest

from paper_1811_05474_amd import rwpt, workloads as W

pytestmark = pytest.mark.gpu

# binary32 FMA issue on gfx950: 256 CUs x 4 SIMDs x 16 lanes per cycle at up
# to 2.4 GHz = 3.9e13 lane operations/s (non-packed)
FMA_CEILING = 256 * 64 * 2.4e9


def test_probe_rates_are_consistent():
    ens = rwpt.Ensemble(dim=2, n_species=2, react=(0, 1), kappa=3.0, precision=rwpt.RWPT_FP32)
    try:
        fma = ens.probe_rate(rwpt.RWPT_PROBE_FMA)
        ex = ens.probe_rate(rwpt.RWPT_PROBE_EXP)
        rs = ens.probe_rate(rwpt.RWPT_PROBE_ROWSUM)
        xc = ens.probe_rate(rwpt.RWPT_PROBE_EXCHANGE)
    finally:
        ens.close()
    print("fma %.3e  exp %.3e  rowsum %.3e  exchange %.3e" % (fma, ex, rs, xc))
    assert 0.25 * FMA_CEILING < fma < 1.1 * FMA_CEILING
    assert 0.0 < ex <= 1.1 * fma
    # at least 8 VALU instructions per row-sum evaluation, more for the exchange
    assert 0.0 < rs < fma / 8.0
    assert 0.0 < xc < rs


def test_rowsum_kernel_below_its_probe():
    """Measured evaluations/s of the row-sum kernel (profiled step of a 2-D
    ensemble of 2^18 particles, row-broadcast tiling) stay below the probe."""
    w = W.WORKLOADS["walk2d_n1e6"]
    n = 1 << 18
    x = W.positions(n, 2, 11)
    M = W.masses(n, 2, 11)
    ens = rwpt.Ensemble(dim=2, n_species=2, react=(0, 1), kappa=3.0, rw_ratio=1.0,
                        precision=rwpt.RWPT_FP32, tile_lanes=4, seed=11)
    try:
        ens.init([n], x, M)
        ens.step(w.dt, w.D, 2)
        rwpt.rwpt_profile_enable(ens.ctx, 1)
        rwpt.rwpt_profile_reset(ens.ctx)
        ens.step(w.dt, w.D, 10)
        st = ens.stats()
        rs_ms, rs_n = st["phases"]["rowsum"]
        ex_ms, ex_n = st["phases"]["exchange"]
        evals = st["candidate_evals"]
        rate_rs = evals * rs_n / (rs_ms * 1e-3)
        rate_ex = evals * ex_n / (ex_ms * 1e-3)
        probe_rs = ens.probe_rate(rwpt.RWPT_PROBE_ROWSUM)
        probe_ex = ens.probe_rate(rwpt.RWPT_PROBE_EXCHANGE)
    finally:
        ens.close()
    print("rowsum %.3e of %.3e, exchange %.3e of %.3e" % (rate_rs, probe_rs, rate_ex, probe_ex))
    assert np.isfinite(rate_rs) and np.isfinite(rate_ex)
    assert 0.0 < rate_rs < 1.05 * probe_rs
    assert 0.0 < rate_ex < 1.05 * probe_ex
