"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/rwpt.h declares, and validates arguments before any
device work."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_1811_05474_amd import rwpt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(rwpt.LIB_PATH):
        from paper_1811_05474_amd import _build
        _build.build()
    return rwpt.load_library()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rwpt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rwpt_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(rwpt.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert "gfx950" in rwpt.rwpt_version()


def test_config_struct_matches_c_layout(lib):
    cfg = rwpt.rwpt_config_default()
    assert cfg.dim == 2 and cfg.n_species == 2 and cfg.react_a == 0 and cfg.react_b == 1
    assert cfg.kappa == 3.0 and cfg.rw_ratio == 1.0 and cfg.use_graph == 1
    assert list(cfg.box_hi) == [1.0, 1.0, 1.0]


@pytest.mark.parametrize("field,value", [
    ("dim", 0), ("dim", 4), ("n_species", 0), ("n_species", 9), ("react_a", 5), ("kappa", 0.0),
    ("kappa", -1.0), ("kappa", float("nan")), ("rw_ratio", -1.0), ("precision", 2), ("norm", 3),
    ("path", 7), ("tile_lanes", 3), ("tile_lanes", 32), ("tile_lanes", -3), ("tile_lanes", 2), ("device", -1), ("use_graph", 2),
    ("alpha_t", -0.1), ("alpha_l", float("nan")),
])
def test_create_rejects_bad_config(lib, field, value):
    cfg = rwpt.rwpt_config_default()
    setattr(cfg, field, value)
    with pytest.raises(rwpt.RwptError) as ei:
        rwpt.rwpt_create(cfg)
    assert ei.value.status == rwpt.RWPT_EINVAL
    assert rwpt.rwpt_last_error(None)


def test_advection_defaults_and_validation(lib):
    cfg = rwpt.rwpt_config_default()
    assert list(cfg.velocity) == [0.0, 0.0, 0.0] and cfg.alpha_l == 0.0 and cfg.alpha_t == 0.0
    cfg.velocity[1] = float("inf")
    with pytest.raises(rwpt.RwptError):
        rwpt.rwpt_create(cfg)
    cfg = rwpt.rwpt_config_default()
    cfg.alpha_l, cfg.alpha_t = 0.1, 0.2   # alpha_l < alpha_t
    with pytest.raises(rwpt.RwptError):
        rwpt.rwpt_create(cfg)
    cfg.alpha_l = 0.3
    rwpt.rwpt_destroy(rwpt.rwpt_create(cfg))


def test_create_rejects_bad_box_and_reaction(lib):
    cfg = rwpt.rwpt_config_default()
    cfg.box_lo[1] = 2.0
    with pytest.raises(rwpt.RwptError):
        rwpt.rwpt_create(cfg)
    cfg = rwpt.rwpt_config_default()
    cfg.react_a, cfg.react_b = 1, 1
    with pytest.raises(rwpt.RwptError):
        rwpt.rwpt_create(cfg)
    cfg = rwpt.rwpt_config_default()
    cfg.react_a, cfg.react_b = 0, -1
    with pytest.raises(rwpt.RwptError):
        rwpt.rwpt_create(cfg)


def test_create_accepts_infinite_kappa_and_touches_no_device(lib):
    cfg = rwpt.rwpt_config_default()
    cfg.kappa = math.inf
    ctx = rwpt.rwpt_create(cfg)
    rwpt.rwpt_destroy(ctx)


def test_validation_before_device(lib):
    ctx = rwpt.rwpt_create(rwpt.rwpt_config_default())
    try:
        x = np.full((4, 2), 0.5)
        M = np.ones((2, 4))
        # state errors
        with pytest.raises(rwpt.RwptError) as ei:
            rwpt.rwpt_step(ctx, 0.1, 1e-5, 1)
        assert ei.value.status == rwpt.RWPT_ESTATE
        with pytest.raises(rwpt.RwptError) as ei:
            rwpt.rwpt_step(ctx, 0.0, 1e-5, 1)
        assert ei.value.status == rwpt.RWPT_EINVAL
        with pytest.raises(rwpt.RwptError) as ei:
            rwpt.rwpt_step(ctx, 0.1, -1.0, 1)
        assert ei.value.status == rwpt.RWPT_EINVAL
        # input errors are reported before any device call
        bad = x.copy()
        bad[2, 1] = 1.5
        with pytest.raises(rwpt.RwptError) as ei:
            rwpt.rwpt_init_ensemble(ctx, [4], bad, M)
        assert ei.value.status == rwpt.RWPT_EINVAL and "outside" in str(ei.value)
        bad = x.copy()
        bad[0, 0] = float("nan")
        with pytest.raises(rwpt.RwptError):
            rwpt.rwpt_init_ensemble(ctx, [4], bad, M)
        badm = M.copy()
        badm[1, 3] = float("inf")
        with pytest.raises(rwpt.RwptError):
            rwpt.rwpt_init_ensemble(ctx, [4], x, badm)
        with pytest.raises(rwpt.RwptError):
            rwpt.rwpt_init_ensemble(ctx, [-1, 5], np.full((4, 2), 0.5), np.ones((2, 4)))
        with pytest.raises(rwpt.RwptError):
            rwpt.rwpt_init_ensemble(ctx, [4], x, M, d_scale=[-2.0])
    finally:
        rwpt.rwpt_destroy(ctx)


def test_valid_init_without_gpu_reports_device_error(lib):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except Exception:
        pass
    ctx = rwpt.rwpt_create(rwpt.rwpt_config_default())
    try:
        with pytest.raises(rwpt.RwptError) as ei:
            rwpt.rwpt_init_ensemble(ctx, [4], np.full((4, 2), 0.5), np.ones((2, 4)))
        assert ei.value.status == rwpt.RWPT_EDEVICE
    finally:
        rwpt.rwpt_destroy(ctx)


def test_destroy_null_is_allowed(lib):
    lib.rwpt_destroy(None)


def test_stats_struct_matches_c_layout(lib):
    # offsets of the C struct: 4 x 8-byte header fields, 3 doubles, 4 int64,
    # two int32, 16 doubles, 16 int64
    assert ctypes.sizeof(rwpt.rwpt_stats_t) == 8 + 4 + 4 + 24 + 8 * 4 + 4 + 4 + 16 * 8 + 16 * 8
    ctx = rwpt.rwpt_create(rwpt.rwpt_config_default())
    try:
        st = rwpt.rwpt_stats(ctx)  # before init: no device work
        assert st["n_particles"] == 0 and st["ordered_pairs"] == -1 and st["n_cells"] == 0
    finally:
        rwpt.rwpt_destroy(ctx)


def test_device_init_validates_before_copy(lib):
    ctx = rwpt.rwpt_create(rwpt.rwpt_config_default())
    try:
        with pytest.raises(rwpt.RwptError) as ei:
            rwpt.rwpt_init_ensemble_device(ctx, [-1], 0, 0)
        assert ei.value.status == rwpt.RWPT_EINVAL
        with pytest.raises(rwpt.RwptError) as ei:
            rwpt.rwpt_init_ensemble_device(ctx, [4], 0, 0)
        assert ei.value.status == rwpt.RWPT_EINVAL and "NULL" in str(ei.value)
    finally:
        rwpt.rwpt_destroy(ctx)


def test_probe_rate_validates_before_device(lib):
    ctx = rwpt.rwpt_create(rwpt.rwpt_config_default())
    try:
        for kind in (-1, 4):
            with pytest.raises(rwpt.RwptError) as ei:
                rwpt.rwpt_probe_rate(ctx, kind)
            assert ei.value.status == rwpt.RWPT_EINVAL
        assert lib.rwpt_probe_rate(ctx, rwpt.RWPT_PROBE_FMA, None) == rwpt.RWPT_EINVAL
        assert lib.rwpt_probe_rate(None, rwpt.RWPT_PROBE_FMA, None) == rwpt.RWPT_EINVAL
        try:
            import torch
            gpu = torch.cuda.is_available()
        except Exception:
            gpu = False
        if not gpu:
            with pytest.raises(rwpt.RwptError) as ei:
                rwpt.rwpt_probe_rate(ctx, rwpt.RWPT_PROBE_ROWSUM)
            assert ei.value.status == rwpt.RWPT_EDEVICE
    finally:
        rwpt.rwpt_destroy(ctx)


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_init_refuses_more_particles_than_32_bit_indices(lib):
    # sorted slots are 32-bit: the size check comes before any array is read,
    # so the one-element buffers here are never touched
    ctx = rwpt.rwpt_create(rwpt.rwpt_config_default())
    try:
        x = np.full((1, 2), 0.5)
        M = np.ones((2, 1))
        for sizes in ([2 ** 31], [2 ** 30, 2 ** 30], [2 ** 31 - 64]):
            with pytest.raises(rwpt.RwptError) as ei:
                rwpt.rwpt_init_ensemble(ctx, sizes, x, M)
            assert ei.value.status == rwpt.RWPT_EINVAL and "too many particles" in str(ei.value)
    finally:
        rwpt.rwpt_destroy(ctx)


def test_missing_library_fails_loudly(tmp_path):
    # no CPU fallback: without the built HIP library the binding refuses to run
    import subprocess
    import sys
    code = ("from paper_1811_05474_amd import rwpt\n"
            "rwpt.LIB_PATH = %r\n"
            "try:\n"
            "    rwpt.Ensemble(dim=2, n_species=2)\n"
            "except ImportError as e:\n"
            "    print('refused:', e)\n"
            "else:\n"
            "    raise SystemExit('ensemble created without the library')\n") % str(tmp_path / "librwpt.so")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "refused:" in r.stdout and "not built" in r.stdout


def test_half_stencil_tiling_is_binary32_only(lib):
    cfg = rwpt.rwpt_config_default()
    cfg.tile_lanes = -2
    ctx = rwpt.rwpt_create(cfg)  # binary32: accepted, no device touched
    rwpt.rwpt_destroy(ctx)
    cfg.precision = rwpt.RWPT_FP64
    with pytest.raises(rwpt.RwptError) as ei:
        rwpt.rwpt_create(cfg)
    assert ei.value.status == rwpt.RWPT_EUNSUPPORTED


def test_noalloc_validates_before_any_device_work(lib):
    # every refusal below happens on the host, before the scratch area is
    # looked up or a kernel is queued (the pointers are never dereferenced)
    cfg = rwpt.rwpt_config_default()
    bad = [dict(n=-1), dict(dt=0.0), dict(D=-1.0), dict(D=float("nan")), dict(pos=0), dict(m_out=2)]
    for kw in bad:
        args = dict(n=10, pos=1, m_in=2, m_out=3, dt=0.1, D=1e-4)
        args.update(kw)
        with pytest.raises(rwpt.RwptError) as ei:
            rwpt.rwpt_transfer_noalloc(cfg, args["n"], args["pos"], args["m_in"], args["m_out"], args["dt"],
                                       args["D"])
        assert ei.value.status == rwpt.RWPT_EINVAL, kw
    cfg.path = rwpt.RWPT_PATH_DENSE
    cfg.kappa = math.inf
    with pytest.raises(rwpt.RwptError) as ei:
        rwpt.rwpt_transfer_noalloc(cfg, 10, 1, 2, 3, 0.1, 1e-4)
    assert ei.value.status == rwpt.RWPT_EUNSUPPORTED
    cfg = rwpt.rwpt_config_default()
    cfg.tile_lanes = -2
    with pytest.raises(rwpt.RwptError) as ei:
        rwpt.rwpt_transfer_noalloc(cfg, 10, 1, 2, 3, 0.1, 1e-4)
    assert ei.value.status == rwpt.RWPT_EUNSUPPORTED
    # beyond the fixed scratch area: refused with the size in the message
    cfg = rwpt.rwpt_config_default()
    cfg.dim, cfg.n_species, cfg.precision = 3, 8, rwpt.RWPT_FP64
    with pytest.raises(rwpt.RwptError) as ei:
        rwpt.rwpt_transfer_noalloc(cfg, 1_000_000, 1, 2, 3, 0.1, 1e-6)
    assert ei.value.status == rwpt.RWPT_EUNSUPPORTED and "scratch" in str(ei.value)
    # n = 0 is a no-op
    rwpt.rwpt_transfer_noalloc(rwpt.rwpt_config_default(), 0, 0, 0, 0, 0.1, 1e-4)
