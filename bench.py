"""Benchmark of the mass-transfer hot path on one MI355X.

Workload (synthetic, seeded): 10^6 particles uniform in the unit square,
species A and B with masses (1/N)(1 + 0.1 xi), D = 1e-5, dt = 0.1,
cutoff 3 sigma, random walk with D_rw = D between transfers, symmetric
normalisation, reaction A + B -> 0.  One step = walk + cell sort + row sums +
exchange + reaction + audit, all on the GPU.

Prints one JSON line.  value = particle-pair interactions per second (unordered
pairs {i, j}, i != j, within the cutoff, counted by the library before and
after the timed region) on the FP32 path; steps/s and the FP64 path's numbers
are reported beside it.

--workload NAME measures another of the named workloads in the same form: the
interface verification problem (75 realisations of 2000 particles in 1-D),
the 64-realisation batch, the 3-D eight-species case, the 1-D sparse case or
the 1-D full matrix on matrix cores.  For the full matrix the pair count is
every pair of the realisation, and the roofline counts the pairs whose weight
is at least 2^-40 (separation within sqrt(40 ln 2) sigma), the ones the kernel
must evaluate to binary32 accuracy.

Besides value, the line carries:
  roofline        the exchange kernel against the FP32 vector peak, or against
                  HBM when its flops per algorithmic byte are below the machine
                  balance; the kernel's duration from HIP events around every
                  kernel phase (on the library's stream) of an eager rerun of
                  the same steps after the timed region; traffic from the
                  committed rocprofv3
                  counter summary while the device sources match it (else null)
  step_roofline   the whole step's algorithmic bytes against HBM
  valu_probe      the row-broadcast pair kernels' evaluation rates against
                  register-only kernels running the same per-candidate code
                  (rwpt_probe_rate)
  host_io         one step fed from and returned to host memory, PCIe included
  err_vs_oracle_fp32, err_vs_oracle_fp64
                  one step from the seeded state, sampled particles against the
                  oracle, on identical positions and with the walk, each with
                  its bar (--no-accuracy skips them)
  fp64            the same run in binary64: its rate and phases, the FP32 path's
                  speedup over it (fp32_speedup, stated only when both paths are
                  within their bars; fp32_speedup_at says so), the two paths'
                  normwise mass difference after the run and both audits' drift
  config.tile_lanes, config.tiling_chosen_by
                  the pair tiling timed and who chose it: the library default, a
                  --tile-lanes flag, or rwpt_autotune (run outside the timed
                  region for the 64-realisation batch; --no-autotune skips it)
  cpu_baseline    the CPU oracle on a bounded sample of the same workload on
                  the host's threads, with the CPU model, the thread count and a
                  single-thread figure on a slab of the same workload
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

WORKLOAD = "walk2d_n1e6"
METRIC = "particle-pair interactions/s and steps/s at 1e6 particles 2D; FP32 vs FP64 path"

# MI355X published peaks used for the roofline fraction
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_HBM_GBPS = 8000.0


def exchange_flops_per_pair(dim: int, S: int) -> int:
    """Algorithmic flops per ordered in-cutoff pair (j != i): one exp, 2 dim
    for the separation (a difference and a square per axis), about 3 for the
    weight's scale, its normalisation factor and its accumulation, and 2 per
    species (a difference and a multiply-accumulate): 1 + 2 dim + 3 + 2 S."""
    return 1 + 2 * dim + 3 + 2 * S


def exchange_bytes_per_particle(dim: int, S: int, tsize: int) -> int:
    """Algorithmic HBM bytes of the transfer per particle: read the position
    and the S masses, write the S masses (tsize (dim + 2 S))."""
    return tsize * (dim + 2 * S)


def step_bytes_per_particle(dim: int, S: int, tsize: int) -> int:
    """Algorithmic HBM bytes of one whole step per particle: the walk reads and
    writes the position, the transfer reads the position and the masses and
    writes the masses (sorting and row sums are implementation overhead)."""
    return tsize * (2 * dim) + tsize * (dim + 2 * S)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-only", action="store_true",
                    help="run only the FP32 timed region (for rocprofv3)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--tile-lanes", type=int, default=0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the batch workload in the default tiling instead of the autotuned one")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the comparison with the oracle")
    ap.add_argument("--workload", default=WORKLOAD,
                    help="workload name (default %s)" % WORKLOAD)
    return ap.parse_args()


def ensemble_for(rwpt, w, precision, tile_lanes, kappa=None):
    kappa = w.kappa if kappa is None else kappa
    return rwpt.Ensemble(dim=w.dim, n_species=w.n_species, react=w.react, kappa=kappa,
                         rw_ratio=w.rw_ratio, precision=precision, seed=w.seed, tile_lanes=tile_lanes,
                         box_lo=w.box_lo, box_hi=w.box_hi, velocity=w.velocity, alpha_l=w.alpha_l,
                         alpha_t=w.alpha_t)


def init_ensemble(ens, W, w):
    x, M, sizes, Ds = W.make_inputs(w)
    d_scale = Ds / w.D if w.D > 0 else None
    ens.init(sizes, x, M, d_scale=d_scale)
    return sizes


def host_io(rwpt, W, w, precision, tile_lanes, repeats=3):
    """One step fed from and returned to host memory: init from the host
    arrays (copy over PCIe, cell grid), one step, masses copied back; the best
    of a few repeats, in ms."""
    import torch

    x, M, sizes, Ds = W.make_inputs(w)
    d_scale = Ds / w.D if w.D > 0 else None
    best = None
    for _ in range(repeats):
        ens = ensemble_for(rwpt, w, precision, tile_lanes)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ens.init(sizes, x, M, d_scale=d_scale)
        ens.sync()
        t1 = time.perf_counter()
        ens.step(w.dt, w.D, 1)
        ens.sync()
        t2 = time.perf_counter()
        ens.masses()
        t3 = time.perf_counter()
        ens.close()
        r = (1e3 * (t1 - t0), 1e3 * (t2 - t1), 1e3 * (t3 - t2))
        if best is None or sum(r) < sum(best):
            best = r
    return {"init_ms": best[0], "first_step_ms": best[1], "query_ms": best[2], "total_ms": sum(best)}


def run_path(rwpt, W, w, precision, steps, warmup, tile_lanes, profile=True, autotune=False):
    import torch

    ens = ensemble_for(rwpt, w, precision, tile_lanes)
    init_ensemble(ens, W, w)
    tuned_s = None
    if autotune:
        # outside the timed region: every candidate tiling is timed on a
        # snapshot of the state, which is then restored
        t0 = time.perf_counter()
        rwpt.rwpt_autotune(ens.ctx, w.dt, w.D, 3)
        tuned_s = time.perf_counter() - t0
    audit0 = ens.audit().sum(axis=0).tolist()
    ens.step(w.dt, w.D, warmup)
    ens.sync()
    pairs0, evals0 = ens.count_pairs(w.dt, w.D)
    torch.cuda.synchronize()
    ens.sync()
    t0 = time.perf_counter()
    ens.step(w.dt, w.D, steps)
    ens.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pairs1, evals1 = ens.count_pairs(w.dt, w.D)
    out = {
        "seconds": t1 - t0,
        "ms_per_step": 1e3 * (t1 - t0) / steps,
        "ordered_pairs_per_step": 0.5 * (pairs0 + pairs1),
        "evaluations_per_step": 0.5 * (evals0 + evals1),
        "masses": ens.masses(),
        "audit0": audit0,
    }
    if profile:
        # same number of steps again, eagerly, with HIP events around every
        # kernel phase on the library's stream
        rwpt.rwpt_profile_reset(ens.ctx)
        rwpt.rwpt_profile_enable(ens.ctx, True)
        ens.step(w.dt, w.D, steps)
        ens.sync()
        prof = rwpt.rwpt_profile_read(ens.ctx)
        rwpt.rwpt_profile_enable(ens.ctx, False)
        out["phases"] = {k: {"ms_total": v[0], "launches": v[1],
                             "us_avg": (1e3 * v[0] / v[1]) if v[1] else 0.0} for k, v in prof.items() if v[1]}
    out["audit"] = ens.audit().sum(axis=0).tolist()
    out["tiling"] = rwpt.rwpt_get_tiling(ens.ctx)
    out["autotune_s"] = tuned_s
    if profile and precision == rwpt.RWPT_FP32 and out["tiling"][0] == 4 and "rowsum" in out.get("phases", {}):
        # attainable rates of the row-broadcast kernels' inner loops on this
        # device, from register-only kernels running the same per-candidate code
        out["probe"] = {k: ens.probe_rate(v) for k, v in (
            ("fma", rwpt.RWPT_PROBE_FMA), ("exp", rwpt.RWPT_PROBE_EXP),
            ("rowsum", rwpt.RWPT_PROBE_ROWSUM), ("exchange", rwpt.RWPT_PROBE_EXCHANGE))}
    ens.close()
    return out


def accuracy(rwpt, W, w, precision, tile_lanes, n_rows=2000):
    """Error of one step of the path against the oracle, normwise over sampled
    particles (max |dM| / max |M|), in two forms:

    * identical positions: the walk switched off, so both sides transfer on
      the seeded positions (binary32-rounded for the FP32 path): the bar is
      1e-5 (FP32) or 1e-12 (FP64);
    * with the walk: the oracle's own walk then its transfer, against the
      path's walked step; positions may differ by an ulp, so the bar adds
      0.3 * 2 kappa * 2 u / sigma (u the ulp of the box's largest coordinate).

    Realisations: the first and, for a batch, the largest.  The full-matrix
    workload is compared with the oracle at kappa = 7, which equals the full
    matrix to e^-49 of the kernel."""
    import oracle

    f32 = precision == rwpt.RWPT_FP32
    p = 32 if f32 else 64
    bar = 1e-5 if f32 else 1e-12
    x, M, sizes, Ds = W.make_inputs(w)
    if f32:
        x = x.astype(np.float32).astype(np.float64)
        M = M.astype(np.float32).astype(np.float64)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    reals = sorted({0, int(np.argmax(sizes))})
    kappa = w.kappa if math.isfinite(w.kappa) else 7.0
    d_scale = Ds / w.D if w.D > 0 else None
    rng = np.random.default_rng(12)
    xmax = max(abs(v) for v in list(w.box_lo[:w.dim]) + list(w.box_hi[:w.dim]))
    u = float(np.spacing(np.float32(xmax))) if f32 else float(np.spacing(np.float64(xmax)))
    out = {}
    for form, rw in (("identical_positions", 0.0), ("with_walk", w.rw_ratio)):
        ens = rwpt.Ensemble(dim=w.dim, n_species=w.n_species, react=w.react, kappa=w.kappa, rw_ratio=rw,
                            precision=precision, seed=w.seed, tile_lanes=tile_lanes, box_lo=w.box_lo,
                            box_hi=w.box_hi, velocity=w.velocity if rw > 0 else (0.0, 0.0, 0.0),
                            alpha_l=w.alpha_l, alpha_t=w.alpha_t)
        ens.init(sizes, x, M, d_scale=d_scale)
        ens.step(w.dt, w.D, 1)
        got = ens.masses()
        ens.close()
        err, allow = 0.0, 0.0
        for r in reals:
            b, e = int(off[r]), int(off[r + 1])
            rows = rng.choice(e - b, min(n_rows, e - b), replace=False)
            Dr = float(Ds[r])
            xr = x[b:e]
            if rw > 0.0:
                xr = oracle.walk(xr, np.arange(b, e, dtype=np.uint32), w.seed, 0, rw * Dr, w.dt, w.box_lo,
                                 w.box_hi, velocity=w.velocity if any(w.velocity) else None,
                                 alpha_l=w.alpha_l, alpha_t=w.alpha_t)
                if f32:
                    xr = xr.astype(np.float32).astype(np.float64)
                allow = max(allow, 0.3 * 2.0 * kappa * 2.0 * u / math.sqrt(8.0 * Dr * w.dt))
            ref = oracle.transfer(xr, M[:, b:e], Dr, w.dt, kappa=kappa, prec=p, react=w.react, rows=rows)
            g = got[:, b + rows]
            err = max(err, float(np.abs(g - ref).max() / np.abs(ref).max()))
        out[form] = {"normwise_err": err, "bar": bar + allow, "within_bar": err < bar + allow}
    out["scope"] = ("one step from the seeded state, %d sampled particles of realisation(s) %s, max |dM| / max |M| "
                    "against the oracle (FP64 weights, cutoff predicate in the path's precision)"
                    % (n_rows, reals))
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_single_thread(W, w, budget_cells=16):
    """The oracle on one thread over a bounded sample: the particles of one
    strip of the box (1/budget_cells of the first axis, same density and
    neighbourhoods, the strip's own edges aside), one full step (walk +
    transfer + reaction); pairs from the oracle's neighbour count of the
    stepped sample."""
    import oracle

    x, M, sizes, Ds = W.make_inputs(w)
    x = x.astype(np.float32).astype(np.float64)
    b, e = 0, int(sizes[0])
    lo, hi = w.box_lo[0], w.box_hi[0]
    sel = np.flatnonzero(x[b:e, 0] < lo + (hi - lo) / budget_cells)
    xs, Ms = x[b:e][sel], M[:, b:e][:, sel]
    Dr = float(Ds[0])
    kappa = w.kappa if math.isfinite(w.kappa) else 7.0
    saved = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        if w.rw_ratio > 0 or any(w.velocity):
            xs = oracle.walk(xs, sel.astype(np.uint32), w.seed, 0, w.rw_ratio * Dr, w.dt, w.box_lo, w.box_hi,
                             velocity=w.velocity if any(w.velocity) else None, alpha_l=w.alpha_l,
                             alpha_t=w.alpha_t)
        oracle.transfer(xs, Ms, Dr, w.dt, kappa=kappa, prec=32, react=w.react)
        dt_s = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(saved)
    rp, _ = oracle.neighbors(xs.astype(np.float32).astype(np.float64), kappa, Dr, w.dt, 32)
    unordered = 0.5 * (rp[-1] - sel.size)
    return {
        "value": unordered / dt_s,
        "unit": "pair-interactions/s",
        "cores": 1,
        "sample": "one full step (walk + transfer + reaction, FP64 weights) of the %d particles in the first "
                  "1/%d of the box along x (%d unordered pairs) on one thread: %.3f s"
                  % (sel.size, budget_cells, int(unordered), dt_s),
    }


def cpu_baseline(W, w, unordered_pairs_per_step, budget_s=15.0):
    """The oracle (unchanged) on the host: one full step (walk + transfer +
    reaction) of the same workload, timed; pairs/s uses the workload's
    in-cutoff pair count per step.  Realisations of a batch are stepped in
    order until the time budget is spent, the pair count scaled by the
    fraction of particles stepped."""
    import oracle

    x, M, sizes, Ds = W.make_inputs(w)
    x = x.astype(np.float32).astype(np.float64)
    N = x.shape[0]
    off = np.concatenate([[0], np.cumsum(sizes)])
    threads = oracle.num_threads()
    done, passes = 0, 0
    t0 = time.perf_counter()
    while True:  # repeat short workloads to at least a second of work
        for r in range(len(sizes)):
            b, e = int(off[r]), int(off[r + 1])
            if e == b:
                continue
            xr = x[b:e]
            if w.rw_ratio > 0 or any(w.velocity):
                ids = np.arange(b, e, dtype=np.uint32)
                xr = oracle.walk(xr, ids, w.seed, 0, w.rw_ratio * Ds[r], w.dt, w.box_lo, w.box_hi,
                                 velocity=w.velocity if any(w.velocity) else None,
                                 alpha_l=w.alpha_l, alpha_t=w.alpha_t)
            oracle.transfer(xr, M[:, b:e], Ds[r], w.dt, kappa=w.kappa, prec=32, react=w.react)
            done += e - b
            if time.perf_counter() - t0 > budget_s:
                break
        passes += 1
        if done < passes * N or time.perf_counter() - t0 > 1.0:
            break
    dt_s = time.perf_counter() - t0
    frac = done / N  # steps' worth of particles processed
    sample = ("%d full step(s) (walk + transfer + reaction, FP64 weights) of %d of %d particles"
              % (passes, min(done, N), N))
    return {
        "value": frac * unordered_pairs_per_step / dt_s,
        "unit": "pair-interactions/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "%s of workload %s on %d OpenMP threads: %.3f s" % (sample, w.name, threads, dt_s),
        "steps_per_s": frac / dt_s,
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
        "single_thread": cpu_single_thread(W, w) if w.n_real == 1 else None,
    }


# the device code and the host code that picks its launch shapes; the counter
# summaries in profiles/ record the SHA-256 of their concatenation, in this order
DEVICE_SOURCES = ("rwpt_device.h", "rwpt_layout.h", "rwpt_pairstep.h", "rwpt_kernels.h", "rwpt_kernels.hip",
                  "rwpt_dense.hip", "rwpt_api.hip")


def measured_traffic(kernel_tag: str):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s.txt" % kernel_tag)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    digest = hashlib.sha256()
    for name in DEVICE_SOURCES:
        digest.update(open(os.path.join(ROOT, "paper_1811_05474_amd", "csrc", name), "rb").read())
    if fields.get("kernel_source_sha256") != digest.hexdigest():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the path runs on one GPU (--gpus %d requested); sharding across GPUs "
              "is not implemented" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1811_05474_amd import rwpt, workloads as W

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.init()
    if args.workload not in W.WORKLOADS:
        print("bench.py: unknown workload %r (known: %s)" % (args.workload, ", ".join(W.WORKLOADS)),
              file=sys.stderr)
        sys.exit(2)
    w = W.WORKLOADS[args.workload]

    if args.copy_calibration_mib:
        nbytes = args.copy_calibration_mib << 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # the batch of uneven realisations is timed in the tiling the autotuner picks
    autotune = w.name == "batch2d_64" and args.tile_lanes == 0 and not args.no_autotune
    r32 = run_path(rwpt, W, w, rwpt.RWPT_FP32, args.steps, args.warmup, args.tile_lanes,
                   profile=not args.profile_only, autotune=autotune)
    if args.profile_only:
        print(json.dumps({"profile_only": True, "ms_per_step": r32["ms_per_step"]}))
        return
    hio = host_io(rwpt, W, w, rwpt.RWPT_FP32, args.tile_lanes)
    r64 = None
    if not args.no_fp64:
        r64 = run_path(rwpt, W, w, rwpt.RWPT_FP64, args.steps, args.warmup, args.tile_lanes, autotune=autotune)

    unordered = 0.5 * r32["ordered_pairs_per_step"]
    steps_per_s = 1e3 / r32["ms_per_step"]
    value = unordered * steps_per_s

    dense = "dense" in r32["phases"]
    if dense:
        # pairs the full-matrix kernel must evaluate: weight >= 2^-40
        counter = ensemble_for(rwpt, w, rwpt.RWPT_FP32, 0, kappa=math.sqrt(40.0 * math.log(2.0)))
        init_ensemble(counter, W, w)
        if w.rw_ratio > 0:  # same walk, same positions as the measured run
            counter.step(w.dt, w.D, args.warmup + 2 * args.steps)
        alg_pairs, _ = counter.count_pairs(w.dt, w.D)
        counter.close()
        ex = r32["phases"]["dense"]
        kernel = "dense path (tile bounds + row sums + bf16-split MFMA exchange + reaction)"
    else:
        alg_pairs = r32["ordered_pairs_per_step"]
        ex = r32["phases"]["exchange"]
        kernel = "k_exchange (weights + exchange + reaction + audit partials)"
    n_total = r32["masses"].shape[1]
    flops_per_launch = exchange_flops_per_pair(w.dim, w.n_species) * alg_pairs
    achieved_tflops = flops_per_launch / (ex["us_avg"] * 1e-6) / 1e12
    alg_bytes = exchange_bytes_per_particle(w.dim, w.n_species, 4) * n_total
    achieved_gbps = alg_bytes / (ex["us_avg"] * 1e-6) / 1e9
    # the roof the kernel's algorithmic intensity puts it under: flops per
    # algorithmic byte against the machine balance (peak flops / peak bytes)
    hbm_bound = flops_per_launch < alg_bytes * (PEAK_FP32_VECTOR_TFLOPS * 1e12) / (PEAK_HBM_GBPS * 1e9)
    roofline = {
        "bound": "hbm" if hbm_bound else "alu",
        "kernel": kernel,
        "achieved": achieved_gbps if hbm_bound else achieved_tflops,
        "peak": PEAK_HBM_GBPS if hbm_bound else PEAK_FP32_VECTOR_TFLOPS,
        "unit": "GB/s" if hbm_bound else "TFLOP/s",
        "frac": achieved_gbps / PEAK_HBM_GBPS if hbm_bound else achieved_tflops / PEAK_FP32_VECTOR_TFLOPS,
        "traffic": measured_traffic(("k_dense_exchange_" if dense else "k_exchange_") + w.name),
        "us_per_launch": ex["us_avg"],
        "flops_per_launch": flops_per_launch,
        "algorithmic_bytes_per_launch": alg_bytes,
        "flops_per_algorithmic_byte": flops_per_launch / alg_bytes,
        "hbm_frac_of_algorithmic_bytes": achieved_gbps / PEAK_HBM_GBPS,
        "alu_frac_of_algorithmic_flops": achieved_tflops / PEAK_FP32_VECTOR_TFLOPS,
    }
    if dense:
        roofline["ordered_pairs_evaluated_per_launch"] = alg_pairs
    valu_probe = None
    if "probe" in r32:
        pr = r32["probe"]
        ev = r32["evaluations_per_step"]
        valu_probe = {
            "scope": "row-broadcast pair kernels: candidate evaluations/s against a register-only kernel "
                     "running the same per-candidate code at full occupancy (rwpt_probe_rate)",
            "fma_lane_ops_per_s": pr["fma"],
            "exp_lane_ops_per_s": pr["exp"],
        }
        for k in ("rowsum", "exchange"):
            got = ev / (r32["phases"][k]["us_avg"] * 1e-6)
            valu_probe[k] = {"achieved": got, "attainable": pr[k], "unit": "evaluations/s",
                             "frac": got / pr[k]}
    step_bytes = step_bytes_per_particle(w.dim, w.n_species, 4) * n_total
    step_gbps = step_bytes / (r32["ms_per_step"] * 1e-3) / 1e9
    step_roofline = {
        "bound": "hbm",
        "scope": "whole step (walk + sort + row sums + exchange + reaction + audit)",
        "algorithmic_bytes_per_step": step_bytes,
        "achieved": step_gbps,
        "peak": PEAK_HBM_GBPS,
        "unit": "GB/s",
        "frac": step_gbps / PEAK_HBM_GBPS,
    }

    line = {
        "metric": METRIC if w.name == WORKLOAD else
        "particle-pair interactions/s and steps/s, workload %s; FP32 vs FP64 path" % w.name,
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "steps_per_s": steps_per_s,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": w.name, "n_particles": n_total, "realisations": w.n_real, "dim": w.dim,
            "species": w.n_species, "D": w.D, "dt": w.dt,
            "kappa": w.kappa if math.isfinite(w.kappa) else "inf", "rw_ratio": w.rw_ratio,
            "norm": "sym", "reaction": "A+B->0" if w.react else "none",
            "path": "dense" if dense else "sparse",
            "tile_lanes": r32["tiling"][0], "cell_refine": r32["tiling"][1],
            "tiling_chosen_by": ("rwpt_autotune (%.1f s, outside the timed region)" % r32["autotune_s"]
                                 if r32["autotune_s"] is not None
                                 else ("--tile-lanes %d" % args.tile_lanes if args.tile_lanes else "default")),
            "unordered_pairs_per_step": unordered,
            "candidate_evaluations_per_step": r32["evaluations_per_step"],
        },
        "phases_us": {k: round(v["us_avg"], 2) for k, v in r32["phases"].items()},
        "roofline": roofline,
        "step_roofline": step_roofline,
        "valu_probe": valu_probe,
        "host_io": dict(hio, scope="one step with host input and output: init from host arrays "
                                   "(PCIe copy + cell grid), the first step (graph capture included), "
                                   "masses copied back",
                        pair_interactions_per_s=unordered / (hio["total_ms"] * 1e-3)),
    }
    acc32 = acc64 = None
    if not args.no_accuracy:
        acc32 = accuracy(rwpt, W, w, rwpt.RWPT_FP32, r32["tiling"][0] if autotune else args.tile_lanes)
        line["err_vs_oracle_fp32"] = acc32
    if r64 is not None:
        m32, m64 = r32["masses"], r64["masses"]
        line["fp64"] = {
            "ms_per_step": r64["ms_per_step"],
            "steps_per_s": 1e3 / r64["ms_per_step"],
            "value": 0.5 * r64["ordered_pairs_per_step"] * 1e3 / r64["ms_per_step"],
            "phases_us": {k: round(v["us_avg"], 2) for k, v in r64["phases"].items()},
            "fp32_vs_fp64_normwise_mass_diff_after_run": float(np.abs(m32 - m64).max() / np.abs(m64).max()),
        }
        if not args.no_accuracy:
            acc64 = accuracy(rwpt, W, w, rwpt.RWPT_FP64, r64["tiling"][0] if autotune else args.tile_lanes)
            line["err_vs_oracle_fp64"] = acc64
        # FP32 over FP64 speedup, stated only where both paths meet their bars
        # against the oracle ("equal accuracy")
        equal = (acc32 is not None and acc64 is not None and
                 all(a[f]["within_bar"] for a in (acc32, acc64) for f in ("identical_positions", "with_walk")))
        line["fp64"]["fp32_speedup"] = r64["ms_per_step"] / r32["ms_per_step"] if equal else None
        line["fp64"]["fp32_speedup_at"] = ("equal accuracy: both paths within their bars against the oracle "
                                           "(FP32 1e-5, FP64 1e-12, plus the walk allowance)" if equal else
                                           "not stated: accuracy not established")
        for tag, r in (("fp32", r32), ("fp64", r64)):
            a0, a1 = r["audit0"], r["audit"]
            if w.react:
                line["fp64"]["a_minus_b_drift_" + tag] = abs(a1[-1] - a0[-1]) / (a0[0] + a0[1])
            else:
                line["fp64"]["species_drift_" + tag] = max(abs(a1[k] - a0[k]) / abs(a0[k])
                                                           for k in range(w.n_species) if a0[k])
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(W, w, unordered)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
