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
    """Algorithmic flops of the exchange pass per ordered in-cutoff pair (j != i):
    dim differences, dim squares + (dim-1) adds, one exponent scale, one exp,
    q_i + q_j, its product with w, and per species a difference, a product and
    an accumulation."""
    return dim + dim + (dim - 1) + 1 + 1 + 1 + 1 + 3 * S


def exchange_bytes_per_particle(dim: int, S: int, tsize: int) -> int:
    """Algorithmic HBM bytes of the exchange pass per particle: read the
    position, q and S masses, write S masses."""
    return tsize * (dim + 1 + S) + tsize * S


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
    return ap.parse_args()


def run_path(rwpt, W, w, precision, steps, warmup, tile_lanes, profile=True):
    import torch

    x, M, sizes, _ = W.make_inputs(w)
    ens = rwpt.Ensemble(dim=w.dim, n_species=w.n_species, react=w.react, kappa=w.kappa,
                        rw_ratio=w.rw_ratio, precision=precision, seed=w.seed, tile_lanes=tile_lanes)
    ens.init(sizes, x, M)
    audit0 = ens.audit()[0].tolist()
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
    out["audit"] = ens.audit()[0].tolist()
    out["tiling"] = rwpt.rwpt_get_tiling(ens.ctx)
    ens.close()
    return out


def cpu_baseline(W, w, unordered_pairs_per_step):
    """The oracle (unchanged) on the host: one full step (walk + transfer +
    reaction) of the same workload, timed; pairs/s uses the workload's
    in-cutoff pair count per step."""
    import oracle

    x, M, sizes, _ = W.make_inputs(w)
    x = x.astype(np.float32).astype(np.float64)
    ids = np.arange(w.n, dtype=np.uint32)
    threads = oracle.num_threads()
    steps = 1
    t0 = time.perf_counter()
    for s in range(steps):
        x = oracle.walk(x, ids, w.seed, s, w.rw_ratio * w.D, w.dt, w.box_lo, w.box_hi)
        M = oracle.transfer(x, M, w.D, w.dt, kappa=w.kappa, prec=32, react=w.react)
    dt_s = (time.perf_counter() - t0) / steps
    return {
        "value": unordered_pairs_per_step / dt_s,
        "unit": "pair-interactions/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "%d full step (walk + transfer + reaction, FP64 weights) of the 1e6-particle 2-D "
                  "workload on %d OpenMP threads: %.3f s/step" % (steps, threads, dt_s),
        "steps_per_s": 1.0 / dt_s,
    }


def measured_traffic(kernel_tag: str):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s.txt" % kernel_tag)
    src = os.path.join(ROOT, "paper_1811_05474_amd", "csrc", "rwpt_kernels.hip")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if fields.get("kernel_source_sha256") != sha:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus %d requested); "
              "the multi-GPU decomposition is described in DESIGN.md" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1811_05474_amd import rwpt, workloads as W

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.init()
    w = W.WORKLOADS[WORKLOAD]

    if args.copy_calibration_mib:
        nbytes = args.copy_calibration_mib << 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    r32 = run_path(rwpt, W, w, rwpt.RWPT_FP32, args.steps, args.warmup, args.tile_lanes,
                   profile=not args.profile_only)
    if args.profile_only:
        print(json.dumps({"profile_only": True, "ms_per_step": r32["ms_per_step"]}))
        return
    r64 = None
    if not args.no_fp64:
        r64 = run_path(rwpt, W, w, rwpt.RWPT_FP64, args.steps, args.warmup, args.tile_lanes)

    unordered = 0.5 * r32["ordered_pairs_per_step"]
    steps_per_s = 1e3 / r32["ms_per_step"]
    value = unordered * steps_per_s

    ex = r32["phases"]["exchange"]
    flops_per_launch = exchange_flops_per_pair(w.dim, w.n_species) * r32["ordered_pairs_per_step"]
    achieved_tflops = flops_per_launch / (ex["us_avg"] * 1e-6) / 1e12
    roofline = {
        "bound": "alu",
        "kernel": "k_exchange (weights + exchange + reaction + audit partials)",
        "achieved": achieved_tflops,
        "peak": PEAK_FP32_VECTOR_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved_tflops / PEAK_FP32_VECTOR_TFLOPS,
        "traffic": measured_traffic("k_exchange_walk2d_n1e6"),
        "us_per_launch": ex["us_avg"],
        "flops_per_launch": flops_per_launch,
        "algorithmic_bytes_per_launch": exchange_bytes_per_particle(w.dim, w.n_species, 4) * w.n,
        "hbm_frac_of_algorithmic_bytes": exchange_bytes_per_particle(w.dim, w.n_species, 4) * w.n
        / (ex["us_avg"] * 1e-6) / 1e9 / PEAK_HBM_GBPS,
    }

    line = {
        "metric": METRIC,
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
            "workload": WORKLOAD, "n_particles": w.n, "dim": w.dim, "species": w.n_species,
            "D": w.D, "dt": w.dt, "kappa": w.kappa, "rw_ratio": w.rw_ratio, "norm": "sym",
            "reaction": "A+B->0", "tile_lanes": r32["tiling"][0], "cell_refine": r32["tiling"][1],
            "unordered_pairs_per_step": unordered,
            "candidate_evaluations_per_step": r32["evaluations_per_step"],
        },
        "phases_us": {k: round(v["us_avg"], 2) for k, v in r32["phases"].items()},
        "roofline": roofline,
    }
    if r64 is not None:
        m32, m64 = r32["masses"], r64["masses"]
        line["fp64"] = {
            "ms_per_step": r64["ms_per_step"],
            "steps_per_s": 1e3 / r64["ms_per_step"],
            "value": 0.5 * r64["ordered_pairs_per_step"] * 1e3 / r64["ms_per_step"],
            "phases_us": {k: round(v["us_avg"], 2) for k, v in r64["phases"].items()},
            "fp32_speedup": r64["ms_per_step"] / r32["ms_per_step"],
            "fp32_vs_fp64_normwise_mass_diff": float(np.abs(m32 - m64).max() / np.abs(m64).max()),
        }
        for tag, r in (("fp32", r32), ("fp64", r64)):
            a0, a1 = r["audit0"], r["audit"]
            line["fp64"]["a_minus_b_drift_" + tag] = abs(a1[2] - a0[2]) / (a0[0] + a0[1])
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(W, w, unordered)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
