"""Benchmark of the CGKS-5th stage sweep on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--grid 256]

Workload: Taylor-Green vortex, Re 1600, Ma 0.1, Pr 0.72, Sutherland, periodic [0, 2pi]^3 at 256^3
(the grid the equal-error target is stated on), initial condition evaluated on the device.  A step is
one CGKS-5th time step: the CFL/viscous time-step reduction and the two stages (reconstruction,
gas-kinetic flux at the face Gauss points, update of averages and gradients).

Metric: Mcell-stage updates/s = cells x 2 stages x K / timed seconds, for
  * the headline form: FP32-bulk with the learned troubled-cell indicator (GENO where the network
    flags a cell), or FP32-bulk GENO everywhere when no trained indicator is present;
  * FP64 plain (GENO everywhere), measured beside it; the line reports the speedup and the relative
    L2 difference of the two velocity fields after the same steps;
  * "at equal L2 error": the record of paper_2508_19911_amd/equal_l2.py (results/tgv_equal_l2.json),
    |u_FP32 - u_FP64| over the FP64 scheme's own error at t = 2.5 per field, attached with the kernel
    digest it was measured on (marked stale when the kernels changed since);
  * with a trained indicator, FP32-bulk GENO everywhere as context (the form without the switch) and
    the flagged fraction of the learned run.
The roofline object is for the face-flux kernel (the dominant one): algorithmic flops per launch
(flops.json, counted from the kernel's own templates) over its mean launch time, taken with HIP events
on the library's stream during the timed region (only the flux launches carry events there).
kernels_ms is a per-class breakdown from as many further steps after the timed region, with every
launch between events.  cpu_baseline times the FP64 oracle on host cores over a bounded sample of
the same flow: one step on all cores, and one step of a smaller grid on one core.
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

PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}   # MI355X vector peaks (FP32 packed-math figure)
HBM_PEAK_GBS = 8000.0

# HBM bytes per k_flux5<float> launch on the 256^3 grid (mean over the three directions, read +
# write), from two rocprofv3 counter passes (FETCH_SIZE, then WRITE_SIZE) scaled by a 1 GiB copy
# kernel: profiles/step_tgv256_hbm_counters.md.  Valid only for the kernel code they were taken on
# (comments aside); any change to that code makes the reported traffic null until the counters are
# retaken.
FLUX_TRAFFIC = {"grid": 256, "bytes_per_launch": 1.9407e+10,
                "sources_sha256": "c710053779141e6d0a23146aee24df841c5220f5f6e9bd47d39e333d9742b7ce"}
KERNEL_SOURCES = ["common.hpp", "gks_flux.hpp", "recon.hpp", "recon_tables.hpp", "kernels.hpp"]


def kernel_digest():
    from paper_2508_19911_amd import equal_l2
    return equal_l2.source_digest(KERNEL_SOURCES)


def load_flops():
    with open(os.path.join(ROOT, "paper_2508_19911_amd", "flops.json")) as f:
        return json.load(f)


def load_indicator():
    path = os.path.join(ROOT, "paper_2508_19911_amd", "indicator.npz")
    if not os.path.exists(path):
        return None
    import numpy as np
    z = np.load(path)
    return z["params"].astype("float32"), float(z["logit_threshold"])


def run_variant(case, precision, steps, warmup, timing, indicator=None, breakdown_steps=0):
    """Time `steps` steps after `warmup`.  timing: True brackets the face-flux launches of the timed
    steps with HIP events (the other kernels run without events between them); breakdown_steps > 0
    then runs that many more steps, after the timed region, with every kernel class timed."""
    import numpy as np
    import torch
    from paper_2508_19911_amd import cgks

    thr = indicator[1] if indicator is not None else 0.0
    s = cgks.Solver(case, precision=precision, indicator_logit=thr)
    if indicator is not None:
        s.indicator_set(indicator[0], indicator[1])
    s.set_ic(cgks.IC_TGV, [case.ma, case.rho0, case.u0])
    s.step(warmup, case.cfl)
    torch.cuda.synchronize()
    if timing:
        s.timing(True, classes=["flux"])
        s.timing_read()
    t0 = time.perf_counter()
    _, done, t_now = s.step(steps, case.cfl)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = s.timing_read() if timing else None
    diag = s.diagnostics(case.rho0, case.u0)
    q, _, _, _ = s.get_state()
    vel = q[1:4] / q[0]
    breakdown = None
    if breakdown_steps:
        s.timing(True)
        s.timing_read()
        s.step(breakdown_steps, case.cfl)
        breakdown = s.timing_read()
    s.timing(False)
    s.close()
    del s
    torch.cuda.empty_cache()
    return {"seconds": t1 - t0, "steps": done, "t": t_now, "kernels": kt, "diag": diag, "vel": vel,
            "breakdown": breakdown, "breakdown_steps": breakdown_steps}


def copy_calibration(nbytes=1 << 30):
    """One plain device-to-device copy of nbytes (a kernel of known HBM traffic: nbytes read, nbytes
    written), so that a hardware-counter pass can scale FETCH_SIZE / WRITE_SIZE."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    torch.cuda.empty_cache()


def _oracle_step_rate(n):
    import oracle
    from paper_2508_19911_amd import inputs

    case = inputs.tgv_case(n).with_(recon=1)
    q, g = inputs.tgv_state(case)
    o = oracle.Oracle(oracle.params_from_config(case))
    o.set_state(q, g)
    t0 = time.perf_counter()
    rc, done, _ = o.step(1, case.cfl)
    dt = time.perf_counter() - t0
    return case.N * 2 * done / dt / 1e6, dt


def cpu_baseline(n=56, n1=24):
    """The FP64 oracle on one CGKS-5th GENO step of the same flow: at n^3 with OpenMP over the host's
    cores, and at n1^3 on one core."""
    import ctypes
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rate, dt = _oracle_step_rate(n)
    out = {"value": rate, "unit": "Mcell-stage/s", "cores": cores, "kind": "oracle",
           "sample": f"TGV Re1600 Ma0.1 {n}^3, 1 CGKS-5th GENO FP64 step (2 stages), {dt:.1f} s"}
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        r1, d1 = _oracle_step_rate(n1)
        gomp.omp_set_num_threads(cores)
        out["single_core"] = {"value": r1, "cores": 1,
                              "sample": f"TGV {n1}^3, 1 CGKS-5th GENO FP64 step, {d1:.1f} s"}
    except OSError:
        pass
    return out


def equal_l2_record(n):
    """The equal-L2 record of paper_2508_19911_amd/equal_l2.py for grid n, if one was written."""
    path = os.path.join(ROOT, "results", "tgv_equal_l2.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    g = rec.get("grids", {}).get(str(n))
    if g is None:
        return None
    from paper_2508_19911_amd import equal_l2
    return {"t": rec["t"], "fields": rec["fields"], "variant": rec["variant"],
            "ratio_fp32_minus_fp64_over_fp64_error": g.get("ratio"), "max_ratio": g.get("max_ratio"),
            "reference": g.get("reference"), "criterion": "max_ratio <= 0.05",
            "other_grids": {k: v.get("max_ratio") for k, v in rec["grids"].items() if k != str(n)},
            "record": "results/tgv_equal_l2.json",
            "stale": rec.get("kernel_sources_sha256") != equal_l2.kernel_digest()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="run the headline variant only")
    ap.add_argument("--no-fp64-plain", action="store_true",
                    help="skip the FP64 plain comparator (it does not fit one GPU above about 400^3)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy first (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the sweep is not sharded across GPUs.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2508_19911_amd import cgks, inputs

    cgks.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    flops = load_flops()
    indicator = load_indicator()
    if args.copy_calibration:
        copy_calibration()
    n = args.grid
    base = inputs.tgv_case(n, ma=0.1, re=1600.0, prandtl=0.72)
    N = base.N

    head_case = base.with_(recon=cgks.RECON_LEARNED if indicator is not None else cgks.RECON_NONLINEAR)
    head = run_variant(head_case, cgks.PREC_FP32_BULK, args.steps, args.warmup, True, indicator,
                       breakdown_steps=args.steps)
    rate = N * 2 * head["steps"] / head["seconds"] / 1e6

    # context: FP32-bulk with GENO everywhere (the same form without the learned switch)
    geno32 = None
    if indicator is not None and not args.no_fp64:
        geno32 = run_variant(base.with_(recon=cgks.RECON_NONLINEAR), cgks.PREC_FP32_BULK, args.steps,
                             args.warmup, True)

    fp64 = None
    if not args.no_fp64 and not args.no_fp64_plain:
        fp64 = run_variant(base.with_(recon=cgks.RECON_NONLINEAR), cgks.PREC_FP64, args.steps, args.warmup, True)

    kc, kms = head["kernels"]["flux"]
    flux_ms = kms / max(kc, 1)
    per_cell = flops["flux_launch_per_cell"]
    achieved = per_cell * N / (flux_ms * 1e-3) / 1e12
    traffic = None
    if n == FLUX_TRAFFIC["grid"] and kernel_digest() == FLUX_TRAFFIC["sources_sha256"]:
        traffic = FLUX_TRAFFIC["bytes_per_launch"]
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_TFLOPS["fp32"], 4), "traffic": traffic, "kernel": "k_flux5<float>",
            "flops_per_launch": per_cell * N, "mean_launch_ms": round(flux_ms, 4)}
    if traffic is not None:  # the same launch against the HBM roof: measured bytes over its mean time
        gbs = traffic / (flux_ms * 1e-3) / 1e9
        roof["hbm_achieved_gbs"] = round(gbs, 1)
        roof["hbm_frac"] = round(gbs / HBM_PEAK_GBS, 4)
    # per-class breakdown from the steps after the timed region, every launch between events
    kernels = {k: {"launches": c, "ms": round(m, 3)} for k, (c, m) in head["breakdown"].items()}
    kernels["steps"] = head["breakdown_steps"]

    line = {
        "metric": "Mcell-stage updates/s at 1 GPU, FP32+learned vs FP64 plain, at equal L2 error",
        "value": round(rate, 3),
        "unit": "Mcell-stage/s",
        "n_gpus": 1,
        "steps": head["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(head["seconds"] / head["steps"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (analytic Taylor-Green initial condition on the device)",
        "config": {"workload": f"Taylor-Green vortex Re1600 Ma0.1 Pr0.72 {n}^3 CGKS-5th",
                   "cells": N, "variant": "fp32_bulk+learned" if indicator is not None else "fp32_bulk+geno(no indicator)",
                   "cfl": base.cfl},
        "roofline": roof,
        "kernels_ms": kernels,
    }
    if indicator is not None:
        line["learned"] = {"flagged_fraction_last_stage": round(head["diag"]["flagged_fraction"], 4),
                           "logit_threshold": indicator[1]}
        if geno32 is not None:
            r32 = N * 2 * geno32["steps"] / geno32["seconds"] / 1e6
            dv32 = np.sqrt(((head["vel"] - geno32["vel"]) ** 2).sum()) / np.sqrt((geno32["vel"] ** 2).sum())
            line["fp32_geno_everywhere"] = {"value": round(r32, 3),
                                            "ms_per_step": round(geno32["seconds"] / geno32["steps"] * 1e3, 3),
                                            "rel_l2_velocity_diff_to_learned": float(dv32)}
    if fp64 is not None:
        rate64 = N * 2 * fp64["steps"] / fp64["seconds"] / 1e6
        dv = np.sqrt(((head["vel"] - fp64["vel"]) ** 2).sum()) / np.sqrt((fp64["vel"] ** 2).sum())
        line["fp64_plain"] = {"value": round(rate64, 3), "ms_per_step": round(fp64["seconds"] / fp64["steps"] * 1e3, 3),
                              "speedup_of_value": round(rate / rate64, 3), "rel_l2_velocity_diff": float(dv)}
        if fp64["kernels"]:
            c64, m64 = fp64["kernels"]["flux"]
            a64 = per_cell * N / (m64 / max(c64, 1) * 1e-3) / 1e12
            line["fp64_plain"]["flux_roofline"] = {"achieved": round(a64, 3), "peak": PEAK_TFLOPS["fp64"],
                                                   "frac": round(a64 / PEAK_TFLOPS["fp64"], 4)}
    eq = equal_l2_record(n)
    if eq is not None:
        line["equal_l2"] = eq
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
