"""The paper's efficiency comparison (Sec. 4.1 and 4.2): CGKS-5th against GKS-2nd at equal
resolution, on one MI355X.

    python -m paper_2508_19911_amd.efficiency [--flow subsonic|supersonic] [--t-end 10] [--out eff.json]

- subsonic Taylor-Green vortex (Re 1600, Ma 0.1): linear CGKS-5th on 96^3 against linear GKS-2nd on
  296^3;
- supersonic Taylor-Green vortex (Re 1600, Ma 2): nonlinear CGKS-5th (GENO) on 116^3 against GKS-2nd
  with the Venkatakrishnan limiter on 384^3.

All runs are FP64, as in the paper, at the CFL of the 3-D cases, from t = 0 to t_end. The line
reports for each run:
- the GPU wall time, steps and Mcell-stage/s;
- E_k(t_end) and the peaks of -dE_k/dt and eps_S.

It also reports the cost ratio GKS-2nd / CGKS-5th. With --fp32, CGKS-5th is also run in the
FP32-bulk form (GENO, or the trained indicator when present) for context.

With --reference N, CGKS-5th FP64 on N^3 (256^3 for the supersonic flow in the paper) is run as well.
Each run's E_k(t), eps_S(t) and eps_D(t) histories are compared with it (max relative difference
over t, and the peak values).

The diagnostics integrate over each cell's reconstruction with the 3x3x3 Gauss rule, as the paper
does (--one-point: the cell-average form instead).  They are outside the timed steps.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def run(cgks, case, precision, t_end, dt_out, label, indicator=None, quad=True):
    import torch
    thr = indicator[1] if indicator is not None else 0.0
    s = cgks.Solver(case, precision=precision, indicator_logit=thr)
    if indicator is not None:
        s.indicator_set(indicator[0], indicator[1])
    ic = cgks.IC_TGV_SUPERSONIC if case.name == "tgv_sup" else cgks.IC_TGV
    s.set_ic(ic, [case.ma, case.rho0, case.u0])
    torch.cuda.synchronize()
    hist = []
    steps = 0
    t, k = 0.0, 0
    gpu_s = 0.0
    while t < t_end - 1e-12:
        k += 1
        t0 = time.perf_counter()
        _, done, t = s.step(10 ** 8, case.cfl, t_stop=min(k * dt_out, t_end))
        torch.cuda.synchronize()
        gpu_s += time.perf_counter() - t0
        steps += done
        d = s.diagnostics(case.rho0, case.u0, quad=quad)
        hist.append([t, d["Ek"], d["epsS"], d["epsD"]])
        if k % 20 == 0:
            print(f"  {label}: t={t:.2f} steps={steps} Ek={d['Ek']:.5f} ({gpu_s:.0f} s)", flush=True)
    s.close()
    h = np.array(hist)
    keep_hist = h.round(8).tolist()
    dek = -np.gradient(h[:, 1], h[:, 0])
    stages = 2 if case.scheme == cgks.SCHEME_CGKS5 else 1
    return {"cells": case.N, "grid": case.nx, "steps": steps, "seconds": gpu_s,
            "mcell_stage_per_s": case.N * stages * steps / gpu_s / 1e6,
            "Ek_end": float(h[-1, 1]), "dEk_peak": float(dek.max()), "t_dEk_peak": float(h[int(np.argmax(dek)), 0]),
            "epsS_peak": float(h[:, 2].max()), "t_epsS_peak": float(h[int(np.argmax(h[:, 2])), 0]),
            "epsD_peak": float(h[:, 3].max()), "history": keep_hist}


def flow_cases(flow):
    """(CGKS-5th case, GKS-2nd case, the paper's table) of one comparison (Sec. 4.1 or 4.2)."""
    from . import cgks, inputs
    if flow == "subsonic":
        c5 = inputs.tgv_case(96).with_(recon=cgks.RECON_LINEAR)
        c2 = inputs.tgv_case(296).with_(scheme=cgks.SCHEME_GKS2, recon=cgks.RECON_LINEAR)
        paper = {"cgks5_seconds": 876, "gks2_seconds": 7746, "ratio": 8.8, "hardware": "2x RTX 4090, FP64"}
    else:
        c5 = inputs.tgv_case(116, ma=2.0, supersonic=True).with_(recon=cgks.RECON_NONLINEAR)
        c2 = inputs.tgv_case(384, ma=2.0, supersonic=True).with_(scheme=cgks.SCHEME_GKS2, recon=cgks.RECON_NONLINEAR)
        paper = {"cgks5_seconds": 407, "gks2_seconds": 2842, "ratio": 7.0, "hardware": "4x RTX 4090, FP64"}
    return c5, c2, paper


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--flow", choices=["subsonic", "supersonic"], default="subsonic")
    ap.add_argument("--t-end", type=float, default=10.0)
    ap.add_argument("--dt-out", type=float, default=0.05)
    ap.add_argument("--fp32", action="store_true")
    ap.add_argument("--reference", type=int, default=0, help="grid of a CGKS-5th FP64 reference run")
    ap.add_argument("--one-point", action="store_true", help="cell-average diagnostics instead of quadrature")
    ap.add_argument("--skip-gks2", action="store_true")
    ap.add_argument("--out", default="efficiency.json")
    args = ap.parse_args()

    from . import cgks, inputs

    cgks.load()
    c5, c2, paper = flow_cases(args.flow)
    quad = not args.one_point
    from .equal_l2 import kernel_digest

    out = {"flow": args.flow, "t_end": args.t_end, "cfl": c5.cfl, "paper_table": paper,
           "diagnostics": "quadrature" if quad else "one-point", "kernel_sources_sha256": kernel_digest(),
           "runs": {}}
    out["runs"]["cgks5_fp64"] = run(cgks, c5, cgks.PREC_FP64, args.t_end, args.dt_out, "cgks5_fp64", quad=quad)
    print(json.dumps({k: v for k, v in out["runs"]["cgks5_fp64"].items() if k != "history"}), flush=True)
    if args.fp32:
        ind = None
        path = os.path.join(HERE, "indicator.npz")
        if c5.recon == cgks.RECON_NONLINEAR and os.path.exists(path):
            z = np.load(path)
            ind = (z["params"].astype(np.float32), float(z["logit_threshold"]))
        c5f = c5.with_(recon=cgks.RECON_LEARNED) if ind is not None else c5
        out["runs"]["cgks5_fp32"] = run(cgks, c5f, cgks.PREC_FP32_BULK, args.t_end, args.dt_out, "cgks5_fp32", ind,
                                        quad=quad)
        print(json.dumps({k: v for k, v in out["runs"]["cgks5_fp32"].items() if k != "history"}), flush=True)
    if not args.skip_gks2:
        out["runs"]["gks2_fp64"] = run(cgks, c2, cgks.PREC_FP64, args.t_end, args.dt_out, "gks2_fp64", quad=quad)
        print(json.dumps({k: v for k, v in out["runs"]["gks2_fp64"].items() if k != "history"}), flush=True)
        out["cost_ratio_gks2_over_cgks5"] = \
            out["runs"]["gks2_fp64"]["seconds"] / out["runs"]["cgks5_fp64"]["seconds"]
    if args.reference:
        cref = c5.with_(nx=args.reference, ny=args.reference, nz=args.reference, recon=cgks.RECON_NONLINEAR)
        ref = run(cgks, cref, cgks.PREC_FP64, args.t_end, args.dt_out, f"cgks5_fp64_{args.reference}", quad=quad)
        out["runs"]["reference"] = ref
        hr = np.array(ref["history"])
        cmp = {}
        for name, r in out["runs"].items():
            if name == "reference":
                continue
            h = np.array(r["history"])
            m = min(len(h), len(hr))
            cmp[name] = {f"max_rel_diff_{q}": float(np.abs(h[:m, c] - hr[:m, c]).max() / np.abs(hr[:m, c]).max())
                         for q, c in (("Ek", 1), ("epsS", 2), ("epsD", 3))}
        out["against_reference"] = cmp
        print("against the reference: " + json.dumps(cmp), flush=True)
    if "cost_ratio_gks2_over_cgks5" in out:
        print(f"cost ratio GKS-2nd / CGKS-5th = {out['cost_ratio_gks2_over_cgks5']:.2f} (paper: {paper['ratio']})",
              flush=True)
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
