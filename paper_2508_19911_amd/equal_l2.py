"""The FP32-bulk + learned form against FP64 plain at equal L2 error, on the Taylor-Green vortex
(Re 1600, Ma 0.1; Sec. 4.1), at a short horizon.

    python -m paper_2508_19911_amd.equal_l2 [--t 2.5] [--grids 64 128 256] [--out results/tgv_equal_l2.json]

For each grid n the script runs CGKS-5th FP64 plain (GENO everywhere) to t, and on the grids of
--fp32 (default: the two finest) the FP32-bulk form with the trained indicator (GENO everywhere when
there is none).  Fields compared: rho, U, V, W, p of the cell averages.

- D_n = |u64_n - R_n|_2 per field, R_n = the FP64 run on 2n restricted by 2^3 block averaging of the
  conservative averages: the scheme's own discretisation error on n, measured against 2n.
- Direct ratio where 2n was run: |u32_n - u64_n|_2 / D_n per field (the criterion is <= 0.05).
- On the finest grid N, whose 2N run does not fit one GPU in FP64 (512^3: ~340 GB of workspace) nor
  finish in one GPU session, D_N is estimated from the measured convergence: with p from
  D_{N/4} / D_{N/2} = 2^p, D_N = D_{N/2} 2^-p = D_{N/2}^2 / D_{N/4} (Richardson); the ratio is
  reported against that estimate and labelled as such.
Writes a JSON record with the kernel-source digest it was measured on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
KERNEL_SOURCES = ["common.hpp", "gks_flux.hpp", "recon.hpp", "recon_tables.hpp", "kernels.hpp", "mlp.hpp"]
FIELDS = ["rho", "U", "V", "W", "p"]


def source_digest(names):
    """SHA-256 of the code of the given csrc files with comments and layout taken out, so that a
    record stays valid across edits that change no code."""
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(HERE, "csrc", name), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def kernel_digest():
    return source_digest(KERNEL_SOURCES)


def prims(q, gamma):
    rho = q[0]
    u = q[1:4] / rho
    p = (gamma - 1.0) * (q[4] - 0.5 * rho * (u ** 2).sum(0))
    return np.stack([rho, u[0], u[1], u[2], p])


def restrict2(q, n):
    """2^3 block average of conservative averages [5][(2n)^3] (indexed [z][y][x]) onto [5][n^3]"""
    return q.reshape(5, n, 2, n, 2, n, 2).mean(axis=(2, 4, 6)).reshape(5, n ** 3)


def l2(a):
    return np.sqrt((a ** 2).sum(axis=1))


def run(cgks, case, precision, t_end, indicator=None):
    thr = indicator[1] if indicator is not None else 0.0
    s = cgks.Solver(case, precision=precision, indicator_logit=thr)
    if indicator is not None:
        s.indicator_set(indicator[0], indicator[1])
    s.set_ic(cgks.IC_TGV, [case.ma, case.rho0, case.u0])
    t0 = time.time()
    steps = 0
    t = 0.0
    while t < t_end - 1e-12:
        _, done, t = s.step(200, case.cfl, t_stop=t_end)
        steps += done
        print(f"  {case.nx}^3 {'fp64' if precision == 0 else 'fp32'} t={t:.3f} ({time.time() - t0:.0f} s)", flush=True)
    q = s.get_state()[0]
    s.close()
    return q, steps, time.time() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--t", type=float, default=2.5)
    ap.add_argument("--grids", type=int, nargs="+", default=[64, 128, 256])
    ap.add_argument("--fp32", type=int, nargs="+", default=None)
    ap.add_argument("--out", default=os.path.join(ROOT, "results", "tgv_equal_l2.json"))
    args = ap.parse_args()
    from . import cgks, inputs

    cgks.load()
    grids = sorted(args.grids)
    fp32_grids = sorted(args.fp32) if args.fp32 else grids[-2:]
    path = os.path.join(HERE, "indicator.npz")
    ind = None
    if os.path.exists(path):
        z = np.load(path)
        ind = (z["params"].astype(np.float32), float(z["logit_threshold"]))
    q64, u64, u32, runs = {}, {}, {}, {}
    for n in grids:
        case = inputs.tgv_case(n).with_(recon=cgks.RECON_NONLINEAR)
        q, steps, secs = run(cgks, case, cgks.PREC_FP64, args.t)
        q64[n], u64[n] = q, prims(q, case.gamma)
        runs[f"fp64_plain_{n}"] = {"steps": steps, "seconds": round(secs, 1)}
    for n in fp32_grids:
        case = inputs.tgv_case(n).with_(recon=cgks.RECON_LEARNED if ind is not None else cgks.RECON_NONLINEAR)
        q, steps, secs = run(cgks, case, cgks.PREC_FP32_BULK, args.t, ind)
        u32[n] = prims(q, case.gamma)
        runs[f"fp32_{'learned' if ind is not None else 'geno'}_{n}"] = {"steps": steps, "seconds": round(secs, 1)}
    gamma = inputs.tgv_case(8).gamma
    D = {}
    for n in grids:
        if 2 * n in q64:
            D[n] = l2(u64[n] - prims(restrict2(q64[2 * n], n), gamma))
    out = {"workload": "Taylor-Green vortex Re1600 Ma0.1 Pr0.72, CGKS-5th", "t": args.t,
           "fields": FIELDS, "variant": "fp32_bulk+learned" if ind is not None else "fp32_bulk+geno",
           "kernel_sources_sha256": kernel_digest(), "runs": runs,
           "fp64_error_vs_2n": {str(n): D[n].tolist() for n in D}, "grids": {}}
    for n in fp32_grids:
        d32 = l2(u32[n] - u64[n])
        g = {"fp32_minus_fp64": d32.tolist()}
        if n in D:
            r = d32 / D[n]
            g.update({"reference": f"FP64 plain on {2 * n}^3, 2^3 block average", "ratio": r.tolist(),
                      "max_ratio": float(r.max())})
        elif n // 2 in D and n // 4 in D:
            order = np.log2(D[n // 4] / D[n // 2])
            Dest = D[n // 2] ** 2 / D[n // 4]
            r = d32 / Dest
            g.update({"reference": f"estimated: FP64 error against {2 * n}^3 from D_{n // 4} and D_{n // 2} "
                                   f"(observed order per field)", "observed_order": order.tolist(),
                      "fp64_error_estimate": Dest.tolist(), "ratio": r.tolist(), "max_ratio": float(r.max())})
        out["grids"][str(n)] = g
        print(n, json.dumps(g), flush=True)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
