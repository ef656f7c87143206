"""Taylor-Green vortex (Re 1600, Ma 0.1, Sec. 4.1): kinetic-energy and dissipation histories, and the
distance between the FP32-bulk + learned form and the FP64 plain scheme measured against the scheme's
own discretisation error.

    python -m paper_2508_19911_amd.tgv_history [--grid 128] [--t-end 10] [--out history.json]

Variants on the grid (CFL of the 3-D cases):
- CGKS-5th FP32-bulk with the trained indicator (when indicator.npz is present);
- CGKS-5th FP32-bulk with GENO everywhere;
- CGKS-5th FP64 plain (GENO everywhere);
- GKS-2nd FP64 (linear, the paper's subsonic comparator).

Diagnostics every dt_out = 0.05: E_k, eps_S, eps_D.

The reference R is CGKS-5th FP64 plain on the doubled grid to t = 2.5, restricted by 2^3 block
averaging. At t = 2.5 the line reports, for the velocity:
- |u_FP32+learned - u_FP64| / |u_FP64 - R|: the extra error of the fast form, relative to the scheme's
  own error on this grid;
- |u_GKS2 - R| / |u_FP64 - R|: how much larger the second-order scheme's error is.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def run(cgks, case, precision, t_marks, dt_out, indicator=None, keep=()):
    """Advance to each mark; diagnostics every dt_out; the velocity field at the times in `keep`."""
    thr = indicator[1] if indicator is not None else 0.0
    s = cgks.Solver(case, precision=precision, indicator_logit=thr)
    if indicator is not None:
        s.indicator_set(indicator[0], indicator[1])
    s.set_ic(cgks.IC_TGV, [case.ma, case.rho0, case.u0])
    hist, fields = [], {}
    t, k = 0.0, 0
    t0 = time.time()
    t_end = max(t_marks)
    while t < t_end - 1e-12:
        k += 1
        t_next = min(k * dt_out, t_end)
        _, _, t = s.step(10 ** 7, case.cfl, t_stop=t_next)
        d = s.diagnostics(case.rho0, case.u0)
        hist.append([t, d["Ek"], d["epsS"], d["epsD"], d["flagged_fraction"]])
        if k % 10 == 0:
            print(f"  t={t:.2f} Ek={d['Ek']:.6f} epsS={d['epsS']:.6f} ({time.time() - t0:.0f} s)", flush=True)
        for tk in keep:
            if abs(t - tk) < 1e-9 and tk not in fields:
                q = s.get_state()[0]
                fields[tk] = q[1:4] / q[0]
    s.close()
    return np.array(hist), fields, time.time() - t0


def restrict2(u, n):
    """2^3 block average of a [3][(2n)^3] field onto [3][n^3] (arrays indexed [z][y][x])."""
    v = u.reshape(3, n, 2, n, 2, n, 2)
    return v.mean(axis=(2, 4, 6)).reshape(3, n ** 3)


def rel(a, b):
    return float(np.sqrt(((a - b) ** 2).sum()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--t-end", type=float, default=10.0)
    ap.add_argument("--t-compare", type=float, default=2.5)
    ap.add_argument("--dt-out", type=float, default=0.05)
    ap.add_argument("--no-reference", action="store_true")
    ap.add_argument("--reference-only", action="store_true",
                    help="only the reference run and the FP64 / FP32 fields at t_compare on the grid")
    ap.add_argument("--out", default="tgv_history.json")
    args = ap.parse_args()

    from . import cgks, inputs

    cgks.load()
    n = args.grid
    base = inputs.tgv_case(n)
    ind = None
    path = os.path.join(HERE, "indicator.npz")
    if os.path.exists(path):
        z = np.load(path)
        ind = (z["params"].astype(np.float32), float(z["logit_threshold"]))
    tc = args.t_compare
    variants = []
    if ind is not None:
        variants.append(("cgks5_fp32_learned", base.with_(recon=cgks.RECON_LEARNED), cgks.PREC_FP32_BULK, ind))
    variants += [
        ("cgks5_fp32_geno", base.with_(recon=cgks.RECON_NONLINEAR), cgks.PREC_FP32_BULK, None),
        ("cgks5_fp64_plain", base.with_(recon=cgks.RECON_NONLINEAR), cgks.PREC_FP64, None),
        ("gks2_fp64_linear", base.with_(scheme=cgks.SCHEME_GKS2, recon=cgks.RECON_LINEAR), cgks.PREC_FP64, None),
    ]
    from .equal_l2 import kernel_digest

    out = {"grid": n, "cfl": base.cfl, "dt_out": args.dt_out, "kernel_sources_sha256": kernel_digest(),
           "variants": {}}
    fields = {}
    t_end = tc if args.reference_only else args.t_end
    for name, case, prec, indicator in variants:
        hist, f, secs = run(cgks, case, prec, [t_end], args.dt_out, indicator, keep=(tc,))
        fields[name] = f.get(tc)
        ipk = int(np.argmax(hist[:, 2]))
        out["variants"][name] = {
            "seconds": secs, "steps_time": float(hist[-1, 0]),
            "Ek_end": float(hist[-1, 1]), "epsS_peak": float(hist[ipk, 2]), "t_epsS_peak": float(hist[ipk, 0]),
            "epsD_max": float(hist[:, 3].max()), "flagged_fraction_mean": float(hist[:, 4].mean()),
            "history": hist.round(8).tolist()}
        print(f"{name}: {secs:.1f} s, Ek(t_end) {hist[-1, 1]:.6f}, eps_S peak {hist[ipk, 2]:.6f} at t={hist[ipk, 0]:.2f}",
              flush=True)
    if not args.no_reference and fields.get("cgks5_fp64_plain") is not None:
        ref = inputs.tgv_case(2 * n).with_(recon=cgks.RECON_NONLINEAR)
        _, fr, secs = run(cgks, ref, cgks.PREC_FP64, [tc], args.dt_out, None, keep=(tc,))
        R = restrict2(fr[tc], n)
        u64 = fields["cgks5_fp64_plain"]
        err64 = rel(u64, R)
        cmp = {"t": tc, "reference": f"CGKS-5th FP64 plain on {2 * n}^3, 2^3 block average", "reference_seconds": secs,
               "abs_l2_fp64_minus_ref": err64, "rel_l2_fp64_minus_ref": err64 / float(np.sqrt((R ** 2).sum()))}
        for name in fields:
            if name != "cgks5_fp64_plain" and fields[name] is not None:
                cmp[f"{name}_minus_fp64_over_fp64_error"] = rel(fields[name], u64) / err64
                cmp[f"{name}_error_over_fp64_error"] = rel(fields[name], R) / err64
        out["compare"] = cmp
        print(json.dumps(cmp, indent=1), flush=True)
    with open(args.out, "w") as fh:
        json.dump(out, fh)
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
