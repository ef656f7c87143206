"""Train the troubled-cell network on the GPU from the scheme's own runs.

    python -m paper_2508_19911_amd.train_indicator [--grid 128] [--epochs 30] [--out .../indicator.npz]

Data: CGKS-5th with GENO everywhere (FP32-bulk, the form the network serves) on two of the paper's
flows:
- the Taylor-Green vortex (Re 1600, Ma 0.1);
- decaying isotropic turbulence (Ma_t 0.5, Re_lambda 72).

At a set of times, cells give one sample each (every positive cell of the Taylor-Green vortex, a seeded
sample of the rest):
- x = the 64 features (59 used) computed on the device;
- y = 1 iff max_v |1 - chi_v| > 0.01 under full GENO (the scheme's own nonlinear-weight outcome).

Training runs in the library's GPU kernels: BF16 matrix-core forward, FP32 backward, Adam. In the
Taylor-Green vortex the positive cells are rare (thin sheets, from t ~ 4), so they are repeated until
they are about a quarter of that flow's samples; at these grids the isotropic turbulence is GENO-active
almost everywhere and contributes a small sample.

The last snapshot of each flow is held out. The logit threshold is the largest value that keeps
recall >= 0.999 on the held-out positives of every flow. The held-out flagged fraction and recall are stored with
the weights, and so are the same figures on the shocklet flow (isotropic turbulence at Ma_t 1.0),
which is not used in training.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def snapshots(cgks, case, state, times, precision):
    """Run GENO from the given state and yield (t, features, labels, q, g) at each requested time."""
    s = cgks.Solver(case.with_(recon=cgks.RECON_NONLINEAR), precision=precision)
    s.set_state(*state)
    t = 0.0
    for tt in times:
        if tt > t:
            _, _, t = s.step(10 ** 7, case.cfl, t_stop=tt)
        q, g, _, _ = s.get_state()
        yield t, s.features(), s.labels(0.01), q, g
    s.close()


def held_out_stats(cgks, case, q, g, params, precision):
    """Flags of the trained network on a held-out state (device inference) against its GENO labels."""
    s = cgks.Solver(case.with_(recon=cgks.RECON_NONLINEAR), precision=precision)
    s.set_state(q, g)
    s.indicator_set(params, 0.0)
    z = s.logits()
    y = s.labels(0.01).astype(bool)
    s.close()
    return z, y


def solution_gap(cgks, case, q, g, params, thr, precision, steps=20):
    """From a held-out state, the velocity after `steps` fixed steps with the network's flags
    (LEARNED), with GENO everywhere and with the linear reconstruction: the L2 distance of LEARNED
    to GENO relative to that of LINEAR to GENO, and the mean flagged fraction."""
    dt = None
    out = {}
    for name, recon in (("geno", cgks.RECON_NONLINEAR), ("linear", cgks.RECON_LINEAR), ("learned", cgks.RECON_LEARNED)):
        s = cgks.Solver(case.with_(recon=recon), precision=precision, indicator_logit=thr)
        if recon == cgks.RECON_LEARNED:
            s.indicator_set(params, thr)
        s.set_state(q, g)
        if dt is None:
            dt = s.compute_dt(case.cfl)
        frac = 0.0
        for _ in range(steps):
            s.step_fixed(1, dt)
            frac += float(s.flags().mean()) / steps
        qq = s.get_state()[0]
        out[name] = (qq[1:4] / qq[0], frac)
        s.close()
    ug = out["geno"][0]
    gap = float(np.sqrt(((out["learned"][0] - ug) ** 2).sum() / ((out["linear"][0] - ug) ** 2).sum()))
    return {"steps": steps, "learned_to_geno_over_linear_to_geno": gap, "flagged_fraction": out["learned"][1]}


def summarize(z, y, thr):
    flag = z > thr
    pos = int(y.sum())
    return {"cells": int(y.size), "positives": pos, "flagged_fraction": float(flag.mean()),
            "recall": float((flag & y).sum() / pos) if pos else 1.0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--sample", type=float, default=0.0625,
                    help="fraction of the other cells per training snapshot")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--recall", type=float, default=0.999)
    ap.add_argument("--out", default=os.path.join(HERE, "indicator.npz"))
    args = ap.parse_args()

    import torch
    from . import cgks, inputs

    cgks.load()
    prec = cgks.PREC_FP32_BULK
    n = args.grid
    flows = [
        ("tgv_ma0.1", inputs.tgv_case(n), [0.0, 3.0, 5.0, 6.0, 7.0, 8.0, 9.0], 1.0),
        ("hit_mat0.5", inputs.hit_case(n, ma_t=0.5), [0.0, 0.1, 0.2, 0.3, 0.5], 0.0),
    ]
    xs, ys, held = [], [], []
    pick = np.random.default_rng(args.seed + 1)
    t0 = time.time()
    for name, case, times, keep_pos in flows:
        state = inputs.initial_state(case)
        snaps = list(snapshots(cgks, case, state, times, prec))
        for k, (t, x, y, q, g) in enumerate(snaps):
            print(f"{name} t={t:.3f}: {y.mean() * 100:.2f}% labelled", flush=True)
            if k == len(snaps) - 1:
                held.append((name, case, q, g))
            else:
                sel = (pick.random(y.size) < args.sample) | ((y > 0) & (keep_pos > 0))
                xs.append((name, x[sel]))
                ys.append((name, y[sel]))
    parts_x, parts_y, reps = [], [], {}
    for name, _, _, keep_pos in flows:
        xf = np.concatenate([a for nm, a in xs if nm == name])
        yf = np.concatenate([a for nm, a in ys if nm == name]).astype(np.float32)
        pos = np.flatnonzero(yf > 0.5)
        r = max(1, int(0.25 * len(yf) / max(len(pos), 1))) if keep_pos else 1
        reps[name] = r
        parts_x += [xf] + [xf[pos]] * (r - 1)
        parts_y += [yf] + [yf[pos]] * (r - 1)
        print(f"{name}: {len(yf)} samples, {len(pos)} positive, positives repeated x{r}", flush=True)
    x = np.concatenate(parts_x)
    y = np.concatenate(parts_y)
    del xs, ys, parts_x, parts_y
    print(f"training set: {len(y)} samples, {int(y.sum())} positive, "
          f"{time.time() - t0:.1f} s of data generation", flush=True)

    xb = cgks.to_bf16_bits(x)
    xd = torch.from_numpy(xb.view(np.int16)).cuda()
    yd = torch.from_numpy(y).cuda()
    trainer = cgks.Solver(inputs.tgv_case(8), precision=prec)
    rng = np.random.default_rng(args.seed)
    p0 = (rng.normal(size=cgks.MLP_NPARAM) * 0.1).astype(np.float32)
    p0[2048:2080] = np.abs(p0[2048:2080])
    trainer.indicator_set(p0, 0.0)
    loss0, _ = trainer.indicator_grad(xd, yd)
    t1 = time.time()
    final = trainer.indicator_train(xd, yd, epochs=args.epochs, lr=args.lr, seed=args.seed)
    torch.cuda.synchronize()
    train_s = time.time() - t1
    params = trainer.indicator_get()
    trainer.close()
    print(f"loss {loss0:.4f} -> {final:.4f} in {args.epochs} epochs, {train_s:.1f} s", flush=True)

    # threshold: recall >= target on the held-out positives of both flows
    zs, yl = [], []
    for name, case, q, g in held:
        z, yy = held_out_stats(cgks, case, q, g, params, prec)
        zs.append(z)
        yl.append(yy)
    thr = float(max(z.max() for z in zs))
    for z, yy in zip(zs, yl):
        zp = np.sort(z[yy])
        if len(zp):
            thr = min(thr, float(zp[int(np.floor((1.0 - args.recall) * len(zp)))]) - 1e-3)
    report = {"held_out": {}, "test": {}, "tradeoff_tgv": {}}
    for (name, case, _, _), z, yy in zip(held, zs, yl):
        report["held_out"][name] = summarize(z, yy, thr)
    # trade-off on the held-out Taylor-Green state: recall target -> flagged fraction, solution gap
    name, case, q, g = held[0]
    zp = np.sort(zs[0][yl[0]])
    for target in (0.9, 0.99, 0.995, args.recall):
        th = float(zp[int(np.floor((1.0 - target) * len(zp)))]) - 1e-3
        rep = summarize(zs[0], yl[0], th)
        rep.update(solution_gap(cgks, case, q, g, params, th, prec))
        rep["logit_threshold"] = th
        report["tradeoff_tgv"][f"recall_{target}"] = rep
        print(f"tgv held-out, recall target {target}: {json.dumps(rep)}", flush=True)
    # generalisation: shocklet-laden isotropic turbulence, not seen in training
    case = inputs.hit_case(n, ma_t=1.0)
    st = inputs.initial_state(case)
    try:
        for t, _, _, q, g in snapshots(cgks, case, st, [0.0, 0.02, 0.05, 0.1], prec):
            z, yy = held_out_stats(cgks, case, q, g, params, prec)
            report["test"][f"hit_mat1.0_t{t:.2f}"] = summarize(z, yy, thr)
    except cgks.CgksError as e:  # the run may leave the physical range before the last time
        report["test"]["hit_mat1.0_stopped"] = str(e)
    meta = {"grid": n, "sample": args.sample, "epochs": args.epochs, "lr": args.lr, "seed": args.seed, "loss_initial": loss0,
            "loss_final": final, "train_seconds": train_s, "samples": int(len(y)), "positive_repeat": reps,
            "recall_target": args.recall, "logit_threshold": thr, **report}
    print(json.dumps(meta, indent=1), flush=True)
    np.savez(args.out, params=params, logit_threshold=np.float64(thr), meta=json.dumps(meta))
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
