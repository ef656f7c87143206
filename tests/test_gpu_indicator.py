"""What the trained troubled-cell network gains over the method without it (GPU).

The committed network (paper_2508_19911_amd/indicator.npz, trained on the GPU by
paper_2508_19911_amd/train_indicator.py from the scheme's own runs) at its stored threshold, on a
Taylor-Green state developed to t = 8 on 64^3 (the network was trained on 128^3 runs):
- LEARNED runs GENO only on the flagged cells, so the fraction of cells that skip the nonlinear
  blend is the saving;
- its velocity after 10 steps stays close to GENO everywhere: much closer than the linear
  reconstruction is (the method without the switch).
"""
import os

import numpy as np
import pytest

from paper_2508_19911_amd import inputs

pytestmark = pytest.mark.gpu

NPZ = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2508_19911_amd",
                   "indicator.npz")


def test_trained_indicator_gain():
    from paper_2508_19911_amd import cgks
    z = np.load(NPZ)
    params, thr = z["params"].astype(np.float32), float(z["logit_threshold"])
    case = inputs.tgv_case(64).with_(recon=cgks.RECON_NONLINEAR)
    s = cgks.Solver(case, precision=cgks.PREC_FP32_BULK)
    s.set_ic(cgks.IC_TGV, [case.ma, case.rho0, case.u0])
    s.step(10 ** 6, case.cfl, t_stop=8.0)
    q, g, _, _ = s.get_state()
    dt = s.compute_dt(case.cfl)
    s.close()
    vel, frac = {}, {}
    for name, recon in (("geno", cgks.RECON_NONLINEAR), ("linear", cgks.RECON_LINEAR),
                        ("learned", cgks.RECON_LEARNED)):
        r = cgks.Solver(case.with_(recon=recon), precision=cgks.PREC_FP32_BULK, indicator_logit=thr)
        if recon == cgks.RECON_LEARNED:
            r.indicator_set(params, thr)
        r.set_state(q, g)
        f = 0.0
        for _ in range(10):
            r.step_fixed(1, dt)
            f += r.flags().mean() / 10
        qq = r.get_state()[0]
        vel[name], frac[name] = qq[1:4] / qq[0], f
        r.close()
    gap_learned = np.linalg.norm(vel["learned"] - vel["geno"])
    gap_linear = np.linalg.norm(vel["linear"] - vel["geno"])
    print(f"flagged {frac['learned']:.3f}, |learned - geno| / |linear - geno| = {gap_learned / gap_linear:.4f}")
    assert abs(frac["geno"] - 1.0) < 1e-12 and frac["linear"] == 0.0
    assert 0.0 < frac["learned"] < 0.9, frac
    assert gap_learned < 0.05 * gap_linear, (gap_learned, gap_linear)
