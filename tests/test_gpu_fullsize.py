"""Parity at the full size of the Taylor-Green workload (128^3, Re 1600, Ma 0.1) in the launch
configuration the benchmark times (the same grid, kernels and launch shapes as its steps).

The device stage operator is compared with the oracle's stage evaluated at sampled cells only
(oracle.stage_cells: each cell from its own neighbourhood). The cells are seeded random ones plus
the 8 corners, the cells next to each periodic seam and the last cell. Bars are as on the small
grids: 1e-12 of the natural scales in FP64, and 100 float roundings of them in the FP32-bulk form.
A few steps of the FP32-bulk form keep the box totals to rounding.
"""
import numpy as np
import pytest

import oracle
from paper_2508_19911_amd import inputs

from test_gpu_parity import scales, scaled_err

pytestmark = pytest.mark.gpu

N1 = 128


def sampled_cells(n, count=160, seed=0):
    rng = np.random.default_rng(seed)
    idx = set(int(c) for c in rng.integers(0, n ** 3, size=count))
    for i in (0, n - 1):
        for j in (0, n - 1):
            for k in (0, n - 1):
                idx.add((k * n + j) * n + i)
    for a in (0, 1, n - 2, n - 1):  # next to each periodic seam, on each axis
        idx.add((5 * n + 7) * n + a)
        idx.add((5 * n + a) * n + 7)
        idx.add((a * n + 7) * n + 5)
    return np.array(sorted(idx), dtype=np.int64)


@pytest.mark.parametrize("precision", [0, 1])
def test_tgv128_stage_at_sampled_cells(precision):
    from paper_2508_19911_amd import cgks
    case = inputs.tgv_case(N1).with_(recon=cgks.RECON_NONLINEAR)
    s = cgks.Solver(case, precision=precision)
    s.set_ic(cgks.IC_TGV, [case.ma, case.rho0, case.u0])
    s.step(2, case.cfl)  # leave the initial symmetry-aligned state
    q, g, _, _ = s.get_state()
    dt = s.compute_dt(case.cfl)
    L, Lt, sqn, sqt = s.stage(dt)
    s.close()
    cells = sampled_cells(N1)
    o = oracle.Oracle(oracle.params_from_config(case))
    o.set_state(q, g)
    Lo, Lto, sqno, sqto = o.stage_cells(dt, cells)
    sc = scales(case, q)
    bar = 1e-12 if precision == 0 else 100 * 2.0 ** -24
    for key, a, b in [("L", L, Lo), ("Lt", Lt, Lto), ("sqn", sqn, sqno), ("sqt", sqt, sqto)]:
        e = scaled_err(a[:, cells], b, sc[key])
        assert e <= bar, (key, e)


def test_tgv128_fp32_conservation():
    from paper_2508_19911_amd import cgks
    case = inputs.tgv_case(N1).with_(recon=cgks.RECON_NONLINEAR)
    s = cgks.Solver(case, precision=cgks.PREC_FP32_BULK)
    s.set_ic(cgks.IC_TGV, [case.ma, case.rho0, case.u0])
    d0 = s.diagnostics()
    s.step(3, case.cfl)
    d1 = s.diagnostics()
    s.close()
    for k in ["mass", "momx", "momy", "momz", "energy"]:
        # FP64 accumulation of telescoping face sums over 2M cells: rounding of the totals
        assert abs(d1[k] - d0[k]) <= 1e-11 * abs(d0["energy"]), (k, d1[k] - d0[k])
