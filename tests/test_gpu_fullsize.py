"""Parity at the full sizes of the workloads, in the launch configurations of their steps:
- the Taylor-Green vortex (Re 1600, Ma 0.1) at 128^3: the benchmark's grid, kernels and launch
  shapes;
- decaying isotropic turbulence (Ma_t 0.5) at 256^3;
- the Taylor-Green vortex at 512^3 in the FP32-bulk form, the largest single-GPU grid (about 185 GB
  of device workspace).

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


def compare_sampled(case, s, dt, precision, seed):
    """Device stage at sampled cells (cgks_stage_sampled) against the oracle's per-cell stage on the
    state the device holds (q, g as stored, so FP32 gradients enter the oracle exactly)."""
    cells = sampled_cells(case.nx, seed=seed)
    got = s.stage_sampled(dt, cells)
    q, g, _, _ = s.get_state()
    o = oracle.Oracle(oracle.params_from_config(case))
    o.set_state(q, g)
    del g
    ref = o.stage_cells(dt, cells)
    sc = scales(case, q)
    bar = 1e-12 if precision == 0 else 100 * 2.0 ** -24
    for key, a, b in zip(["L", "Lt", "sqn", "sqt"], got, ref):
        e = scaled_err(a, b, sc[key])
        assert e <= bar, (key, e)


def test_sampled_entry_point_equals_full_stage():
    from paper_2508_19911_amd import cgks
    case = inputs.tgv_case(24, ma=0.3).with_(recon=cgks.RECON_NONLINEAR, nx=24, ny=20, nz=18)
    st = inputs.seeded_smooth_state(case, seed=3, amp=0.1)
    s = cgks.Solver(case)
    s.set_state(*st)
    dt = s.compute_dt(case.cfl)
    full = s.stage(dt)
    cells = np.array([0, 5, 777, case.N - 1, 4242, 8191])
    part = s.stage_sampled(dt, cells)
    s.close()
    for a, b in zip(full, part):
        assert np.array_equal(a[:, cells], b)


@pytest.mark.parametrize("precision", [0, 1])
def test_hit256_stage_at_sampled_cells(precision):
    from paper_2508_19911_amd import cgks
    case = inputs.hit_case(256).with_(recon=cgks.RECON_NONLINEAR)
    s = cgks.Solver(case, precision=precision)
    s.set_ic(cgks.IC_HIT, [case.ma], seed=case.seed)
    s.step(1, case.cfl)
    dt = s.compute_dt(case.cfl)
    compare_sampled(case, s, dt, precision, seed=1)
    s.close()


def test_tgv512_fp32_stage_at_sampled_cells():
    from paper_2508_19911_amd import cgks
    case = inputs.tgv_case(512).with_(recon=cgks.RECON_NONLINEAR)
    s = cgks.Solver(case, precision=cgks.PREC_FP32_BULK)
    s.set_ic(cgks.IC_TGV, [case.ma, case.rho0, case.u0])
    d0 = s.diagnostics()
    s.step(1, case.cfl)
    d1 = s.diagnostics()
    for k in ["mass", "momx", "momy", "momz", "energy"]:
        assert abs(d1[k] - d0[k]) <= 1e-11 * abs(d0["energy"]), (k, d1[k] - d0[k])
    dt = s.compute_dt(case.cfl)
    compare_sampled(case, s, dt, 1, seed=2)
    s.close()


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
