"""GPU unit parity: the device flux routine and the device reconstruction, each against the oracle
on the same inputs (FP64 <= 1e-12 relative), so a stage-level difference can be located."""
import numpy as np
import pytest

import oracle
from paper_2508_19911_amd import gen_recon, inputs

pytestmark = pytest.mark.gpu

GAMMA = 1.4


def cons(rho, U, V, W, p):
    return np.array([rho, rho * U, rho * V, rho * W, p / (GAMMA - 1) + 0.5 * rho * (U * U + V * V + W * W)])


def side(rng, base, scale=0.3):
    return np.concatenate([cons(*base), rng.normal(scale=scale, size=15)])


FLUX_CASES = {
    "continuous_viscous": dict(mu0=0.013, prandtl=1.0, sutherland_tref=0.0, same=True),
    "viscous_jump": dict(mu0=0.01, prandtl=1.0, sutherland_tref=0.0, same=False),
    "viscous_prandtl_sutherland": dict(mu0=0.02, prandtl=0.7, sutherland_tref=0.9, same=False),
    "inviscid_jump": dict(mu0=0.0, prandtl=1.0, sutherland_tref=0.0, same=False),
    "inviscid_tau0": dict(mu0=0.0, prandtl=1.0, sutherland_tref=0.0, same=True, tau_eps=0.0),
}


@pytest.mark.parametrize("name", list(FLUX_CASES))
@pytest.mark.parametrize("precision", [0, 1])
def test_point_flux(name, precision):
    from paper_2508_19911_amd import cgks
    c = FLUX_CASES[name]
    case = inputs.tgv_case(8).with_(mu0=c["mu0"], prandtl=c["prandtl"], sutherland_tref=c["sutherland_tref"],
                                    tau_eps=c.get("tau_eps", 0.05))
    P = oracle.params_from_config(case)
    rng = np.random.default_rng(7)
    dt = 0.01
    n = 40
    wl = np.array([side(rng, (1.0 + 0.2 * rng.uniform(), 0.5 * rng.normal(), 0.3 * rng.normal(), -0.2, 1.0)) for _ in range(n)])
    if c["same"]:
        wr = wl.copy()
    else:
        wr = np.array([side(rng, (0.9 + 0.3 * rng.uniform(), 0.4 * rng.normal(), 0.1, 0.2 * rng.normal(), 0.8 + 0.3 * rng.uniform())) for _ in range(n)])
    ref = np.array([oracle.point_flux(P, dt, wl[i], wr[i]) for i in range(n)])
    s = cgks.Solver(case, precision=precision)
    got = s.point_flux(dt, wl, wr)
    # each output component against its largest magnitude over the points
    scale = np.maximum(np.abs(ref).max(axis=0, keepdims=True), 1e-300)
    err = (np.abs(got - ref) / scale).max()
    # FP32: the time-derivative terms combine g0 and g_{l,r} pieces with weights ~ tau/dt^2 that
    # cancel to O(1): float rounding ~ 2^-24 x (1 + tau/dt) x O(100) terms
    tau_dt = 1.5
    bar = 1e-12 if precision == 0 else 100 * 2.0 ** -24 * (1 + tau_dt) * 10
    assert err <= bar, (name, err, np.unravel_index(np.argmax(np.abs(got - ref) / scale), got.shape))


def test_reconstruction_coefficients():
    """Device coefficients evaluated at the face Gauss points (with the generated basis tables) equal
    the oracle's reconstruction of the same cell, linear and GENO."""
    from paper_2508_19911_amd import cgks
    PV, PD = gen_recon.basis_tables()
    case0 = inputs.tgv_case(8, ma=0.3).with_(nx=9, ny=7, nz=6, lx=2.0, ly=1.7, lz=1.3)
    q, g = inputs.seeded_smooth_state(case0, seed=3, amp=0.2)
    off = oracle.stencil_offsets()
    h = np.array(case0.h)
    nx, ny, nz = case0.nx, case0.ny, case0.nz
    for recon in (0, 1):
        case = case0.with_(recon=recon)
        s = cgks.Solver(case)
        s.set_state(q, g)
        C = s.coefficients()  # [5][34][N]
        P = oracle.params_from_config(case)
        for cell in [0, 5, 17, 100, case.N - 1]:
            i, j, k = cell % nx, (cell // nx) % ny, cell // (nx * ny)
            for v in range(5):
                qs = np.zeros(19); gs = np.zeros((19, 3))
                for si, o in enumerate(off):
                    c2 = ((k + o[2]) % nz) * nx * ny + ((j + o[1]) % ny) * nx + (i + o[0]) % nx
                    qs[si] = q[v, c2]
                    gs[si] = [g[5 * e + v, c2] for e in range(3)]
                ref, _ = oracle.recon_cell(P, qs, gs, h, recon, scale=oracle.geno_scale(q[:, cell], v))
                a = C[v, :, cell]
                for f in range(6):
                    for kk in range(4):
                        val = q[v, cell] + np.dot(PV[f][kk], a)
                        der = [np.dot(PD[f][kk][e], a) / h[e] for e in range(3)]
                        sc = max(abs(ref[f, kk, 0]), 1.0)
                        assert abs(val - ref[f, kk, 0]) <= 1e-12 * sc, (recon, cell, v, f, kk, val, ref[f, kk, 0])
                        assert np.allclose(der, ref[f, kk, 1:], rtol=1e-11, atol=1e-12 * np.abs(ref[f, :, 1:]).max())
