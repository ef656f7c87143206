"""The library's device formulation, compiled for the host CPU, against the oracle (no GPU needed).

The gas-kinetic flux and the parity-class face evaluation of the flux kernel are __host__ __device__
templates; tests/host/device_code_on_host.hip instantiates them on the host (double and float). This
file compares them with the oracle's point flux and with a direct evaluation of the generated basis
tables:
- FP64: <= 1e-12 relative;
- float: the bar of the FP32-bulk form.
The GPU tests repeat the comparison for the code the device actually runs.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2508_19911_amd import gen_recon, inputs

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
GAMMA = 1.4


@pytest.fixture(scope="module")
def lib():
    src = os.path.join(HERE, "host", "device_code_on_host.hip")
    out_dir = os.path.join(ROOT, "_build")
    os.makedirs(out_dir, exist_ok=True)
    so = os.path.join(out_dir, "device_code_on_host.so")
    if not os.path.exists(so) or os.path.getmtime(so) < max(
            os.path.getmtime(p) for p in [src] + [os.path.join(ROOT, "paper_2508_19911_amd", "csrc", f) for f in
                                                  ("gks_flux.hpp", "recon.hpp", "common.hpp", "recon_tables.hpp")]):
        subprocess.run(["/opt/rocm/bin/hipcc", "-O1", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", so, src],
                       check=True, capture_output=True)
    L = ctypes.CDLL(so)
    D, P = ctypes.c_double, ctypes.c_void_p
    L.host_point_flux.argtypes = [ctypes.c_int] + [D] * 7 + [P, P, P]
    L.host_eval_face.argtypes = [ctypes.c_int, D, P, P, P]
    L.host_normal_split.argtypes = [D, D, P]
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def cons(rho, U, V, W, p):
    return np.array([rho, rho * U, rho * V, rho * W, p / (GAMMA - 1) + 0.5 * rho * (U * U + V * V + W * W)])


CASES = {
    "continuous_viscous": dict(mu0=0.013, prandtl=1.0, tref=0.0, tau_eps=0.05, same=True),
    "viscous_jump": dict(mu0=0.01, prandtl=1.0, tref=0.0, tau_eps=0.05, same=False),
    "viscous_prandtl_sutherland": dict(mu0=0.02, prandtl=0.7, tref=0.9, tau_eps=0.05, same=False),
    "inviscid_jump": dict(mu0=0.0, prandtl=1.0, tref=0.0, tau_eps=0.05, same=False),
    "inviscid_tau0": dict(mu0=0.0, prandtl=1.0, tref=0.0, tau_eps=0.0, same=True),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", [0, 1])
def test_host_flux_matches_oracle(lib, name, precision):
    c = CASES[name]
    case = inputs.tgv_case(8).with_(mu0=c["mu0"], prandtl=c["prandtl"], sutherland_tref=c["tref"],
                                    tau_eps=c["tau_eps"])
    P = oracle.params_from_config(case)
    rng = np.random.default_rng(11)
    dt = 0.01
    worst = 0.0
    ref, got = [], []
    for _ in range(30):
        wl = np.concatenate([cons(1.0 + 0.2 * rng.uniform(), 0.5 * rng.normal(), 0.3 * rng.normal(), -0.2, 1.0),
                             rng.normal(scale=0.3, size=15)])
        wr = wl.copy() if c["same"] else np.concatenate(
            [cons(0.9 + 0.3 * rng.uniform(), 0.4 * rng.normal(), 0.1, 0.2 * rng.normal(), 0.8 + 0.3 * rng.uniform()),
             rng.normal(scale=0.3, size=15)])
        ref.append(oracle.point_flux(P, dt, wl, wr))
        o = np.zeros(30)
        lib.host_point_flux(precision, GAMMA, case.mu0, case.sutherland_tref, case.prandtl, case.tau_eps,
                            case.tau_c, dt, _p(wl), _p(wr), _p(o))
        got.append(o)
    ref, got = np.array(ref), np.array(got)
    scale = np.maximum(np.abs(ref).max(axis=0, keepdims=True), 1e-300)
    err = (np.abs(got - ref) / scale).max()
    bar = 1e-12 if precision == 0 else 100 * 2.0 ** -24 * 2.5 * 10
    assert err <= bar, (name, err)


@pytest.mark.parametrize("e", [0, 1, 2])
def test_parity_class_face_evaluation_matches_tables(lib, e):
    """Both sides of an axis from the + face tables with a sign: equal to the table of each face."""
    PV, PD = gen_recon.basis_tables()
    PV = np.array(PV, dtype=float)
    PD = np.array([[[[x if x is not None else 0.0 for x in r] for r in q] for q in p] for p in PD])
    rng = np.random.default_rng(e)
    a = rng.normal(size=34)
    for sn, f in ((1.0, 2 * e + 1), (-1.0, 2 * e)):
        val = np.zeros(4); der = np.zeros(12)
        lib.host_eval_face(e, sn, _p(a), _p(val), _p(der))
        for g in range(4):
            assert abs(val[g] - PV[f][g] @ a) <= 1e-13 * np.abs(a).sum()
            for x in range(3):
                assert abs(der[g * 3 + x] - PD[f][g][x] @ a) <= 1e-13 * np.abs(a).sum()


def test_fp32_form_keeps_the_pressure_scale_in_fp64(lib):
    """FP32-bulk flux at Ma 0.1 (p ~ 71 against O(1) velocity variations): the pressure-sized parts
    (W0, its Euler flux, the half-space sums, the assembly of F^n and of the interface values) are
    FP64, so F^n and the interface values match the FP64 oracle far below FP32 rounding of p
    (6e-8 * 71 = 4e-6).  With those parts in FP32 the errors were 1e-6 (mass) to 2e-4 (energy)."""
    case = inputs.tgv_case(8)
    P = oracle.params_from_config(case)
    rng = np.random.default_rng(3)
    p0 = 1.0 / (GAMMA * 0.01)
    err = np.zeros(30)
    for _ in range(40):
        base = cons(1 + 0.05 * rng.normal(), rng.normal(), rng.normal(), rng.normal(), p0 * (1 + 0.01 * rng.normal()))
        d = rng.normal(scale=1e-6, size=5) * np.array([1, 1, 1, 1, 100])
        wl = np.concatenate([base + d, rng.normal(scale=1e-3, size=15)])
        wr = np.concatenate([base - d, rng.normal(scale=1e-3, size=15)])
        ref = oracle.point_flux(P, 1e-3, wl, wr)
        o = np.zeros(30)
        lib.host_point_flux(1, GAMMA, case.mu0, case.sutherland_tref, case.prandtl, case.tau_eps, case.tau_c,
                            1e-3, _p(wl), _p(wr), _p(o))
        err = np.maximum(err, np.abs(o - ref))
    # F^n and the two sides' interface values (absolute; |F| and |Q| up to ~250)
    assert err[0:5].max() <= 1e-9, err[0:5]
    assert err[10:15].max() <= 1e-9 and err[20:25].max() <= 1e-9, (err[10:15], err[20:25])


def test_normal_split_series_and_library_branches(lib):
    """The FP64 split at u = 0 (probabilities of u > 0 and u < 0, and the half-range tail) on both sides
    of the two series branches (|x| = 1/8 and 1/2, x = U / sqrt(2 var)) and on the library branch,
    against erfc and exp evaluated by SciPy: the short series (7 and 8 terms below |x| = 1/8) and the
    long one (12 and 13 terms) must both be exact to FP64 rounding, and pp + pm = 1."""
    from scipy.special import erfc

    var = 1.7
    xs = np.concatenate([np.linspace(-1.3, 1.3, 261), [0.0, 0.1249999, 0.1250001, -0.1250001, 0.4999999, 0.5000001,
                                                         -0.4999999, 1e-9, -3e-5, 0.07, 0.3]])
    out = np.zeros(3)
    for x in xs:
        U = x * np.sqrt(2.0 * var)
        lib.host_normal_split(U, var, _p(out))
        pp, pm = 0.5 * erfc(-x), 0.5 * erfc(x)
        tail = np.exp(-x * x) * np.sqrt(var / (2.0 * np.pi))
        # a few ulp: x itself carries the rounding of U / sqrt(2 var); the library branch's erfc and
        # SciPy's differ by up to a few ulp where erfc is steep
        bar = 6e-16 if abs(x) < 0.5 else 3e-15
        assert abs(out[0] - pp) <= bar * pp, (x, out[0], pp)
        assert abs(out[1] - pm) <= bar * pm, (x, out[1], pm)
        assert abs(out[2] - tail) <= bar * tail, (x, out[2], tail)
        assert abs(out[0] + out[1] - 1.0) <= 4e-16
