"""CPU-side checks of the HIP library: it loads, exports every entry point that include/cgks.h
declares, validates parameters on the host, and its exact-rational reconstruction tables agree with
the oracle's floating-point least-squares solve (two independent constructions of the same operator).
No compute call runs here (no GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "cgks.h")).read()
    return sorted(set(re.findall(r"\b(cgks_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2508_19911_amd import cgks
    lib = cgks.load()
    names = header_symbols()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(cgks.SYMBOLS) == names


def test_workspace_size_and_parameter_validation():
    from paper_2508_19911_amd import cgks, inputs
    lib = cgks.load()
    case = inputs.tgv_case(16)
    p = cgks.params_from_case(case)
    n = ctypes.c_size_t()
    assert lib.cgks_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == 0
    # FP64 CGKS-5th: 60 state doubles + 170 coefficient + 90 face planes per cell, plus small buffers
    assert 320 * 8 * case.N <= n.value <= 320 * 8 * case.N + 4 * 1024 * 1024
    p32 = cgks.params_from_case(case, precision=1)
    n32 = ctypes.c_size_t()
    assert lib.cgks_workspace_bytes(ctypes.byref(p32), ctypes.byref(n32)) == 0 and n32.value < n.value
    bad = cgks.params_from_case(case.with_(nx=0))
    assert lib.cgks_workspace_bytes(ctypes.byref(bad), ctypes.byref(n)) == -1
    bad = cgks.params_from_case(case.with_(gamma=1.0))
    assert lib.cgks_workspace_bytes(ctypes.byref(bad), ctypes.byref(n)) == -1
    bad = cgks.params_from_case(case.with_(scheme=1, recon=2))
    assert lib.cgks_workspace_bytes(ctypes.byref(bad), ctypes.byref(n)) == -1
    assert lib.cgks_strerror(-4).decode().startswith("non-physical")


def test_exact_tables_match_oracle_operator():
    from paper_2508_19911_amd import gen_recon
    R_exact, stencil, neigh, basis = gen_recon.exact_operator()
    Ro = oracle.recon_operator()
    off = [tuple(o) for o in oracle.stencil_offsets()]
    # oracle basis order: by degree, then d1 descending, d2 descending
    ob = [(a, b, dg - a - b) for dg in range(1, 5) for a in range(dg, -1, -1) for b in range(dg - a, -1, -1)]
    assert sorted(ob) == sorted(basis)
    worst = 0.0
    for i, d in enumerate(basis):
        io = ob.index(d)
        for c in range(75):
            if c < 18:
                co = off.index(neigh[c]) - 1
            else:
                s, e = divmod(c - 18, 3)
                co = 18 + 3 * off.index(stencil[s]) + e
            worst = max(worst, abs(float(R_exact[i][c]) - Ro[io, co]))
    assert worst <= 1e-12, worst
    nnz = sum(1 for row in R_exact for v in row if v != 0)
    assert nnz == 678


def test_generated_header_is_current():
    from paper_2508_19911_amd import gen_recon
    path = os.path.join(ROOT, "paper_2508_19911_amd", "csrc", "recon_tables.hpp")
    assert open(path).read() == gen_recon.generate()


def test_flop_counts_are_current():
    """flops.json (used by bench.py for the roofline) equals a fresh count from the kernel templates."""
    import json
    from paper_2508_19911_amd import build
    path = os.path.join(ROOT, "paper_2508_19911_amd", "flops.json")
    stored = json.load(open(path))
    fresh = build.count_flops(verbose=False)
    assert fresh == stored
    # the face flux dominates a stage: three launches per stage
    assert 3 * fresh["flux_launch_per_cell"] > 0.7 * fresh["cell_stage_geno"]


def test_grid_limit_rejected_before_any_device_work():
    """Planes are addressed with 32-bit byte offsets: N >= 2^29 is refused by the parameter check."""
    from paper_2508_19911_amd import cgks, inputs
    lib = cgks.load()
    n = ctypes.c_size_t()
    big = cgks.params_from_case(inputs.tgv_case(8).with_(nx=1024, ny=1024, nz=512))
    assert lib.cgks_workspace_bytes(ctypes.byref(big), ctypes.byref(n)) == -1
    ok = cgks.params_from_case(inputs.tgv_case(8).with_(nx=1024, ny=1024, nz=511))
    assert lib.cgks_workspace_bytes(ctypes.byref(ok), ctypes.byref(n)) == 0 and n.value > 0


def test_null_context_is_rejected_without_device_work():
    """Every entry point taking a context returns EINVAL for NULL (checked before any HIP call)."""
    from paper_2508_19911_amd import cgks
    lib = cgks.load()
    z = ctypes.c_void_p(None)
    d = ctypes.c_double()
    assert lib.cgks_compute_dt(z, 0.5, ctypes.byref(d)) == -1
    assert lib.cgks_step_fixed(z, 1, 0.1) == -1
    assert lib.cgks_stage(z, 0.1, None, None, None, None) == -1
    assert lib.cgks_set_ic(z, 1, None, 0, 0) == -1
    assert lib.cgks_get_flags(z, None) == -1
    assert lib.cgks_diagnostics_quad(z, 1.0, 1.0, None) == -1
    assert lib.cgks_timing_enable(z, 1) == -1
    assert lib.cgks_destroy(z) == 0  # destroying nothing is a no-op


def test_reflection_orbits_reproduce_the_operator():
    """The kernels apply a = R d over the reflection orbits of the data columns (sign-pattern sums
    times the reduced operator RS).  Expanded back, RS and the patterns give R exactly (rationals),
    every column sits in one orbit, and the reduced operator has 216 nonzeros against R's 678."""
    from fractions import Fraction as Fr
    from paper_2508_19911_amd import gen_recon
    R, _, _, _ = gen_recon.exact_operator()
    orbits, patterns, RS = gen_recon.orbit_tables(R)
    cols = sorted(c for o in orbits for c in o)
    assert cols == list(range(75))
    back = [[Fr(0)] * 75 for _ in range(34)]
    for k, (o, signs) in enumerate(patterns):
        for r, c in enumerate(orbits[o]):
            for m in range(34):
                back[m][c] += RS[m][k] * signs[r]
    assert back == R
    assert sum(1 for row in RS for v in row if v != 0) == 216
    assert sum(1 for row in R for v in row if v != 0) == 678


@pytest.mark.parametrize("n", [8, 16, 32])
def test_host_turbulence_field_matches_inputs(n):
    """cgks_ic_host (C++ in the library: counter-based normals, radix-2 FFTs) against inputs.hit_state
    (numpy FFTs) on the same seed: the same field to rounding.  A host computation; no GPU."""
    from paper_2508_19911_amd import cgks, inputs
    case = inputs.hit_case(n, ma_t=0.5, seed=20250827 + n)
    q, g = cgks.ic_host(case, cgks.IC_HIT, [case.ma, 8.0], case.seed)
    qp, gp = inputs.hit_state(case)
    assert np.abs(q - qp).max() <= 1e-12 * np.abs(qp).max()
    assert np.abs(g - gp).max() <= 1e-12 * np.abs(gp).max()
    # the field itself: zero mean velocity, u_rms = 1 per component on average, divergence-free
    # cell-averaged gradients (to rounding), uniform density and pressure
    u = q[1:4] / q[0]
    assert np.abs(u.mean(axis=1)).max() <= 1e-12
    assert abs((u ** 2).sum(0).mean() - 3.0) <= 1e-12
    div = g[1] + g[7] + g[13]
    assert np.abs(div).max() <= 1e-10 * np.abs(g[1]).max()
    assert np.all(q[0] == 1.0)
    # another seed gives another field
    q2, _ = cgks.ic_host(case, cgks.IC_HIT, [case.ma], case.seed + 1)
    assert np.abs(q2[1] - q[1]).max() > 0.1


def test_host_turbulence_field_rejects_bad_grids():
    from paper_2508_19911_amd import cgks, inputs
    lib = cgks.load()
    q = np.zeros((5, 24 ** 3)); g = np.zeros((15, 24 ** 3))
    prm = np.array([0.5])
    P = ctypes.c_void_p
    for case in (inputs.hit_case(24), inputs.hit_case(16).with_(nz=8), inputs.hit_case(16).with_(lz=1.0)):
        p = cgks.params_from_case(case)
        assert lib.cgks_ic_host(ctypes.byref(p), cgks.IC_HIT, prm.ctypes.data_as(P), 1, 1,
                                q.ctypes.data_as(P), g.ctypes.data_as(P)) == -1
    p = cgks.params_from_case(inputs.hit_case(16))
    for kind in (cgks.IC_TGV, cgks.IC_VORTEX2D, 7):
        assert lib.cgks_ic_host(ctypes.byref(p), kind, prm.ctypes.data_as(P), 1, 1,
                                q.ctypes.data_as(P), g.ctypes.data_as(P)) == -1
    bad = np.array([0.0])
    assert lib.cgks_ic_host(ctypes.byref(p), cgks.IC_HIT, bad.ctypes.data_as(P), 1, 1,
                            q.ctypes.data_as(P), g.ctypes.data_as(P)) == -1
