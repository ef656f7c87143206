"""The Taylor-Green workloads against the set-ups the paper prints (Sec. 4.1 and 4.2), read from
tests/golden/tgv_setups.txt: flow constants, initial fields at scattered points, the grids of the
efficiency comparison and the paper's cost tables."""
import math
import os

import numpy as np
import pytest

from paper_2508_19911_amd import cgks, efficiency, inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tgv_setups.txt")
GAMMA = 1.4


def golden():
    out = {}
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        k, v = (s.strip() for s in line.split("=", 1))
        out[k] = v
    return out


def value(g, key, ma=None):
    """A fixture value: a number, or one of the two closed forms the paper writes."""
    v = g[key]
    forms = {"gamma*Ma^2/16": lambda: GAMMA * ma * ma / 16.0, "1/16": lambda: 1.0 / 16.0,
             "sqrt(gamma)*Ma": lambda: math.sqrt(GAMMA) * ma}
    return forms[v]() if v in forms else float(v)


def primitive(case, x, y, z):
    """rho, velocity, p of the workload's initial field at points (inverting the conservative form)."""
    q = np.asarray(inputs.tgv_field(case)(x, y, z))
    rho = q[0]
    u = q[1:4] / rho
    p = (case.gamma - 1.0) * (q[4] - 0.5 * rho * (u * u).sum(axis=0))
    return rho, u, p


@pytest.mark.parametrize("flow", ["subsonic", "supersonic"])
def test_flow_constants(flow):
    g = golden()
    sup = flow == "supersonic"
    ma = value(g, f"{flow}.Ma")
    c = inputs.tgv_case(16, ma=ma, supersonic=sup)
    assert c.gamma == GAMMA
    assert c.lx == c.ly == c.lz == pytest.approx(2 * math.pi, rel=0, abs=1e-15)
    rho0 = value(g, f"{flow}.rho0")
    assert c.rho0 == rho0
    p0 = c.sutherland_tref * c.rho0  # the Sutherland reference temperature is T0 = p0 / rho0 (R = 1)
    if sup:
        assert p0 == value(g, "supersonic.p0") and c.sutherland_tref == value(g, "supersonic.T0")
        assert c.u0 == pytest.approx(value(g, "supersonic.U0", ma), rel=1e-15)
        assert c.prandtl == value(g, "supersonic.Pr")
    else:
        assert c.u0 == value(g, "subsonic.U0")
    # Ma = U0 / sqrt(gamma p0 / rho0), Re = rho0 U0 L / mu0 with L = 1
    assert c.u0 / math.sqrt(GAMMA * p0 / rho0) == pytest.approx(ma, rel=1e-14)
    assert rho0 * c.u0 * 1.0 / c.mu0 == pytest.approx(value(g, f"{flow}.Re"), rel=1e-14)


@pytest.mark.parametrize("flow", ["subsonic", "supersonic"])
def test_initial_field(flow):
    g = golden()
    sup = flow == "supersonic"
    ma = value(g, f"{flow}.Ma")
    c = inputs.tgv_case(16, ma=ma, supersonic=sup)
    rng = np.random.default_rng(7)
    x, y, z = rng.uniform(-math.pi, 3 * math.pi, size=(3, 50))
    rho, u, p = primitive(c, x, y, z)
    a = value(g, f"{flow}.density_amplitude", ma)
    s = (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    p0 = c.sutherland_tref * c.rho0
    np.testing.assert_allclose(rho, c.rho0 * (1 + a * s), rtol=1e-14)
    np.testing.assert_allclose(p, p0 * (1 + a * s), rtol=1e-12)
    np.testing.assert_allclose(u[0], c.u0 * np.sin(x) * np.cos(y) * np.cos(z), rtol=0, atol=1e-14 * c.u0)
    np.testing.assert_allclose(u[1], -c.u0 * np.cos(x) * np.sin(y) * np.cos(z), rtol=0, atol=1e-14 * c.u0)
    np.testing.assert_allclose(u[2], 0.0, atol=1e-15 * c.u0)
    if sup:  # T = p / rho = 1 everywhere
        np.testing.assert_allclose(p / rho, value(g, "supersonic.T0"), rtol=1e-13)


@pytest.mark.parametrize("flow", ["subsonic", "supersonic"])
def test_efficiency_comparison_cases(flow):
    """The comparison runs the paper's grids and schemes and quotes the paper's table."""
    g = golden()
    c5, c2, paper = efficiency.flow_cases(flow)
    assert (c5.nx, c5.ny, c5.nz) == (int(value(g, f"{flow}.cgks5_grid")),) * 3
    assert (c2.nx, c2.ny, c2.nz) == (int(value(g, f"{flow}.gks2_grid")),) * 3
    assert c5.scheme == cgks.SCHEME_CGKS5 and c2.scheme == cgks.SCHEME_GKS2
    nonlinear = flow == "supersonic"
    assert c5.recon == c2.recon == (cgks.RECON_NONLINEAR if nonlinear else cgks.RECON_LINEAR)
    assert c5.ma == c2.ma == value(g, f"{flow}.Ma")
    assert paper["cgks5_seconds"] == value(g, f"{flow}.cgks5_seconds")
    assert paper["gks2_seconds"] == value(g, f"{flow}.gks2_seconds")
    assert paper["ratio"] == value(g, f"{flow}.ratio")
    assert round(paper["gks2_seconds"] / paper["cgks5_seconds"], 1) == paper["ratio"]
