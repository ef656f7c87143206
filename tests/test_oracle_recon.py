"""Pins of the oracle's reconstruction (arXiv 2508.19911, Sec. 3.2-3.3).

* P^4 reproduces any quartic exactly from exact cell averages and exact cell-averaged gradients
  (the constrained least-squares problem of eq. (compact-big-5) is consistent for quartics);
* the 18 neighbour averages are matched exactly (the "satisfied exactly" rows);
* Gauss-point values converge at fifth order and derivatives at fourth order on smooth data;
* GENO special cases: constant and linear data give chi = 1 and exact values; a jump gives chi ~ 0
  and the blend falls back to the averaged linear sub-stencil polynomials;
* GKS-2nd (Sec. 3.3): central slopes reproduce linear data, and the Venkatakrishnan factor is 1
  there; with eps = 0 the limited face values never leave the range of the 7-cell stencil (the
  factor phi(y) = (y^2 + 2y)/(y^2 + y + 2) of y = Delta1/Delta2 never exceeds y) and an extremum
  cell keeps its average on every face; a hand-worked case fixes eps^2 = (K h)^3 and the sign rule
  of Delta1; phi is the minimum over the six face midpoints.
"""
import math

import numpy as np
import pytest

import oracle

P = oracle.make_params(8, 8, 8, 1, 1, 1, gamma=1.4)
OFF = oracle.stencil_offsets()
GP = oracle.face_gauss_points()


def face_points(h):
    """Physical coordinates (relative to the cell centre) of the 24 face Gauss points, faces
    (-x,+x,-y,+y,-z,+z) x 4, tangential axes cyclic."""
    pts = np.zeros((6, 4, 3))
    for f in range(6):
        e = f // 2
        for k in range(4):
            x = np.zeros(3)
            x[e] = 0.5 if f % 2 else -0.5
            x[(e + 1) % 3] = GP[k, 0]
            x[(e + 2) % 3] = GP[k, 1]
            pts[f, k] = x * h
    return pts


def exact_box_avg_monomial(d, lo, hi):
    r = 1.0
    for k in range(3):
        n = d[k]
        r *= (hi[k] ** (n + 1) - lo[k] ** (n + 1)) / (n + 1) / (hi[k] - lo[k])
    return r


def quartic(rng):
    terms = []
    for a in range(5):
        for b in range(5 - a):
            for c in range(5 - a - b):
                terms.append(((a, b, c), rng.normal()))
    return terms


def poly_avg(terms, lo, hi):
    return sum(c * exact_box_avg_monomial(d, lo, hi) for d, c in terms)


def poly_grad_avg(terms, lo, hi):
    g = np.zeros(3)
    for d, c in terms:
        for e in range(3):
            if d[e] == 0:
                continue
            dd = list(d); dd[e] -= 1
            g[e] += c * d[e] * exact_box_avg_monomial(dd, lo, hi)
    return g


def poly_val(terms, x):
    return sum(c * x[0] ** d[0] * x[1] ** d[1] * x[2] ** d[2] for d, c in terms)


def poly_grad(terms, x):
    g = np.zeros(3)
    for d, c in terms:
        for e in range(3):
            if d[e] == 0:
                continue
            dd = list(d); dd[e] -= 1
            g[e] += c * d[e] * x[0] ** dd[0] * x[1] ** dd[1] * x[2] ** dd[2]
    return g


def stencil_data(terms, h):
    q = np.zeros(19); g = np.zeros((19, 3))
    for s in range(19):
        lo = (OFF[s] - 0.5) * h; hi = (OFF[s] + 0.5) * h
        q[s] = poly_avg(terms, lo, hi)
        g[s] = poly_grad_avg(terms, lo, hi)
    return q, g


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_quartic_reproduced_exactly(seed):
    rng = np.random.default_rng(seed)
    h = np.array([0.3, 0.5, 0.4])
    terms = quartic(rng)
    q, g = stencil_data(terms, h)
    out, info = oracle.recon_cell(P, q, g, h, 0)
    pts = face_points(h)
    for f in range(6):
        for k in range(4):
            x = pts[f, k]
            assert abs(out[f, k, 0] - poly_val(terms, x)) <= 1e-12 * 30
            assert np.allclose(out[f, k, 1:], poly_grad(terms, x), rtol=0, atol=1e-11 * 30)


def test_operator_matches_neighbour_averages_exactly():
    """The constraint rows: the mean of P^4 over every neighbour equals its average (any data)."""
    R = oracle.recon_operator()
    rng = np.random.default_rng(5)
    data = rng.normal(size=75)
    a = R @ data
    # basis means over the neighbour cells, built here from the definition of eq. (base)
    idx = [(x, y, dg - x - y) for dg in range(1, 5) for x in range(dg, -1, -1) for y in range(dg - x, -1, -1)]
    fact = math.factorial
    for n in range(18):
        o = OFF[n + 1]
        s = 0.0
        for j, d in enumerate(idx):
            m_o = exact_box_avg_monomial(d, o - 0.5, o + 0.5) / (fact(d[0]) * fact(d[1]) * fact(d[2]))
            m_0 = exact_box_avg_monomial(d, -0.5 * np.ones(3), 0.5 * np.ones(3)) / (fact(d[0]) * fact(d[1]) * fact(d[2]))
            s += a[j] * (m_o - m_0)
        assert abs(s - data[n]) <= 1e-12 * np.abs(data).max() * 10


def _trig_data(h, k, phase):
    """Exact cell averages / cell-averaged gradients of f = sin(k.x + phase) on the stencil."""
    def avg_sin_cos(lo, hi):
        # average of exp(i(k.x + phase)) over the box: product of 1-D averages
        z = np.exp(1j * phase)
        for e in range(3):
            if k[e] == 0:
                continue
            z *= (np.exp(1j * k[e] * hi[e]) - np.exp(1j * k[e] * lo[e])) / (1j * k[e] * (hi[e] - lo[e]))
        return z
    q = np.zeros(19); g = np.zeros((19, 3))
    for s in range(19):
        lo = (OFF[s] - 0.5) * h; hi = (OFF[s] + 0.5) * h
        z = avg_sin_cos(lo, hi)
        q[s] = z.imag
        g[s] = (1j * np.array(k) * z).imag
    return q, g


@pytest.mark.parametrize("mode", [0, 1])
def test_convergence_order(mode):
    k = np.array([1.1, -0.7, 0.9])
    errs_v, errs_d = [], []
    for h0 in (0.2, 0.1, 0.05):
        h = np.array([h0, h0, h0])
        q, g = _trig_data(h, k, 0.3)
        out, _ = oracle.recon_cell(P, q, g, h, mode)
        pts = face_points(h)
        ev = ed = 0.0
        for f in range(6):
            for j in range(4):
                x = pts[f, j]
                ev = max(ev, abs(out[f, j, 0] - math.sin(k @ x + 0.3)))
                ed = max(ed, np.abs(out[f, j, 1:] - k * math.cos(k @ x + 0.3)).max())
        errs_v.append(ev); errs_d.append(ed)
    ov = math.log2(errs_v[1] / errs_v[2])
    od = math.log2(errs_d[1] / errs_d[2])
    assert ov > 4.6, errs_v
    assert od > 3.6, errs_d


def test_geno_constant_and_linear_data():
    h = np.array([0.1, 0.2, 0.15])
    q = np.full(19, 2.5); g = np.zeros((19, 3))
    out, info = oracle.recon_cell(P, q, g, h, 1)
    assert info[0] == 1.0
    assert np.all(out[:, :, 0] == 2.5) and np.all(out[:, :, 1:] == 0.0)
    grad = np.array([0.7, -1.2, 0.4])
    terms = [((0, 0, 0), 1.3), ((1, 0, 0), grad[0]), ((0, 1, 0), grad[1]), ((0, 0, 1), grad[2])]
    q, g = stencil_data(terms, h)
    out, info = oracle.recon_cell(P, q, g, h, 1)
    assert abs(info[0] - 1.0) <= 1e-12
    pts = face_points(h)
    for f in range(6):
        for j in range(4):
            assert abs(out[f, j, 0] - poly_val(terms, pts[f, j])) <= 1e-13
            assert np.allclose(out[f, j, 1:], grad, atol=1e-12)
    lin, _ = oracle.recon_cell(P, q, g, h, 0)
    assert np.allclose(out, lin, atol=1e-13)


def test_geno_jump_falls_back_to_low_order():
    h = np.array([0.1, 0.1, 0.1])
    q = np.array([0.0 if o[0] <= 0 else 1.0 for o in OFF], dtype=float)  # jump at the +x face
    g = np.zeros((19, 3))
    out, info = oracle.recon_cell(P, q, g, h, 1)
    assert info[0] < 1e-3
    # values stay within the stencil's range (the linear part is almost flat: omega_{+x} ~ 0)
    assert out[:, :, 0].min() > -1e-3 and out[:, :, 0].max() < 1 + 1e-3
    lin, _ = oracle.recon_cell(P, q, g, h, 0)
    assert lin[:, :, 0].min() < -0.05 or lin[:, :, 0].max() > 1.05  # the quartic overshoots


def test_geno_chi_is_one_when_selected_data_is_smooth():
    # smooth quartic data: chi stays within O(h^4) of 1
    rng = np.random.default_rng(9)
    terms = [((0, 0, 0), 1.0), ((1, 0, 0), 0.8), ((0, 1, 0), -0.5), ((0, 0, 1), 0.3)] + [
        (d, 0.1 * c) for d, c in quartic(rng) if sum(d) >= 2]
    chis = []
    for h0 in (0.1, 0.05):
        h = np.full(3, h0)
        q, g = stencil_data(terms, h)
        _, info = oracle.recon_cell(P, q, g, h, 1)
        chis.append(abs(1 - info[0]))
    assert chis[0] < 1e-2 and chis[1] < chis[0] / 8


@pytest.mark.parametrize("k", [(1.0, 0.0, 0.0), (0.8, 0.6, 0.5)])
def test_geno_smoothness_floor_at_smooth_extremum(k):
    """At a smooth extremum every linear sub-stencil slope vanishes, so with the bare epsilon the
    path function drops to the low-order blend (chi = 0) however fine the grid; with the floor
    eps + h_max^2 S (S = the variable's magnitude squared) 1 - chi falls at least as h^5."""
    k = np.array(k)
    bare, floor = [], []
    for h0 in (0.1, 0.05):
        h = np.full(3, h0)
        q, g = _trig_data(h, k, np.pi / 2)  # cos(k.x): extremum at the cell centre
        q = q + 2.0
        _, i0 = oracle.recon_cell(P, q, g, h, 1, scale=0.0)
        _, i1 = oracle.recon_cell(P, q, g, h, 1, scale=4.0)
        bare.append(1 - i0[0]); floor.append(1 - i1[0])
    assert min(bare) > 0.5, bare
    assert floor[0] < 1e-6 and floor[1] < floor[0] / 32, floor


def test_geno_scale_definition():
    q5 = np.array([1.2, 0.3, -0.1, 0.2, 2.5])
    assert oracle.geno_scale(q5, 0) == 1.2 ** 2
    assert oracle.geno_scale(q5, 4) == 2.5 ** 2
    for v in (1, 2, 3):
        assert oracle.geno_scale(q5, v) == 2 * 1.2 * 2.5


# ---------------------------------------------------------------------------------------------------
# GKS-2nd P^1 and the Venkatakrishnan limiter (Sec. 3.3, reading R13).  q7 = (cell, -x, +x, -y, +y,
# -z, +z); faces in the same order as the neighbours.
FACE_SIGN = np.array([-0.5, 0.5, -0.5, 0.5, -0.5, 0.5])


def test_gks2_linear_data_exact_and_unlimited():
    rng = np.random.default_rng(21)
    for _ in range(20):
        h = rng.uniform(0.05, 0.4, size=3)
        grad = rng.normal(size=3)
        q0 = rng.normal()
        q7 = np.array([q0] + [q0 + sgn * grad[e] * h[e] for e in range(3) for sgn in (-1.0, 1.0)])
        for limited in (0, 1):
            P = oracle.make_params(8, 8, 8, 1, 1, 1, vk_k=rng.uniform(0.0, 3.0))
            out, phi = oracle.recon_cell_gks2(P, q7, h, limited)
            # the direction of the largest slope has Delta1 = 2 Delta2 exactly, where the factor
            # is 1 in exact arithmetic
            assert abs(phi - 1.0) <= 1e-14
            for f in range(6):
                e = f // 2
                assert abs(out[f, 0] - (q0 + FACE_SIGN[f] * grad[e] * h[e])) <= 1e-14 * (1 + abs(q0))
                assert np.allclose(out[f, 1:], grad, rtol=1e-13, atol=1e-13)
    # constant data: no slope, factor 1
    out, phi = oracle.recon_cell_gks2(oracle.make_params(8, 8, 8, 1, 1, 1), np.full(7, 2.5), np.ones(3), 1)
    assert phi == 1.0 and np.all(out[:, 0] == 2.5) and np.all(out[:, 1:] == 0.0)


def test_vk_without_eps_keeps_face_values_in_the_stencil_range():
    """eps = 0 (K = 0): the limited value at every face midpoint lies in [min q7, max q7]."""
    P = oracle.make_params(8, 8, 8, 1, 1, 1, vk_k=0.0)
    rng = np.random.default_rng(22)
    h = np.array([0.1, 0.2, 0.15])
    clipped = 0
    for _ in range(400):
        q7 = rng.normal(size=7) * rng.uniform(0.01, 10.0)
        out, phi = oracle.recon_cell_gks2(P, q7, h, 1)
        lo, hi = q7.min(), q7.max()
        tol = 1e-14 * np.abs(q7).max()
        assert np.all(out[:, 0] >= lo - tol) and np.all(out[:, 0] <= hi + tol), (q7, out[:, 0])
        unl, _ = oracle.recon_cell_gks2(P, q7, h, 0)
        clipped += (unl[:, 0].min() < lo - tol) or (unl[:, 0].max() > hi + tol)
    assert clipped > 100  # the unlimited P^1 does overshoot on such data


def test_vk_extremum_cell_keeps_its_average():
    """A strict local maximum (or minimum) with eps = 0: Delta1 = 0 on the faces the slope points
    up, so phi = 0 and every face takes the cell average."""
    P = oracle.make_params(8, 8, 8, 1, 1, 1, vk_k=0.0)
    rng = np.random.default_rng(23)
    for sign in (1.0, -1.0):
        q7 = np.concatenate([[sign * 2.0], sign * rng.uniform(0.0, 1.5, size=6)])
        out, phi = oracle.recon_cell_gks2(P, q7, np.ones(3), 1)
        assert phi == 0.0
        assert np.all(out[:, 0] == q7[0]) and np.all(out[:, 1:] == 0.0)


def test_vk_hand_worked_case():
    """q7 = (1; 0, 4 along x; 1, 1, 1, 1), cubic cells h = 1/4, K = 2, so eps^2 = (K h)^3 = 1/8.
    x slope b = (4 - 0)/2 = 2 (per unit of the normalised coordinate).
      -x face: Delta2 = -1 < 0, so Delta1 = min - Q0 = -1:
               phi = (1 + 1/8 + 2) / (1 + 2 + 1 + 1/8) = 25/33;
      +x face: Delta2 = +1, Delta1 = max - Q0 = 3: (9 + 1/8 + 6)/(9 + 2 + 3 + 1/8) = 121/113 > 1;
      y, z faces: Delta2 = 0, factor 1.
    So phi = 25/33: face values 1 -+ 25/33, d/dx = (25/33) 2 / h."""
    P = oracle.make_params(8, 8, 8, 1, 1, 1, vk_k=2.0)
    h = np.full(3, 0.25)
    out, phi = oracle.recon_cell_gks2(P, [1, 0, 4, 1, 1, 1, 1], h, 1)
    assert abs(phi - 25.0 / 33.0) <= 1e-15
    assert abs(out[0, 0] - (1 - 25.0 / 33.0)) <= 1e-15 and abs(out[1, 0] - (1 + 25.0 / 33.0)) <= 1e-15
    assert np.all(out[2:, 0] == 1.0)
    assert abs(out[0, 1] - 25.0 / 33.0 * 2 / 0.25) <= 1e-13 and np.all(out[:, 2:] == 0.0)
    # the same data with eps^2 read as (K h)^2 = 1/4 would give 13/17
    assert abs(phi - 13.0 / 17.0) > 5e-3


def _vk_face_factor(d1, d2, e2):
    return 1.0 if d2 == 0.0 else ((d1 * d1 + e2) + 2 * d1 * d2) / (d1 * d1 + 2 * d2 * d2 + d1 * d2 + e2)


def test_vk_factor_is_the_minimum_over_the_six_faces():
    """Every face scales its slope by one common phi, the smallest of the six face factors, so the
    ratio (face value - Q0) / (face offset x slope) is the same on all faces."""
    rng = np.random.default_rng(24)
    K = 1.0
    h = np.full(3, 0.1)
    P = oracle.make_params(8, 8, 8, 1, 1, 1, vk_k=K)
    seen_different = 0
    for _ in range(100):
        q7 = rng.normal(size=7)
        out, phi = oracle.recon_cell_gks2(P, q7, h, 1)
        b = np.array([0.5 * (q7[2 + 2 * e] - q7[1 + 2 * e]) for e in range(3)])
        e2 = (K * 0.1) ** 3
        fac = []
        for f in range(6):
            d2 = FACE_SIGN[f] * b[f // 2]
            d1 = (q7.max() - q7[0]) if d2 > 0 else (q7.min() - q7[0])
            fac.append(_vk_face_factor(d1, d2, e2))
        assert abs(phi - min(1.0, min(fac))) <= 1e-14
        for f in range(6):
            assert abs(out[f, 0] - (q7[0] + phi * FACE_SIGN[f] * b[f // 2])) <= 1e-14
        seen_different += np.ptp(np.minimum(fac, 1.0)) > 1e-3
    assert seen_different > 50
