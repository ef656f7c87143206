"""Build-time generator of the compact reconstruction tables used by the HIP kernels.

Solves the constrained least-squares problem of the fifth-order compact reconstruction
(arXiv 2508.19911, Sec. 3.2, eq. (compact-big-5)) once, in exact rational arithmetic, for a uniform
Cartesian cell in normalised coordinates (delta = (x - x0)/h on [-1/2, 1/2]^3):

* unknowns: the 34 coefficients a_d of the zero-mean basis p_d = delta^d/d! - mean, 1 <= |d| <= 4
  (eq. (base));
* exact rows: the mean of P^4 over each of the 18 neighbours (6 face, 12 edge) equals Q_k - Q0;
* least-squares rows (unit weight): the mean of h_e dP/dx_e over each of the 19 cells equals
  h_e (dQ/dx_e) of that cell, all three components (the cell-averaged gradient is the derivative
  data of every stencil cell).

The solution a = R d is linear in the 75 data; R is emitted with the basis values and derivatives
at the 2x2 Gauss points of the six faces (exact in Q(sqrt 3)), at the 3x3x3 Gauss-Legendre points
of the cell (for the quadrature of the diagnostics), and the Gram matrix of the higher-order
smoothness indicator sum_{1<=|alpha|<=4} int (D^alpha P)^2.  Output:
``csrc/recon_tables.hpp``.  Run: ``python -m paper_2508_19911_amd.gen_recon``.
"""
from __future__ import annotations

import decimal
import os
from fractions import Fraction as Fr
from math import factorial

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "csrc", "recon_tables.hpp")

# stencil in memory order (z, then y, then x) with |dx|+|dy|+|dz| <= 2
STENCIL = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
           if abs(dx) + abs(dy) + abs(dz) <= 2]
CENTRE = STENCIL.index((0, 0, 0))
NEIGH = [s for s in STENCIL if s != (0, 0, 0)]
# basis multi-indices: by degree, then lexicographic in (d3, d2, d1)
BASIS = sorted([(a, b, c) for a in range(5) for b in range(5) for c in range(5) if 1 <= a + b + c <= 4],
               key=lambda d: (sum(d), d[2], d[1], d[0]))
NB = len(BASIS)
assert NB == 34 and len(STENCIL) == 19


def interval_mean(n: int, o: int) -> Fr:
    """Mean of x^n over [o - 1/2, o + 1/2]."""
    hi, lo = Fr(2 * o + 1, 2), Fr(2 * o - 1, 2)
    return (hi ** (n + 1) - lo ** (n + 1)) / (n + 1)


def mono_mean(d, o) -> Fr:
    r = Fr(1)
    for k in range(3):
        r *= interval_mean(d[k], o[k]) / factorial(d[k])
    return r


CELL_MEAN = [mono_mean(d, (0, 0, 0)) for d in BASIS]


def basis_mean_over(j, o) -> Fr:
    return mono_mean(BASIS[j], o) - CELL_MEAN[j]


def dbasis_mean_over(j, e, o) -> Fr:
    d = list(BASIS[j])
    if d[e] == 0:
        return Fr(0)
    d[e] -= 1
    return mono_mean(d, o)


def solve_exact(A, B):
    """Gauss-Jordan elimination over the rationals: returns X with A X = B."""
    n = len(A)
    M = [row[:] + brow[:] for row, brow in zip(A, B)]
    m = len(B[0])
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        inv = 1 / M[c][c]
        M[c] = [v * inv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [vr - f * vc for vr, vc in zip(M[r], M[c])]
    return [row[n:n + m] for row in M]


def build_operator():
    # exact rows C (18 x NB), least-squares rows A (57 x NB)
    C = [[basis_mean_over(j, o) for j in range(NB)] for o in NEIGH]
    A = [[dbasis_mean_over(j, e, o) for j in range(NB)] for o in STENCIL for e in range(3)]
    nA = len(A)
    n = NB + len(C)
    K = [[Fr(0)] * n for _ in range(n)]
    for i in range(NB):
        for j in range(NB):
            K[i][j] = sum(A[r][i] * A[r][j] for r in range(nA))
    for r, row in enumerate(C):
        for j in range(NB):
            K[NB + r][j] = row[j]
            K[j][NB + r] = row[j]
    ncol = len(C) + nA
    rhs = [[Fr(0)] * ncol for _ in range(n)]
    for r in range(len(C)):
        rhs[NB + r][r] = Fr(1)
    for r in range(nA):
        for i in range(NB):
            rhs[i][len(C) + r] = A[r][i]
    X = solve_exact(K, rhs)
    return [X[i] for i in range(NB)]  # NB x 75


# ---- numbers a + b sqrt(3) ------------------------------------------------------------------------
class Q3:
    __slots__ = ("a", "b")

    def __init__(self, a, b=Fr(0)):
        self.a, self.b = Fr(a), Fr(b)

    def __mul__(self, o):
        o = o if isinstance(o, Q3) else Q3(o)
        return Q3(self.a * o.a + 3 * self.b * o.b, self.a * o.b + self.b * o.a)

    def __add__(self, o):
        o = o if isinstance(o, Q3) else Q3(o)
        return Q3(self.a + o.a, self.b + o.b)

    def __sub__(self, o):
        o = o if isinstance(o, Q3) else Q3(o)
        return Q3(self.a - o.a, self.b - o.b)

    def pow(self, n):
        r = Q3(1)
        for _ in range(n):
            r = r * self
        return r

    def to_float(self) -> float:
        with decimal.localcontext() as ctx:
            ctx.prec = 60
            v = decimal.Decimal(self.a.numerator) / decimal.Decimal(self.a.denominator) + \
                decimal.Decimal(self.b.numerator) / decimal.Decimal(self.b.denominator) * decimal.Decimal(3).sqrt()
            return float(v)


G = Q3(0, Fr(1, 6))  # Gauss-Legendre 2-point abscissa on [-1/2,1/2]: 1/(2 sqrt 3) = sqrt(3)/6
# Gauss points of a face: tangential signs (s1, s2) along the cyclic tangential axes
GP_SIGNS = [(-1, -1), (-1, 1), (1, -1), (1, 1)]


def gauss_point(f, k):
    e = f // 2
    x = [None, None, None]
    x[e] = Q3(Fr(1, 2) if f % 2 else Fr(-1, 2))
    s1, s2 = GP_SIGNS[k]
    x[(e + 1) % 3] = G * s1
    x[(e + 2) % 3] = G * s2
    return x


def mono_at(d, x):
    r = Q3(1)
    for k in range(3):
        r = r * x[k].pow(d[k]) * Fr(1, factorial(d[k]))
    return r


def basis_tables():
    PV = [[[None] * NB for _ in range(4)] for _ in range(6)]
    PD = [[[[None] * NB for _ in range(4)] for _ in range(4)] for _ in range(6)]
    for f in range(6):
        for k in range(4):
            x = gauss_point(f, k)
            for j, d in enumerate(BASIS):
                PV[f][k][j] = (mono_at(d, x) - CELL_MEAN[j]).to_float()
                for e in range(3):
                    if d[e] == 0:
                        PD[f][k][e][j] = 0.0
                    else:
                        dd = list(d); dd[e] -= 1
                        PD[f][k][e][j] = mono_at(dd, x).to_float()
    return PV, PD


# ---- 3x3x3 Gauss-Legendre points of the cell (volume quadrature of the diagnostics) ----------------
# abscissae 0, +-sqrt(15)/10 on [-1/2, 1/2], weights 4/9 and 5/18 (exact for degree 5 per axis)
VQ_ABS = [-1, 0, 1]          # multiples of sqrt(15)/10
VQ_W1 = [Fr(5, 18), Fr(4, 9), Fr(5, 18)]


def _dec(fr):
    return decimal.Decimal(fr.numerator) / decimal.Decimal(fr.denominator)


def volume_tables():
    """Points (x fastest), weights, basis values p_m and derivatives d p_m / d delta_e at the 27 points."""
    with decimal.localcontext() as ctx:
        ctx.prec = 60
        r = decimal.Decimal(15).sqrt() / 10
        pts, wts, PVQ, PDQ = [], [], [], []
        for kz in range(3):
            for ky in range(3):
                for kx in range(3):
                    x = [VQ_ABS[kx] * r, VQ_ABS[ky] * r, VQ_ABS[kz] * r]
                    pts.append([float(v) for v in x])
                    wts.append(float(_dec(VQ_W1[kx] * VQ_W1[ky] * VQ_W1[kz])))

                    def mono(d):
                        v = decimal.Decimal(1)
                        for k in range(3):
                            if d[k]:
                                v *= x[k] ** d[k] / factorial(d[k])
                        return v
                    PVQ.append([float(mono(d) - _dec(CELL_MEAN[j])) for j, d in enumerate(BASIS)])
                    der = []
                    for e in range(3):
                        row = []
                        for d in BASIS:
                            if d[e] == 0:
                                row.append(0.0)
                            else:
                                dd = list(d)
                                dd[e] -= 1
                                row.append(float(mono(dd)))
                        der.append(row)
                    PDQ.append(der)
    return pts, wts, PVQ, PDQ


def gram():
    def cell_int(n):  # integral of x^n over [-1/2,1/2]
        return Fr(0) if n % 2 else Fr(2, n + 1) * Fr(1, 2) ** (n + 1)
    Gm = [[Fr(0)] * NB for _ in range(NB)]
    for al in BASIS:
        for i, di in enumerate(BASIS):
            for j, dj in enumerate(BASIS):
                r = Fr(1)
                for k in range(3):
                    mi, mj = di[k] - al[k], dj[k] - al[k]
                    if mi < 0 or mj < 0:
                        r = Fr(0)
                        break
                    r *= cell_int(mi + mj) / (factorial(mi) * factorial(mj))
                Gm[i][j] += r
    return Gm


def fmt(v: float) -> str:
    return repr(float(v))


def generate() -> str:
    R = build_operator()
    PV, PD = basis_tables()
    Gm = gram()
    L = []
    L.append("// Generated by paper_2508_19911_amd/gen_recon.py -- do not edit.")
    L.append("// Compact fifth-order reconstruction on a uniform Cartesian cell (arXiv 2508.19911, Sec. 3.2):")
    L.append("// exact-rational solution of the constrained least-squares system, basis values at the face")
    L.append("// Gauss points, and the Gram matrix of the smoothness indicator.")
    L.append("#pragma once")
    L.append("namespace cgks {")
    L.append("namespace tab {")
    L.append(f"constexpr int NB = {NB};        // basis functions, 1 <= |d| <= 4")
    L.append("constexpr int NSTEN = 19;      // stencil cells")
    L.append("constexpr int NDATA = 75;      // 18 value differences + 19 x 3 normalised gradients")
    L.append(f"constexpr int CENTRE = {CENTRE}; // index of the cell itself in SOFF")
    L.append("// stencil offsets (dx, dy, dz) in memory order")
    L.append("constexpr int SOFF[19][3] = {" + ", ".join("{%d,%d,%d}" % s for s in STENCIL) + "};")
    L.append("// basis exponents (d1, d2, d3): p_d = dx^d1 dy^d2 dz^d3 / (d1! d2! d3!) - cell mean")
    L.append("constexpr int BD[34][3] = {" + ", ".join("{%d,%d,%d}" % d for d in BASIS) + "};")
    L.append("// data vector: d[n] = Q(neighbour n) - Q0 for n < 18 (SOFF order without the centre);")
    L.append("//              d[18 + 3 s + e] = h_e dQ/dx_e of stencil cell s")
    L.append("constexpr int NEIGH_SLOT[19] = {" + ", ".join(
        str(NEIGH.index(s)) if s != (0, 0, 0) else "-1" for s in STENCIL) + "};")
    L.append("// a = R d")
    L.append("constexpr double R[34][75] = {")
    for i in range(NB):
        L.append("  {" + ", ".join(fmt(v) for v in R[i]) + "},")
    L.append("};")
    nnz = sum(1 for i in range(NB) for v in R[i] if v != 0)
    L.append(f"constexpr int R_NNZ = {nnz};")
    orbits, patterns, RS = orbit_tables(R)
    L.append("// reflection orbits of the data columns (members, -1 unused), their sign patterns (each a run")
    L.append("// of patterns per orbit) and the reduced operator: a[m] += RS[m][k] * sum_r PAT_SIGN[k][r] d[ORB_COL[o][r]]")
    L.append(f"constexpr int NORB = {len(orbits)};")
    L.append(f"constexpr int NPAT = {len(patterns)};")
    L.append("constexpr int ORB_SIZE[NORB] = {" + ", ".join(str(len(o)) for o in orbits) + "};")
    L.append("constexpr int ORB_COL[NORB][4] = {" + ", ".join(
        "{" + ", ".join(str(c) for c in (o + [-1] * (4 - len(o)))) + "}" for o in orbits) + "};")
    first = [next(k for k, p in enumerate(patterns) if p[0] == o) for o in range(len(orbits))]
    count = [sum(1 for p in patterns if p[0] == o) for o in range(len(orbits))]
    L.append("constexpr int ORB_PAT0[NORB] = {" + ", ".join(map(str, first)) + "};")
    L.append("constexpr int ORB_NPAT[NORB] = {" + ", ".join(map(str, count)) + "};")
    L.append("constexpr int PAT_SIGN[NPAT][4] = {" + ", ".join(
        "{" + ", ".join(str(v) for v in (list(p[1]) + [0] * (4 - len(p[1])))) + "}" for p in patterns) + "};")
    L.append("constexpr double RS[34][NPAT] = {")
    for i in range(NB):
        L.append("  {" + ", ".join(fmt(v) for v in RS[i]) + "},")
    L.append("};")
    L.append(f"constexpr int RS_NNZ = {sum(1 for i in range(NB) for v in RS[i] if v != 0)};")
    L.append("// faces f = (-x,+x,-y,+y,-z,+z); Gauss point k: tangential signs along ((e+1)%3, (e+2)%3)")
    L.append("constexpr int GP_SIGN[4][2] = {" + ", ".join("{%d,%d}" % s for s in GP_SIGNS) + "};")
    L.append("// PV[f][k][m] = p_m at Gauss point k of face f; PD[f][k][e][m] = d p_m / d delta_e there")
    L.append("constexpr double PV[6][4][34] = {")
    for f in range(6):
        L.append("  {" + ", ".join("{" + ", ".join(fmt(v) for v in PV[f][k]) + "}" for k in range(4)) + "},")
    L.append("};")
    L.append("constexpr double PD[6][4][3][34] = {")
    for f in range(6):
        L.append("  {" + ", ".join("{" + ", ".join("{" + ", ".join(fmt(v) for v in PD[f][k][e]) + "}"
                                                 for e in range(3)) + "}" for k in range(4)) + "},")
    L.append("};")
    vp, vw, PVQ, PDQ = volume_tables()
    L.append("// 3x3x3 Gauss-Legendre points of the cell (x fastest): normalised coordinates, weights (sum 1),")
    L.append("// PVQ[q][m] = p_m there, PDQ[q][e][m] = d p_m / d delta_e there")
    L.append("constexpr int NVQ = 27;")
    L.append("constexpr double VQ_X[27][3] = {" + ", ".join("{" + ", ".join(fmt(v) for v in x) + "}" for x in vp) + "};")
    L.append("constexpr double VQ_W[27] = {" + ", ".join(fmt(v) for v in vw) + "};")
    L.append("constexpr double PVQ[27][34] = {")
    for q in range(27):
        L.append("  {" + ", ".join(fmt(v) for v in PVQ[q]) + "},")
    L.append("};")
    L.append("constexpr double PDQ[27][3][34] = {")
    for q in range(27):
        L.append("  {" + ", ".join("{" + ", ".join(fmt(v) for v in PDQ[q][e]) + "}" for e in range(3)) + "},")
    L.append("};")
    L.append("// IS_H = a^T GR a, GR[i][j] = sum_{1<=|alpha|<=4} int_cell D^alpha p_i D^alpha p_j")
    L.append("constexpr double GR[34][34] = {")
    for i in range(NB):
        L.append("  {" + ", ".join(fmt(v) for v in Gm[i]) + "},")
    L.append("};")
    L.append("}  // namespace tab")
    L.append("}  // namespace cgks")
    return "\n".join(L) + "\n"


# ---- reflection symmetry of the operator ----------------------------------------------------------
# The stencil, the basis and the least-squares weights are invariant under the reflections x -> -x,
# y -> -y, z -> -z, so R is equivariant: a column's image under a reflection g (the datum at the
# reflected offset; a gradient component along a flipped axis changes sign) carries R[m][c] times the
# basis function's parity chi_m(g).  Grouping the 75 columns into orbits, sum_c R[m][c] d_c becomes
# sum over orbits of R[m][c0] D_{o,k(m)} with D_{o,k} = sum_{c in o} s_k(c) d_c: 216 FMAs and the
# pattern sums instead of 678 FMAs.  Checked exactly here.
def data_columns():
    cols = [("v", o, -1) for o in NEIGH] + [("g", o, e) for o in STENCIL for e in range(3)]
    return cols


def orbit_tables(R=None):
    """Orbits of the data columns, their sign patterns and the reduced operator (exact Fractions).
    Returns (orbits: list of member-column lists, patterns: list of (orbit, signs), RS[m][k])."""
    import itertools
    R = R if R is not None else build_operator()
    cols = data_columns()
    index = {c: i for i, c in enumerate(cols)}
    group = list(itertools.product((1, -1), repeat=3))

    def image(c, g):
        t, o, e = c
        o2 = (g[0] * o[0], g[1] * o[1], g[2] * o[2])
        return index[(t, o2, e)], (1 if t == "v" else g[e])

    seen, orbits, maps = set(), [], []
    for i, c in enumerate(cols):
        if i in seen:
            continue
        mem = {}
        for g in group:
            j, sg = image(c, g)
            mem.setdefault(j, (g, sg))
        members = [i] + sorted(j for j in mem if j != i)
        orbits.append(members)
        maps.append(mem)
        seen |= set(mem)
    patterns, RS = [], [[Fr(0)] * 0 for _ in range(NB)]
    rs_cols = []
    for o, (members, mem) in enumerate(zip(orbits, maps)):
        c0 = members[0]
        pats = {}
        for m in range(NB):
            if all(R[m][j] == 0 for j in members):
                continue
            assert R[m][c0] != 0
            d = BASIS[m]
            sig = []
            for j in members:
                g, sg = mem[j]
                sgn = g[0] ** d[0] * g[1] ** d[1] * g[2] ** d[2] * sg
                assert R[m][j] == sgn * R[m][c0], (m, j)
                sig.append(sgn)
            pats.setdefault(tuple(sig), []).append(m)
        for sig, ms in pats.items():
            patterns.append((o, sig))
            col = [Fr(0)] * NB
            for m in ms:
                col[m] = R[m][c0]
            rs_cols.append(col)
    RS = [[rs_cols[k][m] for k in range(len(rs_cols))] for m in range(NB)]
    return orbits, patterns, RS


def exact_operator():
    """The exact-rational operator (for tests): R[34][75] as Fractions, with STENCIL and BASIS."""
    return build_operator(), STENCIL, NEIGH, BASIS


def main():
    src = generate()
    with open(OUT, "w") as f:
        f.write(src)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
