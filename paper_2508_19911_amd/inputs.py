"""Seeded synthetic inputs for the CGKS-5th / GKS-2nd sweep.

Initial conditions of the workloads, delivered as FP64 cell averages of the conservative variables
``q[5][N]`` and cell-averaged gradients ``g[15][N]`` (d/dx of the 5 variables, then d/dy, d/dz),
SoA with x fastest.  This module is the only code shared by the oracle tests and the HIP path: it
holds none of the scheme's arithmetic, only the analytic flow fields and their cell averaging.

* isentropic vortex (Shu): free stream (rho,u,v,p) = (1,1,1,1), strength 5, periodic [0,10]^2;
* Taylor-Green vortex (Sec. 4.1 of arXiv 2508.19911; the Ma = 2 variant of Sec. 4.2), periodic
  [0, 2 pi]^3 -- a shift of the paper's [-pi, pi]^3 by half the box, the same cells for even n;
* decaying isotropic turbulence: seeded random solenoidal velocity with E(k) ~ k^4 exp(-2k^2/k0^2),
  uniform density and pressure.

Cell averages use 4-point Gauss-Legendre per direction; gradients use Gauss's theorem with 4x4
Gauss points per face, (face average(+) - face average(-)) / h.  The turbulence field uses exact
Fourier cell averages (sinc factors).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np

SCHEME_CGKS5, SCHEME_GKS2 = 0, 1
RECON_LINEAR, RECON_NONLINEAR, RECON_LEARNED = 0, 1, 2


@dataclass
class Case:
    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    gamma: float = 1.4
    mu0: float = 0.0
    prandtl: float = 1.0
    sutherland_tref: float = 0.0
    tau_eps: float = 0.05
    tau_c: float = 10.0
    vk_k: float = 1.0
    geno_dh: float = 0.85
    geno_eps: float = 1e-15
    scheme: int = SCHEME_CGKS5
    recon: int = RECON_LINEAR
    cfl: float = 0.5
    rho0: float = 1.0
    u0: float = 1.0
    # flow-specific parameters
    ma: float = 0.1
    seed: int = 0

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def h(self):
        return (self.lx / self.nx, self.ly / self.ny, self.lz / self.nz)

    def with_(self, **kw) -> "Case":
        return replace(self, **kw)


# ---- cases ----------------------------------------------------------------------------------------
# CFL number of the 3-D cases.  The convective step is dt = CFL min_cells min_d h_d / (|U_d| + c)
# (per direction).  With this form, grid-scale 3-D noise on a uniform flow grows for CFL >= 0.34
# (acoustic-dominated, Ma 0.1) and >= 0.38 (Ma 0.5) but decays at 0.30-0.32; 1-D and 2-D noise
# decay up to 0.6.  The 2-D vortex keeps 0.5, the 3-D cases run at 0.3.
CFL_3D = 0.3

def vortex_case(n: int = 64, **kw) -> Case:
    """2-D isentropic vortex on [0,10]^2 with one cell in z (h_z = h_x); inviscid."""
    L = 10.0
    c = Case("vortex2d", n, n, 1, L, L, L / n, gamma=1.4, mu0=0.0, prandtl=1.0, cfl=0.5)
    return c.with_(**kw) if kw else c


def tgv_case(n: int = 128, ma: float = 0.1, re: float = 1600.0, prandtl: float | None = None,
             supersonic: bool = False, **kw) -> Case:
    """Taylor-Green vortex, periodic [0, 2pi]^3; mu0 = rho0 U0 L / Re, Sutherland with T_ref = p0/rho0.

    Subsonic (Sec. 4.1): rho0 = U0 = 1, p0 from the Mach number.  Supersonic (Sec. 4.2): rho0 = p0 = 1,
    U0 = sqrt(gamma) Ma.  The Prandtl number defaults to the supersonic section's 0.7; Sec. 4.1 states
    none, and the subsonic flow takes air's 0.72."""
    gamma = 1.4
    if prandtl is None:
        prandtl = 0.7 if supersonic else 0.72
    if supersonic:
        rho0, p0, u0 = 1.0, 1.0, math.sqrt(gamma) * ma
    else:
        rho0, u0 = 1.0, 1.0
        p0 = rho0 * u0 * u0 / (gamma * ma * ma)
    mu0 = rho0 * u0 * 1.0 / re
    c = Case("tgv_sup" if supersonic else "tgv", n, n, n, 2 * math.pi, 2 * math.pi, 2 * math.pi,
             gamma=gamma, mu0=mu0, prandtl=prandtl, sutherland_tref=p0 / rho0, cfl=CFL_3D, rho0=rho0,
             u0=u0, ma=ma)
    return c.with_(**kw) if kw else c


def hit_case(n: int = 256, ma_t: float = 0.5, re_lambda: float = 72.0, k0: float = 8.0,
             seed: int = 20250827, prandtl: float = 0.7, **kw) -> Case:
    """Decaying isotropic turbulence: u_rms = 1 per component, rho = 1, Ma_t = sqrt(<|u|^2>)/c.
    Taylor microscale lambda = 2/k0 for this spectrum, mu0 = rho u_rms lambda / Re_lambda."""
    gamma = 1.4
    c_snd = math.sqrt(3.0) / ma_t
    p = c_snd * c_snd / gamma
    lam = 2.0 / k0
    mu0 = 1.0 * 1.0 * lam / re_lambda
    c = Case("hit", n, n, n, 2 * math.pi, 2 * math.pi, 2 * math.pi, gamma=gamma, mu0=mu0,
             prandtl=prandtl, sutherland_tref=p / 1.0, cfl=CFL_3D, rho0=1.0, u0=1.0, ma=ma_t, seed=seed)
    return c.with_(**kw) if kw else c


# ---- analytic fields (conservative variables) -----------------------------------------------------
def _cons(gamma, rho, u, v, w, p):
    return (rho, rho * u, rho * v, rho * w, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w))


def vortex_field(case: Case, t: float = 0.0, strength: float = 5.0):
    """Shu's isentropic vortex translated by (t, t) at unit free-stream speed (exact Euler solution)."""
    g = case.gamma
    L = case.lx
    xc = (0.5 * L + t) % L
    yc = (0.5 * case.ly + t) % case.ly

    def fn(x, y, z):
        dx = (x - xc + 0.5 * L) % L - 0.5 * L
        dy = (y - yc + 0.5 * case.ly) % case.ly - 0.5 * case.ly
        r2 = dx * dx + dy * dy
        f = strength / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
        u = 1.0 - f * dy
        v = 1.0 + f * dx
        T = 1.0 - (g - 1.0) * strength ** 2 / (8.0 * g * math.pi ** 2) * np.exp(1.0 - r2)
        rho = T ** (1.0 / (g - 1.0))
        p = rho * T
        return _cons(g, rho, u, v, np.zeros_like(u), p)

    return fn


def tgv_field(case: Case):
    g = case.gamma
    rho0, u0 = case.rho0, case.u0
    if case.name == "tgv":
        p0 = rho0 * u0 * u0 / (g * case.ma ** 2)
        amp = g * case.ma ** 2 / 16.0
    else:
        p0 = 1.0
        amp = 1.0 / 16.0

    def fn(x, y, z):
        s = (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
        rho = rho0 * (1.0 + amp * s)
        p = p0 * (1.0 + amp * s)
        u = u0 * np.sin(x) * np.cos(y) * np.cos(z)
        v = -u0 * np.cos(x) * np.sin(y) * np.cos(z)
        return _cons(g, rho, u, v, np.zeros_like(u), p)

    return fn


# ---- cell averaging ------------------------------------------------------------------------------
def _gl4():
    x, w = np.polynomial.legendre.leggauss(4)
    return 0.5 * x, 0.5 * w


def cell_average(case: Case, fn, chunk_planes: int = 8):
    """q[5][N]: 4x4x4 Gauss-Legendre averages of fn over every cell."""
    xg, wg = _gl4()
    hx, hy, hz = case.h
    xc = (np.arange(case.nx) + 0.5) * hx
    yc = (np.arange(case.ny) + 0.5) * hy
    zc = (np.arange(case.nz) + 0.5) * hz
    q = np.zeros((5, case.nz, case.ny, case.nx))
    X = xc[None, None, :, None, None, None] + hx * xg[None, None, None, None, None, :]
    Y = yc[None, :, None, None, None, None] + hy * xg[None, None, None, None, :, None]
    W = wg[:, None, None] * wg[None, :, None] * wg[None, None, :]
    for k0 in range(0, case.nz, chunk_planes):
        zz = zc[k0:k0 + chunk_planes]
        Z = zz[:, None, None, None, None, None] + hz * xg[None, None, None, :, None, None]
        vals = fn(X, Y, Z)
        for v in range(5):
            arr = np.broadcast_to(vals[v], (len(zz), case.ny, case.nx, 4, 4, 4))
            q[v, k0:k0 + len(zz)] = np.einsum("kjiabc,abc->kji", arr, W)
    return q.reshape(5, -1)


def gauss_gradient(case: Case, fn, chunk_planes: int = 8):
    """g[15][N]: (average over face +d - average over face -d)/h_d, 4x4 Gauss points per face."""
    xg, wg = _gl4()
    h = case.h
    cen = [(np.arange(n) + 0.5) * hh for n, hh in zip((case.nx, case.ny, case.nz), h)]
    out = np.zeros((15, case.nz, case.ny, case.nx))
    W2 = wg[:, None] * wg[None, :]
    for k0 in range(0, case.nz, chunk_planes):
        zsl = cen[2][k0:k0 + chunk_planes]
        nzc = len(zsl)
        for d in range(3):
            t1, t2 = [e for e in range(3) if e != d]
            acc = np.zeros((5, nzc, case.ny, case.nx))
            for sgn in (-1.0, 1.0):
                coords = []
                for e in range(3):
                    c = (zsl if e == 2 else cen[e])
                    shape = [1, 1, 1, 1, 1]
                    shape[2 - e] = len(c)
                    base = c.reshape(shape)
                    if e == d:
                        coords.append(base + sgn * 0.5 * h[e])
                    else:
                        sh = [1, 1, 1, 1, 1]
                        sh[3 if e == t1 else 4] = 4
                        coords.append(base + h[e] * xg.reshape(sh))
                vals = fn(coords[0], coords[1], coords[2])
                for v in range(5):
                    arr = np.broadcast_to(vals[v], (nzc, case.ny, case.nx, 4, 4))
                    acc[v] += sgn * np.einsum("kjiab,ab->kji", arr, W2)
            out[5 * d:5 * d + 5, k0:k0 + nzc] = acc / h[d]
    return out.reshape(15, -1)


def vortex_state(case: Case, t: float = 0.0):
    fn = vortex_field(case, t)
    return cell_average(case, fn), gauss_gradient(case, fn)


def tgv_state(case: Case):
    fn = tgv_field(case)
    return cell_average(case, fn), gauss_gradient(case, fn)


def _counter_uniform(seed: int, i: np.ndarray) -> np.ndarray:
    """Uniforms in (0, 1) of a counter-based generator: the SplitMix64 output function (Steele, Lea and
    Flood, OOPSLA 2014) of seed + (i + 1) * 0x9e3779b97f4a7c15 (mod 2^64), top 53 bits plus 1/2."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (i + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return ((z >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53


def counter_normals(seed: int, start: int, count: int) -> np.ndarray:
    """Standard normals j = start .. start + count - 1: the Box-Muller pair of the uniforms 2m, 2m+1
    (m = j // 2), cos for even j and sin for odd j."""
    j = np.arange(start, start + count, dtype=np.uint64)
    m = j >> np.uint64(1)
    u1 = _counter_uniform(seed, np.uint64(2) * m)
    u2 = _counter_uniform(seed, np.uint64(2) * m + np.uint64(1))
    r = np.sqrt(-2.0 * np.log(u1))
    th = 2.0 * np.pi * u2
    return np.where((j & np.uint64(1)) == 1, r * np.sin(th), r * np.cos(th))


def hit_state(case: Case):
    """Seeded random solenoidal velocity with E(k) ~ k^4 exp(-2 k^2/k0^2), 1 <= |k| <= n/2, exact
    Fourier cell averages and cell-averaged gradients, one global scale so <|u|^2> = 3; rho = 1,
    uniform p; energy from the cell-averaged velocity.  The white noise of component c at cell m
    (x fastest) is counter_normals(seed) number c N + m."""
    n = case.nx
    assert case.ny == n and case.nz == n
    N = n ** 3
    k0 = 8.0
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    KZ, KY, KX = np.meshgrid(k1, k1, k1, indexing="ij")
    K2 = KX ** 2 + KY ** 2 + KZ ** 2
    Km = np.sqrt(K2)
    amp = np.where((Km >= 1.0) & (Km <= n / 2), Km ** 2 * np.exp(-(Km / k0) ** 2), 0.0)
    amp = np.where(Km > 0, amp / np.maximum(Km, 1.0), 0.0)  # |u_k| ~ sqrt(E(k) / k^2)
    uh = []
    for c in range(3):
        noise = counter_normals(case.seed, c * N, N).reshape(n, n, n)
        uh.append(np.fft.fftn(noise) * amp)
    kv = (KX, KY, KZ)
    kdu = sum(kv[i] * uh[i] for i in range(3))
    K2s = np.where(K2 > 0, K2, 1.0)
    uh = [uh[i] - kv[i] * kdu / K2s for i in range(3)]  # solenoidal projection
    hcell = 2 * np.pi / n
    sinc = [np.sinc(kk * hcell / (2 * np.pi)) for kk in kv]  # sin(k h/2)/(k h/2)
    cavg = sinc[0] * sinc[1] * sinc[2]
    u = [np.real(np.fft.ifftn(uh[i] * cavg)) for i in range(3)]
    scale = math.sqrt(3.0 / np.mean(u[0] ** 2 + u[1] ** 2 + u[2] ** 2))
    u = [ui * scale for ui in u]
    du = [[np.real(np.fft.ifftn(uh[i] * cavg * 1j * kv[d])) * scale for d in range(3)] for i in range(3)]
    # arrays are indexed [z][y][x] (KZ first axis)
    g = case.gamma
    c_snd = math.sqrt(3.0) / case.ma
    p = c_snd ** 2 / g
    q = np.zeros((5, n, n, n))
    q[0] = 1.0
    q[1], q[2], q[3] = u[0], u[1], u[2]
    q[4] = p / (g - 1.0) + 0.5 * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    gr = np.zeros((15, n, n, n))
    for d in range(3):
        for i in range(3):
            gr[5 * d + 1 + i] = du[i][d]
        gr[5 * d + 4] = u[0] * du[0][d] + u[1] * du[1][d] + u[2] * du[2][d]
    return q.reshape(5, -1), gr.reshape(15, -1)


def initial_state(case: Case):
    if case.name == "vortex2d":
        return vortex_state(case)
    if case.name in ("tgv", "tgv_sup"):
        return tgv_state(case)
    if case.name == "hit":
        return hit_state(case)
    raise ValueError(case.name)


def uniform_state(case: Case, rho=1.0, u=(0.3, -0.2, 0.1), p=1.0):
    """Free stream: every cell the same state, zero gradients."""
    q = np.zeros((5, case.N))
    q[:] = np.array(_cons(case.gamma, rho, u[0], u[1], u[2], p)).reshape(5, 1)
    return q, np.zeros((15, case.N))


def seeded_smooth_state(case: Case, seed: int = 1, amp: float = 0.05):
    """A smooth random periodic perturbation of a uniform state (few Fourier modes): general data for
    parity tests that exercise every term of the flux."""
    rng = np.random.Generator(np.random.PCG64(seed))
    modes = []
    for _ in range(4):
        k = rng.integers(-2, 3, size=3)
        if case.nz == 1:
            k[2] = 0
        ph = rng.uniform(0, 2 * np.pi, size=5)
        a = rng.uniform(-1, 1, size=5)
        modes.append((k, ph, a))
    L = (case.lx, case.ly, case.lz)
    base = np.array([1.0, 0.4, -0.3, 0.2, 1.0])  # rho, u, v, w, p

    def fn(x, y, z):
        prim = []
        for v in range(5):
            s = 0.0
            for k, ph, a in modes:
                s = s + a[v] * np.cos(2 * np.pi * (k[0] * x / L[0] + k[1] * y / L[1] + k[2] * z / L[2]) + ph[v])
            prim.append(base[v] + amp * s)
        return _cons(case.gamma, prim[0], prim[1], prim[2], prim[3] * (case.nz > 1), prim[4])

    return cell_average(case, fn), gauss_gradient(case, fn)
