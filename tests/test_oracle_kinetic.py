"""Pins of the oracle's gas-kinetic flux (arXiv 2508.19911, Sec. 2) against independent mathematics.

* Maxwellian moments vs brute-force velocity-space quadrature (Gauss-Hermite / -Laguerre, adaptive
  quadrature for half ranges);
* micro-slopes: the solved polynomial reproduces the requested moments (quadrature check);
* time integrals of the six time functions of eq. (flux) vs adaptive quadrature in t;
* continuous limit: equal sides give the Navier-Stokes flux with mu = tau p (Chapman-Enskog of the
  BGK model), and F_t equals the Euler-flux Jacobian times the Euler time derivative;
* the full flux vs a brute-force re-implementation in which every moment is a phase-space
  quadrature and every slope a dense linear solve.
"""
import math

import numpy as np
import pytest
from numpy.polynomial.hermite import hermgauss
from numpy.polynomial.laguerre import laggauss
from scipy import integrate
from scipy.special import gamma as Gamma

import oracle

GAMMA = 1.4
K = (5 - 3 * GAMMA) / (GAMMA - 1)  # = 2


def prim_of(W, gamma=GAMMA):
    rho = W[0]
    U, V, Wv = W[1] / rho, W[2] / rho, W[3] / rho
    p = (gamma - 1) * (W[4] - 0.5 * rho * (U * U + V * V + Wv * Wv))
    return np.array([rho, U, V, Wv, rho / (2 * p)]), p


def cons_of(rho, U, V, W, p, gamma=GAMMA):
    return np.array([rho, rho * U, rho * V, rho * W, p / (gamma - 1) + 0.5 * rho * (U * U + V * V + W * W)])


# ---------------------------------------------------------------------------------------------------
# phase-space quadrature (K = 2 internal degrees of freedom: xi^2 = s has density lam exp(-lam s))
class PhaseQuad:
    def __init__(self, prim, half=0, n_gh=24, n_gl=24, n_half=160):
        rho, U, V, W, lam = prim
        x, w = hermgauss(n_gh)
        sig = 1.0 / math.sqrt(lam)
        if half == 0:
            uu, wu = U + x * sig, w / math.sqrt(math.pi)
        else:
            # Gauss-Legendre on the half line truncated 14 standard deviations out
            lo, hi = (0.0, max(U, 0.0) + 14 * sig) if half > 0 else (min(U, 0.0) - 14 * sig, 0.0)
            xl, wl = np.polynomial.legendre.leggauss(n_half)
            uu = 0.5 * (hi - lo) * xl + 0.5 * (hi + lo)
            wu = 0.5 * (hi - lo) * wl * math.sqrt(lam / math.pi) * np.exp(-lam * (uu - U) ** 2)
        vv, wv = V + x * sig, w / math.sqrt(math.pi)
        ww, www = W + x * sig, w / math.sqrt(math.pi)
        xs, ws = laggauss(n_gl)
        ss = xs / lam
        self.u, self.v, self.w, self.s = np.meshgrid(uu, vv, ww, ss, indexing="ij")
        self.wt = (wu[:, None, None, None] * wv[None, :, None, None] * www[None, None, :, None]
                   * ws[None, None, None, :])

    def psi(self):
        return [np.ones_like(self.u), self.u, self.v, self.w,
                0.5 * (self.u ** 2 + self.v ** 2 + self.w ** 2 + self.s)]

    def mom(self, fun):
        """<fun psi> (5-vector) of the normalised Maxwellian."""
        f = fun * self.wt
        return np.array([np.sum(f * p) for p in self.psi()])

    def slope(self, a):
        return a[0] + a[1] * self.u + a[2] * self.v + a[3] * self.w + a[4] * 0.5 * (
            self.u ** 2 + self.v ** 2 + self.w ** 2 + self.s)


def brute_slope(prim, r):
    """Solve <a psi> = r with the moment matrix from quadrature."""
    Q = PhaseQuad(prim)
    ps = Q.psi()
    M = np.array([[np.sum(Q.wt * ps[i] * ps[j]) for j in range(5)] for i in range(5)])
    return np.linalg.solve(M, r)


# ---------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("half", [0, 1, -1])
@pytest.mark.parametrize("U", [-1.3, 0.0, 0.4, 2.5])
def test_moments_vs_quadrature(half, U):
    lam = 0.37
    prim = np.array([1.0, U, -0.2, 0.6, lam])
    mu, mv, mw, mxi = oracle.moments(prim, K, half, nmax=7)
    for k in range(8):
        if half == 0:
            ref = integrate.quad(lambda u: u ** k * math.sqrt(lam / math.pi) * math.exp(-lam * (u - U) ** 2),
                                 -np.inf, np.inf, epsabs=1e-15, epsrel=1e-14)[0]
        else:
            lo, hi = (0, np.inf) if half > 0 else (-np.inf, 0)
            ref = integrate.quad(lambda u: u ** k * math.sqrt(lam / math.pi) * math.exp(-lam * (u - U) ** 2),
                                 lo, hi, epsabs=1e-15, epsrel=1e-14)[0]
        scale = max(1.0, abs(U) + 3 / math.sqrt(lam)) ** k
        assert abs(mu[k] - ref) <= 1e-12 * scale, (k, mu[k], ref)
        refv = integrate.quad(lambda v: v ** k * math.sqrt(lam / math.pi) * math.exp(-lam * (v + 0.2) ** 2),
                              -np.inf, np.inf, epsabs=1e-15, epsrel=1e-14)[0]
        assert abs(mv[k] - refv) <= 1e-12 * max(1.0, 0.2 + 3 / math.sqrt(lam)) ** k


@pytest.mark.parametrize("Kdof", [0.0, 2.0, 3.0])
def test_internal_dof_moments(Kdof):
    lam = 0.8
    _, _, _, mxi = oracle.moments(np.array([1, 0, 0, 0, lam]), Kdof, 0)
    for l in range(4):
        # xi^2 ~ Gamma(K/2, 1/lam) for K internal degrees of freedom
        ref = 1.0 if (Kdof == 0 and l == 0) else (Gamma(Kdof / 2 + l) / Gamma(Kdof / 2) / lam ** l if Kdof > 0 else 0.0)
        assert abs(mxi[l] - ref) <= 1e-13 * max(1, abs(ref))


def test_micro_slope_reproduces_moments():
    rng = np.random.default_rng(3)
    for _ in range(4):
        prim = np.array([1.3, rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.2, 2.0)])
        r = rng.normal(size=5)
        a = oracle.micro_slope(prim, K, r)
        Q = PhaseQuad(prim)
        got = Q.mom(Q.slope(a))
        assert np.allclose(got, r, rtol=0, atol=1e-11 * max(1, np.abs(r).max())), (got, r)
        assert np.allclose(a, brute_slope(prim, r), rtol=1e-10, atol=1e-12)


def _time_functions(t, tau):
    e = math.exp(-t / tau)
    return [1 - e, (t + tau) * e - tau, t - tau + tau * e, e, -(tau + t) * e, -tau * e]


def _tquad(i, T, tau):
    """Adaptive quadrature of a time function, split at 50 tau so the boundary layer is resolved."""
    cut = min(T, 50.0 * tau)
    f = lambda t: _time_functions(t, tau)[i]
    r = integrate.quad(f, 0, cut, epsabs=1e-18, epsrel=1e-14, limit=200)[0]
    if cut < T:
        r += integrate.quad(f, cut, T, epsabs=1e-18, epsrel=1e-14, limit=200)[0]
    return r


@pytest.mark.parametrize("tau", [0.0, 1e-6, 0.013, 0.4, 3.0])
@pytest.mark.parametrize("T", [0.01, 0.2])
def test_time_integrals(T, tau):
    c = oracle.time_integrals(T, tau)
    assert np.all(np.isfinite(c))
    if tau == 0.0:
        assert np.allclose(c, [T, 0, 0.5 * T * T, 0, 0, 0], atol=0)
        return
    for i in range(6):
        ref = _tquad(i, T, tau)
        assert abs(c[i] - ref) <= 1e-12 * max(abs(ref), T * max(T, tau))
    # continuous limit: the g0 and g_{l,r} coefficients add up to the collisionless/equilibrium sums
    assert abs(c[0] + c[3] - T) <= 1e-14 * T
    assert abs(c[1] + c[4] + tau * T) <= 1e-13 * max(T * tau, T * T)
    assert abs(c[2] + c[5] - (0.5 * T * T - tau * T)) <= 1e-13 * max(T * T, T * tau)


# ---------------------------------------------------------------------------------------------------
def _params(mu0=0.01, prandtl=1.0):
    return oracle.make_params(8, 8, 8, 1, 1, 1, gamma=GAMMA, mu0=mu0, prandtl=prandtl, tau_c=10.0)


def _random_side(rng, base=None):
    if base is None:
        rho, U, V, W, p = 1.1, 0.3, -0.4, 0.2, 0.9
    else:
        rho, U, V, W, p = base
    Wc = cons_of(rho, U, V, W, p)
    D = rng.normal(scale=0.3, size=(3, 5))
    return np.concatenate([Wc, D.ravel()])


def euler_flux(Wc, d=0, gamma=GAMMA):
    prim, p = prim_of(Wc, gamma)
    rho, U = prim[0], prim[1:4]
    F = np.zeros(5)
    F[0] = rho * U[d]
    F[1:4] = rho * U[d] * U
    F[1 + d] += p
    F[4] = (Wc[4] + p) * U[d]
    return F


def jac(fun, W, eps=1e-6):
    J = np.zeros((5, 5))
    for j in range(5):
        dw = np.zeros(5); dw[j] = eps * max(1.0, abs(W[j]))
        J[:, j] = (fun(W + dw) - fun(W - dw)) / (2 * dw[j])
    return J


def ns_flux(Wc, D, mu, Kdof, prandtl=1.0, gamma=GAMMA):
    """Navier-Stokes flux normal to x from the BGK model's Chapman-Enskog expansion:
    stress mu (du_i/dx_j + du_j/dx_i - 2/(K+3) div u delta_ij), heat flux -mu c_p/Pr dT/dx, c_p = (K+5)/2."""
    prim, p = prim_of(Wc, gamma)
    rho, U = prim[0], prim[1:4]
    # primitive gradients: dU_i/dx_d, dT/dx_d (R = 1, T = p/rho)
    dU = np.zeros((3, 3)); dT = np.zeros(3)
    for d in range(3):
        dr, dm, dE = D[d, 0], D[d, 1:4], D[d, 4]
        dUd = (dm - U * dr) / rho
        dp = (gamma - 1) * (dE - U @ dm + 0.5 * (U @ U) * dr)
        dU[:, d] = dUd
        dT[d] = (dp - (p / rho) * dr) / rho
    div = np.trace(dU)
    sig = mu * (dU + dU.T) - mu * 2.0 / (Kdof + 3) * div * np.eye(3)
    cp = (Kdof + 5) / 2
    q = -mu * cp / prandtl * dT
    F = euler_flux(Wc, 0, gamma)
    F[1:4] -= sig[0, :]
    F[4] += -sig[0, :] @ U + q[0]
    return F


@pytest.mark.parametrize("prandtl", [1.0, 0.72])
def test_continuous_limit_is_navier_stokes(prandtl):
    rng = np.random.default_rng(11)
    P = _params(mu0=0.013, prandtl=prandtl)
    dt = 0.004
    side = _random_side(rng)
    out, dbg = oracle.point_flux(P, dt, side, side, debug=True)
    W = side[:5]
    D = side[5:].reshape(3, 5)
    prim, p = prim_of(W)
    tau = dbg["tau"]
    assert abs(tau - 0.013 / p) <= 1e-15  # no pressure jump: tau = mu / p
    Fns = ns_flux(W, D, mu=tau * p, Kdof=K, prandtl=prandtl)
    assert np.allclose(out[:5], Fns, rtol=1e-12, atol=1e-12), (out[:5], Fns)
    # F_t = dF^E/dW . W_t with the Euler time derivative W_t = -sum_d dF_d^E/dW . dW/dx_d
    Wt = -sum(jac(lambda w: euler_flux(w, d), W) @ D[d] for d in range(3))
    Ft_ref = jac(lambda w: euler_flux(w, 0), W) @ Wt
    assert np.allclose(out[5:10], Ft_ref, rtol=1e-6, atol=1e-7), (out[5:10], Ft_ref)
    # interface values: Q^n = W - tau W_t (first-order CE correction of the moments vanishes: Q^n = W)
    assert np.allclose(out[10:15], W, rtol=1e-12, atol=1e-12)
    assert np.allclose(out[15:20], Wt, rtol=1e-6, atol=1e-7)
    assert np.allclose(out[10:20], out[20:30], rtol=0, atol=0)


def brute_point_flux(P, dt, wl, wr, full_step=False):
    """Independent implementation of the interface flux: every moment by phase-space quadrature, every
    slope by a dense solve, the time integrals by adaptive quadrature of the time functions.
    full_step: also return the time-integrated flux over the whole step, Fbar(dt)."""
    gamma = P.gamma
    sides = [wl, wr]
    prim, pres, Qh, Qf, a = [], [], [], [], []
    for s in range(2):
        pr, p = prim_of(sides[s][:5], gamma)
        prim.append(pr); pres.append(p)
        Qh.append(PhaseQuad(pr, half=1 if s == 0 else -1))
        Qf.append(PhaseQuad(pr))
        a.append([brute_slope(pr, sides[s][5 + 5 * d:10 + 5 * d] / pr[0]) for d in range(3)])
    rho = [prim[0][0], prim[1][0]]
    W0 = rho[0] * Qh[0].mom(1.0) + rho[1] * Qh[1].mom(1.0)
    dW0 = [rho[0] * Qh[0].mom(Qh[0].slope(a[0][d])) + rho[1] * Qh[1].mom(Qh[1].slope(a[1][d])) for d in range(3)]
    prim0, p0 = prim_of(W0, gamma)
    Q0 = PhaseQuad(prim0)
    abar = [brute_slope(prim0, dW0[d] / prim0[0]) for d in range(3)]

    def adotu(Q, sl):
        return Q.slope(sl[0]) * Q.u + Q.slope(sl[1]) * Q.v + Q.slope(sl[2]) * Q.w

    A = [brute_slope(prim[s], -Qf[s].mom(adotu(Qf[s], a[s]))) for s in range(2)]
    Abar = brute_slope(prim0, -Q0.mom(adotu(Q0, abar)))
    jump = abs(pres[0] - pres[1]) / (pres[0] + pres[1])
    T0 = p0 / prim0[0]
    mu = P.mu0 if P.sutherland_tref <= 0 else P.mu0 * 1.4042 * (T0 / P.sutherland_tref) ** 1.5 / (T0 / P.sutherland_tref + 0.4042)
    tau = (mu / p0 if P.mu0 > 0 else P.tau_eps * dt) + P.tau_c * jump * dt
    # velocity-space pieces of eq. (flux)
    pieces = [
        (Q0, prim0[0], [1.0, adotu(Q0, abar), Q0.slope(Abar)]),
    ]
    Fp = np.zeros((6, 5)); Qp = np.zeros((6, 5))
    for i, fun in enumerate([1.0, adotu(Q0, abar), Q0.slope(Abar)]):
        Fp[i] = prim0[0] * Q0.mom(Q0.u * fun)
        Qp[i] = prim0[0] * Q0.mom(fun * np.ones_like(Q0.u))
    for s in range(2):
        Q = Qh[s]
        for i, fun in enumerate([1.0, adotu(Q, a[s]), Q.slope(A[s])]):
            Fp[3 + i] += rho[s] * Q.mom(Q.u * fun)
            Qp[3 + i] += rho[s] * Q.mom(fun * np.ones_like(Q.u))

    def tint(T):
        if tau == 0:
            return np.array([T, 0, 0.5 * T * T, 0, 0, 0])
        return np.array([_tquad(i, T, tau) for i in range(6)])

    Fb, Qb = [], []
    for T in (0.5 * dt, dt):
        c = tint(T)
        Fb.append(c @ Fp); Qb.append(c @ Qp)
    Fn = (4 * Fb[0] - Fb[1]) / dt
    Ft = 4 * (Fb[1] - 2 * Fb[0]) / dt ** 2
    Qn = (4 * Qb[0] - Qb[1]) / dt
    Qt = 4 * (Qb[1] - 2 * Qb[0]) / dt ** 2
    if P.mu0 > 0 and P.prandtl not in (0.0, 1.0):
        # heat flux of f^n in the frame of the interface equilibrium velocity
        U = prim0[1:4]
        k2 = 0.5 * U @ U
        qf = Fn[4] - U @ Fn[1:4] + k2 * Fn[0]
        qq = Qn[4] - U @ Qn[1:4] + k2 * Qn[0]
        Fn = Fn.copy(); Fn[4] += (1 / P.prandtl - 1) * (qf - U[0] * qq)
    tau0 = P.tau_c * jump * dt
    w = math.exp(-dt / tau0) if tau0 > 0 else 0.0
    eul = [-rho[s] * Qf[s].mom(adotu(Qf[s], a[s])) for s in range(2)]
    if full_step:
        return Fb[1]
    return np.concatenate([Fn, Ft, (1 - w) * Qn + w * wl[:5], (1 - w) * Qt + w * eul[0],
                           (1 - w) * Qn + w * wr[:5], (1 - w) * Qt + w * eul[1]])


@pytest.mark.parametrize("case", ["viscous_jump", "inviscid_jump", "viscous_prandtl", "strong_jump"])
def test_flux_vs_bruteforce_quadrature(case):
    rng = np.random.default_rng({"viscous_jump": 1, "inviscid_jump": 2, "viscous_prandtl": 3, "strong_jump": 4}[case])
    if case == "inviscid_jump":
        P = oracle.make_params(8, 8, 8, 1, 1, 1, gamma=GAMMA, mu0=0.0, tau_eps=0.05)
    elif case == "viscous_prandtl":
        P = oracle.make_params(8, 8, 8, 1, 1, 1, gamma=GAMMA, mu0=0.02, prandtl=0.7, sutherland_tref=0.9)
    else:
        P = oracle.make_params(8, 8, 8, 1, 1, 1, gamma=GAMMA, mu0=0.01)
    dt = 0.01
    wl = _random_side(rng, (1.0, 0.5, 0.1, -0.3, 1.0))
    if case == "strong_jump":
        wr = _random_side(rng, (0.3, -0.2, 0.4, 0.1, 0.4))
    else:
        wr = _random_side(rng, (1.04, 0.45, 0.12, -0.28, 0.97))
    got = oracle.point_flux(P, dt, wl, wr)
    ref = brute_point_flux(P, dt, wl, wr)
    scale = np.maximum(np.abs(ref), 1.0)
    err = np.abs(got - ref) / scale
    assert err.max() <= 1e-9, (np.argmax(err), got, ref)
    # the two sides differ exactly where the pressure jump switches the l/r model on
    assert not np.allclose(got[10:20], got[20:30])


@pytest.mark.parametrize("case", ["viscous", "inviscid", "strong_jump"])
def test_linearised_flux_reproduces_the_full_step_integral(case):
    """P5c: dt F^n + dt^2/2 F_t^n equals the time integral of the interface flux over the whole step,
    Fbar(dt) (Sec. 2: F^n and F_t^n are fixed by Fbar(dt/2) and Fbar(dt)).  GKS-2nd's one-stage
    update Q^{n+1} = Q^n + dt L + dt^2/2 L_t rests on this identity.  Fbar(dt) comes from the
    independent phase-space / adaptive time quadrature; Prandtl number 1 (the heat-flux correction
    acts on F^n alone)."""
    rng = np.random.default_rng({"viscous": 11, "inviscid": 12, "strong_jump": 13}[case])
    if case == "inviscid":
        P = oracle.make_params(8, 8, 8, 1, 1, 1, gamma=GAMMA, mu0=0.0, tau_eps=0.05)
    else:
        P = oracle.make_params(8, 8, 8, 1, 1, 1, gamma=GAMMA, mu0=0.01)
    dt = 0.02
    wl = _random_side(rng, (1.0, 0.5, 0.1, -0.3, 1.0))
    wr = _random_side(rng, (0.3, -0.2, 0.4, 0.1, 0.4) if case == "strong_jump" else (1.03, 0.47, 0.12, -0.28, 0.98))
    out = oracle.point_flux(P, dt, wl, wr)
    fbar = brute_point_flux(P, dt, wl, wr, full_step=True)
    lhs = dt * out[0:5] + 0.5 * dt * dt * out[5:10]
    assert np.allclose(lhs, fbar, rtol=1e-9, atol=1e-11 * np.abs(fbar).max()), (lhs, fbar)
