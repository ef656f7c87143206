/*
 * kinetic.cpp -- oracle: Maxwellian moments, micro-slopes and the gas-kinetic
 * interface flux (arXiv 2508.19911, Sec. 2).  TEST INFRASTRUCTURE ONLY.
 *
 * Everything is written in the plainest form: the distribution function of
 * eq. (flux) is assembled as a sum of (polynomial in u, v, w, xi^2) x (Maxwellian)
 * terms, and every moment is the generic expectation of a polynomial against the
 * Maxwellian's moment table.  No hand-expanded moment formula is used.
 *
 * Readings where the paper defers to its references (GKS-Xu1/2, CGKS-high-4/5):
 *  R5  interface equilibrium g0: its macroscopic state is the half-space split
 *      W0 = rho_l <psi>_{l,u>0} + rho_r <psi>_{r,u<0}, and its spatial slopes are
 *      the kinetic weighting of the one-sided slopes rho_s <a_d^s psi>_{s,half}.
 *  R6  micro-slopes a solve <a psi>_g = dW/rho; the time slopes A solve the
 *      compatibility condition <(a.u + A) psi>_g = 0 (Sec. 2).
 *  R7  face frame: cyclic permutation (the caller rotates).
 *  R8  f(Delta t) and f(Delta t/2) are integrated with the full step in both stages.
 *  R9  Prandtl number: the energy flux F^n gains (1/Pr - 1) times the heat flux of f^n in the
 *      frame of the interface equilibrium velocity; F_t is left as is.  (Correcting the two
 *      time-integrated fluxes instead adds an O(1) term to F_t whenever the interface velocity
 *      changes in time, which breaks the F_t = dF/dW W_t limit and the scheme's time order.)
 *  R10 l/r interface values: Q^s(t) = (1-w) Q^e(t) + w Q_0^s(t), w = exp(-dt/tau0),
 *      tau0 = C |p_l-p_r|/(p_l+p_r) dt; Q^e are the moments of the linearised f,
 *      Q_0^s = W^s + t (Euler time derivative of side s).
 *  Collision time (Sec. 4 opening): viscous tau = mu/p + C|dp|/(sum p) dt with mu
 *  from the interface equilibrium; inviscid tau = eps dt + C|dp|/(sum p) dt.
 */
#include "oracle_internal.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace cgkso {

/* ---- polynomials in (u, v, w, xi^2) -------------------------------------- */
struct Term {
  double c;
  int i, j, k, l;  // u^i v^j w^k (xi^2)^l
};
typedef std::vector<Term> Poly;

static Poly psi_poly(int a) {
  // psi = (1, u, v, w, (u^2+v^2+w^2+xi^2)/2)   (Sec. 2)
  switch (a) {
    case 0: return {{1.0, 0, 0, 0, 0}};
    case 1: return {{1.0, 1, 0, 0, 0}};
    case 2: return {{1.0, 0, 1, 0, 0}};
    case 3: return {{1.0, 0, 0, 1, 0}};
    default:
      return {{0.5, 2, 0, 0, 0}, {0.5, 0, 2, 0, 0}, {0.5, 0, 0, 2, 0}, {0.5, 0, 0, 0, 1}};
  }
}

// a1 + a2 u + a3 v + a4 w + a5 (u^2+v^2+w^2+xi^2)/2
static Poly slope_poly(const double* a) {
  Poly p = {{a[0], 0, 0, 0, 0}, {a[1], 1, 0, 0, 0}, {a[2], 0, 1, 0, 0}, {a[3], 0, 0, 1, 0}};
  Poly e = psi_poly(4);
  for (auto& t : e) p.push_back({t.c * a[4], t.i, t.j, t.k, t.l});
  return p;
}

static Poly mul(const Poly& p, const Poly& q) {
  Poly r;
  r.reserve(p.size() * q.size());
  for (auto& a : p)
    for (auto& b : q) r.push_back({a.c * b.c, a.i + b.i, a.j + b.j, a.k + b.k, a.l + b.l});
  return r;
}

static Poly add(const Poly& p, const Poly& q) {
  Poly r = p;
  r.insert(r.end(), q.begin(), q.end());
  return r;
}

static const Poly U1 = {{1.0, 1, 0, 0, 0}};
static const Poly V1 = {{1.0, 0, 1, 0, 0}};
static const Poly W1 = {{1.0, 0, 0, 1, 0}};
static const Poly ONE = {{1.0, 0, 0, 0, 0}};

// (a_n u + a_t1 v + a_t2 w) for the three directional slope polynomials
static Poly adotu(const double* an, const double* at1, const double* at2) {
  return add(add(mul(slope_poly(an), U1), mul(slope_poly(at1), V1)), mul(slope_poly(at2), W1));
}

/* ---- Maxwellian moments --------------------------------------------------- */
struct Moments {
  double u[12], v[12], w[12], xi[5];
};

// g = rho (lambda/pi)^{(K+3)/2} exp(-lambda((u-U)^2 + xi^2))   (Sec. 2); moments of g/rho.
static void maxwell_moments(const double prim[5], double K, int half, Moments& m) {
  const double U = prim[1], V = prim[2], W = prim[3], lam = prim[4];
  const double var = 1.0 / (2.0 * lam);
  const int n = 12;
  if (half == 0) {
    m.u[0] = 1.0;
    m.u[1] = U;
  } else {
    const double tail = std::exp(-lam * U * U) / (2.0 * std::sqrt(M_PI * lam));
    if (half > 0) {
      m.u[0] = 0.5 * std::erfc(-std::sqrt(lam) * U);
      m.u[1] = U * m.u[0] + tail;
    } else {
      m.u[0] = 0.5 * std::erfc(std::sqrt(lam) * U);
      m.u[1] = U * m.u[0] - tail;
    }
  }
  m.v[0] = 1.0;
  m.v[1] = V;
  m.w[0] = 1.0;
  m.w[1] = W;
  for (int k = 2; k < n; ++k) {
    // Gaussian recursion <x^k> = X <x^{k-1}> + (k-1) var <x^{k-2}>; also exact for a half
    // range bounded at 0 once k >= 2 (the boundary term vanishes).
    m.u[k] = U * m.u[k - 1] + (k - 1) * var * m.u[k - 2];
    m.v[k] = V * m.v[k - 1] + (k - 1) * var * m.v[k - 2];
    m.w[k] = W * m.w[k - 1] + (k - 1) * var * m.w[k - 2];
  }
  m.xi[0] = 1.0;
  for (int l = 1; l < 5; ++l) m.xi[l] = m.xi[l - 1] * (K + 2.0 * (l - 1)) * var;
}

static double expect(const Poly& p, const Moments& m) {
  double s = 0.0;
  for (auto& t : p) s += t.c * m.u[t.i] * m.v[t.j] * m.w[t.k] * m.xi[t.l];
  return s;
}

// <p psi_alpha> for alpha = 0..4
static void moment_vec(const Poly& p, const Moments& m, double out[5]) {
  for (int a = 0; a < 5; ++a) out[a] = expect(mul(p, psi_poly(a)), m);
}

/* ---- small dense solver ---------------------------------------------------- */
void solve_dense(int n, double* A, double* b, int nrhs) {
  // Gaussian elimination with partial pivoting; A is n x n row-major, b is n x nrhs.
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
      for (int k = 0; k < nrhs; ++k) std::swap(b[c * nrhs + k], b[piv * nrhs + k]);
    }
    for (int r = c + 1; r < n; ++r) {
      const double f = A[r * n + c] / A[c * n + c];
      if (f == 0.0) continue;
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      for (int k = 0; k < nrhs; ++k) b[r * nrhs + k] -= f * b[c * nrhs + k];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    for (int k = 0; k < nrhs; ++k) {
      double s = b[c * nrhs + k];
      for (int j = c + 1; j < n; ++j) s -= A[c * n + j] * b[j * nrhs + k];
      b[c * nrhs + k] = s / A[c * n + c];
    }
  }
}

// Micro-slope: the polynomial a with <a psi>_g = r, the 5x5 moment system solved directly.
static void micro_slope(const double prim[5], double K, const double r[5], double a[5]) {
  Moments m;
  maxwell_moments(prim, K, 0, m);
  double M[25], b[5];
  for (int al = 0; al < 5; ++al) {
    for (int be = 0; be < 5; ++be) M[al * 5 + be] = expect(mul(psi_poly(al), psi_poly(be)), m);
    b[al] = r[al];
  }
  solve_dense(5, M, b, 1);
  for (int i = 0; i < 5; ++i) a[i] = b[i];
}

void cons_to_prim(const double* Q, double gamma, double prim[5], double* p_out) {
  const double rho = Q[0];
  const double U = Q[1] / rho, V = Q[2] / rho, W = Q[3] / rho;
  const double p = (gamma - 1.0) * (Q[4] - 0.5 * rho * (U * U + V * V + W * W));
  prim[0] = rho;
  prim[1] = U;
  prim[2] = V;
  prim[3] = W;
  prim[4] = rho / (2.0 * p);  // lambda = rho / (2p)
  if (p_out) *p_out = p;
}

double viscosity(const cgkso_params& P, double T) {
  if (P.sutherland_tref > 0.0) {
    const double th = T / P.sutherland_tref;
    return P.mu0 * 1.4042 * std::pow(th, 1.5) / (th + 0.4042);  // Sutherland law (Sec. 4.2)
  }
  return P.mu0;
}

// Integrals over [0,T] of the six time functions multiplying g0, (abar.u) g0, Abar g0,
// g_s, (a^s.u) g_s and A^s g_s in eq. (flux).
void time_integrals(double T, double tau, double c[6]) {
  const double e = std::exp(-T / tau);  // tau = 0 gives exp(-inf) = 0
  c[0] = T - tau * (1.0 - e);
  c[1] = 2.0 * tau * tau * (1.0 - e) - tau * T * (1.0 + e);
  c[2] = 0.5 * T * T - tau * T + tau * tau * (1.0 - e);
  c[3] = tau * (1.0 - e);
  c[4] = tau * T * e - 2.0 * tau * tau * (1.0 - e);
  c[5] = -tau * tau * (1.0 - e);
}

/* ---- the interface flux ---------------------------------------------------- */
void point_flux(const cgkso_params& P, double dt, const double* wl, const double* wr, double* out,
                double* dbg) {
  const double gamma = P.gamma;
  const double K = (5.0 - 3.0 * gamma) / (gamma - 1.0);
  const double* wside[2] = {wl, wr};

  double prim[2][5], pres[2];
  Moments mh[2], mf[2];
  for (int s = 0; s < 2; ++s) {
    cons_to_prim(wside[s], gamma, prim[s], &pres[s]);
    maxwell_moments(prim[s], K, s == 0 ? +1 : -1, mh[s]);  // left: u > 0, right: u < 0
    maxwell_moments(prim[s], K, 0, mf[s]);
  }
  const double rho[2] = {prim[0][0], prim[1][0]};

  // micro-slopes of both sides in the three face-frame directions
  double a[2][3][5];
  for (int s = 0; s < 2; ++s)
    for (int d = 0; d < 3; ++d) {
      double r[5];
      for (int v = 0; v < 5; ++v) r[v] = wside[s][5 + 5 * d + v] / rho[s];
      micro_slope(prim[s], K, r, a[s][d]);
    }

  // interface equilibrium state and its slopes (R5)
  double W0[5], dW0[3][5];
  {
    double ml[5], mr[5];
    moment_vec(ONE, mh[0], ml);
    moment_vec(ONE, mh[1], mr);
    for (int v = 0; v < 5; ++v) W0[v] = rho[0] * ml[v] + rho[1] * mr[v];
    for (int d = 0; d < 3; ++d) {
      moment_vec(slope_poly(a[0][d]), mh[0], ml);
      moment_vec(slope_poly(a[1][d]), mh[1], mr);
      for (int v = 0; v < 5; ++v) dW0[d][v] = rho[0] * ml[v] + rho[1] * mr[v];
    }
  }
  double prim0[5], p0;
  cons_to_prim(W0, gamma, prim0, &p0);
  const double rho0 = prim0[0];
  Moments m0;
  maxwell_moments(prim0, K, 0, m0);
  double abar[3][5];
  for (int d = 0; d < 3; ++d) {
    double r[5];
    for (int v = 0; v < 5; ++v) r[v] = dW0[d][v] / rho0;
    micro_slope(prim0, K, r, abar[d]);
  }

  // time slopes from the compatibility condition <(a.u + A) psi> = 0 (R6)
  const Poly adu_l = adotu(a[0][0], a[0][1], a[0][2]);
  const Poly adu_r = adotu(a[1][0], a[1][1], a[1][2]);
  const Poly adu_0 = adotu(abar[0], abar[1], abar[2]);
  double A[2][5], Abar[5], eul[2][5];
  {
    double r[5];
    moment_vec(adu_l, mf[0], r);
    for (int v = 0; v < 5; ++v) {
      eul[0][v] = -rho[0] * r[v];  // Euler time derivative of side l
      r[v] = -r[v];
    }
    micro_slope(prim[0], K, r, A[0]);
    moment_vec(adu_r, mf[1], r);
    for (int v = 0; v < 5; ++v) {
      eul[1][v] = -rho[1] * r[v];
      r[v] = -r[v];
    }
    micro_slope(prim[1], K, r, A[1]);
    moment_vec(adu_0, m0, r);
    for (int v = 0; v < 5; ++v) r[v] = -r[v];
    micro_slope(prim0, K, r, Abar);
  }

  // collision time (Sec. 4 opening)
  const double jump = std::fabs(pres[0] - pres[1]) / (pres[0] + pres[1]);
  double tau;
  if (P.mu0 > 0.0) {
    const double mu = viscosity(P, p0 / rho0);
    tau = mu / p0 + P.tau_c * jump * dt;
  } else {
    tau = P.tau_eps * dt + P.tau_c * jump * dt;
  }
  const double tau0 = P.tau_c * jump * dt;

  // the nine (polynomial, Maxwellian) pieces of f, in the order of the c_i:
  // g0, (abar.u) g0, Abar g0 and, per side, g_s, (a^s.u) g_s, A^s g_s on the half space
  double Fpiece[9][5], Qpiece[9][5];
  const Poly pieces0[3] = {ONE, adu_0, slope_poly(Abar)};
  for (int i = 0; i < 3; ++i) {
    moment_vec(mul(U1, pieces0[i]), m0, Fpiece[i]);
    moment_vec(pieces0[i], m0, Qpiece[i]);
    for (int v = 0; v < 5; ++v) {
      Fpiece[i][v] *= rho0;
      Qpiece[i][v] *= rho0;
    }
  }
  const Poly pl[3] = {ONE, adu_l, slope_poly(A[0])};
  const Poly pr[3] = {ONE, adu_r, slope_poly(A[1])};
  for (int i = 0; i < 3; ++i) {
    double fl[5], fr[5], ql[5], qr[5];
    moment_vec(mul(U1, pl[i]), mh[0], fl);
    moment_vec(mul(U1, pr[i]), mh[1], fr);
    moment_vec(pl[i], mh[0], ql);
    moment_vec(pr[i], mh[1], qr);
    for (int v = 0; v < 5; ++v) {
      Fpiece[3 + i][v] = rho[0] * fl[v] + rho[1] * fr[v];
      Qpiece[3 + i][v] = rho[0] * ql[v] + rho[1] * qr[v];
    }
  }

  // time-integrated flux and interface moments over [0, T] for T = dt/2 and dt
  double Fbar[2][5], Qbar[2][5];
  const double Ts[2] = {0.5 * dt, dt};
  const bool prfix = P.mu0 > 0.0 && P.prandtl > 0.0 && P.prandtl != 1.0;
  for (int it = 0; it < 2; ++it) {
    double c[6];
    time_integrals(Ts[it], tau, c);
    for (int v = 0; v < 5; ++v) {
      double f = 0.0, q = 0.0;
      // pieces 0..2 use c1..c3; pieces 3..5 (half-space sides) use c4..c6
      for (int i = 0; i < 6; ++i) {
        f += c[i] * Fpiece[i][v];
        q += c[i] * Qpiece[i][v];
      }
      Fbar[it][v] = f;
      Qbar[it][v] = q;
    }
  }

  // time linearisation f(t) ~ f^n + t f_t^n (Sec. 2)
  double Fn[5], Ft[5], Qn[5], Qt[5];
  for (int v = 0; v < 5; ++v) {
    Fn[v] = (4.0 * Fbar[0][v] - Fbar[1][v]) / dt;
    Ft[v] = 4.0 * (Fbar[1][v] - 2.0 * Fbar[0][v]) / (dt * dt);
    Qn[v] = (4.0 * Qbar[0][v] - Qbar[1][v]) / dt;
    Qt[v] = 4.0 * (Qbar[1][v] - 2.0 * Qbar[0][v]) / (dt * dt);
  }
  if (prfix) {
    // heat flux of f^n in the frame of the interface equilibrium velocity (R9)
    const double U = prim0[1], V = prim0[2], W = prim0[3];
    const double k2 = 0.5 * (U * U + V * V + W * W);
    const double qf = Fn[4] - (U * Fn[1] + V * Fn[2] + W * Fn[3]) + k2 * Fn[0];
    const double qq = Qn[4] - (U * Qn[1] + V * Qn[2] + W * Qn[3]) + k2 * Qn[0];
    Fn[4] += (1.0 / P.prandtl - 1.0) * (qf - U * qq);
  }

  // two-sided interface values (R10)
  const double w = std::exp(-dt / tau0);  // tau0 = 0 gives w = 0
  for (int v = 0; v < 5; ++v) {
    out[v] = Fn[v];
    out[5 + v] = Ft[v];
    out[10 + v] = (1.0 - w) * Qn[v] + w * wl[v];
    out[15 + v] = (1.0 - w) * Qt[v] + w * eul[0][v];
    out[20 + v] = (1.0 - w) * Qn[v] + w * wr[v];
    out[25 + v] = (1.0 - w) * Qt[v] + w * eul[1][v];
  }

  if (dbg) {
    int o = 0;
    dbg[o++] = tau;
    dbg[o++] = tau0;
    for (int v = 0; v < 5; ++v) dbg[o++] = W0[v];
    for (int d = 0; d < 3; ++d)
      for (int v = 0; v < 5; ++v) dbg[o++] = dW0[d][v];
    for (int d = 0; d < 3; ++d)
      for (int v = 0; v < 5; ++v) dbg[o++] = abar[d][v];
    for (int v = 0; v < 5; ++v) dbg[o++] = Abar[v];
    for (int d = 0; d < 3; ++d)
      for (int v = 0; v < 5; ++v) dbg[o++] = a[0][d][v];
    for (int v = 0; v < 5; ++v) dbg[o++] = A[0][v];
    for (int d = 0; d < 3; ++d)
      for (int v = 0; v < 5; ++v) dbg[o++] = a[1][d][v];
    for (int v = 0; v < 5; ++v) dbg[o++] = A[1][v];
  }
}

}  // namespace cgkso

using namespace cgkso;

extern "C" {

void cgkso_moments(const double prim[5], double K, int half, int nmax, double* mu, double* mv,
                   double* mw, double* mxi) {
  Moments m;
  maxwell_moments(prim, K, half, m);
  for (int k = 0; k <= nmax && k < 12; ++k) {
    mu[k] = m.u[k];
    mv[k] = m.v[k];
    mw[k] = m.w[k];
  }
  for (int l = 0; l < 4; ++l) mxi[l] = m.xi[l];
}

void cgkso_micro_slope(const double prim[5], double K, const double r[5], double a[5]) {
  micro_slope(prim, K, r, a);
}

void cgkso_time_integrals(double T, double tau, double c[6]) { time_integrals(T, tau, c); }

void cgkso_point_flux(const cgkso_params* p, double dt, const double* wl, const double* wr,
                      double* out, double* dbg) {
  point_flux(*p, dt, wl, wr, out, dbg);
}

}  // extern "C"
