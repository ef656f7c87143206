// gks_flux.hpp -- gas-kinetic interface flux at one Gauss point (arXiv 2508.19911, Sec. 2).
//
// Device routine, templated on the bulk arithmetic type T (double, or float in the FP32-bulk
// form).  The Gauss-point states arrive as FP64 conservative values plus T derivatives; the
// conversion to primitive variables is done in FP64 and everything after it in T.
//
// f at the interface is eq. (flux): an equilibrium part built on g0 and the left/right parts on
// g_l (u > 0) and g_r (u < 0).  Its time integrals over [0, dt/2] and [0, dt] give the linearised
// f^n and f_t^n, whose moments are F^n, F_t^n (eq. deri-t-f) and Q^n, Q_t^n (eq. deri-t-q).  The
// coefficients of the six time functions are used in closed form (no cancellation).
//
// Readings where the paper defers to its references:
//  * g0 is the half-space split of the two sides, W0 = rho_l <psi>_{l,u>0} + rho_r <psi>_{r,u<0};
//    its slopes are the kinetic weighting rho_l <a^l psi>_{l,u>0} + rho_r <a^r psi>_{r,u<0};
//  * micro-slopes a solve <a psi> = dW/rho; time slopes A solve <(a.u + A) psi> = 0;
//  * collision time tau = mu(T0)/p0 + C |p_l-p_r|/(p_l+p_r) dt (viscous) or eps dt + C|..| dt;
//  * Prandtl number: F^n_E gains (1/Pr - 1) times the heat flux of f^n in the g0 frame;
//  * l/r interface values Q^s = (1-w) Q^e + w (W^s, Euler time derivative of side s),
//    w = exp(-dt/tau0), tau0 = C |p_l-p_r|/(p_l+p_r) dt.
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace cgks {

// Moments of a normalised Maxwellian: <u^k> (the half range for the l/r sides), <v^k>, <w^k>,
// <xi^2>, <xi^4>.
template <class T>
struct Mom {
  T u[7];
  T v[6];
  T w[6];
  T xi2, xi4;
};

// primitive state of a Maxwellian; var = 1/(2 lam) = p/rho is kept beside lam
template <class T>
struct Prim {
  T rho, U, V, W, lam, var;
};

// velocity moments by the Gaussian recursion <x^{k}> = X <x^{k-1}> + (k-1)/(2 lam) <x^{k-2}>
// (exact for a half range bounded at 0 once k >= 2); HALF = +1 (u > 0), -1 (u < 0) or 0 (full)
template <int HALF, class T>
__host__ __device__ __forceinline__ void maxwell_moments(const Prim<T>& p, T Kdof, Mom<T>& m) {
  const T var = p.var;
  if constexpr (HALF == 0) {
    m.u[0] = T(1);
    m.u[1] = p.U;
  } else {
    const T sl = dsqrt(p.lam);
    // e^{-lam U^2} / (2 sqrt(pi lam)) = e^{-lam U^2} sqrt(var / (2 pi))
    const T tail = dexp(-p.lam * p.U * p.U) * (T(0.39894228040143267794) * dsqrt(var));
    if constexpr (HALF > 0) {
      m.u[0] = T(0.5) * derfc(-sl * p.U);
      m.u[1] = p.U * m.u[0] + tail;
    } else {
      m.u[0] = T(0.5) * derfc(sl * p.U);
      m.u[1] = p.U * m.u[0] - tail;
    }
  }
#pragma unroll
  for (int k = 2; k < 7; ++k) m.u[k] = p.U * m.u[k - 1] + T(k - 1) * var * m.u[k - 2];
  m.v[0] = T(1);
  m.v[1] = p.V;
  m.w[0] = T(1);
  m.w[1] = p.W;
#pragma unroll
  for (int k = 2; k < 6; ++k) {
    m.v[k] = p.V * m.v[k - 1] + T(k - 1) * var * m.v[k - 2];
    m.w[k] = p.W * m.w[k - 1] + T(k - 1) * var * m.w[k - 2];
  }
  m.xi2 = Kdof * var;
  m.xi4 = Kdof * (Kdof + T(2)) * var * var;
}

// <u^A v^B w^C psi>, psi = (1, u, v, w, (u^2+v^2+w^2+xi^2)/2).  Products are formed as
// <u^A> (<v^B> <w^C>): the tangential pairs are few and shared by every normal order A.
template <int A, int B, int C, class T>
__host__ __device__ __forceinline__ void mvec(const Mom<T>& m, T o[5]) {
  const T vw = m.v[B] * m.w[C];
  const T b = m.u[A] * vw;
  o[0] = b;
  o[1] = m.u[A + 1] * vw;
  o[2] = m.u[A] * (m.v[B + 1] * m.w[C]);
  o[3] = m.u[A] * (m.v[B] * m.w[C + 1]);
  o[4] = T(0.5) * (m.u[A + 2] * vw + m.u[A] * (m.v[B + 2] * m.w[C]) + m.u[A] * (m.v[B] * m.w[C + 2]) +
                   b * m.xi2);
}

// <xi^2 u^A v^B w^C psi>
template <int A, int B, int C, class T>
__host__ __device__ __forceinline__ void mvec_xi(const Mom<T>& m, T o[5]) {
  T t[5];
  mvec<A, B, C>(m, t);
  const T b = t[0];
#pragma unroll
  for (int i = 0; i < 4; ++i) o[i] = m.xi2 * t[i];
  // <xi^2 psi_4> = (xi2 <(u^2+v^2+w^2) ...> + xi4 <...>)/2 = xi2 (t4 - b xi2/2) + xi4 b/2
  o[4] = m.xi2 * (t[4] - T(0.5) * b * m.xi2) + T(0.5) * m.xi4 * b;
}

// <s u^A v^B w^C psi> for the slope polynomial s = s1 + s2 u + s3 v + s4 w + s5 (u^2+v^2+w^2+xi^2)/2;
// accumulated into o with weight wgt
template <int A, int B, int C, class T>
__host__ __device__ __forceinline__ void smom_acc(const Mom<T>& m, const T s[5], T wgt, T o[5]) {
  T t0[5], t1[5], t2[5], t3[5], tu[5], tv[5], tw[5], tx[5];
  mvec<A, B, C>(m, t0);
  mvec<A + 1, B, C>(m, t1);
  mvec<A, B + 1, C>(m, t2);
  mvec<A, B, C + 1>(m, t3);
  mvec<A + 2, B, C>(m, tu);
  mvec<A, B + 2, C>(m, tv);
  mvec<A, B, C + 2>(m, tw);
  mvec_xi<A, B, C>(m, tx);
  const T h5 = T(0.5) * s[4];
#pragma unroll
  for (int i = 0; i < 5; ++i)
    o[i] += wgt * (s[0] * t0[i] + s[1] * t1[i] + s[2] * t2[i] + s[3] * t3[i] +
                   h5 * (tu[i] + tv[i] + tw[i] + tx[i]));
}

// Closed-form micro-slope solver: the polynomial a with <a psi> = R for a Maxwellian.
// ik3 = 1/(K+3).
template <class T>
__host__ __device__ __forceinline__ void micro_slope(const Prim<T>& p, T Kdof, T ik3, const T R[5],
                                                     T a[5]) {
  const T Ad = R[1] - p.U * R[0];
  const T Cd = R[2] - p.V * R[0];
  const T Dd = R[3] - p.W * R[0];
  const T q = p.U * p.U + p.V * p.V + p.W * p.W + (Kdof + T(3)) * p.var;
  const T Bd = T(2) * R[4] - q * R[0];
  a[4] = T(4) * p.lam * p.lam * (Bd - T(2) * (p.U * Ad + p.V * Cd + p.W * Dd)) * ik3;
  a[1] = T(2) * p.lam * Ad - p.U * a[4];
  a[2] = T(2) * p.lam * Cd - p.V * a[4];
  a[3] = T(2) * p.lam * Dd - p.W * a[4];
  a[0] = R[0] - p.U * a[1] - p.V * a[2] - p.W * a[3] - T(0.5) * a[4] * q;
}

struct FluxParams {
  double gamma;
  double Kdof;       // internal degrees of freedom
  double mu0;        // 0 => inviscid collision time
  double tref;       // Sutherland reference temperature (<= 0: constant mu0)
  double prandtl;
  double tau_eps, tau_c;
  double ik3;        // 1 / (Kdof + 3)
  double itref;      // 1 / tref (0 when tref <= 0)
};

inline FluxParams make_flux_params(double gamma, double mu0, double tref, double prandtl,
                                   double tau_eps, double tau_c) {
  FluxParams f;
  f.gamma = gamma;
  f.Kdof = (5.0 - 3.0 * gamma) / (gamma - 1.0);
  f.mu0 = mu0;
  f.tref = tref;
  f.prandtl = prandtl;
  f.tau_eps = tau_eps;
  f.tau_c = tau_c;
  f.ik3 = 1.0 / (f.Kdof + 3.0);
  f.itref = tref > 0.0 ? 1.0 / tref : 0.0;
  return f;
}

template <class T>
__host__ __device__ __forceinline__ T viscosity(const FluxParams& P, T Temp) {
  if (P.tref > 0.0) {
    const T th = Temp * T(P.itref);
    return T(P.mu0) * T(1.4042) * th * dsqrt(th) * drcp(th + T(0.4042));
  }
  return T(P.mu0);
}

// Interface flux at one point in the face frame (first axis = face normal).
// WL/WR: conservative values (FP64); DL/DR[d*5+v]: derivative of variable v along face-frame axis d.
// out: Fn[5], Ft[5], QLn[5], QLt[5], QRn[5], QRt[5].  NOUT = 10 skips the interface values.
template <class T, int NOUT>
__host__ __device__ __forceinline__ void gks_flux(const FluxParams& P, double dt, const double* WL,
                                         const T* DL, const double* WR, const T* DR, T* out) {
  const T K = T(P.Kdof);
  const T ik3 = T(P.ik3);
  const double gm1 = P.gamma - 1.0;
  // primitive variables in FP64
  double pres[2];
  Prim<T> pr[2];
  {
    const double* Ws[2] = {WL, WR};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const double rho = Ws[s][0];
      const double ir = 1.0 / rho;
      const double U = Ws[s][1] * ir, V = Ws[s][2] * ir, W = Ws[s][3] * ir;
      const double p = gm1 * (Ws[s][4] - 0.5 * rho * (U * U + V * V + W * W));
      pres[s] = p;
      pr[s].rho = data<T>(rho);
      pr[s].U = data<T>(U);
      pr[s].V = data<T>(V);
      pr[s].W = data<T>(W);
      pr[s].var = data<T>(p * ir);
      pr[s].lam = T(0.5) * drcp(pr[s].var);
    }
  }

  T W0[5] = {0, 0, 0, 0, 0};
  T dW0[3][5] = {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};
  T SP[6][5];  // sums over the sides of rho_s x {<u psi>, <u (a.u) psi>, <u A psi>, <psi>, <(a.u) psi>, <A psi>}
  T eul[2][5];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int v = 0; v < 5; ++v) SP[i][v] = T(0);

#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const Prim<T>& p = pr[s];
    const T* D = s ? DR : DL;
    Mom<T> mh, mf;
    if (s == 0)
      maxwell_moments<+1>(p, K, mh);
    else
      maxwell_moments<-1>(p, K, mh);
    maxwell_moments<0>(p, K, mf);
    const T irho = drcp(p.rho);
    T a[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T R[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) R[v] = D[d * 5 + v] * irho;
      micro_slope(p, K, ik3, R, a[d]);
    }
    // W0 and its slopes (half-space split)
    T t[5];
    mvec<0, 0, 0>(mh, t);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      W0[v] += p.rho * t[v];
      SP[3][v] += p.rho * t[v];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) smom_acc<0, 0, 0>(mh, a[d], p.rho, dW0[d]);
    // Euler time derivative of the side: -rho <(a.u) psi> over the full space; A from compatibility
    T E[5] = {0, 0, 0, 0, 0};
    smom_acc<1, 0, 0>(mf, a[0], T(1), E);
    smom_acc<0, 1, 0>(mf, a[1], T(1), E);
    smom_acc<0, 0, 1>(mf, a[2], T(1), E);
    T RA[5], A[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      RA[v] = -E[v];
      eul[s][v] = -p.rho * E[v];
    }
    micro_slope(p, K, ik3, RA, A);
    // the side's pieces of f on its half space
    mvec<1, 0, 0>(mh, t);
#pragma unroll
    for (int v = 0; v < 5; ++v) SP[0][v] += p.rho * t[v];
    smom_acc<2, 0, 0>(mh, a[0], p.rho, SP[1]);
    smom_acc<1, 1, 0>(mh, a[1], p.rho, SP[1]);
    smom_acc<1, 0, 1>(mh, a[2], p.rho, SP[1]);
    smom_acc<1, 0, 0>(mh, A, p.rho, SP[2]);
    // interface moments (needed for Q^n, which also enters the heat-flux correction)
    smom_acc<1, 0, 0>(mh, a[0], p.rho, SP[4]);
    smom_acc<0, 1, 0>(mh, a[1], p.rho, SP[4]);
    smom_acc<0, 0, 1>(mh, a[2], p.rho, SP[4]);
    smom_acc<0, 0, 0>(mh, A, p.rho, SP[5]);
  }

  // interface equilibrium g0
  Prim<T> p0;
  p0.rho = W0[0];
  const T ir0 = drcp(W0[0]);
  p0.U = W0[1] * ir0;
  p0.V = W0[2] * ir0;
  p0.W = W0[3] * ir0;
  const T pe = T(gm1) * (W0[4] - T(0.5) * W0[0] * (p0.U * p0.U + p0.V * p0.V + p0.W * p0.W));
  p0.var = pe * ir0;
  p0.lam = T(0.5) * drcp(p0.var);
  Mom<T> m0;
  maxwell_moments<0>(p0, K, m0);
  T ab[3][5];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T R[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) R[v] = dW0[d][v] * ir0;
    micro_slope(p0, K, ik3, R, ab[d]);
  }
  T G[6][5];  // rho0 x {<u psi>, <u (ab.u) psi>, <u Ab psi>, <psi>, <(ab.u) psi>, <Ab psi>}
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int v = 0; v < 5; ++v) G[i][v] = T(0);
  T Ab[5];
  {
    T E[5] = {0, 0, 0, 0, 0};
    smom_acc<1, 0, 0>(m0, ab[0], T(1), E);
    smom_acc<0, 1, 0>(m0, ab[1], T(1), E);
    smom_acc<0, 0, 1>(m0, ab[2], T(1), E);
    T RA[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      RA[v] = -E[v];
      G[4][v] = p0.rho * E[v];
      G[3][v] = W0[v];
    }
    micro_slope(p0, K, ik3, RA, Ab);
  }
  {
    T t[5];
    mvec<1, 0, 0>(m0, t);
#pragma unroll
    for (int v = 0; v < 5; ++v) G[0][v] = p0.rho * t[v];
  }
  smom_acc<2, 0, 0>(m0, ab[0], p0.rho, G[1]);
  smom_acc<1, 1, 0>(m0, ab[1], p0.rho, G[1]);
  smom_acc<1, 0, 1>(m0, ab[2], p0.rho, G[1]);
  smom_acc<1, 0, 0>(m0, Ab, p0.rho, G[2]);
  smom_acc<0, 0, 0>(m0, Ab, p0.rho, G[5]);

  // collision time (Sec. 4 opening)
  // relative pressure jump |p_l - p_r| / (p_l + p_r): the difference in FP64, the ratio in T
  const T jump = data<T>(fabs(pres[0] - pres[1])) * drcp(data<T>(pres[0] + pres[1]));
  const T Dt = T(dt);
  T tau;
  if (P.mu0 > 0.0)
    tau = viscosity(P, p0.var) * drcp(pe) + T(P.tau_c) * jump * Dt;
  else
    tau = (T(P.tau_eps) + T(P.tau_c) * jump) * Dt;

  // closed-form coefficients of f^n and f_t^n (time integrals over [0,dt/2] and [0,dt] combined)
  const T iDt = T(1.0 / dt);
  const T om = -dexpm1(T(-0.5) * Dt * drcp(tau));  // 1 - e^{-dt/(2 tau)}; tau = 0 gives 1
  const T e1 = T(1) - om;
  const T r = tau * iDt;
  const T rq = r * om * (T(3) - e1);
  T cn[6], ct[6];
  cn[0] = T(1) - rq;
  cn[1] = T(2) * tau * rq + tau * (e1 * e1 - T(2) * e1 - T(1));
  cn[2] = tau * (rq - T(1));
  cn[3] = rq;
  cn[4] = tau * e1 * (T(2) - e1) - T(2) * tau * rq;
  cn[5] = -tau * rq;
  const T rom = r * om;
  ct[0] = T(4) * rom * om * iDt;
  ct[1] = T(4) * rom * (e1 - T(2) * rom);
  ct[2] = T(1) - T(4) * rom * rom;
  ct[3] = -ct[0];
  ct[4] = -ct[1];
  ct[5] = T(4) * rom * rom;

  T Fn[5], Ft[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    Fn[v] = cn[0] * G[0][v] + cn[1] * G[1][v] + cn[2] * G[2][v] + cn[3] * SP[0][v] +
            cn[4] * SP[1][v] + cn[5] * SP[2][v];
    Ft[v] = ct[0] * G[0][v] + ct[1] * G[1][v] + ct[2] * G[2][v] + ct[3] * SP[0][v] +
            ct[4] * SP[1][v] + ct[5] * SP[2][v];
  }
  T Qn[5];
#pragma unroll
  for (int v = 0; v < 5; ++v)
    Qn[v] = cn[0] * G[3][v] + cn[1] * G[4][v] + cn[2] * G[5][v] + cn[3] * SP[3][v] +
            cn[4] * SP[4][v] + cn[5] * SP[5][v];
  if (P.mu0 > 0.0 && P.prandtl > 0.0 && P.prandtl != 1.0) {
    const T k2 = T(0.5) * (p0.U * p0.U + p0.V * p0.V + p0.W * p0.W);
    const T qf = Fn[4] - (p0.U * Fn[1] + p0.V * Fn[2] + p0.W * Fn[3]) + k2 * Fn[0];
    const T qq = Qn[4] - (p0.U * Qn[1] + p0.V * Qn[2] + p0.W * Qn[3]) + k2 * Qn[0];
    Fn[4] += T(1.0 / P.prandtl - 1.0) * (qf - p0.U * qq);
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    out[v] = Fn[v];
    out[5 + v] = Ft[v];
  }
  if constexpr (NOUT > 10) {
    T Qt[5];
#pragma unroll
    for (int v = 0; v < 5; ++v)
      Qt[v] = ct[0] * G[3][v] + ct[1] * G[4][v] + ct[2] * G[5][v] + ct[3] * SP[3][v] +
              ct[4] * SP[4][v] + ct[5] * SP[5][v];
    // w = e^{-dt/tau0}, tau0 = C jump dt; a zero jump gives w = 0
    const T w = dexp(-drcp(T(P.tau_c) * jump));
    const T w1 = T(1) - w;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      out[10 + v] = w1 * Qn[v] + w * data<T>(WL[v]);
      out[15 + v] = w1 * Qt[v] + w * eul[0][v];
      out[20 + v] = w1 * Qn[v] + w * data<T>(WR[v]);
      out[25 + v] = w1 * Qt[v] + w * eul[1][v];
    }
  }
}

}  // namespace cgks
